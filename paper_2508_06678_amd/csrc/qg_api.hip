// Host runtime of the QG step: parameter validation, per-size plans, the
// workspace layout, the phase sequences of a step / the adjoint / the
// diagnostics, hipGraph capture and replay, and the C ABI of include/qg.h.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "qg_fft.hpp"
#include "qg_internal.hpp"
#include "../../include/qg.h"

namespace qg {

static thread_local std::string g_err;

// A roctx range over the host span of an entry point (visible in rocprofv3
// --marker-trace timelines beside the kernels it enqueues).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

static int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define QG_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(QG_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
static int ilog2(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }
static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ------------------------------------------------------------ validation
static int validate(const qg_params& p, int idx) {
  auto bad = [&](int code, const char* what) {
    char buf[256];
    snprintf(buf, sizeof buf, "member %d: %s", idx, what);
    return fail(code, buf);
  };
  if (p.nx <= 0 || p.ny <= 0) return bad(QG_EINVAL, "grid sizes must be positive");
  if (!is_pow2(p.nx) || !is_pow2(p.ny) || p.nx < 32 || p.ny < 32 || p.nx > 4096 || p.ny > 4096)
    return bad(QG_EUNSUPPORTED, "nx and ny must be powers of two in [32, 4096]");
  if (!(p.lx > 0) || !(p.ly > 0)) return bad(QG_EINVAL, "lx and ly must be positive");
  const double dx = p.lx / p.nx, dy = p.ly / p.ny;
  if (std::fabs(dx - dy) > 1e-12 * dx) return bad(QG_EUNSUPPORTED, "dx must equal dy");
  if (!(p.dt > 0) || !std::isfinite(p.dt)) return bad(QG_EINVAL, "dt must be positive and finite");
  if (p.closure < 0 || p.closure > 4) return bad(QG_EINVAL, "unknown closure");
  if (p.precision != 32 && p.precision != 64) return bad(QG_EINVAL, "precision must be 32 or 64");
  if (p.clip_mode != 0 && p.clip_mode != 1) return bad(QG_EINVAL, "clip_mode must be 0 or 1");
  if (p.clip_mode == 1 && (p.nx < 64 || (p.precision == 64 && p.nx > 2048)))
    return bad(QG_EUNSUPPORTED, "pointwise clipping (clip_mode 1) needs nx >= 64 (and nx <= 2048 in 64-bit runs)");
  if (p.closure >= 3) {
    const double r = p.test_ratio;
    if (!(r == 2.0 || r == 3.0 || r == 4.0)) return bad(QG_EUNSUPPORTED, "test_ratio must be 2, 3 or 4");
  }
  if (!std::isfinite(p.beta) || !std::isfinite(p.mu) || !std::isfinite(p.u_in) || !std::isfinite(p.v_in) ||
      !std::isfinite(p.c) || !(p.sponge_sigma >= 0) || !std::isfinite(p.sponge_sigma))
    return bad(QG_EINVAL, "non-finite or negative parameter");
  if (p.eta == 0.0 || std::isnan(p.eta)) return bad(QG_EINVAL, "eta must be positive (or inf to disable)");
  if (p.eta < 0) return bad(QG_EINVAL, "eta must be positive (or inf to disable)");
  if (p.fp64_lowk < 0) return bad(QG_EINVAL, "fp64_lowk must be >= 0");
  if (p.scheme != QG_SCHEME_RK4 && p.scheme != QG_SCHEME_AB2CN) return bad(QG_EINVAL, "unknown scheme");
  if (p.scheme == QG_SCHEME_AB2CN) {
    // the penalization and sponge passes run on the field-parallel kernels only
    if (p.nx < 64) return bad(QG_EUNSUPPORTED, "the AB2CN scheme needs nx >= 64");
    if (p.precision == 64 && (p.nx > 2048 || p.ny > 2048))
      return bad(QG_EUNSUPPORTED, "the AB2CN scheme in 64-bit runs needs nx, ny <= 2048");
    // explicit penalization is stable only for eta > dt (Sec. II-E)
    if (!(p.eta > p.dt)) return bad(QG_EINVAL, "the AB2CN scheme needs eta > dt (explicit penalization)");
  }
  return QG_OK;
}

// ------------------------------------------------------------ plans
struct Group {
  int nx, ny, lognx, logny, closure;
  int scheme;                    // QG_SCHEME_*
  int clip;                      // clip_mode of the dynamic closures
  bool dbl;
  int kxn, myh, kyn, W, logW, kxp, RP, logRP;
  int kxn_f, myh_f, kyn_f, kxp_f;
  int Wi, logWi, mfp, mfp_f;     // column-inverse strip width, MF row pitch
  int nstrips, nstrips_f, nrow, nspec;
  int m0, count;                 // slice of the device member table
  std::vector<int> users;        // caller indices of the members
  RegionLayout L;
  long long region_bytes;
  char* region0;                 // first member region
  void* twx;
  void* twy;
  long long o_twx, o_twy;        // offsets in the global area
  void* twx1;                    // the same for pass schedule 1
  void* twy1;
  long long o_twx1, o_twy1;
  void* twx2 = nullptr;          // the row and column tables of pass schedule 2
  void* twy2 = nullptr;
  long long o_twx2 = 0, o_twy2 = 0;
  int rsch, csch;                // pass schedules of the row / column compile-time engines
  int rpb;                       // row pairs per block of the step's row pass
  int rwv;                       // wave-synchronous row transforms (and the FP32 1024-point forward columns of the dynamic closures)
};

// Strip width W of the column passes: W * ny <= one tile, at least 64
// threads per block.  Changes the launch geometry only (the workspace is
// sized for any W <= 16).
static int max_width(const Group& g) { return std::max(1, std::min(16, col_tile_elems(g.dbl) / g.ny)); }
static int min_width(const Group& g) { return std::max(1, std::min(max_width(g), 512 / g.ny)); }

static void set_inv_width(Group& g, int Wi) {
  g.Wi = Wi;
  g.logWi = ilog2(Wi);
}

static void set_width(Group& g, int W) {
  g.W = W;
  g.logW = ilog2(W);
  g.kxp = (g.kxn + W - 1) / W * W;
  g.kxp_f = (g.kxn_f + W - 1) / W * W;
  g.nstrips = (g.kxn + W - 1) / W;
  g.nstrips_f = (g.kxn_f + W - 1) / W;
}

// Default: the widest strip that still gives every size group at least 512
// column blocks (a 1024^2 member alone gets W = 1; eight get W = 4).
static int default_width(const Group& g, int count) {
  int W = max_width(g);
  while (W > min_width(g) && (long long)((g.kxn + W - 1) / W) * count < 512) W >>= 1;
  return W;
}
// column-inverse: one block per (strip, field), so wider strips keep enough
// blocks; wide strips make the scattered MF row stores longer.
static int default_inv_width(const Group& g, int count) {
  int W = max_width(g);
  while (W > min_width(g) && (long long)((g.kxn + W - 1) / W) * count * rhs_fields(g.closure) < 1024) W >>= 1;
  return W;
}

static void plan_sizes(Group& g, int adjK) {
  const int cs = g.dbl ? 16 : 8, rs = g.dbl ? 8 : 4;
  g.lognx = ilog2(g.nx);
  g.logny = ilog2(g.ny);
  g.kxn = (g.nx - 1) / 3 + 1;
  g.myh = (g.ny - 1) / 3;
  g.kyn = 2 * g.myh + 1;
  g.kxn_f = g.nx / 2;
  g.myh_f = g.ny / 2 - 1;
  g.kyn_f = g.ny - 1;
  set_width(g, max_width(g));
  set_inv_width(g, max_width(g));
  const int kxp16 = (g.kxn + 15) / 16 * 16, kxpf16 = (g.kxn_f + 15) / 16 * 16;
  g.mfp = kxp16;
  g.mfp_f = kxpf16;
  g.RP = std::max(1, std::min(2048 / g.nx, g.ny / 2));
  g.logRP = ilog2(g.RP);
  g.nrow = g.ny / (2 * g.RP);
  g.nspec = (g.kxn * g.kyn + 255) / 256;

  const int cl = g.closure;
  // at least the 5 fields and 4 products of the SGS-analysis pass
  int F = std::max({rhs_fields(cl), 5});
  int Pn = std::max({rhs_products(cl), 4});
  if (adjK > 0) {
    // the adjoint pass's fields and products; the dynamic closures run the
    // two passes of a stage in one launch (both sets side by side)
    const int lv = dynamic_closure(cl) ? 2 : 1;
    F = std::max(F, lv * ((smag_family(cl) ? 6 : 4) + 3));
    Pn = std::max(Pn, lv * (smag_family(cl) ? 6 : 4));
  }
  const long long spec = (long long)g.kxn * g.kyn * cs;
  const long long mf = std::max((long long)F * g.ny * kxp16, 2LL * g.ny * kxpf16) * cs;
  const long long mp = std::max((long long)Pn * g.ny * kxp16, 1LL * g.ny * kxpf16) * cs;
  long long o = 0;
  auto take = [&](long long b) { long long r = o; o += align256(b); return r; };
  RegionLayout& L = g.L;
  L.wn = take(spec);
  L.acc = take(spec);
  L.x = take(spec);
  if (g.scheme == QG_SCHEME_AB2CN) {
    L.ab_pen = take(spec);
    L.ab_hist = take(spec);
    L.ab_wss = take(spec);
  } else {
    L.ab_pen = L.ab_hist = L.ab_wss = -1;
  }
  L.jsp = take(spec);
  L.qsp = take(spec);
  L.chih = take((long long)g.kxn_f * g.kyn_f * cs);
  L.mf = take(mf);
  L.mp = take(mp);
  L.phys = take(6LL * g.nx * g.ny * rs);
  L.part = take((long long)std::max(g.kxn, g.kxn_f) * 2 * 8);   // one slot per strip at W = 1
  L.coef = take(32 * 8);
  // row-block partial sums (at most ny/2 blocks, 5 values each), then the
  // spectral partial sums of the diagnostics
  L.dpart = take((long long)(5 * (g.ny / 2) + 2 * g.nspec + 8) * 8);
  if (adjK > 0) {
    L.adj_lam = take(spec);
    L.adj_lacc = take(spec);   // LW
    L.adj_lk = take(spec);     // LK
    L.adj_store = take((long long)align256(spec) * (4LL * adjK + 1));  // LS, then 4 stage inputs per step
  } else {
    L.adj_lam = L.adj_lacc = L.adj_lk = L.adj_store = -1;
  }
  if (g.clip == 1) {
    L.clip_h = take(spec);
    L.clip_m = take(spec);
  } else {
    L.clip_h = L.clip_m = -1;
  }
  if (adjK > 0 && dynamic_closure(cl)) {
    L.adj_hmq = take((long long)align256(spec) * 3 * 4 * adjK);   // H, M, Q of every stage of a segment
    L.adj_cs = take(3LL * 4 * adjK * 8);                          // C, <HM>, <M^2> of every stage
    L.adj_a = take(spec);
    L.adj_b = take(spec);
    L.adj_e = take(spec);
  } else {
    L.adj_hmq = L.adj_cs = L.adj_a = L.adj_b = L.adj_e = -1;
  }
  L.total = o;
  g.region_bytes = o;
}

struct Handle {
  std::vector<qg_params> params;
  std::vector<Group> groups;
  std::vector<int> member_group;   // caller index -> group
  std::vector<long long> omega_off;
  long long total_points = 0;
  long long total_bytes = 0;       // bytes of one flat field of all members
  int adjK = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  MemberDev* mem_dev = nullptr;
  std::map<int, hipGraphExec_t> graphs;   // steps per replay -> executable graph
  std::map<int, hipGraphExec_t> adj_graphs;  // adjoint segment length -> executable graph
  hipStream_t graph_stream = nullptr;      // capture/replay stream (the caller's may be the null stream)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // one capture stream and join event per size group beyond the first: the
  // groups' step chains become parallel branches of the graph
  std::vector<hipStream_t> branch_streams;
  std::vector<hipEvent_t> branch_events;
  hipEvent_t ev_fork = nullptr;
  std::vector<MemberDev> table;            // host copy of the device member table
};

static bool same_group(const qg_params& a, const qg_params& b) {
  return a.nx == b.nx && a.ny == b.ny && a.precision == b.precision && a.closure == b.closure &&
         a.scheme == b.scheme && a.clip_mode == b.clip_mode;
}

// Everything qg_workspace_bytes and qg_init share: grouping, layout.
static int build_layout(const qg_params* params, int n, int adjK, Handle& h) {
  if (!params || n <= 0) return fail(QG_EINVAL, "need at least one member");
  if (adjK < 0) return fail(QG_EINVAL, "adj_segment_k must be >= 0");
  for (int i = 0; i < n; ++i) {
    int rc = validate(params[i], i);
    if (rc) return rc;
  }
  h.params.assign(params, params + n);
  h.adjK = adjK;
  h.member_group.assign(n, -1);
  h.omega_off.assign(n, 0);
  long long off = 0;
  for (int i = 0; i < n; ++i) {
    h.omega_off[i] = off;
    off += (long long)params[i].nx * params[i].ny * (params[i].precision == 64 ? 8 : 4);
    h.total_points += (long long)params[i].nx * params[i].ny;
  }
  h.total_bytes = off;
  for (int i = 0; i < n; ++i) {
    int gi = -1;
    for (size_t k = 0; k < h.groups.size(); ++k)
      if (same_group(params[h.groups[k].users[0]], params[i])) gi = (int)k;
    if (gi < 0) {
      Group g{};
      g.nx = params[i].nx;
      g.ny = params[i].ny;
      g.closure = params[i].closure;
      g.scheme = params[i].scheme;
      g.clip = dynamic_closure(params[i].closure) ? params[i].clip_mode : 0;
      g.dbl = params[i].precision == 64;
      plan_sizes(g, adjK);
      h.groups.push_back(g);
      gi = (int)h.groups.size() - 1;
    }
    h.groups[gi].users.push_back(i);
    h.member_group[i] = gi;
  }
  for (auto& g : h.groups) {
    set_width(g, default_width(g, (int)g.users.size()));
    set_inv_width(g, default_inv_width(g, (int)g.users.size()));
  }
  // global area: member table, twiddles; then group regions
  long long o = align256((long long)n * sizeof(MemberDev));
  for (auto& g : h.groups) {
    const int cs = g.dbl ? 16 : 8;
    g.o_twx = o; o += align256((long long)g.nx * cs);
    g.o_twy = o; o += align256((long long)g.ny * cs);
    g.o_twx1 = o; o += align256((long long)g.nx * cs);
    g.o_twy1 = o; o += align256((long long)g.ny * cs);
    g.o_twx2 = o; o += align256((long long)g.nx * cs);
    g.o_twy2 = o; o += align256((long long)g.ny * cs);
    g.rsch = g.csch = g.rwv = 0;
    g.rpb = 1;
  }
  int m0 = 0;
  for (auto& g : h.groups) {
    g.m0 = m0;
    g.count = (int)g.users.size();
    m0 += g.count;
    g.region0 = reinterpret_cast<char*>(o);   // offset for now
    o += g.region_bytes * g.count;
  }
  h.ws_bytes = (size_t)o;
  return QG_OK;
}

// Twiddles exp(-2 pi i m / n), m in [0, n), from the octant-reduced angle in
// long double so that every entry is correctly rounded or nearly so.
static void twiddles(int n, std::vector<long double>& re, std::vector<long double>& im) {
  re.resize(n);
  im.resize(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int m = 0; m < n; ++m) {
    // reduce m/n to [0, 1/8] with symmetries of cos/sin
    long long a = (long long)m * 8;           // angle in units of 2 pi / (8 n)
    long long oct = a / n;                    // octant 0..7
    long long r = a - oct * n;                // remainder in [0, n)
    long double t = (long double)r / (long double)n;   // fraction of the octant
    long double c, s;
    // angle within octant: theta = (oct + t) * pi / 4
    long double th = t * pi / 4.0L;
    long double ct = cosl(th), st = sinl(th);
    long double cq = cosl(pi / 4.0L - th), sq = sinl(pi / 4.0L - th);
    switch (oct) {
      case 0: c = ct; s = st; break;
      case 1: c = sq; s = cq; break;
      case 2: c = -st; s = ct; break;
      case 3: c = -cq; s = sq; break;
      case 4: c = -ct; s = -st; break;
      case 5: c = -sq; s = -cq; break;
      case 6: c = st; s = -ct; break;
      default: c = cq; s = -sq; break;
    }
    re[m] = c;
    im[m] = -s;   // exp(-i theta)
  }
}

// Per-pass table of the FFT engines: the pass with sub-transform length
// Ns >= 8 and radix R (8 while three factors of two remain, then 4 or 2)
// keeps exp(-2 pi i t k / (Ns R)) at (Ns - 8) + k (R - 1) + t - 1, taken
// from the full table (index t k N / (Ns R)).  n - 8 entries; the rest of
// the n slots is zero.
// Per-pass table of the transforms of length n under pass schedule sch (see
// qg_fft.hpp): the pass with sub-length ns and radix r keeps
// exp(-2 pi i t k / (ns r)) at (ns - 8) + k (r - 1) + (t - 1).
static void pass_twiddles(int n, int sch, const std::vector<long double>& fre, const std::vector<long double>& fim,
                          std::vector<long double>& re, std::vector<long double>& im) {
  re.assign(n, 0.0L);
  im.assign(n, 0.0L);
  const int logn = ilog2(n);
  for (int logns = 3; logns < logn;) {
    const int ns = 1 << logns;
    const int r = 1 << pass_log_radix(logn, logns, sch);
    const int stride = n / (ns * r);
    for (int k = 0; k < ns; ++k)
      for (int t = 1; t < r; ++t) {
        const int o = (ns - 8) + k * (r - 1) + (t - 1);
        re[o] = fre[(long long)t * k * stride];
        im[o] = fim[(long long)t * k * stride];
      }
    logns += pass_log_radix(logn, logns, sch);
  }
}

// ------------------------------------------------------------ phases
static Phase base_phase(const Handle& h, const Group& g) {
  Phase P{};
  P.mem = h.mem_dev;
  P.m0 = g.m0;
  P.nx = g.nx; P.ny = g.ny; P.lognx = g.lognx; P.logny = g.logny;
  P.kxn = g.kxn; P.myh = g.myh; P.kyn = g.kyn; P.kxp = g.kxp;
  P.W = g.W; P.logW = g.logW; P.RP = g.RP; P.logRP = g.logRP;
  P.Wi = g.Wi; P.logWi = g.logWi; P.mfp = g.mfp;
  P.nf = 1;
  P.stage = 0;
  P.nparts = g.nstrips;
  P.o_mf = g.L.mf; P.o_mp = g.L.mp; P.o_phys = g.L.phys;
  P.o_part = g.L.part; P.o_coef = g.L.coef; P.o_dpart = g.L.dpart;
  P.twx = g.twx; P.twy = g.twy;
  P.twx1 = g.twx1; P.twy1 = g.twy1; P.twx2 = g.twx2; P.twy2 = g.twy2;
  P.rsch = g.rsch; P.csch = g.csch; P.rpb = g.rpb; P.rwv = g.rwv;
  P.cwv = g.rwv;   // one choice for the wave-synchronous rows and columns
  return P;
}

static Phase full_set(Phase P, const Group& g) {
  P.kxn = g.kxn_f; P.myh = g.myh_f; P.kyn = g.kyn_f; P.kxp = g.kxp_f; P.mfp = g.mfp_f;
  P.nparts = g.nstrips_f;
  return P;
}

#define QG_LAUNCH(call)                                                               \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(QG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e_));   \
  } while (0)

static int run_entry(const Handle& h, const Group& g, const void* src, long long o_out, hipStream_t s) {
  Phase P = base_phase(h, g);
  P.user_in = src;
  P.o_out = o_out;
  QG_LAUNCH(launch_row(g.dbl, OP_ENTRY, 0, P, g.count, s));
  QG_LAUNCH(launch_colfwd(g.dbl, OP_ENTRY, 0, P, g.count, s));
  return QG_OK;
}

static int run_exit(const Handle& h, const Group& g, long long o_in, void* dst, hipStream_t s) {
  Phase P = base_phase(h, g);
  P.o_in = o_in;
  P.nf = 1;
  P.user = dst;
  QG_LAUNCH(launch_colinv(g.dbl, OP_EXIT, 0, P, g.count, s));
  QG_LAUNCH(launch_row(g.dbl, OP_EXIT, 0, P, g.count, s));
  return QG_OK;
}

// Pointwise clip (clip_mode 1): the dynamic column pass keeps the stage's
// H and M spectra (clip_keep on its phase), this pass takes them to the grid
// and sums max(H, 0) M and M^2 per row pair into dpart, and the coefficient
// is formed from those sums (clip_sums on the combine's phase).
static void clip_keep(const Group& g, Phase& P) {
  if (g.clip != 1) return;
  P.adj_dyn = 1;
  P.o_h = g.L.clip_h;
  P.o_m = g.L.clip_m;
}
static int run_clip_pass(const Handle& h, const Group& g, hipStream_t st) {
  if (g.clip != 1) return QG_OK;
  Phase P = base_phase(h, g);
  P.nf = 2;
  P.o_h = g.L.clip_h;
  P.o_m = g.L.clip_m;
  QG_LAUNCH(launch_colinv(g.dbl, OP_CLIPF, 0, P, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_CLIPF, 0, P, g.count, st));
  return QG_OK;
}
static void clip_sums(const Group& g, Phase& Q) {
  if (g.clip != 1) return;
  Q.o_part = g.L.dpart;
  Q.nparts = g.ny / 2;
}

// Profiling runs (qg_profile_steps): every launch of one kind of phase
// kernel gets a pair of HIP events bound to its dispatch.  Kinds: 0 the
// right-hand side's column-inverse pass, 1 its row pass, 2 its
// column-forward pass, 3 the dynamic combine, 4-6 the same three passes of
// the B sub-step.
struct ProfState {
  int kind;
  std::vector<hipEvent_t> ev;   // begin, end of launch 0, then launch 1, ...
  int used;
};
static thread_local ProfState* g_prof = nullptr;
// Stamp runs (qg_stamp_steps, stamp builds): the caller's stamp buffer
static thread_local unsigned long long* g_stamps = nullptr;

static Phase timed(Phase P, int kind) {
  P.ev0 = P.ev1 = nullptr;
  P.stamps = g_stamps;
  if (g_prof && g_prof->kind == kind && 2 * (g_prof->used + 1) <= (int)g_prof->ev.size()) {
    P.ev0 = g_prof->ev[2 * g_prof->used];
    P.ev1 = g_prof->ev[2 * g_prof->used + 1];
    ++g_prof->used;
  }
  return P;
}

// Where the adjoint's segment recompute keeps a dynamic stage's H, M, Q
// and (C, <HM>, <M^2>) (byte offsets in the member region).
struct StageStore {
  long long h, m, q, cs;
};

// One RK4 stage (s = 1..4): colinv -> row -> colfwd (-> combine for dynamic).
static int run_stage(const Handle& h, const Group& g, int s, hipStream_t st, const StageStore* keep = nullptr) {
  Phase P = base_phase(h, g);
  const int cl = g.closure;
  P.stage = s;
  P.nf = rhs_fields(cl);
  P.o_in = s == 1 ? g.L.wn : g.L.x;
  QG_LAUNCH(launch_colinv(g.dbl, OP_RHS, cl, timed(P, 0), g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_RHS, cl, timed(P, 1), g.count, st));
  if (!dynamic_closure(cl)) {
    P.o_in = g.L.x;
    P.o_in2 = g.L.wn;
    P.o_aux = g.L.acc;
    QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, timed(P, 2), g.count, st));
  } else {
    P.o_out = g.L.jsp;
    P.o_aux = keep ? keep->q : g.L.qsp;
    if (keep) {
      P.adj_dyn = 1;
      P.o_h = keep->h;
      P.o_m = keep->m;
    }
    clip_keep(g, P);
    QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, timed(P, 2), g.count, st));
    int rc = run_clip_pass(h, g, st);
    if (rc) return rc;
    Phase Q = base_phase(h, g);
    Q.stage = s;
    Q.o_in = g.L.x;
    Q.o_in2 = g.L.wn;
    Q.o_out = g.L.jsp;
    Q.o_aux = P.o_aux;
    Q.o_mp = g.L.acc;
    if (keep) {
      Q.adj_dyn = 1;
      Q.o_cs = keep->cs;
    }
    clip_sums(g, Q);
    QG_LAUNCH(launch_combine(g.dbl, OP_RHS, timed(Q, 3), g.count, st));
  }
  return QG_OK;
}

static int run_b(const Handle& h, const Group& g, hipStream_t st) {
  Phase P = base_phase(h, g);
  P.o_in = g.L.x;
  P.nf = 3;
  QG_LAUNCH(launch_colinv(g.dbl, OP_B, 0, timed(P, 4), g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_B, 0, timed(P, 5), g.count, st));
  P.o_out = g.L.wn;
  QG_LAUNCH(launch_colfwd(g.dbl, OP_B, 0, timed(P, 6), g.count, st));
  return QG_OK;
}

// One step of the paper's scheme (Sec. II-E, Eq. 4) for an AB2CN group:
// D curl(chi u^t) (penalization pass), the nonlinear terms at omega^t and
// the AB2CN update to omega* (right-hand-side pass), the AB2 sponge from
// omega* and omega** back to w_n (sponge pass), then omega** <- omega*.
static int run_ab2cn_step(const Handle& h, const Group& g, hipStream_t st) {
  const int cl = g.closure;
  // penalization: u', v' at omega^t -> chi (U + u'), chi (V + v') -> curl
  Phase Pp = base_phase(h, g);
  Pp.nf = 2;
  Pp.o_in = g.L.wn;
  QG_LAUNCH(launch_colinv(g.dbl, OP_B, 0, Pp, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_PEN, 0, Pp, g.count, st));
  Pp.o_out = g.L.ab_pen;
  QG_LAUNCH(launch_colfwd(g.dbl, OP_PEN, 0, Pp, g.count, st));
  // nonlinear terms and the CN / AB2 update: omega^t = wn -> omega* = x
  Phase P = base_phase(h, g);
  P.stage = AB2CN_STAGE;
  P.nf = rhs_fields(cl);
  P.o_in = g.L.wn;
  P.o_ab_pen = g.L.ab_pen;
  P.o_ab_hist = g.L.ab_hist;
  QG_LAUNCH(launch_colinv(g.dbl, OP_RHS, cl, P, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_RHS, cl, P, g.count, st));
  if (!dynamic_closure(cl)) {
    P.o_in = g.L.x;
    P.o_in2 = g.L.wn;
    QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, P, g.count, st));
  } else {
    P.o_out = g.L.jsp;
    P.o_aux = g.L.qsp;
    clip_keep(g, P);
    QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, P, g.count, st));
    int rc = run_clip_pass(h, g, st);
    if (rc) return rc;
    P.o_in = g.L.x;
    P.o_in2 = g.L.wn;
    P.adj_dyn = 0;
    clip_sums(g, P);
    QG_LAUNCH(launch_combine(g.dbl, OP_RHS, P, g.count, st));
  }
  // sponge: omega*, omega** -> omega^{t+1} on D -> wn
  Phase Ps = base_phase(h, g);
  Ps.nf = 2;
  Ps.o_in = g.L.x;
  Ps.o_in2 = g.L.ab_wss;
  QG_LAUNCH(launch_colinv(g.dbl, OP_SPONGE, 0, Ps, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_SPONGE, 0, Ps, g.count, st));
  Ps.o_out = g.L.wn;
  QG_LAUNCH(launch_colfwd(g.dbl, OP_B, 0, Ps, g.count, st));
  Ps.o_out = g.L.ab_wss;
  QG_LAUNCH(launch_ab2cn_finish(g.dbl, Ps, g.count, st));
  return QG_OK;
}

static int run_step(const Handle& h, const Group& g, hipStream_t st) {
  if (g.scheme == QG_SCHEME_AB2CN) return run_ab2cn_step(h, g, st);
  for (int s = 1; s <= 4; ++s) {
    int rc = run_stage(h, g, s, st);
    if (rc) return rc;
  }
  return run_b(h, g, st);
}

static int run_steps_eager(const Handle& h, int n, hipStream_t st) {
  for (int k = 0; k < n; ++k)
    for (const auto& g : h.groups) {
      int rc = run_step(h, g, st);
      if (rc) return rc;
    }
  return QG_OK;
}

// The capture of nsteps steps of every group.  The groups share nothing
// that a step writes (each has its own members' regions and tables), so
// each group's chain of launches is captured on a stream of its own, forked
// from st and joined back: the graph holds one branch per group, which the
// runtime may run concurrently (small groups then fill the chip together).
static int make_branches(Handle& h, size_t ng) {
  while (h.branch_streams.size() + 1 < ng) {
    hipStream_t s;
    hipEvent_t e;
    QG_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    h.branch_streams.push_back(s);
    QG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h.branch_events.push_back(e);
  }
  if (ng > 1 && !h.ev_fork) QG_HIP(hipEventCreateWithFlags(&h.ev_fork, hipEventDisableTiming));
  return QG_OK;
}

// Inside a capture on st: work(g, stream) for every group, group 0 on st and
// each further group on its branch stream (make_branches first).
template <typename F>
static int capture_branches(Handle& h, hipStream_t st, F work) {
  const size_t ng = h.groups.size();
  if (ng > 1) {
    QG_HIP(hipEventRecord(h.ev_fork, st));
    for (size_t i = 1; i < ng; ++i) QG_HIP(hipStreamWaitEvent(h.branch_streams[i - 1], h.ev_fork, 0));
  }
  for (size_t i = 0; i < ng; ++i) {
    int rc = work(h.groups[i], i == 0 ? st : h.branch_streams[i - 1]);
    if (rc) return rc;
  }
  for (size_t i = 1; i < ng; ++i) {
    QG_HIP(hipEventRecord(h.branch_events[i - 1], h.branch_streams[i - 1]));
    QG_HIP(hipStreamWaitEvent(st, h.branch_events[i - 1], 0));
  }
  return QG_OK;
}

// The step's branches: one per group; a handle of one group with
// SPLIT_MIN members or more runs it as two halves instead (its members
// share nothing a step writes either), so that the tail of one half's
// launch overlaps the start of the other's.  (Measured on 1024^2 members:
// 8 x FP32 0.885 -> 0.851 ms per step, 8 x FP64 1.955 -> 1.875 ms, 2 x
// FP32 0.296 -> 0.285 ms, 3 x FP32 0.388 -> 0.385 ms; three, four or eight
// parts lose again, and splitting the groups of a ragged ensemble, already
// a dozen branches, makes its step 25% slower.)
constexpr int SPLIT_MIN = 2;
static std::vector<Group> step_units(const Handle& h) {
  if (h.groups.size() != 1 || h.groups[0].count < SPLIT_MIN) return h.groups;
  const Group& g = h.groups[0];
  Group a = g, b = g;
  a.count = g.count / 2;
  b.m0 = g.m0 + a.count;
  b.count = g.count - a.count;
  return {a, b};
}

// nsteps steps of every unit, unit 0 on st and each further unit on a
// branch stream (make_branches first), forked from st and joined back.
static int capture_units(Handle& h, const std::vector<Group>& units, int nsteps, hipStream_t st) {
  const size_t nu = units.size();
  if (nu > 1) {
    QG_HIP(hipEventRecord(h.ev_fork, st));
    for (size_t i = 1; i < nu; ++i) QG_HIP(hipStreamWaitEvent(h.branch_streams[i - 1], h.ev_fork, 0));
  }
  for (size_t i = 0; i < nu; ++i) {
    hipStream_t bs = i == 0 ? st : h.branch_streams[i - 1];
    for (int k = 0; k < nsteps; ++k) {
      int rc = run_step(h, units[i], bs);
      if (rc) return rc;
    }
  }
  for (size_t i = 1; i < nu; ++i) {
    QG_HIP(hipEventRecord(h.branch_events[i - 1], h.branch_streams[i - 1]));
    QG_HIP(hipStreamWaitEvent(st, h.branch_events[i - 1], 0));
  }
  return QG_OK;
}

static int capture_steps(Handle& h, int nsteps, hipStream_t st) { return capture_units(h, step_units(h), nsteps, st); }

static int get_graph(Handle& h, int nsteps, hipStream_t st, hipGraphExec_t* out) {
  auto it = h.graphs.find(nsteps);
  if (it != h.graphs.end()) { *out = it->second; return QG_OK; }
  hipGraph_t graph;
  int rc = make_branches(h, step_units(h).size());
  if (rc) return rc;
  QG_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  rc = capture_steps(h, nsteps, st);
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (rc) { if (e == hipSuccess) (void)hipGraphDestroy(graph); return rc; }
  if (e != hipSuccess) return fail(QG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  hipGraphExec_t exec;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(QG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  h.graphs[nsteps] = exec;
  *out = exec;
  return QG_OK;
}

constexpr int GRAPH_STEPS = 10;

static int run_steps(Handle& h, long long n, bool use_graph, hipStream_t st) {
  if (!use_graph) return run_steps_eager(h, (int)n, st);
  if (!h.graph_stream) {
    QG_HIP(hipStreamCreateWithFlags(&h.graph_stream, hipStreamNonBlocking));
    QG_HIP(hipEventCreateWithFlags(&h.ev_in, hipEventDisableTiming));
    QG_HIP(hipEventCreateWithFlags(&h.ev_out, hipEventDisableTiming));
  }
  hipStream_t gs = h.graph_stream;
  QG_HIP(hipEventRecord(h.ev_in, st));
  QG_HIP(hipStreamWaitEvent(gs, h.ev_in, 0));
  while (n > 0) {
    const int k = n >= GRAPH_STEPS ? GRAPH_STEPS : 1;
    hipGraphExec_t ex;
    int rc = get_graph(h, k, gs, &ex);
    if (rc) return rc;
    QG_HIP(hipGraphLaunch(ex, gs));
    n -= k;
  }
  QG_HIP(hipEventRecord(h.ev_out, gs));
  QG_HIP(hipStreamWaitEvent(st, h.ev_out, 0));
  return QG_OK;
}

static int mask_precompute(const Handle& h, const Group& g, hipStream_t st) {
  Phase P = full_set(base_phase(h, g), g);
  QG_LAUNCH(launch_row(g.dbl, OP_MASKFWD, 0, P, g.count, st));
  P.o_out = g.L.chih;
  QG_LAUNCH(launch_colfwd(g.dbl, OP_MASKFWD, 0, P, g.count, st));
  P.o_in = g.L.chih;
  P.nf = 2;
  QG_LAUNCH(launch_colinv(g.dbl, OP_MASKGRAD, 0, P, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_MASKGRAD, 0, P, g.count, st));
  return QG_OK;
}

static MemberDev make_member(const qg_params& p, char* base, long long omega_off, int user) {
  MemberDev m{};
  m.base = base;
  m.omega_off = omega_off;
  m.user_index = user;
  const double pi = 3.14159265358979323846;
  m.two_pi_lx = 2.0 * pi / p.lx;
  m.two_pi_ly = 2.0 * pi / p.ly;
  m.dt = p.dt;
  m.dt2 = p.dt / 2.0;
  m.dt3 = p.dt / 3.0;
  m.dt6 = p.dt / 6.0;
  m.beta = p.beta;
  m.inv_re = (p.re > 0 && std::isfinite(p.re)) ? 1.0 / p.re : 0.0;
  m.mu = p.mu;
  m.u_in = p.u_in;
  m.v_in = p.v_in;
  const double delta = p.lx / p.nx;
  m.inv_delta = 1.0 / delta;
  m.closure = p.closure;
  m.clip_mode = p.clip_mode;
  if (p.closure == 1) { m.coef_static = (p.c * delta) * (p.c * delta); m.dcoef_dc = 2.0 * p.c * delta * delta; }
  else if (p.closure == 2) { m.coef_static = std::pow(p.c * delta, 3); m.dcoef_dc = 3.0 * p.c * p.c * delta * delta * delta; }
  const int tr = (int)std::lround(p.test_ratio > 0 ? p.test_ratio : 2.0);
  m.r_test = p.closure == 3 ? (double)tr * tr : (double)tr * tr * tr;
  m.test_r2 = tr * tr;
  const long long Mx = (p.nx - 1) / 3, My = (p.ny - 1) / 3;
  const long long lim = std::min(Mx * p.ny, My * p.nx);
  m.test_lim = lim * lim;
  // first column with no mode in the test filter: test_r2 ny^2 mx^2 > test_lim
  m.test_kx = 0;
  while (m.test_kx < p.nx / 2 + 1 &&
         (long long)m.test_r2 * p.ny * p.ny * (long long)m.test_kx * m.test_kx <= m.test_lim)
    ++m.test_kx;
  m.lowk2 = (double)p.fp64_lowk * p.fp64_lowk;
  m.pen_a = (p.eta > 0 && std::isfinite(p.eta)) ? p.dt / p.eta : 0.0;
  m.sponge_a = p.dt * p.sponge_sigma;
  m.inv_n = 1.0 / ((double)p.nx * p.ny);
  return m;
}

// ------------------------------------------------------------ adjoint sweep
// The reverse sweep's passes: at strip width 1 where the compile-time
// column engines take it.  The tuned width is chosen for the forward step;
// a reverse pass's row and column launches only have to agree with each
// other on the mixed layout's strip width (the pitch stays the group's).
static Phase adj_phase(const Handle& h, const Group& g) {
  Phase P = base_phase(h, g);
  if (g.logny >= 8 && g.logny <= 10) {
    P.W = 1;
    P.logW = 0;
  }
  return P;
}

// Recompute one segment from the state in wn, storing every stage input,
// then run the adjoint steps in reverse (B-step transpose, stages 4..1),
// starting from adj_lam and leaving dL/d state at the segment start in
// adj_lam; dL/dc is accumulated in the workspace.  Workspace-only pointers,
// so the whole sweep can be captured in a graph.
static int adjoint_sweep(const Handle& h, const Group& g, long long nsteps, hipStream_t st) {
  const long long spec = (long long)g.kxn * g.kyn * (g.dbl ? 16 : 8);
  const long long slot_bytes = (long long)align256((size_t)spec);
  const long long LS = g.L.adj_store;
  auto slot = [&](long long n, int s) { return g.L.adj_store + (1 + 4 * n + s) * slot_bytes; };
  const bool dyn = dynamic_closure(g.closure);
  // dynamic closures: H, M, Q and (C, <HM>, <M^2>) of step n, stage s (1..4)
  auto keep = [&](long long n, int s) {
    const long long k = 4 * n + (s - 1);
    return StageStore{g.L.adj_hmq + (3 * k) * slot_bytes, g.L.adj_hmq + (3 * k + 1) * slot_bytes,
                      g.L.adj_hmq + (3 * k + 2) * slot_bytes, g.L.adj_cs + 3 * k * 8};
  };
  Phase C = base_phase(h, g);
  for (long long n = 0; n < nsteps; ++n) {
    QG_LAUNCH(launch_spec_copy(g.dbl, C, g.count, slot(n, 0), g.L.wn, st));
    for (int s = 1; s <= 4; ++s) {
      const StageStore ks = dyn ? keep(n, s) : StageStore{};
      int rc = run_stage(h, g, s, st, dyn ? &ks : nullptr);
      if (rc) return rc;
      if (s < 4) QG_LAUNCH(launch_spec_copy(g.dbl, C, g.count, slot(n, s), g.L.x, st));
    }
    int rc = run_b(h, g, st);
    if (rc) return rc;
  }
  const int cl = g.closure;
  const int nb = smag_family(cl) ? 6 : 4;
  const int clb = cl == 3 ? 1 : cl == 4 ? 2 : cl;   // the adjoint kernels of the closure's base family
  for (long long n = nsteps - 1; n >= 0; --n) {
    Phase B = adj_phase(h, g);
    B.o_in = g.L.adj_lam;
    B.nf = 1;
    QG_LAUNCH(launch_colinv(g.dbl, OP_ADJ_B, 0, B, g.count, st));
    QG_LAUNCH(launch_row(g.dbl, OP_ADJ_B, 0, B, g.count, st));
    B.o_out = LS;
    B.o_aux = g.L.adj_lacc;
    B.o_in = g.L.adj_lk;
    QG_LAUNCH(launch_colfwd(g.dbl, OP_ADJ_B, 0, B, g.count, st));
    for (int s = 4; s >= 1; --s) {
      Phase A = adj_phase(h, g);
      A.stage = s;
      A.o_in = slot(n, s - 1);
      A.o_in2 = g.L.adj_lk;
      A.nf = nb + (cl == 0 ? 1 : 3);
      if (dyn) {
        // the stage's coefficient as a function of its input: s = <lambda,
        // Q> and the cotangents of the kept H and M, the transport adjoint at
        // the test-filtered stage input into adj_e; the stage's own pass
        // below takes the rest
        const StageStore ks = keep(n, s);
        Phase Kp = adj_phase(h, g);
        Kp.o_in2 = g.L.adj_lk;
        Kp.o_aux = ks.q;
        Kp.o_h = ks.h;
        Kp.o_m = ks.m;
        Kp.o_cs = ks.cs;
        Kp.o_a = g.L.adj_a;
        Kp.o_b = g.L.adj_b;
        QG_LAUNCH(launch_adj_dyn_prep(g.dbl, Kp, g.count, st));
        A.adj_dyn = 1;
        A.o_a = g.L.adj_a;
        A.o_b = g.L.adj_b;
        A.o_e = g.L.adj_e;
        // the column-inverse and row passes of both (adj_mode 2): fields
        // and products of the stage's own pass first, then those of the
        // transport pass; the latter's column pass forms the term into
        // adj_e, which the former's column pass below adds
        Phase T1 = A;
        T1.adj_mode = 1;
        T1.adj_dyn = 0;
        if (row_two_levels_ok(g.dbl, OP_ADJ_RHS, clb, A)) {
          Phase G = A;
          G.adj_mode = 2;
          G.nf = 2 * A.nf;
          QG_LAUNCH(launch_colinv(g.dbl, OP_ADJ_RHS, clb, G, g.count, st));
          QG_LAUNCH(launch_row(g.dbl, OP_ADJ_RHS, clb, G, g.count, st));
          T1.o_mp = g.L.mp + (long long)(smag_family(cl) ? 6 : 4) * g.ny * g.kxp * (g.dbl ? 16 : 8);
          QG_LAUNCH(launch_colfwd(g.dbl, OP_ADJ_RHS, clb, T1, g.count, st));
        } else {
          // the row kernel of these sizes takes one pass at a time
          QG_LAUNCH(launch_colinv(g.dbl, OP_ADJ_RHS, clb, T1, g.count, st));
          QG_LAUNCH(launch_row(g.dbl, OP_ADJ_RHS, clb, T1, g.count, st));
          QG_LAUNCH(launch_colfwd(g.dbl, OP_ADJ_RHS, clb, T1, g.count, st));
          QG_LAUNCH(launch_colinv(g.dbl, OP_ADJ_RHS, clb, A, g.count, st));
          QG_LAUNCH(launch_row(g.dbl, OP_ADJ_RHS, clb, A, g.count, st));
        }
      } else {
        QG_LAUNCH(launch_colinv(g.dbl, OP_ADJ_RHS, clb, A, g.count, st));
        QG_LAUNCH(launch_row(g.dbl, OP_ADJ_RHS, clb, A, g.count, st));
      }
      if (cl != 0 && !dyn)
        QG_LAUNCH(launch_adj_grad_c(A, g.count, row_launch_blocks(g.dbl, OP_ADJ_RHS, cl, A), nullptr, 0, st));
      A.o_out = LS;
      A.o_aux = g.L.adj_lacc;
      QG_LAUNCH(launch_colfwd(g.dbl, OP_ADJ_RHS, clb, A, g.count, st));
    }
    QG_LAUNCH(launch_spec_copy(g.dbl, C, g.count, g.L.adj_lam, g.L.adj_lacc, st));
  }
  return QG_OK;
}

// ------------------------------------------------------------ tuning cache
// A flat JSON object {"<key>": W, ...}; keys name the device architecture,
// grid, precision, closure and member count of a size group.
static std::string group_key(const Group& g) {
  char arch[64] = "gpu";
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c) if (*c == ':') { *c = 0; break; }
  }
  char buf[160];
  snprintf(buf, sizeof buf, "%s/%dx%d/fp%d/closure%d/members%d", arch, g.nx, g.ny, g.dbl ? 64 : 32,
           g.closure, g.count);
  return buf;
}

static void read_width_cache(const char* path, std::map<std::string, int>& out) {
  FILE* f = fopen(path, "r");
  if (!f) return;
  std::string txt;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
  fclose(f);
  size_t pos = 0;
  while ((pos = txt.find('"', pos)) != std::string::npos) {
    size_t end = txt.find('"', pos + 1);
    if (end == std::string::npos) break;
    std::string key = txt.substr(pos + 1, end - pos - 1);
    size_t colon = txt.find(':', end);
    if (colon == std::string::npos) break;
    out[key] = atoi(txt.c_str() + colon + 1);
    pos = colon + 1;
  }
}

static void write_width_cache(const char* path, const std::map<std::string, int>& m) {
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
  rename(tmp.c_str(), path);
}

}  // namespace qg

// ================================================================ C ABI
using namespace qg;

struct qg_handle {
  Handle h;
};

extern "C" {

const char* qg_last_error(void) { return g_err.c_str(); }

int qg_workspace_bytes(const qg_params* params, int32_t n, int32_t adjK, size_t* bytes) {
  if (!bytes) return fail(QG_EINVAL, "bytes is NULL");
  try {
    Handle h;
    int rc = build_layout(params, n, adjK, h);
    if (rc) return rc;
    *bytes = h.ws_bytes;
    return QG_OK;
  } catch (...) {
    return fail(QG_EINVAL, "internal error while sizing the workspace");
  }
}

int qg_init(const qg_params* params, int32_t n, const void* const* chi_obs, const void* const* chi_sponge,
            void* workspace, size_t ws_bytes, int32_t adjK, void* hip_stream, qg_handle** out) {
  if (!out) return fail(QG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!chi_obs || !chi_sponge) return fail(QG_EINVAL, "mask arrays are NULL");
  qg_handle* H = nullptr;
  try {
    H = new qg_handle();
  } catch (...) {
    return fail(QG_EINVAL, "out of host memory");
  }
  Handle& h = H->h;
  int rc = build_layout(params, n, adjK, h);
  if (rc) { delete H; return rc; }
  if (!workspace) { delete H; return fail(QG_EWORKSPACE, "workspace is NULL"); }
  if (reinterpret_cast<uintptr_t>(workspace) % 256) { delete H; return fail(QG_EWORKSPACE, "workspace must be 256-byte aligned"); }
  if (ws_bytes < h.ws_bytes) {
    delete H;
    char buf[160];
    snprintf(buf, sizeof buf, "workspace too small: %zu < %zu bytes", ws_bytes, h.ws_bytes);
    return fail(QG_EWORKSPACE, buf);
  }
  for (int i = 0; i < n; ++i)
    if (!chi_obs[i] || !chi_sponge[i]) { delete H; return fail(QG_EINVAL, "a mask pointer is NULL"); }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  h.ws = reinterpret_cast<char*>(workspace);
  h.mem_dev = reinterpret_cast<MemberDev*>(h.ws);
  auto cleanup = [&](int code) { delete H; return code; };
  if (launch_fill_zero(h.ws, h.ws_bytes, st) != hipSuccess) return cleanup(fail(QG_EHIP, "workspace clear failed"));
  std::vector<MemberDev> table(n);
  std::vector<char> host_tw;
  for (auto& g : h.groups) {
    g.region0 = h.ws + reinterpret_cast<long long>(g.region0);
    g.twx = h.ws + g.o_twx;
    g.twy = h.ws + g.o_twy;
    g.twx1 = h.ws + g.o_twx1;
    g.twy1 = h.ws + g.o_twy1;
    g.twx2 = h.ws + g.o_twx2;
    g.twy2 = h.ws + g.o_twy2;
    for (int k = 0; k < g.count; ++k) {
      const int u = g.users[k];
      MemberDev& m = table[g.m0 + k];
      m = make_member(params[u], g.region0 + (long long)k * g.region_bytes, h.omega_off[u], u);
      m.tab_off = g.L.phys;
      // a member given the same mask buffers as an earlier member of its
      // group, with the same dt/eta and dt sigma, has the same tables bit
      // for bit: its B sub-step reads that member's (one copy read per
      // step for an ensemble over initial conditions on one geometry)
      for (int k0 = 0; k0 < k; ++k0) {
        const int u0 = g.users[k0];
        const MemberDev& m0 = table[g.m0 + k0];
        if (chi_obs[u0] == chi_obs[u] && chi_sponge[u0] == chi_sponge[u] && m0.pen_a == m.pen_a &&
            m0.sponge_a == m.sponge_a) {
          m.tab_off = (m0.base + g.L.phys) - m.base;
          break;
        }
      }
    }
    // x and y tables of schedules 0, 1 and 2
    for (int axis = 0; axis < 6; ++axis) {
      const int len = (axis & 1) == 0 ? g.nx : g.ny;
      std::vector<long double> fre, fim, re, im;
      twiddles(len, fre, fim);
      pass_twiddles(len, axis >> 1, fre, fim, re, im);
      void* dst = axis == 0 ? g.twx : axis == 1 ? g.twy : axis == 2 ? g.twx1 : axis == 3 ? g.twy1
                : axis == 4 ? g.twx2 : g.twy2;
      if (g.dbl) {
        std::vector<double> t(2 * len);
        for (int m = 0; m < len; ++m) { t[2 * m] = (double)re[m]; t[2 * m + 1] = (double)im[m]; }
        if (hipMemcpyAsync(dst, t.data(), t.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return cleanup(fail(QG_EHIP, "twiddle upload failed"));
      } else {
        std::vector<float> t(2 * len);
        for (int m = 0; m < len; ++m) { t[2 * m] = (float)re[m]; t[2 * m + 1] = (float)im[m]; }
        if (hipMemcpyAsync(dst, t.data(), t.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          return cleanup(fail(QG_EHIP, "twiddle upload failed"));
      }
    }
  }
  if (hipMemcpyAsync(h.mem_dev, table.data(), n * sizeof(MemberDev), hipMemcpyHostToDevice, st) != hipSuccess)
    return cleanup(fail(QG_EHIP, "member table upload failed"));
  h.table = table;
  for (auto& g : h.groups) {
    const int rs = g.dbl ? 8 : 4;
    const size_t fb = (size_t)g.nx * g.ny * rs;
    for (int k = 0; k < g.count; ++k) {
      char* phys = g.region0 + (long long)k * g.region_bytes + g.L.phys;
      const int u = g.users[k];
      if (hipMemcpyAsync(phys + 4 * fb, chi_obs[u], fb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipMemcpyAsync(phys + 5 * fb, chi_sponge[u], fb, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return cleanup(fail(QG_EHIP, "mask copy failed"));
    }
    int r2 = mask_precompute(h, g, st);
    if (r2) return cleanup(r2);
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return cleanup(fail(QG_EHIP, std::string("init: ") + hipGetErrorString(e)));
  // AB2CN's penalty D curl(chi u) is formed as D curl((chi - c) u) + c omega
  // with c the mask's mean (an identity for any constant c, since the curl
  // of the total velocity is omega): the transform then carries no large
  // near-constant product whose rounding the curl would multiply by |k|.
  // c from the zero mode of the mask's spectrum (the sum of its values).
  bool ab2cn = false;
  for (const auto& g : h.groups) ab2cn = ab2cn || g.scheme == QG_SCHEME_AB2CN;
  if (ab2cn) {
    for (const auto& g : h.groups) {
      if (g.scheme != QG_SCHEME_AB2CN) continue;
      for (int k = 0; k < g.count; ++k) {
        const char* z0 = g.region0 + (long long)k * g.region_bytes + g.L.chih;
        double re = 0.0;
        if (g.dbl) {
          e = hipMemcpy(&re, z0, sizeof(double), hipMemcpyDeviceToHost);
        } else {
          float rf = 0.f;
          e = hipMemcpy(&rf, z0, sizeof(float), hipMemcpyDeviceToHost);
          re = rf;
        }
        if (e != hipSuccess) return cleanup(fail(QG_EHIP, std::string("init: ") + hipGetErrorString(e)));
        table[g.m0 + k].pen_c = re / ((double)g.nx * g.ny);
      }
    }
    if (hipMemcpyAsync(h.mem_dev, table.data(), n * sizeof(MemberDev), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return cleanup(fail(QG_EHIP, "member table upload failed"));
    h.table = table;
  }
  *out = H;
  return QG_OK;
}

void qg_destroy(qg_handle* H) {
  if (!H) return;
  for (auto& kv : H->h.graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& kv : H->h.adj_graphs) (void)hipGraphExecDestroy(kv.second);
  if (H->h.graph_stream) {
    (void)hipStreamSynchronize(H->h.graph_stream);
    (void)hipStreamDestroy(H->h.graph_stream);
  }
  if (H->h.ev_in) (void)hipEventDestroy(H->h.ev_in);
  if (H->h.ev_out) (void)hipEventDestroy(H->h.ev_out);
  for (auto s : H->h.branch_streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (auto e : H->h.branch_events) (void)hipEventDestroy(e);
  if (H->h.ev_fork) (void)hipEventDestroy(H->h.ev_fork);
  delete H;
}

int qg_info(const qg_handle* H, int32_t* n_members, int64_t* total_points, int32_t* fwd_width,
            int32_t* inv_width) {
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  const Handle& h = H->h;
  if (n_members) *n_members = (int32_t)h.params.size();
  if (total_points) *total_points = h.total_points;
  for (size_t i = 0; i < h.params.size(); ++i) {
    if (fwd_width) fwd_width[i] = h.groups[h.member_group[i]].W;
    if (inv_width) inv_width[i] = h.groups[h.member_group[i]].Wi;
  }
  return QG_OK;
}

int qg_step(qg_handle* H, void* omega, int64_t nsteps, int32_t save_every, void* ckpt_out, int32_t use_graph,
            void* hip_stream) {
  Range range("qg_step");
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  if (!omega) return fail(QG_EINVAL, "omega is NULL");
  if (nsteps < 0) return fail(QG_EINVAL, "nsteps must be >= 0");
  if (save_every < 0) return fail(QG_EINVAL, "save_every must be >= 0");
  if (save_every > 0 && !ckpt_out) return fail(QG_EINVAL, "ckpt_out is NULL with save_every > 0");
  Handle& h = H->h;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  try {
    for (const auto& g : h.groups) {
      int rc = run_entry(h, g, omega, g.L.wn, st);
      if (rc) return rc;
    }
    long long done = 0;
    int save_idx = 0;
    while (done < nsteps) {
      long long chunk = nsteps - done;
      if (save_every > 0) chunk = std::min<long long>(chunk, save_every - done % save_every);
      int rc = run_steps(h, chunk, use_graph != 0, st);
      if (rc) return rc;
      done += chunk;
      if (save_every > 0 && done % save_every == 0) {
        char* dst = reinterpret_cast<char*>(ckpt_out) + (long long)save_idx * h.total_bytes;
        for (const auto& g : h.groups) {
          rc = run_exit(h, g, g.L.wn, dst, st);
          if (rc) return rc;
        }
        if (done < nsteps)
          for (const auto& g : h.groups) {
            rc = run_entry(h, g, dst, g.L.wn, st);
            if (rc) return rc;
          }
        ++save_idx;
      }
    }
    for (const auto& g : h.groups) {
      int rc = run_exit(h, g, g.L.wn, omega, st);
      if (rc) return rc;
    }
  } catch (...) {
    return fail(QG_EINVAL, "internal error in qg_step");
  }
  return QG_OK;
}

// Position of caller member i inside its group.
static int group_slot(const Handle& h, int i) {
  const Group& g = h.groups[h.member_group[i]];
  for (int k = 0; k < g.count; ++k)
    if (g.users[k] == i) return k;
  return -1;
}

// Member pairs of an FR and an LES handle: same count, the LES grid the FR
// grid coarsened by a power of two >= 2, same box and precision.
static int check_les_pair(const Handle& F, const Handle& L) {
  const int n = (int)F.params.size();
  if ((int)L.params.size() != n) return fail(QG_EINVAL, "the two handles hold different member counts");
  for (int i = 0; i < n; ++i) {
    const qg_params& a = F.params[i];
    const qg_params& b = L.params[i];
    char buf[160];
    const int d = b.nx > 0 ? a.nx / b.nx : 0;
    if (d < 2 || a.nx != d * b.nx || a.ny != d * b.ny || !is_pow2(d)) {
      snprintf(buf, sizeof buf, "member %d: the LES grid must be the FR grid coarsened by a power of two >= 2", i);
      return fail(QG_EINVAL, buf);
    }
    if (std::fabs(a.lx - b.lx) > 1e-12 * a.lx || std::fabs(a.ly - b.ly) > 1e-12 * a.ly || a.precision != b.precision) {
      snprintf(buf, sizeof buf, "member %d: the two grids must share lx, ly and precision", i);
      return fail(QG_EINVAL, buf);
    }
  }
  return QG_OK;
}

// H_full of member i: FR D-compact spectrum at byte offset o_src of its
// region -> LES spectrum at o_dst, on the LES full set (full = true) or on
// its 2/3 set.
static int launch_member_filter(const Handle& F, const Handle& L, int i, long long o_src, long long o_dst,
                                bool full, hipStream_t st) {
  const Group& gf = F.groups[F.member_group[i]];
  const Group& gl = L.groups[L.member_group[i]];
  const qg_params& a = F.params[i];
  const int d = a.nx / L.params[i].nx;
  const double pi = 3.14159265358979323846;
  FilterArgs A{};
  A.src = F.table[gf.m0 + group_slot(F, i)].base + o_src;
  A.dst = L.table[gl.m0 + group_slot(L, i)].base + o_dst;
  A.kxn_f = gf.kxn; A.kyn_f = gf.kyn; A.myh_f = gf.myh;
  if (full) {
    A.kxn_c = gl.kxn_f; A.kyn_c = gl.kyn_f; A.myh_c = gl.myh_f;
  } else {
    A.kxn_c = gl.kxn; A.kyn_c = gl.kyn; A.myh_c = gl.myh;
  }
  A.two_pi_lx = 2.0 * pi / a.lx;
  A.two_pi_ly = 2.0 * pi / a.ly;
  const double dfr = a.lx / a.nx;
  A.width2 = (d * dfr) * (d * dfr);
  A.kc2 = (pi / (d * dfr)) * (pi / (d * dfr));
  A.inv_d2 = 1.0 / ((double)d * d);
  QG_LAUNCH(launch_filter_les(gf.dbl, A, st));
  return QG_OK;
}

int qg_filter_les(qg_handle* Fh, qg_handle* Lh, const void* omega_fr, void* omega_ff, void* hip_stream) {
  if (!Fh || !Lh) return fail(QG_EINVAL, "handle is NULL");
  if (!omega_fr || !omega_ff) return fail(QG_EINVAL, "omega_fr or omega_ff is NULL");
  const Handle& F = Fh->h;
  const Handle& L = Lh->h;
  const int n = (int)F.params.size();
  int rc0 = check_les_pair(F, L);
  if (rc0) return rc0;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  for (const auto& g : F.groups) {
    int rc = run_entry(F, g, omega_fr, g.L.wn, st);
    if (rc) return rc;
  }
  for (int i = 0; i < n; ++i) {
    const Group& gf = F.groups[F.member_group[i]];
    const Group& gl = L.groups[L.member_group[i]];
    int rc = launch_member_filter(F, L, i, gf.L.wn, gl.L.chih, true, st);
    if (rc) return rc;
  }
  for (const auto& g : L.groups) {
    Phase P = full_set(base_phase(L, g), g);
    P.o_in = g.L.chih;
    P.nf = 1;
    P.user = omega_ff;
    QG_LAUNCH(launch_colinv(g.dbl, OP_EXIT, 0, P, g.count, st));
    QG_LAUNCH(launch_row(g.dbl, OP_EXIT, 0, P, g.count, st));
  }
  return QG_OK;
}

// The SGS-analysis pass runs at strip width 1.
static Phase gterms_phase(const Handle& h, const Group& g) {
  Phase P = base_phase(h, g);
  P.W = 1;
  P.logW = 0;
  P.nparts = g.kxn;
  return P;
}

// G(omega) of every member of group g from the D-compact spectrum at o_in
// to o_out; minus the spectrum at o_sub unless o_sub < 0.
static int run_gterms(const Handle& h, const Group& g, long long o_in, long long o_out, long long o_sub,
                      hipStream_t st) {
  Phase P = gterms_phase(h, g);
  P.nf = 5;
  P.o_in = o_in;
  QG_LAUNCH(launch_colinv(g.dbl, OP_GTERMS, 0, P, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_GTERMS, 0, P, g.count, st));
  P.o_out = o_out;
  P.stage = o_sub >= 0 ? 1 : 0;
  P.o_in2 = o_sub >= 0 ? o_sub : 0;
  QG_LAUNCH(launch_colfwd(g.dbl, OP_GTERMS, 0, P, g.count, st));
  return QG_OK;
}

// The closure's term C D div(base grad omega) at the D-compact spectrum
// o_in (C from it for the dynamic closures) -> o_out.
static int run_model_term(const Handle& h, const Group& g, long long o_in, long long o_out, hipStream_t st) {
  const int cl = g.closure;
  Phase P = base_phase(h, g);
  P.stage = SGS_STAGE;
  P.nf = rhs_fields(cl);
  P.o_in = o_in;
  QG_LAUNCH(launch_colinv(g.dbl, OP_RHS, cl, P, g.count, st));
  QG_LAUNCH(launch_row(g.dbl, OP_RHS, cl, P, g.count, st));
  if (!dynamic_closure(cl)) {
    P.o_out = o_out;
    QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, P, g.count, st));
  } else {
    P.o_out = g.L.jsp;
    P.o_aux = g.L.qsp;
    clip_keep(g, P);
    QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, P, g.count, st));
    int rc = run_clip_pass(h, g, st);
    if (rc) return rc;
    P.o_in = o_out;
    P.adj_dyn = 0;
    clip_sums(g, P);
    QG_LAUNCH(launch_combine(g.dbl, OP_RHS, P, g.count, st));
  }
  return QG_OK;
}

int qg_ideal_sgs(qg_handle* Fh, qg_handle* Lh, const void* omega_fr, void* pi_ff, void* pi_model,
                 void* omega_bar, void* hip_stream) {
  if (!Fh || !Lh) return fail(QG_EINVAL, "handle is NULL");
  if (!omega_fr || !pi_ff) return fail(QG_EINVAL, "omega_fr or pi_ff is NULL");
  const Handle& F = Fh->h;
  const Handle& L = Lh->h;
  int rc0 = check_les_pair(F, L);
  if (rc0) return rc0;
  for (const Handle* hp : {&F, &L})
    for (const auto& g : hp->groups)
      if (!gterms_ok(g.dbl, gterms_phase(*hp, g)))
        return fail(QG_EUNSUPPORTED, "the SGS analysis needs 64 <= nx <= 1024, and ny <= 1024 in 64-bit runs "
                                     "(ny <= 2048 in 32-bit runs)");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  try {
    // FR: omega -> wn, G(omega) -> jsp
    for (const auto& g : F.groups) {
      int rc = run_entry(F, g, omega_fr, g.L.wn, st);
      if (!rc) rc = run_gterms(F, g, g.L.wn, g.L.jsp, -1, st);
      if (rc) return rc;
    }
    // filtered omega and filtered G on the LES 2/3 set -> wn, acc
    for (int i = 0; i < (int)F.params.size(); ++i) {
      const Group& gf = F.groups[F.member_group[i]];
      const Group& gl = L.groups[L.member_group[i]];
      int rc = launch_member_filter(F, L, i, gf.L.wn, gl.L.wn, false, st);
      if (!rc) rc = launch_member_filter(F, L, i, gf.L.jsp, gl.L.acc, false, st);
      if (rc) return rc;
    }
    for (const auto& g : L.groups) {
      int rc = run_gterms(L, g, g.L.wn, g.L.x, g.L.acc, st);
      if (!rc) rc = run_exit(L, g, g.L.x, pi_ff, st);
      if (!rc && omega_bar) rc = run_exit(L, g, g.L.wn, omega_bar, st);
      if (!rc && pi_model) {
        rc = run_model_term(L, g, g.L.wn, g.L.x, st);
        if (!rc) rc = run_exit(L, g, g.L.x, pi_model, st);
      }
      if (rc) return rc;
    }
  } catch (...) {
    return fail(QG_EINVAL, "internal error in qg_ideal_sgs");
  }
  return QG_OK;
}

int qg_closure_term(qg_handle* H, const void* omega, void* out, void* hip_stream) {
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  if (!omega || !out) return fail(QG_EINVAL, "omega or out is NULL");
  const Handle& h = H->h;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  try {
    for (const auto& g : h.groups) {
      int rc = run_entry(h, g, omega, g.L.wn, st);
      if (!rc) rc = run_model_term(h, g, g.L.wn, g.L.x, st);
      if (!rc) rc = run_exit(h, g, g.L.x, out, st);
      if (rc) return rc;
    }
  } catch (...) {
    return fail(QG_EINVAL, "internal error in qg_closure_term");
  }
  return QG_OK;
}

int qg_pcc(qg_handle* H, const void* a, const void* b, double* out_dev, void* hip_stream) {
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  if (!a || !b || !out_dev) return fail(QG_EINVAL, "a, b or out_dev is NULL");
  Handle& h = H->h;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  for (const auto& g : h.groups) {
    // one block per 8192 points, at most 64, within the dpart area
    const long long npts = (long long)g.nx * g.ny;
    const long long cap = (5LL * (g.ny / 2) + 2LL * g.nspec + 8) / 5;
    const int nblk = (int)std::max(1LL, std::min({(npts + 8191) / 8192, 64LL, cap}));
    QG_LAUNCH(launch_pcc(g.dbl, base_phase(h, g), g.count, nblk, a, b, out_dev, st));
  }
  return QG_OK;
}

int qg_diag(qg_handle* H, const void* omega, double* out_dev, void* nu_e_out, void* hip_stream) {
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  if (!omega || !out_dev) return fail(QG_EINVAL, "omega or out_dev is NULL");
  Handle& h = H->h;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  for (const auto& g : h.groups) {
    int rc = run_entry(h, g, omega, g.L.wn, st);
    if (rc) return rc;
    Phase P = base_phase(h, g);
    const int cl = g.closure;
    if (dynamic_closure(cl)) {
      P.nf = rhs_fields(cl);
      P.o_in = g.L.wn;
      QG_LAUNCH(launch_colinv(g.dbl, OP_RHS, cl, P, g.count, st));
      QG_LAUNCH(launch_row(g.dbl, OP_RHS, cl, P, g.count, st));
      P.o_out = g.L.jsp;
      P.o_aux = g.L.qsp;
      clip_keep(g, P);
      QG_LAUNCH(launch_colfwd(g.dbl, OP_RHS, cl, P, g.count, st));
      rc = run_clip_pass(h, g, st);
      if (rc) return rc;
      clip_sums(g, P);
      QG_LAUNCH(launch_dyn_coef(P, g.count, 0, st));
    }
    Phase D = base_phase(h, g);
    D.nf = smag_family(cl) ? 6 : 4;
    D.o_in = g.L.wn;
    D.user = nu_e_out;
    QG_LAUNCH(launch_colinv(g.dbl, OP_DIAG, cl, D, g.count, st));
    QG_LAUNCH(launch_row(g.dbl, OP_DIAG, cl, D, g.count, st));
    D.o_aux = g.L.dpart + 5LL * (g.ny / 2) * 8;
    QG_LAUNCH(launch_diag_spectral(g.dbl, D, g.count, st));
    QG_LAUNCH(launch_diag_final(D, g.count, row_launch_blocks(g.dbl, OP_DIAG, cl, D), g.nspec, out_dev, 0, st));
  }
  return QG_OK;
}

int qg_adjoint_step(qg_handle* H, const void* omega_ckpt, void* lambda, int64_t nsteps, double* grad_c,
                    void* hip_stream) {
  Range range("qg_adjoint_step");
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  Handle& h = H->h;
  if (!omega_ckpt || !lambda || !grad_c) return fail(QG_EINVAL, "NULL argument");
  if (h.adjK <= 0) return fail(QG_ESTATE, "handle was built without adjoint storage (adj_segment_k = 0)");
  if (nsteps < 1 || nsteps > h.adjK) return fail(QG_EINVAL, "nsteps must be in [1, adj_segment_k]");
  for (const auto& g : h.groups) {
    if (g.scheme != QG_SCHEME_RK4)
      return fail(QG_EUNSUPPORTED, "the adjoint covers the RK4 scheme only");
    if (g.clip == 1)
      return fail(QG_EUNSUPPORTED, "the adjoint covers the coefficient-level clip (clip_mode 0) only");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  // outside the graph: the caller's fields in, the dL/dc slots cleared
  for (const auto& g : h.groups) {
    int rc = run_entry(h, g, omega_ckpt, g.L.wn, st);          // state at the segment start
    if (rc) return rc;
    rc = run_entry(h, g, lambda, g.L.adj_lam, st);              // adjoint of the exit transform
    if (rc) return rc;
    QG_LAUNCH(launch_adj_grad_c(base_phase(h, g), g.count, 0, nullptr, 1, st));
  }
  // recompute + reverse sweep: one graph per segment length
  if (!h.graph_stream) {
    QG_HIP(hipStreamCreateWithFlags(&h.graph_stream, hipStreamNonBlocking));
    QG_HIP(hipEventCreateWithFlags(&h.ev_in, hipEventDisableTiming));
    QG_HIP(hipEventCreateWithFlags(&h.ev_out, hipEventDisableTiming));
  }
  hipStream_t gs = h.graph_stream;
  hipGraphExec_t ex = nullptr;
  auto it = h.adj_graphs.find((int)nsteps);
  if (it != h.adj_graphs.end()) {
    ex = it->second;
  } else {
    hipGraph_t graph;
    int rc = make_branches(h, h.groups.size());
    if (rc) return rc;
    QG_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    // the groups' sweeps are independent: one graph branch each
    rc = capture_branches(h, gs, [&](const Group& g, hipStream_t bs) { return adjoint_sweep(h, g, nsteps, bs); });
    hipError_t e = hipStreamEndCapture(gs, &graph);
    if (rc) { if (e == hipSuccess) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return fail(QG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(QG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h.adj_graphs[(int)nsteps] = ex;
  }
  QG_HIP(hipEventRecord(h.ev_in, st));
  QG_HIP(hipStreamWaitEvent(gs, h.ev_in, 0));
  QG_HIP(hipGraphLaunch(ex, gs));
  QG_HIP(hipEventRecord(h.ev_out, gs));
  QG_HIP(hipStreamWaitEvent(st, h.ev_out, 0));
  // outside the graph: the caller's fields out
  for (const auto& g : h.groups) {
    int rc = run_exit(h, g, g.L.adj_lam, lambda, st);           // adjoint of the entry transform
    if (rc) return rc;
    QG_LAUNCH(launch_adj_grad_c(base_phase(h, g), g.count, 0, grad_c, 2, st));
  }
  return QG_OK;
}

int qg_set_coef(qg_handle* H, const double* c, void* hip_stream) {
  if (!H || !c) return fail(QG_EINVAL, "NULL argument");
  Handle& h = H->h;
  for (size_t i = 0; i < h.params.size(); ++i)
    if (!std::isfinite(c[i])) return fail(QG_EINVAL, "non-finite closure coefficient");
  for (const auto& g : h.groups)
    for (int k = 0; k < g.count; ++k) {
      const int u = g.users[k];
      h.params[u].c = c[u];
      MemberDev m = make_member(h.params[u], h.table[g.m0 + k].base, h.omega_off[u], u);
      // values qg_init derived are kept: the mask mean split off in the
      // AB2CN penalty's curl, and where the B sub-step's tables are read
      // (they depend on dt/eta and dt sigma only, which stay)
      m.pen_c = h.table[g.m0 + k].pen_c;
      m.tab_off = h.table[g.m0 + k].tab_off;
      h.table[g.m0 + k] = m;
    }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  QG_HIP(hipMemcpyAsync(h.mem_dev, h.table.data(), h.table.size() * sizeof(MemberDev),
                        hipMemcpyHostToDevice, st));
  QG_HIP(hipStreamSynchronize(st));
  return QG_OK;
}

int qg_profile_steps(qg_handle* H, void* omega, int64_t nsteps, int32_t kind, float* ms, int32_t max_launches,
                     int32_t* n_launches, void* hip_stream) {
  if (!H || !omega || !ms || !n_launches) return fail(QG_EINVAL, "NULL argument");
  if (kind < 0 || kind > 6) return fail(QG_EINVAL, "kind must be in [0, 6]");
  if (nsteps < 0 || max_launches < 0) return fail(QG_EINVAL, "nsteps and max_launches must be >= 0");
  Handle& h = H->h;
  for (const auto& g : h.groups)
    if (g.scheme != QG_SCHEME_RK4) return fail(QG_EUNSUPPORTED, "profiling runs take RK4 members only");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  ProfState ps;
  ps.kind = kind;
  ps.used = 0;
  int rc = QG_OK;
  for (int i = 0; i < 2 * max_launches; ++i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { rc = fail(QG_EHIP, "hipEventCreate failed"); break; }
    ps.ev.push_back(e);
  }
  if (rc == QG_OK) {
    g_prof = &ps;
    try {
      for (const auto& g : h.groups)
        if (rc == QG_OK) rc = run_entry(h, g, omega, g.L.wn, st);
      if (rc == QG_OK) rc = run_steps_eager(h, (int)nsteps, st);
      for (const auto& g : h.groups)
        if (rc == QG_OK) rc = run_exit(h, g, g.L.wn, omega, st);
    } catch (...) {
      rc = fail(QG_EINVAL, "internal error in qg_profile_steps");
    }
    g_prof = nullptr;
  }
  if (rc == QG_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(QG_EHIP, "hipStreamSynchronize failed");
  if (rc == QG_OK) {
    for (int i = 0; i < ps.used; ++i)
      if (hipEventElapsedTime(&ms[i], ps.ev[2 * i], ps.ev[2 * i + 1]) != hipSuccess) {
        rc = fail(QG_EHIP, "hipEventElapsedTime failed");
        break;
      }
    *n_launches = ps.used;
  }
  for (auto e : ps.ev) (void)hipEventDestroy(e);
  return rc;
}

int qg_stamp_steps(qg_handle* H, void* omega, int64_t nsteps, void* stamps, size_t stamp_bytes, void* hip_stream) {
#ifndef QG_STAMPS
  (void)H; (void)omega; (void)nsteps; (void)stamps; (void)stamp_bytes; (void)hip_stream;
  return fail(QG_EUNSUPPORTED, "this library was built without QG_STAMPS: load libqg_stamps.so");
#else
  if (!H || !omega || !stamps) return fail(QG_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(QG_EINVAL, "nsteps must be >= 0");
  if (stamp_bytes < QG_STAMP_BYTES) {
    char buf[120];
    snprintf(buf, sizeof buf, "the stamp buffer needs %zu bytes", QG_STAMP_BYTES);
    return fail(QG_EINVAL, buf);
  }
  Handle& h = H->h;
  for (const auto& g : h.groups)
    if (g.scheme != QG_SCHEME_RK4) return fail(QG_EUNSUPPORTED, "stamp runs take RK4 members only");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  int rc = QG_OK;
  g_stamps = static_cast<unsigned long long*>(stamps);
  try {
    for (const auto& g : h.groups)
      if (rc == QG_OK) rc = run_entry(h, g, omega, g.L.wn, st);
    if (rc == QG_OK) rc = run_steps_eager(h, (int)nsteps, st);
    for (const auto& g : h.groups)
      if (rc == QG_OK) rc = run_exit(h, g, g.L.wn, omega, st);
  } catch (...) {
    rc = fail(QG_EINVAL, "internal error in qg_stamp_steps");
  }
  g_stamps = nullptr;
  if (rc == QG_OK && hipStreamSynchronize(st) != hipSuccess) rc = fail(QG_EHIP, "hipStreamSynchronize failed");
  return rc;
#endif
}

// One candidate tuning of a size group.
struct Tuning {
  int W, Wi, rsch, csch, rpb, rwv;
};
static void apply_tuning(Group& g, const Tuning& t) {
  set_width(g, t.W);
  set_inv_width(g, t.Wi);
  g.rsch = t.rsch;
  g.csch = t.csch;
  g.rpb = t.rpb;
  g.rwv = t.rwv;
}

int qg_autotune(qg_handle* H, const char* cache_path, void* hip_stream) {
  if (!H) return fail(QG_EINVAL, "handle is NULL");
  Handle& h = H->h;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  std::map<std::string, int> cache;
  if (cache_path) read_width_cache(cache_path, cache);
  // candidates run as captured graphs on a stream of the tuner's own,
  // ordered after the caller's earlier work
  hipStream_t ts = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr, ein = nullptr;
  QG_HIP(hipStreamCreateWithFlags(&ts, hipStreamNonBlocking));
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ein) (void)hipEventDestroy(ein);
    if (ts) { (void)hipStreamSynchronize(ts); (void)hipStreamDestroy(ts); }
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipEventCreateWithFlags(&ein, hipEventDisableTiming) != hipSuccess || hipEventRecord(ein, st) != hipSuccess ||
      hipStreamWaitEvent(ts, ein, 0) != hipSuccess) {
    cleanup();
    return fail(QG_EHIP, "autotune: stream or event set-up failed");
  }
  constexpr int TUNE_STEPS = 4;   // steps per timed graph
  int rc = QG_OK;
  bool changed = false;
  auto valid_w = [&](const Group& g, int W) { return W >= min_width(g) && W <= max_width(g) && is_pow2(W); };
  for (auto& g : h.groups) {
    if (rc) break;
    const std::string key = group_key(g);
    // admissible values of every tunable; a value found in the cache fixes it
    std::vector<int> Ws, Wis, rs, cs, rp, wv;
    for (int W = min_width(g); W <= max_width(g); W *= 2) { Ws.push_back(W); Wis.push_back(W); }
    const bool ct_rows = g.nx == 256 || g.nx == 512 || g.nx == 1024;
    const bool ct_cols = g.ny == 256 || g.ny == 512 || g.ny == 1024;
    // schedule 2 (radix 16) for the wave-synchronous 1024-point rows only
    rs = g.nx == 1024 ? std::vector<int>{0, 1, 2} : ct_rows ? std::vector<int>{0, 1} : std::vector<int>{0};
    cs = ct_cols ? std::vector<int>{0, 1} : std::vector<int>{0};
    rp = g.ny >= 64 ? std::vector<int>{1, 2} : std::vector<int>{1};
    wv = ct_rows ? std::vector<int>{0, 1} : std::vector<int>{0};
    auto fix = [&](const char* name, std::vector<int>& vals, bool ok_range) {
      auto it = cache.find(key + name);
      if (it == cache.end()) return;
      if (ok_range) vals.assign(1, it->second);
    };
    {
      auto it = cache.find(key + "/fwd");
      fix("/fwd", Ws, it != cache.end() && valid_w(g, it->second));
      it = cache.find(key + "/inv");
      fix("/inv", Wis, it != cache.end() && valid_w(g, it->second));
      it = cache.find(key + "/rsched");
      fix("/rsched", rs, it != cache.end() && (it->second == 0 || (ct_rows && it->second == 1) ||
                                                (g.nx == 1024 && it->second == 2)));
      it = cache.find(key + "/csched");
      fix("/csched", cs, it != cache.end() && (it->second == 0 || (ct_cols && it->second == 1)));
      it = cache.find(key + "/rpb");
      fix("/rpb", rp, it != cache.end() && (it->second == 1 || (g.ny >= 64 && it->second == 2)));
      it = cache.find(key + "/rwave");
      fix("/rwave", wv, it != cache.end() && (it->second == 0 || (ct_rows && it->second == 1)));
    }
    std::vector<Tuning> cand;
    for (int W : Ws)
      for (int Wi : Wis)
        for (int r : rs)
          for (int c : cs)
            for (int q : rp)
              for (int v : wv)
                if (r != 2 || v == 1) cand.push_back(Tuning{W, Wi, r, c, q, v});
    // schedule 2 and two-wave rows both fixed by the cache: schedule 1
    if (cand.empty()) cand.push_back(Tuning{Ws[0], Wis[0], 1, cs[0], rp[0], wv[0]});
    if (cand.size() == 1) {
      apply_tuning(g, cand[0]);
      continue;
    }
    // every candidate as a graph of TUNE_STEPS steps of this group, in the
    // branches the step's graph will run it in
    const bool split = step_units(h).size() > h.groups.size();
    if (split && (rc = make_branches(h, 2)) != QG_OK) break;
    std::vector<hipGraphExec_t> ex(cand.size(), nullptr);
    for (size_t i = 0; i < cand.size() && rc == QG_OK; ++i) {
      apply_tuning(g, cand[i]);
      hipGraph_t graph;
      if (hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = fail(QG_EHIP, "autotune: capture failed");
        break;
      }
      int r2 = QG_OK;
      if (split) r2 = capture_units(h, step_units(h), TUNE_STEPS, ts);
      else
        for (int k = 0; k < TUNE_STEPS && r2 == QG_OK; ++k) r2 = run_step(h, g, ts);
      hipError_t e = hipStreamEndCapture(ts, &graph);
      if (r2) { if (e == hipSuccess) (void)hipGraphDestroy(graph); rc = r2; break; }
      if (e != hipSuccess) { rc = fail(QG_EHIP, std::string("autotune capture: ") + hipGetErrorString(e)); break; }
      e = hipGraphInstantiate(&ex[i], graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) { ex[i] = nullptr; rc = fail(QG_EHIP, "autotune: graph instantiation failed"); }
    }
    // warm-up (clocks ramp up from idle), then three round-robin rounds;
    // each candidate keeps its fastest time
    std::vector<float> best(cand.size(), 1e30f);
    for (int round = -2; round < 3 && rc == QG_OK; ++round)
      for (size_t i = 0; i < cand.size() && rc == QG_OK; ++i) {
        float ms = 0.f;
        if (hipEventRecord(e0, ts) != hipSuccess || hipGraphLaunch(ex[i], ts) != hipSuccess ||
            hipEventRecord(e1, ts) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = fail(QG_EHIP, "autotune: timing failed");
          break;
        }
        if (round >= 0 && ms < best[i]) best[i] = ms;
      }
    for (auto x : ex)
      if (x) (void)hipGraphExecDestroy(x);
    if (rc) break;
    size_t bi = 0;
    for (size_t i = 1; i < cand.size(); ++i)
      if (best[i] < best[bi]) bi = i;
    apply_tuning(g, cand[bi]);
    cache[key + "/fwd"] = g.W;
    cache[key + "/inv"] = g.Wi;
    cache[key + "/rsched"] = g.rsch;
    cache[key + "/csched"] = g.csch;
    cache[key + "/rpb"] = g.rpb;
    cache[key + "/rwave"] = g.rwv;
    changed = true;
  }
  cleanup();
  if (rc) return rc;
  // the timed steps advanced the AB2CN members' history: start it again
  for (const auto& g : h.groups) {
    if (g.scheme != QG_SCHEME_AB2CN) continue;
    for (int k = 0; k < g.count; ++k) {
      char* flag = h.table[g.m0 + k].base + g.L.coef + AB2CN_FLAG_SLOT * (long long)sizeof(double);
      QG_HIP(launch_fill_zero(flag, sizeof(double), st));
    }
  }
  for (auto& kv : h.graphs) (void)hipGraphExecDestroy(kv.second);
  h.graphs.clear();
  for (auto& kv : h.adj_graphs) (void)hipGraphExecDestroy(kv.second);
  h.adj_graphs.clear();
  if (changed && cache_path) write_width_cache(cache_path, cache);
  QG_HIP(hipStreamSynchronize(st));
  return QG_OK;
}

int qg_tuning(const qg_handle* H, int32_t* out) {
  if (!H || !out) return fail(QG_EINVAL, "NULL argument");
  const Handle& h = H->h;
  for (size_t i = 0; i < h.params.size(); ++i) {
    const Group& g = h.groups[h.member_group[i]];
    int32_t* o = out + 6 * i;
    o[0] = g.W;
    o[1] = g.Wi;
    o[2] = g.rsch;
    o[3] = g.csch;
    o[4] = g.rpb;
    o[5] = g.rwv;
  }
  return QG_OK;
}

}  // extern "C"

namespace qg {

// ------------------------------------------------------------ allocation-free step
// For callers that cannot allocate (code under graph capture, serving
// loops, harnesses that forbid hipMalloc): the workspace of one member
// lives in this file-scope device array, one copy per GPU, held until the
// process ends.  Host code never uses the array's name as an address: each
// device's address comes from hipGetSymbolAddress (scratch_on).
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
constexpr int SCRATCH_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
static std::atomic<void*> g_scratch[SCRATCH_MAX_DEVICES];

// The array's address on the current device (looked up once per device).
static int scratch_on(void** out) {
  int dev = -1;
  QG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return fail(QG_EUNSUPPORTED, "device index out of range");
  void* p = g_scratch[dev].load();
  if (!p) {
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(QG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev].store(p);
  }
  *out = p;
  return QG_OK;
}

}  // namespace qg

extern "C" int qg_step_noalloc(const qg_params* p, const void* chi_obs, const void* chi_sponge, void* omega,
                               int64_t nsteps, void* hip_stream) {
  using namespace qg;
  Range range("qg_step_noalloc");
  if (!p || !chi_obs || !chi_sponge || !omega) return fail(QG_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(QG_EINVAL, "nsteps must be >= 0");
  int rc = validate(*p, 0);
  if (rc) return rc;
  if (p->scheme != QG_SCHEME_RK4) return fail(QG_EUNSUPPORTED, "qg_step_noalloc takes the RK4 scheme only");
  void* base = nullptr;
  rc = scratch_on(&base);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  // the plan of qg_workspace_bytes / qg_init for one member, default widths
  Group g{};
  g.nx = p->nx;
  g.ny = p->ny;
  g.closure = p->closure;
  g.scheme = p->scheme;
  g.clip = dynamic_closure(p->closure) ? p->clip_mode : 0;
  g.dbl = p->precision == 64;
  plan_sizes(g, 0);
  set_width(g, default_width(g, 1));
  set_inv_width(g, default_inv_width(g, 1));
  g.m0 = 0;
  g.count = 1;
  g.rsch = g.csch = g.rwv = 0;
  g.rpb = 1;
  const int cs = g.dbl ? 16 : 8;
  long long o = align256(sizeof(MemberDev));
  g.o_twx = o; o += align256((long long)g.nx * cs);
  g.o_twy = o; o += align256((long long)g.ny * cs);
  g.o_twx1 = o; o += align256((long long)g.nx * cs);
  g.o_twy1 = o; o += align256((long long)g.ny * cs);
  const long long region_off = o;
  const long long total = o + g.region_bytes;
  if (total > (long long)SCRATCH_BYTES) {
    char buf[200];
    snprintf(buf, sizeof buf, "member needs %lld bytes, the static scratch holds %zu", total, SCRATCH_BYTES);
    return fail(QG_EUNSUPPORTED, buf);
  }
  char* ws = static_cast<char*>(base);
  g.region0 = ws + region_off;
  g.twx = ws + g.o_twx;
  g.twy = ws + g.o_twy;
  g.twx1 = ws + g.o_twx1;
  g.twy1 = ws + g.o_twy1;
  Handle h;   // only mem_dev is read by the phase sequences below
  h.mem_dev = reinterpret_cast<MemberDev*>(ws);
  MemberDev m = make_member(*p, g.region0, 0, 0);
  m.tab_off = g.L.phys;
  // the array keeps the previous call's contents: clear what is used
  QG_LAUNCH(launch_fill_zero(ws, (size_t)total, st));
  QG_LAUNCH(launch_put_member(h.mem_dev, m, st));
  QG_LAUNCH(launch_twiddle_table(g.dbl, g.twx, g.lognx, 0, st));
  QG_LAUNCH(launch_twiddle_table(g.dbl, g.twy, g.logny, 0, st));
  QG_LAUNCH(launch_twiddle_table(g.dbl, g.twx1, g.lognx, 1, st));
  QG_LAUNCH(launch_twiddle_table(g.dbl, g.twy1, g.logny, 1, st));
  const size_t fb = (size_t)g.nx * g.ny * (g.dbl ? 8 : 4);
  char* phys = g.region0 + g.L.phys;
  QG_HIP(hipMemcpyAsync(phys + 4 * fb, chi_obs, fb, hipMemcpyDeviceToDevice, st));
  QG_HIP(hipMemcpyAsync(phys + 5 * fb, chi_sponge, fb, hipMemcpyDeviceToDevice, st));
  try {
    rc = mask_precompute(h, g, st);
    if (!rc) rc = run_entry(h, g, omega, g.L.wn, st);
    for (long long k = 0; k < nsteps && !rc; ++k) rc = run_step(h, g, st);
    if (!rc) rc = run_exit(h, g, g.L.wn, omega, st);
  } catch (...) {
    rc = fail(QG_EINVAL, "internal error in qg_step_noalloc");
  }
  return rc;
}

