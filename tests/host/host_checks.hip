// Host-side checks of the runtime under AddressSanitizer, UndefinedBehavior-
// Sanitizer and libstdc++ assertions (built by tests/test_host_sanitizers.py
// with the sanitizers on the host pass only).  The runtime's source is
// included so that its internal functions can be called directly; nothing
// here touches a GPU.
#include "../../paper_2508_06678_amd/csrc/qg_api.hip"

#include <cstdlib>
#include <set>

using namespace qg;

static int failures = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);       \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static qg_params member(int nx, int ny, int closure, int precision, int scheme) {
  qg_params p{};
  p.nx = nx;
  p.ny = ny;
  p.lx = 2.0 * M_PI;
  p.ly = 2.0 * M_PI * ny / nx;
  p.beta = 1.0;
  p.re = 1e3;
  p.u_in = 1.0;
  p.eta = 1e-2;
  p.sponge_sigma = 10.0;
  p.dt = 1e-3;
  p.c = 0.17;
  p.closure = closure;
  p.precision = precision;
  p.test_ratio = 2.0;
  p.fp64_lowk = 8;
  p.scheme = scheme;
  return p;
}

// every admitted size, closure, precision and scheme, alone and in ragged
// batches, with and without adjoint storage: the plan must be consistent
static void check_layouts() {
  for (int lnx = 5; lnx <= 12; ++lnx)
    for (int lny = 5; lny <= 12; ++lny)
      for (int cl = 0; cl <= 4; ++cl)
        for (int prec : {32, 64})
          for (int sch : {QG_SCHEME_RK4, QG_SCHEME_AB2CN})
            for (int adj : {0, 3}) {
              qg_params p = member(1 << lnx, 1 << lny, cl, prec, sch);
              size_t b = 0;
              const int rc = qg_workspace_bytes(&p, 1, adj, &b);
              const bool ab_ok = !(sch == QG_SCHEME_AB2CN &&
                                   ((1 << lnx) < 64 || (prec == 64 && ((1 << lnx) > 2048 || (1 << lny) > 2048))));
              CHECK(ab_ok ? rc == QG_OK && b > 0 : rc == QG_EUNSUPPORTED);
              if (rc != QG_OK) continue;
              Handle h;
              CHECK(build_layout(&p, 1, adj, h) == QG_OK);
              const Group& g = h.groups[0];
              CHECK(g.kxn == ((1 << lnx) - 1) / 3 + 1 && g.kyn == 2 * (((1 << lny) - 1) / 3) + 1);
              CHECK(g.L.total == g.region_bytes && g.L.mp > g.L.mf && g.L.phys > g.L.mp);
              CHECK((size_t)g.o_twy1 + (size_t)(1 << lny) * (prec == 64 ? 16 : 8) <= h.ws_bytes);
            }
  // a ragged batch: members grouped by size, closure, precision and scheme
  std::vector<qg_params> batch;
  for (int i = 0; i < 12; ++i) batch.push_back(member(64 << (i % 3), 32 << (i % 3), i % 5, i % 2 ? 32 : 64, 0));
  Handle h;
  CHECK(build_layout(batch.data(), (int)batch.size(), 2, h) == QG_OK);
  int members = 0;
  for (const auto& g : h.groups) members += (int)g.users.size();
  CHECK(members == 12 && h.groups.size() <= 12);
}

static void check_rejections() {
  size_t b = 0;
  qg_params p = member(96, 64, 1, 64, 0);
  CHECK(qg_workspace_bytes(&p, 1, 0, &b) == QG_EUNSUPPORTED);
  p = member(128, 64, 1, 64, 0);
  p.dt = std::nan("");
  CHECK(qg_workspace_bytes(&p, 1, 0, &b) == QG_EINVAL);
  p = member(128, 64, 1, 64, 0);
  p.eta = -1.0;
  CHECK(qg_workspace_bytes(&p, 1, 0, &b) == QG_EINVAL);
  p = member(128, 64, 1, 64, QG_SCHEME_AB2CN);
  p.eta = p.dt;
  CHECK(qg_workspace_bytes(&p, 1, 0, &b) == QG_EINVAL);
  p = member(128, 64, 9, 64, 0);
  CHECK(qg_workspace_bytes(&p, 1, 0, &b) == QG_EINVAL);
  CHECK(qg_workspace_bytes(nullptr, 1, 0, &b) == QG_EINVAL);
  CHECK(qg_workspace_bytes(&p, 0, 0, &b) == QG_EINVAL);
  CHECK(qg_workspace_bytes(&p, 1, -1, &b) == QG_EINVAL);
  CHECK(std::string(qg_last_error()).size() > 0);
  CHECK(qg_step_noalloc(nullptr, nullptr, nullptr, nullptr, 1, nullptr) == QG_EINVAL);
}

// every slot of every per-pass twiddle table written once, values on the
// unit circle
static void check_twiddles() {
  for (int logn = 5; logn <= 12; ++logn) {
    const int n = 1 << logn;
    std::vector<long double> fre, fim, re, im;
    twiddles(n, fre, fim);
    for (int m = 0; m < n; ++m) CHECK(std::fabs((double)(fre[m] * fre[m] + fim[m] * fim[m] - 1.0L)) < 1e-15);
    for (int sch = 0; sch < NSCHED; ++sch) {
      pass_twiddles(n, sch, fre, fim, re, im);
      CHECK((int)re.size() == n);
      int filled = 0;
      for (int o = 0; o < n - 8; ++o) filled += (re[o] != 0.0L || im[o] != 0.0L) ? 1 : 0;
      // the slots of k = 0 hold exp(0) = 1, so every one of the n - 8 slots is nonzero
      CHECK(filled == n - 8);
    }
  }
}

// the tuning cache: round trip, then malformed and hostile files
static void check_cache(const char* dir) {
  const std::string path = std::string(dir) + "/cache.json";
  std::map<std::string, int> m{{"gfx950/1024x1024/fp32/closure4/members1/fwd", 1},
                               {"gfx950/1024x1024/fp32/closure4/members1/rsched", 1},
                               {"gfx950/256x128/fp64/closure0/members9/inv", 16}};
  write_width_cache(path.c_str(), m);
  std::map<std::string, int> back;
  read_width_cache(path.c_str(), back);
  CHECK(back == m);
  const char* bad[] = {"", "{", "{\"", "{\"a", "{\"a\"", "{\"a\":", "{\"a\": }", "\"\"\"\"::::",
                       "{\"a\": 99999999999999999999}", "{\"a\": -3, \"b\" 4, \"c\": x}", "[1, 2, 3]",
                       "{\"k\": 1}}}}}}\"", "\xff\xfe\"z\":7"};
  for (const char* t : bad) {
    FILE* f = fopen(path.c_str(), "w");
    fputs(t, f);
    fclose(f);
    std::map<std::string, int> out;
    read_width_cache(path.c_str(), out);   // must neither crash nor read out of bounds
    CHECK(out.size() <= 4);
  }
  std::map<std::string, int> none;
  read_width_cache((std::string(dir) + "/missing.json").c_str(), none);
  CHECK(none.empty());
}

int main(int argc, char** argv) {
  check_layouts();
  check_rejections();
  check_twiddles();
  check_cache(argc > 1 ? argv[1] : ".");
  if (failures) {
    fprintf(stderr, "%d host check(s) failed\n", failures);
    return 1;
  }
  printf("host checks ok\n");
  return 0;
}
