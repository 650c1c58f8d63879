// HIP kernels of the QG step for gfx950.
//
// Data layout (per member, inside the caller's workspace):
//   spectral state   D-compact complex [kx][iy]: m_x in [0, kxn), m_y in
//                    [-myh, myh] stored as iy = m_y (m_y >= 0) or
//                    iy = m_y + kyn (m_y < 0), kyn = 2 myh + 1.
//                    The 2/3 set D is kxn = (nx-1)/3 + 1, myh = (ny-1)/3.
//   mixed fields     the output of a column-inverse pass / input of a row
//                    pass (MF) is row-major complex [field][y][kx] with row
//                    pitch kxp; the output of a row pass / input of a
//                    column-forward pass (MP) is strip-major complex
//                    [field][strip][y][w], kx = strip * W + w.  So every read
//                    of a mixed field is contiguous (row passes read rows,
//                    column-forward passes read strips) and only the writes
//                    are scattered (they do not stall the waves and merge in
//                    L2, see the XCD-aware block order).
//   physical tables  real [y][x]: S E, S E_x, S E_y (the B sub-step
//                    with the sponge factor folded in), a spare slot, chi,
//                    chi_sponge.
//
// Kernel kinds (Sec. II-C: derivatives in Fourier space, products by
// collocation, 2/3 de-aliasing of every product):
//   k_colinv  one block per (kx strip, field, member): builds the field's
//             spectral column from the state (Poisson inversion, spectral
//             derivatives, test filter), scales by 1/(nx ny), inverse FFT
//             along y in LDS, writes the strip of the mixed layout.
//   k_row     one block per (group of row pairs, member): for each field,
//             two rows packed as one complex row are taken to physical space
//             (c2r), the pointwise physics of the phase is applied, and each
//             product goes back to the retained half spectrum (r2c).
//   k_colfwd  one block per (kx strip, member): forward FFT along y of each
//             product, extraction of the retained modes, then the spectral
//             combine of the phase (right-hand side and RK4 update, dynamic
//             coefficient partial sums, B-step projection, adjoint sums).
#include <hip/hip_ext.h>

#include <cstdint>

#include "qg_fft.hpp"
#include "qg_internal.hpp"

// The library compiles this file once per slice (QG_PART = 0..4): the
// column and row launchers per precision in slices 0-3, everything else in
// slice 4, so that the kernel instantiations build in parallel.  Without
// QG_PART every slice is compiled.
#ifndef QG_PART
#define QG_PART -1
#endif
#define QG_HAS(p) (QG_PART < 0 || QG_PART == (p))

// LDS pad period (one slot every 2^P elements) of the compile-time-length
// row and column transforms
#ifndef QG_ROW_PADS
#define QG_ROW_PADS 4
#endif
#ifndef QG_COL_PADS
#define QG_COL_PADS 4
#endif

namespace qg {

// LDS column stride of the compile-time column-inverse path (elements)
__host__ __device__ constexpr int colinv_stride(int ny) { return ny + (ny >> QG_COL_PADS) + 16; }

// LDS poison (debug builds with QG_LDS_POISON): a kernel with dynamic LDS
// first sets all of it to NaN (bytes 0xff), so that a read of an element
// nothing has written yet carries NaN into the result; the transform passes
// poison their buffers again before each write phase (lds_poison).
__device__ __forceinline__ void lds_poison_all(unsigned char* lds, unsigned bytes) {
#ifdef QG_LDS_POISON
  unsigned* w = reinterpret_cast<unsigned*>(lds);
  for (unsigned i = threadIdx.x; i < bytes / 4; i += blockDim.x) w[i] = 0xffffffffu;
  __syncthreads();
#else
  (void)lds; (void)bytes;
#endif
}

// Phase stamps (debug builds with QG_STAMPS, for qg_stamp_steps): lane 0 of
// every wave of member 0 writes the real-time counter (100 MHz) at the
// phase boundaries of the four right-hand-side kernels, after an empty asm
// that takes `dep` as an operand, so that the stamp follows the work that
// produced it.  Slot 0 (the wave's start) also records the wave's hardware
// ids.  The stamps' own waits perturb the timing slightly.
#ifdef QG_STAMPS
__device__ __forceinline__ void stamp_write(unsigned long long* buf, int kind, int slot) {
  const unsigned long long t = __builtin_amdgcn_s_memrealtime();
  if (buf && (threadIdx.x & 63) == 0 && blockIdx.z == 0) {
    const unsigned w = (blockIdx.y * gridDim.x + blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w < (unsigned)QG_STAMP_WAVES) {
      unsigned long long* s = buf + ((size_t)kind * QG_STAMP_WAVES + w) * 8;
      s[slot] = t;
      if (slot == 0)   // hwreg(HW_REG_HW_ID, 0, 32) and hwreg(HW_REG_XCC_ID, 0, 16)
        s[7] = (unsigned long long)__builtin_amdgcn_s_getreg(63492) |
               ((unsigned long long)__builtin_amdgcn_s_getreg(30740) << 32);
    }
  }
}
#define QG_STAMP(kind, slot, dep)                 \
  do {                                            \
    asm volatile("" ::"v"(dep) : "memory");       \
    stamp_write(P.stamps, (kind), (slot));        \
  } while (0)
#define QG_STAMP_DRAIN(kind, slot)                    \
  do {                                                \
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  \
    stamp_write(P.stamps, (kind), (slot));            \
  } while (0)
#define QG_STAMP_LDS(kind, slot)                        \
  do {                                                  \
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  \
    stamp_write(P.stamps, (kind), (slot));              \
  } while (0)
#else
#define QG_STAMP(kind, slot, dep) do {} while (0)
#define QG_STAMP_DRAIN(kind, slot) do {} while (0)
#define QG_STAMP_LDS(kind, slot) do {} while (0)
#endif

// ---------------------------------------------------------------- helpers
// Workspace pointers come from the member table, so the compiler cannot see
// that they address global memory and would emit flat loads/stores (which
// also hold up every LDS wait).  Hot loads and stores go through explicit
// global-address-space pointers instead.
__device__ __forceinline__ char* as_global(char* p) { return p; }
template <typename S> struct nvec2;
template <> struct nvec2<float> { typedef float __attribute__((ext_vector_type(2))) t; };
template <> struct nvec2<double> { typedef double __attribute__((ext_vector_type(2))) t; };
template <typename V> __device__ __forceinline__ V gld(const V* p) {
  using N = typename nvec2<decltype(V{}.x)>::t;
  const N v = *(const __attribute__((address_space(1))) N*)(p);
  V r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
template <typename V> __device__ __forceinline__ void gst(V* p, const V& v) {
  using N = typename nvec2<decltype(V{}.x)>::t;
  N n;
  n.x = v.x;
  n.y = v.y;
  *(__attribute__((address_space(1))) N*)(p) = n;
}
template <typename S> struct nvec4;
template <> struct nvec4<float> { typedef float __attribute__((ext_vector_type(4))) t; };
template <> struct nvec4<double> { typedef double __attribute__((ext_vector_type(4))) t; };
// a at p, b at p + 1 as one vector store (p aligned to two elements)
template <typename V> __device__ __forceinline__ void gst_pair(V* p, const V& a, const V& b) {
  using N = typename nvec4<decltype(V{}.x)>::t;
  N n; n.x = a.x; n.y = a.y; n.z = b.x; n.w = b.y;
  *(__attribute__((address_space(1))) N*)(p) = n;
}

template <typename T> __device__ __forceinline__ cpx<T>* cptr(const MemberDev& M, long long off) {
  return reinterpret_cast<cpx<T>*>(as_global(M.base + off));
}
template <typename T> __device__ __forceinline__ T* rptr(const MemberDev& M, long long off) {
  return reinterpret_cast<T*>(as_global(M.base + off));
}

// Member table entry read through the constant address space: the table is
// written by the host only, so block-uniform reads of it become scalar
// loads (which neither wait for nor hold back the vector-memory counter).
__device__ __forceinline__ MemberDev member_const(const Phase& P, int m) {
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(4))) MemberDev* CT;
  return ((CT)(P.mem))[P.m0 + m];
#else
  return P.mem[P.m0 + m];   // host pass of the device code (never executed)
#endif
}

// XCD-aware block order: the hardware deals consecutive blocks to the 8
// XCDs in turn; with n a multiple of 8 this gives XCD x the contiguous range
// [x n/8, (x+1) n/8) of logical indices, so neighbouring strips (or rows)
// that share cache lines run on the same L2.
__device__ __forceinline__ int xcd_order(int b, int n) {
  return (n & 7) == 0 ? (b & 7) * (n >> 3) + (b >> 3) : b;
}

// signed m_y of compact index iy
__device__ __forceinline__ int my_of_iy(int iy, int myh, int kyn) { return iy <= myh ? iy : iy - kyn; }

// q / kyn for 0 <= q < kxn kyn (below 2^23 at every admitted size): the
// hardware reciprocal puts the quotient within 1e-3 of the truth, one exact
// 24-bit correction step makes it the integer quotient.  (A 32-bit integer
// division costs tens of instructions, several of them quarter rate.)
__device__ __forceinline__ int div_kyn(int q, int kyn) {
  int m = (int)((float)q * __builtin_amdgcn_rcpf((float)kyn));
  if (__umul24((unsigned)(m + 1), (unsigned)kyn) <= (unsigned)q) ++m;
  else if (__umul24((unsigned)m, (unsigned)kyn) > (unsigned)q) --m;
  return m;
}

__device__ __forceinline__ float qrcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double qrcp(double x) { return 1.0 / x; }

// Wavenumbers of mode (mx, my), in the arithmetic type of the run.  The
// double-precision 1/|k|^2 of the lowest modes (Poisson inversion of 32-bit
// runs) is formed separately in poisson().
template <typename T> struct Wave {
  T kx, ky, k2, inv_k2;
};
template <typename T> __device__ __forceinline__ Wave<T> wave(const MemberDev& M, int mx, int my) {
  Wave<T> w;
  w.kx = T(M.two_pi_lx) * T(mx);
  w.ky = T(M.two_pi_ly) * T(my);
  w.k2 = w.kx * w.kx + w.ky * w.ky;
  // 32-bit runs: the hardware reciprocal (about 1 ulp), 64-bit runs: division
  w.inv_k2 = (mx == 0 && my == 0) ? T(0) : qrcp(w.k2);
  return w;
}

// test filter T: test_ratio^2 (ny^2 mx^2 + nx^2 my^2) <= min(Mx ny, My nx)^2.
// The integer test is evaluated in double precision: with nx, ny <= 4096,
// |m| <= 2048 and test_ratio <= 4 every product is an integer of at most 2^51,
// so each operation is exact (and full rate, where 64-bit integer
// multiplies are not).
__device__ __forceinline__ bool in_test(const MemberDev& M, int nx, int ny, int mx, int my) {
  const double fx = (double)ny * (double)mx, fy = (double)nx * (double)my;
  return (double)M.test_r2 * (fx * fx + fy * fy) <= (double)M.test_lim;
}

// The same set, column by column: the largest |m_y| that passes in column
// m_x (-1 if none), so that in_test(mx, my) == (|my| <= test_mylim(mx));
// exact double arithmetic as in in_test.
__device__ __forceinline__ int test_mylim(const MemberDev& M, int nx, int ny, int mx) {
  const double fx = (double)ny * (double)mx;
  const double a = (double)M.test_r2 * (fx * fx);
  const double lim = (double)M.test_lim;
  if (a > lim) return -1;
  const double den = (double)M.test_r2 * ((double)nx * (double)nx);
  const double rem = lim - a;
  double s = floor(sqrt(rem / den));
  while (s > 0.0 && s * s * den > rem) s -= 1.0;
  while ((s + 1.0) * (s + 1.0) * den <= rem) s += 1.0;
  return (int)s;
}

// Band-limited transform inputs.  A length-N transform of the compile-time
// engines takes element t of thread j at index j + t N/8.  On the 2/3 set
// the nonzero indices are |m| <= (N - 1)/3 (m = index, or index - N in the
// upper half), so the blocks t = 3, 4 are empty; the test filter (test
// ratio >= 2) keeps |m| <= (N - 1)/6 + 1 <= N/4, so the blocks t = 2..5 are
// empty.  Bit t of the mask marks an empty block.
template <bool TEST> __host__ __device__ constexpr int band_zero_mask() { return TEST ? 0x3c : 0x18; }

// psi_hat = -x / |k|^2, in double precision for the lowest modes of 32-bit runs
template <typename T>
__device__ __forceinline__ cpx<T> poisson(const MemberDev& M, cpx<T> x, const Wave<T>& w, int mx, int my) {
  using V = cpx<T>;
  if (sizeof(T) == 4 && w.k2 <= T(M.lowk2) && (mx | my) != 0) {
    const double kx = M.two_pi_lx * mx, ky = M.two_pi_ly * my;
    const double ik2 = 1.0 / (kx * kx + ky * ky);
    return cmake<V>(T(-(double)x.x * ik2), T(-(double)x.y * ik2));
  }
  const T s = -w.inv_k2;
  return cmake<V>(x.x * s, x.y * s);
}

// multiply by i a (a real)
template <typename V, typename S> __device__ __forceinline__ V mul_ia(V z, S a) {
  return cmake<V>(-z.y * a, z.x * a);
}

// ---------------------------------------------------------------- fields
// Spectral field f of a column-inverse launch at mode (mx, my), before the
// 1/(nx ny) scaling.  x: state (or stage input) at the mode; l: adjoint
// variable at the mode (adjoint ops only).
//
// RHS / DIAG fields, per level (grid, then test-filtered for the dynamic
// closures): 0 u' = -i ky psi, 1 v' = i kx psi, 2 omega_x = i kx x,
// 3 omega_y = i ky x, and for the Smagorinsky family 4 psi_xx - psi_yy =
// (ky^2 - kx^2) psi, 5 psi_xy = -kx ky psi (Eq. 1, Eq. 9).
template <typename T, int CL>
__device__ __forceinline__ cpx<T> rhs_field(const MemberDev& M, int f, cpx<T> x, const Wave<T>& w, int mx, int my,
                                            bool test) {
  using V = cpx<T>;
  constexpr int nb = (CL == 1 || CL == 3) ? 6 : 4;
  const int kind = f % nb;
  if (f >= nb && !test) return cmake<V>(T(0), T(0));
  const T kx = T(w.kx), ky = T(w.ky);
  if (kind == 2) return mul_ia(x, kx);
  if (kind == 3) return mul_ia(x, ky);
  V psi = poisson<T>(M, x, w, mx, my);
  if (kind == 0) return mul_ia(psi, -ky);
  if (kind == 1) return mul_ia(psi, kx);
  if (kind == 4) { T a = T(w.ky * w.ky - w.kx * w.kx); return cmake<V>(psi.x * a, psi.y * a); }
  T a = T(-w.kx * w.ky);
  return cmake<V>(psi.x * a, psi.y * a);
}

// Flux coefficient of the adjoint right-hand-side pass: 1 for the dynamic
// closures (their flux cotangent carries C), else the static coefficient.
template <typename T>
__device__ __forceinline__ T adj_coef(const MemberDev& M, const Phase& P) {
  if (P.adj_mode != 0 || P.adj_dyn) return T(1);
  return T(M.coef_static);
}

// A right-hand-side (or diagnostics) field at a test-filtered mode from
// its already loaded spectral value x (the caller's loads run ahead of the
// test set's extent).
template <typename T, int CL>
__device__ __forceinline__ cpx<T> rhs_test_value(const MemberDev& M, const Phase& P, int f, int mx, int iy, cpx<T> x) {
  const int my = my_of_iy(iy, P.myh, P.kyn);
  return rhs_field<T, CL>(M, f, x, wave<T>(M, mx, my), mx, my, true);
}

// A column-inverse field outside the test set (right-hand side,
// diagnostics, B sub-step) from its already loaded spectral value x.
template <typename T, int OP, int CL>
__device__ __forceinline__ cpx<T> colinv_field(const MemberDev& M, const Phase& P, int f, int mx, int iy, cpx<T> x) {
  const int my = my_of_iy(iy, P.myh, P.kyn);
  const Wave<T> w = wave<T>(M, mx, my);
  if constexpr (OP == OP_B) {
    if (f == 2) return x;
    const cpx<T> psi = poisson<T>(M, x, w, mx, my);
    return f == 0 ? mul_ia(psi, T(-w.ky)) : mul_ia(psi, T(w.kx));
  } else {
    return rhs_field<T, CL>(M, f, x, w, mx, my, false);
  }
}

// mylim: test_mylim(mx) of the dynamic closures (-2: evaluate in_test)
template <typename T, int OP, int CL>
__device__ __forceinline__ cpx<T> colinv_value(const MemberDev& M, const Phase& P, int f, int mx, int iy,
                                               int mylim = -2) {
  using V = cpx<T>;
  const int my = my_of_iy(iy, P.myh, P.kyn);
  const int idx = mx * P.kyn + iy;   // < 2^31 for every admissible size
  const Wave<T> w = wave<T>(M, mx, my);
  const bool zero_mean = (mx == 0 && my == 0);
  if constexpr (OP == OP_RHS || OP == OP_DIAG) {
    V x = gld(cptr<T>(M, P.o_in) + idx);
    const bool test = dynamic_closure(CL)
                          ? (mylim >= -1 ? (my <= mylim && -my <= mylim) : in_test(M, P.nx, P.ny, mx, my))
                          : false;
    return rhs_field<T, CL>(M, f, x, w, mx, my, test);
  } else if constexpr (OP == OP_B) {
    V x = gld(cptr<T>(M, P.o_in) + idx);
    if (f == 2) return x;
    V psi = poisson<T>(M, x, w, mx, my);
    return f == 0 ? mul_ia(psi, T(-w.ky)) : mul_ia(psi, T(w.kx));
  } else if constexpr (OP == OP_EXIT) {
    V x = gld(cptr<T>(M, P.o_in) + idx);
    return zero_mean ? cmake<V>(T(0), T(0)) : x;
  } else if constexpr (OP == OP_SPONGE) {
    // field 0: omega*, field 1: omega** (omega* itself before any history)
    const bool first = rptr<double>(M, P.o_coef)[AB2CN_FLAG_SLOT] == 0.0;
    V x = gld(cptr<T>(M, (f == 0 || first) ? P.o_in : P.o_in2) + idx);
    return zero_mean ? cmake<V>(T(0), T(0)) : x;
  } else if constexpr (OP == OP_CLIPF) {
    // the stage's H (field 0) and M (field 1), mean modes included
    return gld(cptr<T>(M, f == 0 ? P.o_h : P.o_m) + idx);
  } else if constexpr (OP == OP_GTERMS) {
    // fields u', v', omega_x, omega_y, omega
    V x = gld(cptr<T>(M, P.o_in) + idx);
    if (f == 4) return zero_mean ? cmake<V>(T(0), T(0)) : x;
    return rhs_field<T, 0>(M, f, x, w, mx, my, false);
  } else if constexpr (OP == OP_MASKGRAD) {
    V x = gld(cptr<T>(M, P.o_in) + idx);
    return f == 0 ? mul_ia(x, T(w.kx)) : mul_ia(x, T(w.ky));
  } else if constexpr (OP == OP_ADJ_B) {
    V l = gld(cptr<T>(M, P.o_in) + idx);
    return zero_mean ? cmake<V>(T(0), T(0)) : l;
  } else {  // OP_ADJ_RHS: forward fields of the stage input, then -l, -i kx l, -i ky l
    constexpr int nb = (CL == 1) ? 6 : 4;
    // adj_mode 2 (dynamic closures): both passes of a stage in one launch,
    // the fields of the stage's own pass (mode 0 with the coefficient's
    // cotangents) first, then those of the transport pass at the
    // test-filtered input (mode 1)
    int mode = P.adj_mode, dynp = P.adj_dyn;
    if (mode == 2) {
      const int nfl = P.nf / 2;
      if (f >= nfl) { f -= nfl; mode = 1; dynp = 0; }
      else { mode = 0; dynp = 1; }
    }
    const bool t = (mode != 0 || dynp) && in_test(M, P.nx, P.ny, mx, my);
    if (f < nb) {
      V x = gld(cptr<T>(M, P.o_in) + idx);
      if (mode == 1 && !t) x = cmake<V>(T(0), T(0));   // the test-filtered stage input
      return rhs_field<T, CL>(M, f, x, w, mx, my, false);
    }
    if (zero_mean) return cmake<V>(T(0), T(0));
    const int a = f - nb;
    // the Jacobian's cotangent cJ and the flux's cQ, given as cJ, -i kx cQ,
    // -i ky cQ (the row pass's flux coefficient is 1 where cQ carries it):
    //   static closures:            cJ = -l,          cQ = l (coefficient c)
    //   dynamic, at the stage input: cJ = -l - T a,   cQ = C l - T b
    //   dynamic, at T x (mode 1):    cJ = a,          cQ = r b
    // with l the stage's cotangent and a, b those of H and M
    V cj, cq;
    if (mode == 1) {
      cj = gld(cptr<T>(M, P.o_a) + idx);
      cq = cscale(gld(cptr<T>(M, P.o_b) + idx), T(M.r_test));
    } else {
      const V l = gld(cptr<T>(M, P.o_in2) + idx);
      cj = cmake<V>(-l.x, -l.y);
      cq = l;
      if (dynp) {
        cq = cscale(l, T(rptr<double>(M, P.o_coef)[ADJ_C_SLOT]));
        if (t) {
          cj = csub(cj, gld(cptr<T>(M, P.o_a) + idx));
          cq = csub(cq, gld(cptr<T>(M, P.o_b) + idx));
        }
      }
    }
    if (a == 0) return cj;
    return mul_ia(cq, a == 1 ? T(-w.kx) : T(-w.ky));
  }
}

// ---------------------------------------------------------------- colinv
// One block per (strip of Wi columns, field f): spectral field values of
// the strip, inverse transform along y, rows written to the field's
// row-major physical-y / spectral-x intermediate.  LOGN = log2(ny) selects
// one compile-time-length transform per column (ny/8 threads each, the
// first pass fed from registers, twiddles from the global table); LOGN = 0
// the run-time engines.
template <typename T, int OP, int CL, int LOGN, int SCH = 0>
__global__ void __launch_bounds__(COL_MAX_THREADS, 4) k_colinv(Phase P) {
  using V = cpx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  lds_poison_all(smem_raw, P.lds_bytes);
  V* tile = reinterpret_cast<V*>(smem_raw);
  if constexpr (OP == OP_RHS) QG_STAMP(1, 0, 0.f);
  const MemberDev M = member_const(P, blockIdx.z);
  const int f = blockIdx.y;
  int strip = xcd_order(blockIdx.x, gridDim.x);
  // test-filtered fields of the dynamic closures vanish beyond column
  // test_kx; the row pass reads no further, so nothing is written there.
  // Their strips are spread over the eight XCDs like the full fields'
  // (consecutive strips on one XCD), not left on the first few.
  if constexpr (OP == OP_RHS && dynamic_closure(CL)) {
    if (f >= rhs_fields(CL) / 2) {
      const int ns = (min(P.kxn, M.test_kx) + P.Wi - 1) / P.Wi;
      const int s8 = (ns + 7) >> 3;
      if ((int)(blockIdx.x >> 3) >= s8) return;
      strip = (blockIdx.x & 7) * s8 + (blockIdx.x >> 3);
      if (strip >= ns) return;
    }
  }
  if (strip * P.Wi >= P.kxn) return;
  const int kx0 = strip * P.Wi;
  const int ny = P.ny;
  const int n = P.Wi * ny;
  const T scale = T(M.inv_n);
  if constexpr (LOGN != 0) {
    constexpr int PD = QG_COL_PADS;
    // column stride: the padded length plus 16 elements, so that columns
    // w and w+1 start 32 banks apart and the strip's row-order read-out
    // below touches each bank twice (the minimum for 8-byte elements)
    // rather than four times
    constexpr int NY = 1 << LOGN, NT = NY / 8, STR = colinv_stride(NY);
    const int w = threadIdx.x >> (LOGN - 3);
    const int j = threadIdx.x & (NT - 1);
    const int mx = kx0 + w;
    V* buf = tile + w * STR;
    // Rows y = j + t NY/8 of the column (m_y = y, or y - NY in the upper
    // half).  The 2/3 set keeps |m_y| <= myh = (NY - 1)/3: the blocks t =
    // 0, 1, 6, 7 hold only such rows, t = 3, 4 none.  The test filter keeps
    // |m_y| <= test_mylim(m_x) <= (NY - 1)/6 (test ratio >= 2): blocks t =
    // 2..5 hold none.  Empty blocks are neither formed nor added in the
    // first radix-8 pass.
    constexpr int MYH = (NY - 1) / 3;
    const bool testf = dynamic_closure(CL) && (OP == OP_RHS || OP == OP_DIAG) && f >= rhs_fields(CL) / 2;
    // the second pass's twiddles, loaded alongside the column's values
    const V* twc = reinterpret_cast<const V*>(SCH ? P.twy1 : P.twy);
    const auto tw1 = fft1c_first_tw<V, LOGN, SCH>(twc, j);
    V v[8];
    if (testf) {
      // the spectral values of the blocks t = 0, 1, 6, 7 (|m_y| < NY/4 <=
      // myh: always inside the stored set) are loaded first, so that their
      // latency overlaps the test set's extent in this column (a double
      // square root and its exact integer correction)
      const int mxl = mx < P.kxn ? mx : P.kxn - 1;
      const V* xin = cptr<T>(M, P.o_in) + (long long)mxl * P.kyn;
      V xr[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t >= 2 && t <= 5) continue;
        const int y = j + t * NT;
        const int my = t < 4 ? y : y - NY;
        xr[t] = gld(xin + (my >= 0 ? my : my + P.kyn));
      }
      const int mylim = mx < P.kxn ? test_mylim(M, P.nx, NY, mx) : -1;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        v[t] = cmake<V>(T(0), T(0));
        if (t >= 2 && t <= 5) continue;
        const int y = j + t * NT;
        const int my = t < 4 ? y : y - NY;
        if (my <= mylim && -my <= mylim) {
          const int iy = my >= 0 ? my : my + P.kyn;
          v[t] = cscale(rhs_test_value<T, CL>(M, P, f, mx, iy, xr[t]), scale);
        }
      }
      if constexpr (OP == OP_RHS) QG_STAMP(1, 1, v[0].x);
      fft1c_pass0<V, true, PD, band_zero_mask<true>(), 8, false, LOGN>(v, buf, j, true);
    } else if constexpr (OP == OP_RHS || OP == OP_DIAG || OP == OP_B) {
      // every load of the column first, then the fields: a field formed
      // right after its (lane-conditional) load would wait there for all
      // loads issued before, one round trip per block of rows
      const V* xin = cptr<T>(M, P.o_in) + (long long)mx * P.kyn;
      V xr[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        xr[t] = cmake<V>(T(0), T(0));
        if (t == 3 || t == 4) continue;
        const int y = j + t * NT;
        const int my = t < 4 ? y : y - NY;
        const bool in = (t <= 1 || t >= 6) || (t == 2 ? my <= MYH : -my <= MYH);
        if (mx < P.kxn && in) xr[t] = gld(xin + (my >= 0 ? my : my + P.kyn));
      }
      asm volatile("" ::: "memory");
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        v[t] = cmake<V>(T(0), T(0));
        if (t == 3 || t == 4) continue;
        const int y = j + t * NT;
        const int my = t < 4 ? y : y - NY;
        const bool in = (t <= 1 || t >= 6) || (t == 2 ? my <= MYH : -my <= MYH);
        if (mx < P.kxn && in) v[t] = cscale(colinv_field<T, OP, CL>(M, P, f, mx, my >= 0 ? my : my + P.kyn, xr[t]), scale);
      }
      if constexpr (OP == OP_RHS) QG_STAMP(1, 1, v[0].x);
      fft1c_pass0<V, true, PD, band_zero_mask<false>(), 8, false, LOGN>(v, buf, j, true);
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        v[t] = cmake<V>(T(0), T(0));
        if (t == 3 || t == 4) continue;
        const int y = j + t * NT;
        const int my = t < 4 ? y : y - NY;
        const bool in = (t <= 1 || t >= 6) || (t == 2 ? my <= MYH : -my <= MYH);
        if (mx < P.kxn && in) {
          const int iy = my >= 0 ? my : my + P.kyn;
          v[t] = cscale(colinv_value<T, OP, CL>(M, P, f, mx, iy, -1), scale);
        }
      }
      fft1c_pass0<V, true, PD, band_zero_mask<false>(), 8, false, LOGN>(v, buf, j, true);
    }
    fft1c_rest<V, LOGN, true, PD, SCH>(buf, twc, j, true, tw1);
    if constexpr (OP == OP_RHS) QG_STAMP_LDS(1, 2);
    // rows of the strip: Wi values of row y per thread group of Wi
    // threads, eight rows NY/8 apart per thread
    V* out = cptr<T>(M, P.o_mf) + (long long)f * NY * P.mfp + kx0;
    const int c = threadIdx.x & (P.Wi - 1);
    const int y0 = threadIdx.x >> P.logWi;
    const V* src = tile + c * STR + padp<PD>(y0);
    V* dst = out + y0 * P.mfp + c;
#pragma unroll
    for (int i = 0; i < 8; ++i) gst(dst + i * (NY / 8) * P.mfp, src[i * (NY / 8 + (NY / 8 >> PD))]);
    if constexpr (OP == OP_RHS) QG_STAMP_DRAIN(1, 3);
    return;
  }
  V* twl = tile + P.Wi * P.ny + (P.Wi == 1 ? P.ny / 8 : 0);
  stage_twiddles<V>(twl, reinterpret_cast<const V*>(P.twy), P.logny);
  if (P.Wi == 1) {
    // one column: padded single-vector transform, first pass from registers
    const int j = threadIdx.x;
    const int n8 = ny >> 3;
    V v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int y = j + t * n8;
      const int my = y < ny / 2 ? y : y - ny;
      V z = cmake<V>(T(0), T(0));
      if (kx0 < P.kxn && my <= P.myh && -my <= P.myh) {
        const int iy = my >= 0 ? my : my + P.kyn;
        z = cscale(colinv_value<T, OP, CL>(M, P, f, kx0, iy), scale);
      }
      v[t] = z;
    }
    __syncthreads();   // twiddles staged
    fft1_pass0<V, true>(v, tile, j, true, P.logny);
    fft1_rest<V, true>(tile, twl, P.logny, j, true);
    V* out = cptr<T>(M, P.o_mf) + (long long)f * ny * P.mfp + kx0;
    for (int y = j; y < ny; y += n8) gst(out + (long long)y * P.mfp, tile[pad8(y)]);
    return;
  }
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int w = q >> P.logny;
    const int y = q & (ny - 1);
    const int mx = kx0 + w;
    const int my = y < ny / 2 ? y : y - ny;
    V v = cmake<V>(T(0), T(0));
    if (mx < P.kxn && my <= P.myh && -my <= P.myh) {
      const int iy = my >= 0 ? my : my + P.kyn;
      v = colinv_value<T, OP, CL>(M, P, f, mx, iy);
      v = cscale(v, scale);
    }
    tile[y * P.Wi + w] = v;
  }
  __syncthreads();
  FftShape s{P.logny, P.Wi, 1, P.logWi, true};
  fft_lds<V, true, COL_EPT>(tile, twl, s);
  V* out = cptr<T>(M, P.o_mf) + (long long)f * ny * P.mfp + kx0;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int w = q & (P.Wi - 1);
    const int y = q >> P.logWi;
    gst(out + (long long)y * P.mfp + w, tile[q]);
  }
}

// ---------------------------------------------------------------- row pass
constexpr int ROW_EPT = 8;

template <typename T> struct RowCtx {
  using V = cpx<T>;
  V* buf;            // RP rows of nx complex
  const V* tw;
  int nx, lognx, RP, logRP, kxn, kxp, ny, logW;
  int kin;           // c2r input columns: m_x < kin (kin <= kxn)
  int y0;            // first row of the block
};

// position of (y, kx) in a strip-major mixed field (fits in 32 bits: at
// most 4096 rows x 1366 columns per field)
template <typename T> __device__ __forceinline__ int mix_at(const RowCtx<T>& C, int y, int k) {
  return (((k >> C.logW) * C.ny + y) << C.logW) + (k & ((1 << C.logW) - 1));
}

// c2r of field src (strip-major mixed layout) for the block's row
// pairs; returns each thread's ROW_EPT elements: .x row 2rp, .y row 2rp+1.
template <typename T>
__device__ __forceinline__ void row_c2r(const RowCtx<T>& C, const cpx<T>* __restrict__ src, cpx<T> (&out)[ROW_EPT]) {
  using V = cpx<T>;
  const int n = C.RP * C.nx;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    const int rp = q >> C.lognx;
    const int k = q & (C.nx - 1);
    const int ya = C.y0 + 2 * rp;
    V z = cmake<V>(T(0), T(0));
    if (k < C.kin) {
      const int o = ya * C.kxp + k;
      V a = gld(src + o);
      V b = gld(src + o + C.kxp);
      if (k == 0) { a.y = T(0); b.y = T(0); }
      z = cmake<V>(a.x - b.y, a.y + b.x);
    } else if (k > C.nx - C.kin) {
      const int kk = C.nx - k;
      const int o = ya * C.kxp + kk;
      V a = gld(src + o);
      V b = gld(src + o + C.kxp);
      z = cmake<V>(a.x + b.y, b.x - a.y);
    }
    C.buf[q] = z;
  }
  __syncthreads();
  FftShape s{C.lognx, 1, C.nx, C.logRP, false};
  fft_lds<V, true, ROW_EPT>(C.buf, C.tw, s);
#pragma unroll
  for (int i = 0; i < ROW_EPT; ++i) {
    const int q = threadIdx.x + i * blockDim.x;
    out[i] = q < n ? C.buf[q] : cmake<V>(T(0), T(0));
  }
  __syncthreads();
}

// r2c of the thread's ROW_EPT product values (.x row 2rp, .y row 2rp+1),
// keeping m_x < kxn, written to dst (mixed layout).
template <typename T>
__device__ __forceinline__ void row_r2c(const RowCtx<T>& C, const cpx<T> (&val)[ROW_EPT], cpx<T>* __restrict__ dst) {
  using V = cpx<T>;
  const int n = C.RP * C.nx;
#pragma unroll
  for (int i = 0; i < ROW_EPT; ++i) {
    const int q = threadIdx.x + i * blockDim.x;
    if (q < n) C.buf[q] = val[i];
  }
  __syncthreads();
  FftShape s{C.lognx, 1, C.nx, C.logRP, false};
  fft_lds<V, false, ROW_EPT>(C.buf, C.tw, s);
  for (int rp = 0; rp < C.RP; ++rp) {
    const V* row = C.buf + rp * C.nx;
    const int ya = C.y0 + 2 * rp;
    for (int k = threadIdx.x; k < C.kxn; k += blockDim.x) {
      V z = row[k];
      V zm = row[(C.nx - k) & (C.nx - 1)];
      V a = cmake<V>(T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y));
      V b = cmake<V>(T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x));
      const int o = mix_at(C, ya, k);
      gst(dst + o, a);
      gst(dst + o + (1 << C.logW), b);
    }
  }
  __syncthreads();
}

template <typename T> __device__ __forceinline__ cpx<T> vmul(cpx<T> a, cpx<T> b) { return cmake<cpx<T>>(a.x * b.x, a.y * b.y); }
template <typename T> __device__ __forceinline__ cpx<T> vadd(cpx<T> a, cpx<T> b) { return cmake<cpx<T>>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cpx<T> vsub(cpx<T> a, cpx<T> b) { return cmake<cpx<T>>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cpx<T> vfma(cpx<T> a, cpx<T> b, cpx<T> c) { return cmake<cpx<T>>(a.x * b.x + c.x, a.y * b.y + c.y); }
// square roots: the hardware instruction in 32-bit runs (about 1 ulp), the
// correctly rounded one in 64-bit runs
__device__ __forceinline__ float qsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double qsqrt(double x) { return sqrt(x); }
template <typename T> __device__ __forceinline__ T strain(T pxy, T pd) { return qsqrt(T(4) * pxy * pxy + pd * pd); }
template <typename T> __device__ __forceinline__ T gradmag(T a, T b) { return qsqrt(a * a + b * b); }

// block-wide fixed-order sum of a double (deterministic)
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t += red[i];
  }
  __syncthreads();
  return t;  // valid in thread 0
}

// two block-wide fixed-order sums in one pass of barriers (the same order as
// two block_sum calls; red: 2 doubles per wave)
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  __syncthreads();
  if (lane == 0) {
    red[2 * wid] = a;
    red[2 * wid + 1] = b;
  }
  __syncthreads();
  double ta = 0.0, tb = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) {
      ta += red[2 * i];
      tb += red[2 * i + 1];
    }
  }
  a = ta;   // valid in thread 0
  b = tb;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = -INFINITY;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) t = fmax(t, red[i]);
  }
  __syncthreads();
  return t;
}

template <typename T, int OP, int CL>
__global__ void __launch_bounds__(512, (sizeof(T) == 4 && OP != OP_ADJ_RHS ? 4 : 2)) k_row(Phase P) {
  using V = cpx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  lds_poison_all(smem_raw, P.lds_bytes);
  const MemberDev M = member_const(P, blockIdx.z);
  RowCtx<T> C;
  C.buf = reinterpret_cast<V*>(smem_raw);
  {
    V* twl = C.buf + P.RP * P.nx;
    stage_twiddles<V>(twl, reinterpret_cast<const V*>(P.twx), P.lognx);
    C.tw = twl;
  }
  C.nx = P.nx; C.lognx = P.lognx; C.RP = P.RP; C.logRP = P.logRP;
  C.kxn = P.kxn; C.kin = P.kxn; C.kxp = P.mfp; C.ny = P.ny; C.logW = P.logW;
  // XCD-aware order: the hardware deals blocks to the 8 XCDs round-robin;
  // give each XCD a contiguous range of rows so mixed-layout lines shared by
  // neighbouring row blocks meet in the same L2.
  int rb = blockIdx.x;
  if ((gridDim.x & 7) == 0) rb = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  C.y0 = rb * 2 * P.RP;
  __shared__ double red[16];
  const long long fstride = (long long)P.ny * P.mfp;   // MF field stride
  const long long pstride = (long long)P.ny * P.kxp;   // MP field stride
  const V* mf = cptr<T>(M, P.o_mf);
  V* mp = cptr<T>(M, P.o_mp);
  const int npts = P.RP * P.nx;
  const long long nxy = (long long)P.nx * P.ny;

  // physical (x, y) of element i of this thread
  auto phys_index = [&](int i) -> long long {
    const int q = threadIdx.x + i * blockDim.x;
    const int rp = q >> P.lognx;
    const int x = q & (P.nx - 1);
    return (long long)(C.y0 + 2 * rp) * P.nx + x;
  };
  auto valid = [&](int i) { return threadIdx.x + i * blockDim.x < npts; };

  if constexpr (OP == OP_RHS || OP == OP_DIAG) {
    constexpr bool smag = (CL == 1 || CL == 3);
    constexpr bool dyn = (CL == 3 || CL == 4);
    constexpr int nb = smag ? 6 : 4;
    constexpr int levels = (OP == OP_RHS && dyn) ? 2 : 1;
    const T U = T(M.u_in), Vv = T(M.v_in);
    double nu_min = INFINITY, nu_max = -INFINITY, nu_sum = 0.0, cfl = 0.0, bad = 0.0;
    T coef = T(0);
    if constexpr (OP == OP_DIAG) coef = dyn ? T(rptr<double>(M, P.o_coef)[0]) : T(M.coef_static);
#pragma unroll 1
    for (int lev = 0; lev < levels; ++lev) {
      const V* F = mf + (long long)lev * nb * fstride;
      V* out = mp + (long long)lev * 3 * pstride;
      C.kin = lev == 0 ? P.kxn : min(P.kxn, M.test_kx);   // test-filtered level: m_x < test_kx
      V base[ROW_EPT], wx[ROW_EPT], wy[ROW_EPT], t0[ROW_EPT], t1[ROW_EPT];
      if constexpr (CL != 0) {
        if constexpr (smag) {
          row_c2r<T>(C, F + 4 * fstride, t0);
          row_c2r<T>(C, F + 5 * fstride, t1);
#pragma unroll
          for (int i = 0; i < ROW_EPT; ++i)
            base[i] = cmake<V>(strain<T>(t1[i].x, t0[i].x), strain<T>(t1[i].y, t0[i].y));
        }
      }
      row_c2r<T>(C, F + 2 * fstride, wx);
      row_c2r<T>(C, F + 3 * fstride, wy);
      if constexpr (CL == 2 || CL == 4) {
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i)
          base[i] = cmake<V>(gradmag<T>(wx[i].x, wy[i].x), gradmag<T>(wx[i].y, wy[i].y));
      }
      if constexpr (OP == OP_RHS && CL != 0) {
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i) t0[i] = vmul<T>(base[i], wx[i]);
        row_r2c<T>(C, t0, out + 1 * pstride);
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i) t0[i] = vmul<T>(base[i], wy[i]);
        row_r2c<T>(C, t0, out + 2 * pstride);
      }
      // advection by the total velocity: J = (U + u') omega_x + (V + v') omega_y
      row_c2r<T>(C, F + 0 * fstride, t0);
      row_c2r<T>(C, F + 1 * fstride, t1);
      if constexpr (OP == OP_RHS) {
        V J[ROW_EPT];
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i) {
          V u = cmake<V>(U + t0[i].x, U + t0[i].y);
          V v = cmake<V>(Vv + t1[i].x, Vv + t1[i].y);
          J[i] = vadd<T>(vmul<T>(u, wx[i]), vmul<T>(v, wy[i]));
        }
        row_r2c<T>(C, J, out);
      } else {
        // diagnostics: nu_e = C base, CFL, non-finite flag
        T* nu_out = P.user ? reinterpret_cast<T*>(reinterpret_cast<char*>(P.user) + M.omega_off) : nullptr;
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i) {
          if (!valid(i)) continue;
          const long long pi = phys_index(i);
          T u0 = U + t0[i].x, u1 = U + t0[i].y, v0 = Vv + t1[i].x, v1 = Vv + t1[i].y;
          T b0 = CL != 0 ? base[i].x : T(0), b1 = CL != 0 ? base[i].y : T(0);
          T n0 = coef * b0, n1 = coef * b1;
          if (nu_out) {
            nu_out[pi] = n0;
            nu_out[pi + P.nx] = n1;
          }
          nu_min = fmin(nu_min, fmin((double)n0, (double)n1));
          nu_max = fmax(nu_max, fmax((double)n0, (double)n1));
          nu_sum += (double)n0 + (double)n1;
          cfl = fmax(cfl, fmax((double)(fabs(u0) + fabs(v0)), (double)(fabs(u1) + fabs(v1))));
          const bool fin = isfinite(u0) && isfinite(u1) && isfinite(v0) && isfinite(v1) &&
                           isfinite(wx[i].x) && isfinite(wx[i].y) && isfinite(wy[i].x) && isfinite(wy[i].y);
          if (!fin) bad = 1.0;
        }
      }
    }
    if constexpr (OP == OP_DIAG) {
      double s0 = block_sum(nu_sum, red);
      double mn = -block_max(-nu_min, red);
      double mx = block_max(nu_max, red);
      double cf = block_max(cfl, red);
      double bd = block_max(bad, red);
      if (threadIdx.x == 0) {
        double* d = rptr<double>(M, P.o_dpart) + 5 * blockIdx.x;
        d[0] = s0; d[1] = mn; d[2] = mx; d[3] = cf; d[4] = bd;
      }
    }
  } else if constexpr (OP == OP_B) {
    // omega'' = S (E omega + E_x v - E_y u) (total velocity), with the
    // tables S E, S E_x, S E_y
    V u[ROW_EPT], v[ROW_EPT], w[ROW_EPT];
    row_c2r<T>(C, mf + 0 * fstride, u);
    row_c2r<T>(C, mf + 1 * fstride, v);
    row_c2r<T>(C, mf + 2 * fstride, w);
    const T* SE = rptr<T>(M, M.tab_off);
    const T* SEx = SE + nxy;
    const T* SEy = SE + 2 * nxy;
    const T U = T(M.u_in), Vv = T(M.v_in);
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) {
      if (!valid(i)) continue;
      const long long a = phys_index(i), b = a + P.nx;
      const T w0 = SE[a] * w[i].x + SEx[a] * (Vv + v[i].x) - SEy[a] * (U + u[i].x);
      const T w1 = SE[b] * w[i].y + SEx[b] * (Vv + v[i].y) - SEy[b] * (U + u[i].y);
      w[i] = cmake<V>(w0, w1);
    }
    row_r2c<T>(C, w, mp);
  } else if constexpr (OP == OP_ENTRY || OP == OP_MASKFWD) {
    const T* src = OP == OP_ENTRY
        ? reinterpret_cast<const T*>(reinterpret_cast<const char*>(P.user_in) + M.omega_off)
        : rptr<T>(M, P.o_phys) + 4 * nxy;
    V w[ROW_EPT];
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) {
      if (!valid(i)) { w[i] = cmake<V>(T(0), T(0)); continue; }
      const long long a = phys_index(i);
      w[i] = cmake<V>(src[a], src[a + P.nx]);
    }
    row_r2c<T>(C, w, mp);
  } else if constexpr (OP == OP_EXIT) {
    V w[ROW_EPT];
    row_c2r<T>(C, mf, w);
    T* dst = reinterpret_cast<T*>(reinterpret_cast<char*>(P.user) + M.omega_off);
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) {
      if (!valid(i)) continue;
      const long long a = phys_index(i);
      dst[a] = w[i].x;
      dst[a + P.nx] = w[i].y;
    }
  } else if constexpr (OP == OP_MASKGRAD) {
    V cx[ROW_EPT], cy[ROW_EPT];
    row_c2r<T>(C, mf + 0 * fstride, cx);
    row_c2r<T>(C, mf + 1 * fstride, cy);
    T* E = rptr<T>(M, P.o_phys);
    const T* chi = E + 4 * nxy;
    const T* chs = E + 5 * nxy;
    const double a = M.pen_a, sa = M.sponge_a;
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) {
      if (!valid(i)) continue;
      const long long p0 = phys_index(i);
      for (int r = 0; r < 2; ++r) {
        const long long p = p0 + r * P.nx;
        const double gx = r ? (double)cx[i].y : (double)cx[i].x;
        const double gy = r ? (double)cy[i].y : (double)cy[i].x;
        // the B sub-step's tables S E, S E_x, S E_y (one rounding each)
        const double e = exp(-a * (double)chi[p]);
        const double sp = exp(-sa * (double)chs[p]);
        E[p] = T(sp * e);
        E[p + nxy] = T(sp * (-a * gx * e));
        E[p + 2 * nxy] = T(sp * (-a * gy * e));
      }
    }
  } else if constexpr (OP == OP_ADJ_B) {
    // lambda'' = c2r(lambda); products (the transposed tables S E, S E_x,
    // S E_y): 0: S E lambda'' (omega), 1: -S E_y lambda'' (u), 2: S E_x lambda'' (v)
    V l[ROW_EPT], a0[ROW_EPT], a1[ROW_EPT];
    row_c2r<T>(C, mf, l);
    const T* SE = rptr<T>(M, M.tab_off);
    const T* SEx = SE + nxy;
    const T* SEy = SE + 2 * nxy;
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) {
      if (!valid(i)) { l[i] = a0[i] = a1[i] = cmake<V>(T(0), T(0)); continue; }
      const long long a = phys_index(i), b = a + P.nx;
      const T s0 = l[i].x, s1 = l[i].y;
      l[i] = cmake<V>(SE[a] * s0, SE[b] * s1);
      a0[i] = cmake<V>(-SEy[a] * s0, -SEy[b] * s1);
      a1[i] = cmake<V>(SEx[a] * s0, SEx[b] * s1);
    }
    row_r2c<T>(C, l, mp);
    row_r2c<T>(C, a0, mp + pstride);
    row_r2c<T>(C, a1, mp + 2 * pstride);
  } else if constexpr (OP == OP_ADJ_RHS) {
    // Adjoint of J = u omega_x + v omega_y, h = base grad omega, base(.)
    constexpr bool smag = (CL == 1);
    constexpr int nb = smag ? 6 : 4;
    const T U = T(M.u_in), Vv = T(M.v_in);
    const T coef = adj_coef<T>(M, P);
    V wx[ROW_EPT], wy[ROW_EPT], lJ[ROW_EPT], t0[ROW_EPT], t1[ROW_EPT];
    row_c2r<T>(C, mf + 2 * fstride, wx);
    row_c2r<T>(C, mf + 3 * fstride, wy);
    row_c2r<T>(C, mf + (long long)nb * fstride, lJ);
    // lambda_u = lambda_J omega_x, lambda_v = lambda_J omega_y
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) t0[i] = vmul<T>(lJ[i], wx[i]);
    row_r2c<T>(C, t0, mp + 0 * pstride);
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) t0[i] = vmul<T>(lJ[i], wy[i]);
    row_r2c<T>(C, t0, mp + 1 * pstride);
    V lwx[ROW_EPT], lwy[ROW_EPT];
    row_c2r<T>(C, mf + 0 * fstride, t0);   // u'
    row_c2r<T>(C, mf + 1 * fstride, t1);   // v'
#pragma unroll
    for (int i = 0; i < ROW_EPT; ++i) {
      lwx[i] = cmake<V>(lJ[i].x * (U + t0[i].x), lJ[i].y * (U + t0[i].y));
      lwy[i] = cmake<V>(lJ[i].x * (Vv + t1[i].x), lJ[i].y * (Vv + t1[i].y));
    }
    double dc = 0.0;
    if constexpr (CL != 0) {
      V gx[ROW_EPT], gy[ROW_EPT], base[ROW_EPT], lb[ROW_EPT];
      row_c2r<T>(C, mf + (long long)(nb + 1) * fstride, gx);
      row_c2r<T>(C, mf + (long long)(nb + 2) * fstride, gy);
      if constexpr (smag) {
        row_c2r<T>(C, mf + 4 * fstride, t0);   // psi_xx - psi_yy
        row_c2r<T>(C, mf + 5 * fstride, t1);   // psi_xy
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i)
          base[i] = cmake<V>(strain<T>(t1[i].x, t0[i].x), strain<T>(t1[i].y, t0[i].y));
      } else {
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i)
          base[i] = cmake<V>(gradmag<T>(wx[i].x, wy[i].x), gradmag<T>(wx[i].y, wy[i].y));
      }
#pragma unroll
      for (int i = 0; i < ROW_EPT; ++i) {
        if (valid(i)) {
          dc += (double)(gx[i].x * base[i].x * wx[i].x + gy[i].x * base[i].x * wy[i].x);
          dc += (double)(gx[i].y * base[i].y * wx[i].y + gy[i].y * base[i].y * wy[i].y);
        }
        V lhx = cmake<V>(coef * gx[i].x, coef * gx[i].y);
        V lhy = cmake<V>(coef * gy[i].x, coef * gy[i].y);
        lwx[i] = vfma<T>(lhx, base[i], lwx[i]);
        lwy[i] = vfma<T>(lhy, base[i], lwy[i]);
        lb[i] = vadd<T>(vmul<T>(lhx, wx[i]), vmul<T>(lhy, wy[i]));
      }
      if constexpr (smag) {
        // lambda_pd = pd/base lambda_b, lambda_pxy = 4 pxy/base lambda_b
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i) {
          T r0 = base[i].x > T(0) ? lb[i].x / base[i].x : T(0);
          T r1 = base[i].y > T(0) ? lb[i].y / base[i].y : T(0);
          gx[i] = cmake<V>(t0[i].x * r0, t0[i].y * r1);
          gy[i] = cmake<V>(T(4) * t1[i].x * r0, T(4) * t1[i].y * r1);
        }
        row_r2c<T>(C, gx, mp + 4 * pstride);
        row_r2c<T>(C, gy, mp + 5 * pstride);
      } else {
#pragma unroll
        for (int i = 0; i < ROW_EPT; ++i) {
          T r0 = base[i].x > T(0) ? lb[i].x / base[i].x : T(0);
          T r1 = base[i].y > T(0) ? lb[i].y / base[i].y : T(0);
          lwx[i] = cmake<V>(lwx[i].x + wx[i].x * r0, lwx[i].y + wx[i].y * r1);
          lwy[i] = cmake<V>(lwy[i].x + wy[i].x * r0, lwy[i].y + wy[i].y * r1);
        }
      }
    }
    row_r2c<T>(C, lwx, mp + 2 * pstride);
    row_r2c<T>(C, lwy, mp + 3 * pstride);
    double s = block_sum(dc, red);
    if (threadIdx.x == 0) rptr<double>(M, P.o_dpart)[blockIdx.x] = s * M.dcoef_dc;
  }
}

// ---------------------------------------------------------------- row pass, field-parallel
// Right-hand side, B sub-step and adjoint right-hand side: one block per row
// pair (.x row ya, .y row ya + 1).  The nb fields are taken to physical space
// at the same time by nb groups of threads (padded single-vector transforms
// whose first pass is fed from the mixed layout directly); then each of the
// first np groups forms one product at its own points straight into the
// registers of its forward transform, and keeps the retained half spectrum.
// Products: J, h_x, h_y per level (right-hand side); the penalized and
// sponged vorticity (B sub-step); l_u, l_v, l_wx, l_wy [, l_pd, l_pxy]
// (adjoint).  nx/8 threads per group; LOGN = log2(nx) selects the
// compile-time-length engine, LOGN = 0 the run-time one.

// one product at point q; dc accumulates the dL/dc integrand (adjoint)
// U, Vv: the member's inflow velocity; coef: its static closure coefficient
template <typename T, int OP, int CL, int PADS>
__device__ __forceinline__ cpx<T> rowp_product(const MemberDev& M, const Phase& P, const cpx<T>* buf, int bstride,
                                               int q, int grp, int ya, double& dc, T U, T Vv, T coef) {
  using V = cpx<T>;
  constexpr bool smag = (CL == 1 || CL == 3);
  constexpr int nbase = smag ? 6 : 4;
  const int nx = P.nx;
  auto F = [&](int f) -> V { return buf[f * bstride + q + (q >> PADS)]; };
  if constexpr (OP == OP_GTERMS) {
    // 0: J = (U + u') omega_x + (V + v') omega_y, 1: chi (U + u'),
    // 2: chi (V + v'), 3: chi_s omega
    const long long a = (long long)ya * nx + q, b = a + nx;
    if (grp == 0) {
      const V u = F(0), vv = F(1), wx = F(2), wy = F(3);
      return vadd<T>(vmul<T>(cmake<V>(U + u.x, U + u.y), wx), vmul<T>(cmake<V>(Vv + vv.x, Vv + vv.y), wy));
    }
    if (grp == 3) {
      const T* chs = rptr<T>(M, P.o_phys) + 5LL * nx * P.ny;
      const V w = F(4);
      return cmake<V>(chs[a] * w.x, chs[b] * w.y);
    }
    const T* chi = rptr<T>(M, P.o_phys) + 4LL * nx * P.ny;
    const V vel = F(grp - 1);
    const T base = grp == 1 ? U : Vv;
    return cmake<V>(chi[a] * (base + vel.x), chi[b] * (base + vel.y));
  } else if constexpr (OP == OP_PEN) {
    // (chi - c) times the total velocity: product 0 (chi - c)(U + u'),
    // 1 (chi - c)(V + v'); c is added back as c omega after the curl
    const long long a = (long long)ya * nx + q, b = a + nx;
    const T* chi = rptr<T>(M, P.o_phys) + 4LL * nx * P.ny;
    const T c = T(M.pen_c);
    const V vel = F(grp);
    const T base = grp == 0 ? U : Vv;
    return cmake<V>((chi[a] - c) * (base + vel.x), (chi[b] - c) * (base + vel.y));
  } else if constexpr (OP == OP_SPONGE) {
    // omega^{t+1} = omega* - dt sigma chi_s (3/2 omega* - 1/2 omega**)
    const long long a = (long long)ya * nx + q, b = a + nx;
    const T* chs = rptr<T>(M, P.o_phys) + 5LL * nx * P.ny;
    const T sa = T(M.sponge_a);
    const V ws = F(0), wss = F(1);
    const T r0 = ws.x - sa * chs[a] * (T(1.5) * ws.x - T(0.5) * wss.x);
    const T r1 = ws.y - sa * chs[b] * (T(1.5) * ws.y - T(0.5) * wss.y);
    return cmake<V>(r0, r1);
  } else if constexpr (OP == OP_B) {
    // omega'' = S (E omega + E_x v - E_y u), total velocity, from the
    // tables S E, S E_x, S E_y
    const long long nxy = (long long)nx * P.ny;
    const T* SE = rptr<T>(M, M.tab_off);
    const V u = F(0), vv = F(1), w = F(2);
    const long long a = (long long)ya * nx + q, b = a + nx;
    const T w0 = SE[a] * w.x + SE[nxy + a] * (Vv + vv.x) - SE[2 * nxy + a] * (U + u.x);
    const T w1 = SE[b] * w.y + SE[nxy + b] * (Vv + vv.y) - SE[2 * nxy + b] * (U + u.y);
    return cmake<V>(w0, w1);
  } else if constexpr (OP == OP_ADJ_B) {
    // transpose of the B sub-step's pointwise update at the cotangent
    // lambda'' (every group holds it; group 0's copy is read): 0: S E
    // lambda'' (omega), 1: -S E_y lambda'' (u), 2: S E_x lambda'' (v)
    const long long nxy = (long long)nx * P.ny;
    const T* SE = rptr<T>(M, M.tab_off);
    const V l = F(0);
    const long long a = (long long)ya * nx + q, b = a + nx;
    if (grp == 0) return cmake<V>(SE[a] * l.x, SE[b] * l.y);
    if (grp == 1) return cmake<V>(-SE[2 * nxy + a] * l.x, -SE[2 * nxy + b] * l.y);
    return cmake<V>(SE[nxy + a] * l.x, SE[nxy + b] * l.y);
  } else if constexpr (OP == OP_RHS) {
    const V wx = F(2), wy = F(3);
    if (grp == 0) {
      const V u = F(0), vv = F(1);
      return vadd<T>(vmul<T>(cmake<V>(U + u.x, U + u.y), wx), vmul<T>(cmake<V>(Vv + vv.x, Vv + vv.y), wy));
    }
    V base;
    if constexpr (smag) {
      const V pd = F(4), pxy = F(5);
      base = cmake<V>(strain<T>(pxy.x, pd.x), strain<T>(pxy.y, pd.y));
    } else {
      base = cmake<V>(gradmag<T>(wx.x, wy.x), gradmag<T>(wx.y, wy.y));
    }
    return vmul<T>(base, grp == 1 ? wx : wy);
  } else {  // OP_ADJ_RHS
    const V u = F(0), vv = F(1), wx = F(2), wy = F(3);
    const V lJ = F(nbase);
    if (grp == 0 && CL == 0) return vmul<T>(lJ, wx);
    if (grp == 1 && CL == 0) return vmul<T>(lJ, wy);
    V lwx = cmake<V>(lJ.x * (U + u.x), lJ.y * (U + u.y));
    V lwy = cmake<V>(lJ.x * (Vv + vv.x), lJ.y * (Vv + vv.y));
    V lpd = cmake<V>(T(0), T(0)), lpxy = lpd;
    if constexpr (CL != 0) {
      const V gx = F(nbase + 1), gy = F(nbase + 2);
      V base, pd, pxy;
      if constexpr (smag) {
        pd = F(4);
        pxy = F(5);
        base = cmake<V>(strain<T>(pxy.x, pd.x), strain<T>(pxy.y, pd.y));
      } else {
        base = cmake<V>(gradmag<T>(wx.x, wy.x), gradmag<T>(wx.y, wy.y));
      }
      if (grp == 0) {
        dc += (double)(gx.x * base.x * wx.x + gy.x * base.x * wy.x);
        dc += (double)(gx.y * base.y * wx.y + gy.y * base.y * wy.y);
        return vmul<T>(lJ, wx);
      }
      if (grp == 1) return vmul<T>(lJ, wy);
      const V lhx = cmake<V>(coef * gx.x, coef * gx.y);
      const V lhy = cmake<V>(coef * gy.x, coef * gy.y);
      lwx = vfma<T>(lhx, base, lwx);
      lwy = vfma<T>(lhy, base, lwy);
      const V lb = vadd<T>(vmul<T>(lhx, wx), vmul<T>(lhy, wy));
      const T r0 = base.x > T(0) ? lb.x / base.x : T(0);
      const T r1 = base.y > T(0) ? lb.y / base.y : T(0);
      if constexpr (smag) {
        lpd = cmake<V>(pd.x * r0, pd.y * r1);
        lpxy = cmake<V>(T(4) * pxy.x * r0, T(4) * pxy.y * r1);
      } else {
        lwx = cmake<V>(lwx.x + wx.x * r0, lwx.y + wx.y * r1);
        lwy = cmake<V>(lwy.x + wy.x * r0, lwy.y + wy.y * r1);
      }
    }
    if (grp == 2) return lwx;
    if (grp == 3) return lwy;
    if (grp == 4) return lpd;
    return lpxy;
  }
}

// c2r input of the packed row pair (rows ya, ya + 1) at column k: the raw
// loads (spectral m_x = k, or its mirror nx - k), then the packing into one
// complex row.
template <typename T, int EPT = 8> struct RowRaw {
  cpx<T> a[EPT], b[EPT];
};
template <typename T>
__device__ __forceinline__ void c2r_load(RowRaw<T>& r, const cpx<T>* src, int pitch, int ya, int j, int ng, int nx,
                                         int kin) {
  using V = cpx<T>;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int k = j + t * ng;
    const int m = k < kin ? k : k > nx - kin ? nx - k : -1;
    if (m >= 0) {
      const int o = ya * pitch + m;
      r.a[t] = gld(src + o);
      r.b[t] = gld(src + o + pitch);
    } else {
      r.a[t] = r.b[t] = cmake<V>(T(0), T(0));
    }
  }
}
template <typename T>
__device__ __forceinline__ cpx<T> c2r_form(cpx<T> a, cpx<T> b, int k, int nx, int kin) {
  using V = cpx<T>;
  if (k < kin) {
    if (k == 0) { a.y = T(0); b.y = T(0); }
    return cmake<V>(a.x - b.y, a.y + b.x);
  }
  if (k > nx - kin) return cmake<V>(a.x + b.y, b.x - a.y);
  return cmake<V>(T(0), T(0));
}

// The same for the compile-time row engine (row length N = 2^LOGN, element t
// of thread j at column k = j + t N/8).  Columns m_x < kin hold modes and
// N - kin < k < N their mirrors; the band between is zero.  At the grid
// level kin = kxn = (N - 1)/3 + 1, so the blocks t = 3, 4 lie inside the
// band and t = 0, 1, 6, 7 wholly outside it; at the test level (test ratio
// >= 2) kin <= (N - 1)/6 + 1 <= N/4, so the blocks t = 2..5 lie inside it.
// Blocks known to be zero (the bits of band_zero_mask) are neither loaded
// nor added in the first radix-8 pass of the transform.

// EPT elements per thread (8, or 16 for one wave per 1024-point row): element
// e of thread j sits at column k = j + e N/EPT, in block t = e / (EPT/8).
template <typename T, int LOGN, bool TL, int EPT = 8>
__device__ __forceinline__ void c2r_loadc(RowRaw<T, EPT>& r, const cpx<T>* row, int pitch, int j, int kin) {
  using V = cpx<T>;
  constexpr int N = 1 << LOGN, GT = N / EPT, NB0 = EPT / 8, KIN = (N - 1) / 3 + 1;
  constexpr int ZM = band_zero_mask<TL>();
  const V* fw = row + j;          // column j + e GT at fw + e GT
  const V* bw = row + (N - j);    // its mirror N - j - e GT at bw - e GT (blocks t >= 4)
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int t = e / NB0;
    r.a[e] = r.b[e] = cmake<V>(T(0), T(0));
    if ((ZM >> t) & 1) continue;
    const bool mirror = t >= 4;
    bool in;
    if (mirror) in = (!TL && t >= 6) || (N - e * GT - j) < (TL ? kin : KIN);
    else in = (!TL && t <= 1) || j + e * GT < (TL ? kin : KIN);
    if (in) {
      const V* q = mirror ? bw - e * GT : fw + e * GT;
      r.a[e] = gld(q);
      r.b[e] = gld(q + pitch);
    }
  }
  // keep every load above the first use of any: the loads of the boundary
  // blocks sit in lane-conditional branches, and a use moved into such a
  // branch waits there for all loads issued before the later ones go out
  asm volatile("" ::: "memory");
}

template <typename T, bool TL, int EPT = 8>
__device__ __forceinline__ void c2r_formc(const RowRaw<T, EPT>& in, cpx<T> (&v)[EPT], int j) {
  using V = cpx<T>;
  constexpr int ZM = band_zero_mask<TL>(), NB0 = EPT / 8;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int t = e / NB0;
    if ((ZM >> t) & 1) { v[e] = cmake<V>(T(0), T(0)); continue; }
    V a = in.a[e], b = in.b[e];
    if (t < 4) {
      if (e == 0 && j == 0) { a.y = T(0); b.y = T(0); }   // the m_x = 0 column is real
      v[e] = cmake<V>(a.x - b.y, a.y + b.x);
    } else {
      v[e] = cmake<V>(a.x + b.y, b.x - a.y);
    }
  }
}

// Column limit of the c2r input: the test-filtered level of a dynamic
// closure's right-hand side holds no mode at m_x >= test_kx (the second
// level of an adjoint stage, adj_mode 2, spans the whole 2/3 set).
__device__ __forceinline__ int rowp_kin(const Phase& P, const MemberDev& M, bool test_level) {
  return test_level ? min(P.kxn, M.test_kx) : P.kxn;
}

// One item of the row pass: row pair rb of member mem at level lev, from
// the packed c2r inputs vin (column j + t nx/8 of the thread's group);
// twl: the x twiddle table (global or staged in LDS).
// EPT points per thread; WV: the transforms synchronise within their wave
// (one wave per transform), the block only around the products.
template <typename T, int OP, int CL, int LOGN, int ZM = 0, int SCH = 0, int EPT = 8, bool WV = false>
__device__ __forceinline__ void rowp_item(const Phase& P, int mem, int rb, int lev, const cpx<T> (&vin)[EPT],
                                          cpx<T>* buf, const cpx<T>* twl, double* red, int item_slot) {
  using V = cpx<T>;
  constexpr int np = rowp_np(OP, CL);
  constexpr int LGE = EPT == 16 ? 4 : 3;        // log2 of the points per thread
  constexpr int PADS = LOGN ? QG_ROW_PADS : 3;  // one pad slot per 2^PADS
  const MemberDev M = member_const(P, mem);
  // member constants read once, not per point
  const T U = T(M.u_in), Vv = T(M.v_in);
  const T coef = OP == OP_ADJ_RHS ? adj_coef<T>(M, P) : T(M.coef_static);
  const int nx = LOGN ? (1 << LOGN) : P.nx;
  const int bstride = nx + (nx >> PADS);
  const int lg = LOGN ? LOGN - LGE : P.lognx - 3;
  const int grp = threadIdx.x >> lg;
  const int j = threadIdx.x & ((1 << lg) - 1);
  const int ng = 1 << lg;                      // threads per group
  const int ya = 2 * rb;
  RowCtx<T> C;
  C.ny = P.ny; C.logW = P.logW; C.kxp = P.mfp;
  const long long pstride = (long long)P.ny * P.kxp;   // MP field stride
  V* mybuf = buf + grp * bstride;
  if constexpr (OP == OP_RHS) QG_STAMP(0, 1, vin[EPT - 1].x);
  // the second pass's twiddles (the same slots serve the c2r and the r2c),
  // loaded before the first pass
  PassTw<V, LOGN ? LOGN : 10, 3, SCH, EPT> tw1;
  if constexpr (LOGN != 0) tw1 = fft1c_first_tw<V, LOGN, SCH, EPT>(twl, j);
  // ---- c2r of field lev * nb + grp
  {
    V v[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) v[t] = vin[t];
    if constexpr (LOGN != 0) {
      fft1c_pass0<V, true, PADS, ZM, EPT, WV, LOGN>(v, mybuf, j, true);
      fft1c_rest<V, LOGN, true, PADS, SCH, EPT, WV>(mybuf, twl, j, true, tw1);
    } else {
      fft1_pass0<V, true>(v, mybuf, j, true, P.lognx);
      fft1_rest<V, true>(mybuf, twl, P.lognx, j, true);
    }
  }
  if constexpr (WV) __syncthreads();   // every field in physical space before the products read them
  if constexpr (OP == OP_RHS) QG_STAMP_LDS(0, 2);
  if constexpr (OP == OP_CLIPF) {
    // sums of max(H, 0) M and M^2 over the two rows (group 0's points)
    double hp = 0.0, mm = 0.0;
    if (grp == 0) {
#pragma unroll
      for (int t = 0; t < EPT; ++t) {
        const int q = j + t * ng;
        const V h = buf[q + (q >> PADS)], m = buf[bstride + q + (q >> PADS)];
        hp += fmax((double)h.x, 0.0) * (double)m.x + fmax((double)h.y, 0.0) * (double)m.y;
        mm += (double)m.x * (double)m.x + (double)m.y * (double)m.y;
      }
    }
    block_sum2(hp, mm, red);
    if (threadIdx.x == 0) {
      double* d = rptr<double>(M, P.o_dpart) + 2 * item_slot;
      d[0] = hp;
      d[1] = mm;
    }
    return;
  }
  // ---- product grp at this thread's points q = j + t ng
  V v[EPT];
  double dc = 0.0;
  const bool act = grp < np;
  if (act) {
#pragma unroll
    for (int t = 0; t < EPT; ++t)
      v[t] = rowp_product<T, OP, CL, PADS>(M, P, buf, bstride, j + t * ng, grp, ya, dc, U, Vv, coef);
  }
  if constexpr (OP == OP_RHS) QG_STAMP(0, 3, v[0].x);
  if constexpr (OP == OP_ADJ_RHS) {
    const double sdc = block_sum(dc, red);
    if (threadIdx.x == 0 && lev == 0) rptr<double>(M, P.o_dpart)[item_slot] = sdc * M.dcoef_dc;
  }
  // ---- r2c of product grp, keep m_x < kxn
  if constexpr (WV) __syncthreads();   // every product formed before the fields' buffers are overwritten
  if constexpr (LOGN != 0) {
    fft1c_pass0<V, false, PADS, 0, EPT, WV, LOGN>(v, mybuf, j, act);
    fft1c_rest<V, LOGN, false, PADS, SCH, EPT, WV, true>(mybuf, twl, j, act, tw1);   // columns of the 2/3 set read
    if constexpr (OP == OP_RHS) QG_STAMP_LDS(0, 4);
  } else {
    fft1_pass0<V, false>(v, mybuf, j, act, P.lognx);
    fft1_rest<V, false>(mybuf, twl, P.lognx, j, act);
  }
  if constexpr (LOGN != 0) {
    // columns k = j + t GT below kxn (GT = N/EPT threads per group); the
    // mirror N - k sits at constant offsets below padp(N - j), except k = 0
    // whose mirror is itself
    constexpr int N = 1 << LOGN, GT = N / EPT, KXN = (N - 1) / 3 + 1;
    constexpr int DPAD = GT + (GT >> PADS);
    if (act) {
      V* dst = cptr<T>(M, P.o_mp) + (long long)(OP == OP_ADJ_RHS ? lev * np + grp : lev * 3 + grp) * pstride;
      const int o0 = mix_at(C, ya, j);
      const int iz = padp<PADS>(j);
      const int izm = padp<PADS>(N - j);
#pragma unroll
      for (int t = 0; t < EPT; ++t) {
        if (t * GT >= KXN || j + t * GT >= KXN) break;
        const V z = mybuf[iz + t * DPAD];
        const V zm = mybuf[(t == 0 && j == 0) ? 0 : izm - t * DPAD];
        const int o = o0 + t * GT * P.ny;
        const V ra = cmake<V>(T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y));     // row ya
        const V rb2 = cmake<V>(T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x));    // row ya + 1
        if (C.logW == 0) {
          gst_pair(dst + o, ra, rb2);
        } else {
          gst(dst + o, ra);
          gst(dst + o + (1 << C.logW), rb2);
        }
      }
    }
    if constexpr (OP == OP_RHS) QG_STAMP_DRAIN(0, 5);
  } else if (act) {
    V* dst = cptr<T>(M, P.o_mp) + (long long)(OP == OP_ADJ_RHS ? lev * np + grp : lev * 3 + grp) * pstride;
    for (int k = j; k < P.kxn; k += ng) {
      const int a = k, b = (nx - k) & (nx - 1);
      const V z = mybuf[a + (a >> PADS)];
      const V zm = mybuf[b + (b >> PADS)];
      const int o = mix_at(C, ya, k);
      const V ra = cmake<V>(T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y));     // row ya
      const V rb2 = cmake<V>(T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x));    // row ya + 1
      if (C.logW == 0) {
        gst_pair(dst + o, ra, rb2);          // the two rows are adjacent
      } else {
        gst(dst + o, ra);
        gst(dst + o + (1 << C.logW), rb2);
      }
    }
  }
}

// packed c2r inputs of the item from its loads
template <typename T>
__device__ __forceinline__ void rowp_form(const Phase& P, int mem, bool test_level, const RowRaw<T>& in,
                                          cpx<T> (&v)[8]) {
  const MemberDev M = member_const(P, mem);
  const int lg = P.lognx - 3;
  const int j = threadIdx.x & ((1 << lg) - 1);
  const int kin = rowp_kin(P, M, test_level);
#pragma unroll
  for (int t = 0; t < 8; ++t) v[t] = c2r_form<T>(in.a[t], in.b[t], j + (t << lg), P.nx, kin);
}

// c2r loads of the item's field (row pair rb, level lev, member mem)
template <typename T, int OP, int CL>
__device__ __forceinline__ void rowp_load(const Phase& P, int mem, int rb, int lev, RowRaw<T>& in) {
  constexpr int nb = rowp_nb(OP, CL);
  const MemberDev M = member_const(P, mem);
  const int lg = P.lognx - 3;
  const int grp = threadIdx.x >> lg;
  const int j = threadIdx.x & ((1 << lg) - 1);
  const long long fstride = (long long)P.ny * P.mfp;   // MF field stride
  // the B sub-step's transpose: every group transforms the one cotangent field
  const cpx<T>* src = cptr<T>(M, P.o_mf) + (long long)(OP == OP_ADJ_B ? 0 : lev * nb + grp) * fstride;
  c2r_load<T>(in, src, P.mfp, 2 * rb, j, 1 << lg, P.nx, rowp_kin(P, M, OP == OP_RHS && lev == 1));
}

// Right-hand side, B sub-step and adjoint right-hand side: one block per
// row pair (grid.x), level (grid.y) and member (grid.z).
// One row pair rb at level lev.
template <typename T, int OP, int CL, int LOGN, int SCH, bool WV>
__device__ __forceinline__ void rowp_pair(const Phase& P, int rb, int lev, cpx<T>* buf, const cpx<T>* twl,
                                          double* red) {
  using V = cpx<T>;
  constexpr bool dyn = OP == OP_RHS && (CL == 3 || CL == 4);
  if constexpr (LOGN != 0) {
    // compile-time row length: loads, packing and the first pass leave out
    // the blocks of columns the 2/3 set (grid level) or the test filter
    // (test level) keep empty.  WV: one wave per transform, 16 points per
    // thread at 1024 (8 below)
    constexpr int EPT = (WV && LOGN >= 10) ? 16 : 8;
    constexpr int LGT = LOGN - (EPT == 16 ? 4 : 3);   // log2 of the threads per transform
    constexpr int nb = rowp_nb(OP, CL);
    const MemberDev M = member_const(P, blockIdx.z);
    const int grp = threadIdx.x >> LGT;
    const int j = threadIdx.x & ((1 << LGT) - 1);
    const cpx<T>* row = cptr<T>(M, P.o_mf) +
                        (long long)(OP == OP_ADJ_B ? 0 : lev * nb + grp) * ((long long)P.ny * P.mfp) +
                        (long long)(2 * rb) * P.mfp;
    RowRaw<T, EPT> in;
    V vin[EPT];
    if (dyn && lev == 1) {
      c2r_loadc<T, LOGN, true, EPT>(in, row, P.mfp, j, min(P.kxn, M.test_kx));
      c2r_formc<T, true, EPT>(in, vin, j);
      rowp_item<T, OP, CL, LOGN, band_zero_mask<true>(), SCH, EPT, WV>(P, blockIdx.z, rb, lev, vin, buf, twl, red,
                                                                        rb);
    } else {
      c2r_loadc<T, LOGN, false, EPT>(in, row, P.mfp, j, P.kxn);
      c2r_formc<T, false, EPT>(in, vin, j);
      rowp_item<T, OP, CL, LOGN, band_zero_mask<false>(), SCH, EPT, WV>(P, blockIdx.z, rb, lev, vin, buf, twl, red,
                                                                         rb);
    }
  } else {
    RowRaw<T> in;
    rowp_load<T, OP, CL>(P, blockIdx.z, rb, lev, in);
    V vin[8];
    rowp_form<T>(P, blockIdx.z, OP == OP_RHS && lev == 1, in, vin);
    rowp_item<T, OP, CL, LOGN>(P, blockIdx.z, rb, lev, vin, buf, twl, red, rb);
  }
}

// Right-hand side, B sub-step and adjoint right-hand side: one block per
// row pair (grid.x, RPB row pairs one after the other when RPB > 1), level
// (grid.y) and member (grid.z).
template <typename T, int OP, int CL, int LOGN, int SCH = 0, bool WV = false, int RPB = 1>
__global__ void __launch_bounds__(1024) k_rowp(Phase P) {
  using V = cpx<T>;
  constexpr bool dyn = OP == OP_RHS && (CL == 3 || CL == 4);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  lds_poison_all(smem_raw, P.lds_bytes);
  __shared__ double red[32];   // 2 doubles per wave (block_sum2), up to 16 waves
  V* buf = reinterpret_cast<V*>(smem_raw);
  if constexpr (OP == OP_RHS) QG_STAMP(0, 0, 0.f);
  // consecutive row pairs on the same XCD: their interleaved output stores
  // meet in one L2
  int rbb = blockIdx.x;
  if ((gridDim.x & 7) == 0) rbb = (blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  // the two levels of the dynamic closures (grid and test filter) are
  // independent: one block each (and the two passes of a dynamic closure's
  // adjoint stage, adj_mode 2)
  const int lev = (dyn || OP == OP_ADJ_RHS) ? (int)blockIdx.y : 0;
  // twiddles straight from the (cached) global table: keeping LDS to the
  // field buffers lets one more block share a compute unit
  const V* twl = reinterpret_cast<const V*>(SCH == 2 ? P.twx2 : SCH ? P.twx1 : P.twx);
  // (no loop at all for one row pair per block: even a loop of one trip
  // changes the register allocation of the body)
  if constexpr (RPB == 1) {
    rowp_pair<T, OP, CL, LOGN, SCH, WV>(P, rbb, lev, buf, twl, red);
  } else {
    for (int r = 0; r < RPB; ++r) rowp_pair<T, OP, CL, LOGN, SCH, WV>(P, rbb * RPB + r, lev, buf, twl, red);
  }
}

// ---------------------------------------------------------------- AB2CN
// One AB2CN step at a mode (Sec. II-E, Eq. 4), given the nonlinear terms
// N = -J_hat + C Q_hat at omega^t: the explicit terms E = N - (1/eta) D
// curl(chi u) (o_ab_pen) go through Adams-Bashforth 2 against the previous
// step's (o_ab_hist; E itself before any history), the linear terms
// L = -(|k|^2/Re + mu) + i beta kx/|k|^2 through Crank-Nicolson:
//   omega* = (omega^t (1 + dt/2 L) + dt (3/2 E - 1/2 E_prev)) / (1 - dt/2 L).
// omega^t from o_in2, omega* to o_in; E replaces the history.  The CN
// factors are formed in double precision.
template <typename T>
__device__ __forceinline__ void ab2cn_update(const MemberDev& M, const Phase& P, int id, int mx, int my, cpx<T> N) {
  using V = cpx<T>;
  const double dt = M.dt;
  const V pen = gld(cptr<T>(M, P.o_ab_pen) + id);
  const T pa = T(M.pen_a / dt);                  // 1/eta
  const V E = csub(N, cscale(pen, pa));
  V* hist = cptr<T>(M, P.o_ab_hist) + id;
  const bool first = rptr<double>(M, P.o_coef)[AB2CN_FLAG_SLOT] == 0.0;
  const V Ep = first ? E : gld(hist);
  gst(hist, E);
  const V w = gld(cptr<T>(M, P.o_in2) + id);
  V out = cmake<V>(T(0), T(0));
  if (mx != 0 || my != 0) {
    const double kx = M.two_pi_lx * mx, ky = M.two_pi_ly * my;
    const double k2 = kx * kx + ky * ky;
    const double lr = -(k2 * M.inv_re + M.mu), li = M.beta * kx / k2;
    const double ar = 1.0 + 0.5 * dt * lr, ai = 0.5 * dt * li;     // 1 + dt/2 L
    const double dr = 1.0 - 0.5 * dt * lr, di = -0.5 * dt * li;    // 1 - dt/2 L
    const double nr = (double)w.x * ar - (double)w.y * ai + dt * (1.5 * (double)E.x - 0.5 * (double)Ep.x);
    const double ni = (double)w.x * ai + (double)w.y * ar + dt * (1.5 * (double)E.y - 0.5 * (double)Ep.y);
    const double den = dr * dr + di * di;
    out = cmake<V>(T((nr * dr + ni * di) / den), T((ni * dr - nr * di) / den));
  }
  gst(cptr<T>(M, P.o_in) + id, out);
}

// End of an AB2CN step: omega* becomes the next step's omega** and the
// history flag is set (after the sponge pass has read the old omega**).
template <typename T>
__global__ void __launch_bounds__(256) k_ab2cn_finish(Phase P) {
  using V = cpx<T>;
  const MemberDev M = member_const(P, blockIdx.z);
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < P.kxn * P.kyn) gst(cptr<T>(M, P.o_out) + q, gld(cptr<T>(M, P.o_in) + q));
  if (blockIdx.x == 0 && threadIdx.x == 0) rptr<double>(M, P.o_coef)[AB2CN_FLAG_SLOT] = 1.0;
}

// ---------------------------------------------------------------- colfwd
// Forward FFT along y of product p's strip into the LDS tile.
template <typename T, int EPT>
__device__ __forceinline__ void colfwd_load_fft(const Phase& P, const MemberDev& M, cpx<T>* tile,
                                                const cpx<T>* twl, int p, int kx0) {
  using V = cpx<T>;
  const int n = P.W * P.ny;
  const V* src = cptr<T>(M, P.o_mp) + (long long)p * P.ny * P.kxp + (long long)kx0 * P.ny;
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += blockDim.x) tile[q] = src[q];
  __syncthreads();
  FftShape s{P.logny, P.W, 1, P.logW, true};
  fft_lds<V, false, EPT>(tile, twl, s);
}

template <typename T, int OP, int CL, int EPT>
__global__ void __launch_bounds__(COL_MAX_THREADS, (sizeof(T) == 4 ? 4 : 2)) k_colfwd(Phase P) {
  using V = cpx<T>;
  constexpr int MAXM = EPT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  lds_poison_all(smem_raw, P.lds_bytes);
  V* tile = reinterpret_cast<V*>(smem_raw);
  V* twl = tile + P.W * P.ny;
  __shared__ double red[32];   // 2 doubles per wave (block_sum2), up to 16 waves
  const MemberDev M = member_const(P, blockIdx.z);
  const int strip = xcd_order(blockIdx.x, gridDim.x);
  if (strip * P.W >= P.kxn) return;
  const int kx0 = strip * P.W;
  const int nmodes = P.W * P.kyn;
  stage_twiddles<V>(twl, reinterpret_cast<const V*>(P.twy), P.logny);
  // owned modes, packed as (m_x << 16) | iy; m_x = kxn marks "not owned"
  int own[MAXM];
#pragma unroll
  for (int i = 0; i < MAXM; ++i) {
    const int q = threadIdx.x + i * blockDim.x;
    const int w = div_kyn(q, P.kyn);
    const int mx = (q < nmodes) ? kx0 + w : P.kxn;
    own[i] = ((mx < P.kxn ? mx : P.kxn) << 16) | (q - (int)__umul24((unsigned)w, (unsigned)P.kyn));
  }
#define mxs_(i) (own[i] >> 16)
#define iys_(i) (own[i] & 0xffff)
  auto tile_at = [&](int i) -> V {
    const int my = my_of_iy(iys_(i), P.myh, P.kyn);
    const int y = my >= 0 ? my : my + P.ny;
    return tile[y * P.W + (mxs_(i) - kx0)];
  };
  auto owned = [&](int i) { return mxs_(i) < P.kxn; };
  auto sidx = [&](int i) { return (long long)mxs_(i) * P.kyn + iys_(i); };

  if constexpr (OP == OP_B || OP == OP_ENTRY || OP == OP_MASKFWD) {
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 0, kx0);
    V* out = cptr<T>(M, P.o_out);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      V v = tile_at(i);
      if (OP != OP_MASKFWD && mxs_(i) == 0 && iys_(i) == 0) v = cmake<V>(T(0), T(0));
      out[sidx(i)] = v;
    }
  } else if constexpr (OP == OP_RHS && !(CL == 3 || CL == 4)) {
    // R = -J + C (i kx h_x + i ky h_y) - (k^2/Re + mu) x - i beta kx psi; RK4 update
    V R[MAXM], Q[MAXM];
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 0, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      V j = tile_at(i);
      R[i] = cmake<V>(-j.x, -j.y);
    }
    if constexpr (CL != 0) {
      colfwd_load_fft<T, EPT>(P, M, tile, twl, 1, kx0);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (!owned(i)) continue;
        const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
        Q[i] = mul_ia(tile_at(i), T(w.kx));
      }
      colfwd_load_fft<T, EPT>(P, M, tile, twl, 2, kx0);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (!owned(i)) continue;
        const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
        Q[i] = cadd(Q[i], mul_ia(tile_at(i), T(w.ky)));
      }
    }
    const T C = T(M.coef_static);
    if (P.stage == AB2CN_STAGE || P.stage == SGS_STAGE) {
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (!owned(i)) continue;
        const int my = my_of_iy(iys_(i), P.myh, P.kyn);
        V cq = cmake<V>(T(0), T(0));
        if constexpr (CL != 0) cq = cscale(Q[i], C);
        if (P.stage == AB2CN_STAGE) {
          ab2cn_update<T>(M, P, (int)sidx(i), mxs_(i), my, cadd(R[i], cq));
        } else {
          if (mxs_(i) == 0 && my == 0) cq = cmake<V>(T(0), T(0));
          gst(cptr<T>(M, P.o_out) + sidx(i), cq);
        }
      }
      return;
    }
    const V* xin = cptr<T>(M, P.stage == 1 ? P.o_in2 : P.o_in);
    const V* wn = cptr<T>(M, P.o_in2);
    V* acc = cptr<T>(M, P.o_aux);
    V* xout = cptr<T>(M, P.o_in);
    const double dt = M.dt;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const int my = my_of_iy(iys_(i), P.myh, P.kyn);
      const Wave<T> w = wave<T>(M, mxs_(i), my);
      const long long id = sidx(i);
      const V x = xin[id];
      V r = R[i];
      const T lin = (w.k2 * T(M.inv_re) + T(M.mu));
      r = csub(r, cscale(x, lin));
      const V psi = poisson<T>(M, x, w, mxs_(i), my);
      r = csub(r, mul_ia(psi, (T(M.beta) * w.kx)));
      if constexpr (CL != 0) r = cadd(r, cscale(Q[i], C));
      if (mxs_(i) == 0 && my == 0) r = cmake<V>(T(0), T(0));
      const V w0 = wn[id];
      if (P.stage == 1) {
        acc[id] = cadd(w0, cscale(r, T(M.dt6)));
        xout[id] = cadd(w0, cscale(r, T(M.dt2)));
      } else if (P.stage == 2) {
        acc[id] = cadd(acc[id], cscale(r, T(M.dt3)));
        xout[id] = cadd(w0, cscale(r, T(M.dt2)));
      } else if (P.stage == 3) {
        acc[id] = cadd(acc[id], cscale(r, T(M.dt3)));
        xout[id] = cadd(w0, cscale(r, T(dt)));
      } else {
        xout[id] = cadd(acc[id], cscale(r, T(M.dt6)));
      }
    }
  } else if constexpr (OP == OP_RHS) {
    // dynamic closures: Q = i k . h and J to the side buffers, then
    // M = r i k . g - T Q and H = FFT(J~) - T J, partial sums of <HM> and
    // <M^2> over the strip (Parseval, weights 1 at m_x = 0 else 2).
    // Products are taken in the order h_x, h_y, g_x, g_y, J~, J so that
    // only two per-mode accumulators are live.
    V A[MAXM], B[MAXM];
    V* jsp = cptr<T>(M, P.o_out);
    V* qsp = cptr<T>(M, P.o_aux);
    const T r = T(M.r_test);
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 1, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      A[i] = mul_ia(tile_at(i), w.kx);
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 2, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      A[i] = cadd(A[i], mul_ia(tile_at(i), w.ky));
      qsp[sidx(i)] = A[i];
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 4, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      B[i] = mul_ia(tile_at(i), w.kx);
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 5, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const int my = my_of_iy(iys_(i), P.myh, P.kyn);
      const Wave<T> w = wave<T>(M, mxs_(i), my);
      V g = cscale(cadd(B[i], mul_ia(tile_at(i), w.ky)), r);
      B[i] = in_test(M, P.nx, P.ny, mxs_(i), my) ? csub(g, A[i]) : g;
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 3, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) if (owned(i)) A[i] = tile_at(i);
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 0, kx0);
    double hm = 0.0, mm = 0.0;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const int my = my_of_iy(iys_(i), P.myh, P.kyn);
      const V j = tile_at(i);
      jsp[sidx(i)] = j;
      const V h = in_test(M, P.nx, P.ny, mxs_(i), my) ? csub(A[i], j) : A[i];
      const V g = B[i];
      if (P.adj_dyn) {
        cptr<T>(M, P.o_h)[sidx(i)] = h;
        cptr<T>(M, P.o_m)[sidx(i)] = g;
      }
      const double wt = mxs_(i) == 0 ? 1.0 : 2.0;
      hm += wt * ((double)h.x * (double)g.x + (double)h.y * (double)g.y);
      mm += wt * ((double)g.x * (double)g.x + (double)g.y * (double)g.y);
    }
    double shm = hm, smm = mm;
    block_sum2(shm, smm, red);
    if (threadIdx.x == 0) {
      double* part = rptr<double>(M, P.o_part) + 2 * strip;
      part[0] = shm;
      part[1] = smm;
    }
  } else if constexpr (OP == OP_ADJ_B) {
    // lambda_s = FFT(lambda_w) - (1/|k|^2)(i ky FFT(lambda_u) - i kx FFT(lambda_v));
    // writes LS (o_out), LW = LS (o_aux), LK = dt/6 LS (o_in)
    V Lw[MAXM];
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 0, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) if (owned(i)) Lw[i] = tile_at(i);
    V Lp[MAXM];
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 1, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      Lp[i] = mul_ia(tile_at(i), T(w.ky));
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 2, kx0);
    V* ls = cptr<T>(M, P.o_out);
    V* lw = cptr<T>(M, P.o_aux);
    V* lk = cptr<T>(M, P.o_in);
    const T c6 = T(M.dt6);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      V lpsi = csub(Lp[i], mul_ia(tile_at(i), T(w.kx)));
      V l = csub(Lw[i], cscale(lpsi, T(w.inv_k2)));
      const long long id = sidx(i);
      ls[id] = l;
      lw[id] = l;
      lk[id] = cscale(l, c6);
    }
  } else if constexpr (OP == OP_ADJ_RHS) {
    // lambda_psi = i beta kx l' + i ky F(l_u) - i kx F(l_v)
    //              [+ (ky^2 - kx^2) F(l_pd) - kx ky F(l_pxy)]
    // lambda_x = -(k^2/Re + mu) l' - i kx F(l_wx) - i ky F(l_wy) - lambda_psi/|k|^2
    // then LW += lambda_x and LK <- c LS + d lambda_x for the previous stage.
    constexpr bool smag = (CL == 1);
    V Lpsi[MAXM], Lx[MAXM];
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 0, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      Lpsi[i] = mul_ia(tile_at(i), T(w.ky));
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 1, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      Lpsi[i] = csub(Lpsi[i], mul_ia(tile_at(i), T(w.kx)));
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 2, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      Lx[i] = mul_ia(tile_at(i), T(-w.kx));
    }
    colfwd_load_fft<T, EPT>(P, M, tile, twl, 3, kx0);
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
      Lx[i] = cadd(Lx[i], mul_ia(tile_at(i), T(-w.ky)));
    }
    if constexpr (smag) {
      colfwd_load_fft<T, EPT>(P, M, tile, twl, 4, kx0);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (!owned(i)) continue;
        const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
        Lpsi[i] = cadd(Lpsi[i], cscale(tile_at(i), T(w.ky * w.ky - w.kx * w.kx)));
      }
      colfwd_load_fft<T, EPT>(P, M, tile, twl, 5, kx0);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (!owned(i)) continue;
        const Wave<T> w = wave<T>(M, mxs_(i), my_of_iy(iys_(i), P.myh, P.kyn));
        Lpsi[i] = cadd(Lpsi[i], cscale(tile_at(i), T(-w.kx * w.ky)));
      }
    }
    if (P.adj_mode != 0) {
      // transport pass at the test-filtered stage input: its term,
      // test-filtered, to o_e
      V* E = cptr<T>(M, P.o_e);
#pragma unroll
      for (int i = 0; i < MAXM; ++i) {
        if (!owned(i)) continue;
        const int my = my_of_iy(iys_(i), P.myh, P.kyn);
        const Wave<T> w = wave<T>(M, mxs_(i), my);
        const V e = csub(Lx[i], cscale(Lpsi[i], T(w.inv_k2)));
        E[sidx(i)] = in_test(M, P.nx, P.ny, mxs_(i), my) ? e : cmake<V>(T(0), T(0));
      }
      return;
    }
    const V* lin = cptr<T>(M, P.o_in2);     // l = LK (stage input adjoint)
    const V* ls = cptr<T>(M, P.o_out);      // LS
    V* lw = cptr<T>(M, P.o_aux);            // LW
    V* lk = cptr<T>(M, P.o_in2);
    const double dt = M.dt;
    const double cs = P.stage == 4 ? M.dt3 : P.stage == 3 ? M.dt3 : M.dt6;
    const double ds = P.stage == 4 ? dt : M.dt2;
#pragma unroll
    for (int i = 0; i < MAXM; ++i) {
      if (!owned(i)) continue;
      const int my = my_of_iy(iys_(i), P.myh, P.kyn);
      const Wave<T> w = wave<T>(M, mxs_(i), my);
      const long long id = sidx(i);
      V l = lin[id];
      if (mxs_(i) == 0 && my == 0) l = cmake<V>(T(0), T(0));
      V lp = cadd(Lpsi[i], mul_ia(l, (T(M.beta) * w.kx)));
      V lx = csub(Lx[i], cscale(l, (w.k2 * T(M.inv_re) + T(M.mu))));
      lx = csub(lx, cscale(lp, T(w.inv_k2)));
      if (P.adj_dyn) lx = cadd(lx, cptr<T>(M, P.o_e)[id]);   // the dynamic coefficient's term
      lw[id] = cadd(lw[id], lx);
      if (P.stage > 1) lk[id] = cadd(cscale(ls[id], T(cs)), cscale(lx, T(ds)));
    }
  }
}
#undef mxs_
#undef iys_

// ---------------------------------------------------------------- colfwd, product-parallel
// All np product strips of a block sit in LDS at once; np groups of
// W ny / 8 threads transform them concurrently, then every thread combines
// the retained modes straight from LDS.  Used when np W ny / 8 <= 1024 and
// the strips fit in LDS (in particular W = 1 at ny <= 1024).
template <typename T, int OP, int CL, int LOGN, int SCH = 0>
__global__ void __launch_bounds__(1024) k_colfwdp(Phase P) {
  using V = cpx<T>;
  constexpr bool dyn = OP == OP_RHS && (CL == 3 || CL == 4);
  constexpr int np = OP == OP_RHS ? (CL == 0 ? 1 : dyn ? 6 : 3)
                   : OP == OP_ADJ_B ? 3 : OP == OP_ADJ_RHS ? (CL == 1 ? 6 : 4) : OP == OP_PEN ? 2
                   : OP == OP_GTERMS ? 4 : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  lds_poison_all(smem_raw, P.lds_bytes);
  __shared__ double red[32];   // 2 doubles per wave (block_sum2), up to 16 waves
  if constexpr (dyn) QG_STAMP(2, 0, 0.f);
  const MemberDev M = member_const(P, blockIdx.z);
  // W = 1: padded single-vector path (compile-time length if LOGN != 0,
  // twiddles then read from the global table)
  const bool one = LOGN != 0 || P.W == 1;
  constexpr int CPD = LOGN ? QG_COL_PADS : 3;   // pad period of the single-column path
  const int n = LOGN ? (1 << LOGN) + (1 << (LOGN - CPD)) : P.W * P.ny + (one ? P.ny >> CPD : 0);
  V* tile = reinterpret_cast<V*>(smem_raw);
  V* twl = tile + np * n;
  if constexpr (LOGN == 0) stage_twiddles<V>(twl, reinterpret_cast<const V*>(P.twy), P.logny);
  const int lg = LOGN ? LOGN - 3 : P.logW + P.logny - 3;     // log2 of the group size W ny/8
  const int grp = threadIdx.x >> lg;
  const int lt = threadIdx.x & ((1 << lg) - 1);
  const int strip = xcd_order(blockIdx.x, gridDim.x);
  if (strip * P.W >= P.kxn) return;
  const int kx0 = strip * P.W;
  const V* src = cptr<T>(M, P.o_mp) + (long long)grp * P.ny * P.kxp + (long long)kx0 * P.ny;
  // test filter of the dynamic closures (one column per block when W = 1),
  // formed while the column's values arrive rather than after the transform
  const int mylim = dyn && one ? test_mylim(M, P.nx, P.ny, kx0) : -2;
  if (one) {
    V v[8];
    // the second pass's twiddles, loaded alongside the column's values
    const V* twc = reinterpret_cast<const V*>(SCH ? P.twy1 : P.twy);
    PassTw<V, LOGN ? LOGN : 10, 3, SCH, 8> tw1;
    if constexpr (LOGN != 0) tw1 = fft1c_first_tw<V, LOGN, SCH>(twc, lt);
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = gld(src + lt + (t << lg));
    if constexpr (LOGN != 0) {
      if constexpr (dyn) QG_STAMP(2, 1, v[7].x);
      fft1c_pass0<V, false, CPD, 0, 8, false, LOGN>(v, tile + grp * n, lt, true);
      // the step's passes read rows of the 2/3 set only
      fft1c_rest<V, LOGN, false, CPD, SCH, 8, false, OP == OP_RHS || OP == OP_B>(tile + grp * n, twc, lt, true, tw1);
      if constexpr (dyn) QG_STAMP_LDS(2, 2);
    } else {
      __syncthreads();   // twiddles staged
      fft1_pass0<V, false>(v, tile + grp * n, lt, true, P.logny);
      fft1_rest<V, false>(tile + grp * n, twl, P.logny, lt, true);
    }
  } else {
    V* dst = tile + grp * n;
    for (int q = lt; q < P.W * P.ny; q += (1 << lg)) dst[q] = gld(src + q);
    __syncthreads();
    const FftShape sh{P.logny, P.W, 1, P.logW, true};
    fft_lds<V, false, COL_EPT>(tile + grp * n, twl, sh, FftGroup{lt, 1 << lg, true});
  }
  // product p at (m_y of row y, kx0 + w)
  auto at = [&](int p, int w, int iy) -> V {
    const int my = my_of_iy(iy, P.myh, P.kyn);
    const int y = my >= 0 ? my : my + P.ny;
    return one ? tile[p * n + padp<CPD>(y)] : tile[p * n + y * P.W + w];
  };
  const int nm = P.W * P.kyn;
  double hm = 0.0, mm = 0.0;
  for (int q = threadIdx.x; q < nm; q += blockDim.x) {
    const int w = one ? 0 : div_kyn(q, P.kyn);
    const int iy = q - (int)__umul24((unsigned)w, (unsigned)P.kyn);
    const int mx = kx0 + w;
    if (mx >= P.kxn) continue;
    const int my = my_of_iy(iy, P.myh, P.kyn);
    const int id = mx * P.kyn + iy;
    if constexpr (OP == OP_B || OP == OP_ENTRY || OP == OP_MASKFWD) {
      V v = at(0, w, iy);
      if (OP != OP_MASKFWD && mx == 0 && my == 0) v = cmake<V>(T(0), T(0));
      gst(cptr<T>(M, P.o_out) + id, v);
    } else if constexpr (OP == OP_PEN) {
      // D curl(chi u) = i kx F((chi - c) v) - i ky F((chi - c) u) + c omega,
      // omega the state the velocity came from (o_in)
      const Wave<T> wv = wave<T>(M, mx, my);
      V v = csub(mul_ia(at(1, w, iy), wv.kx), mul_ia(at(0, w, iy), wv.ky));
      v = cadd(v, cscale(gld(cptr<T>(M, P.o_in) + id), T(M.pen_c)));
      if (mx == 0 && my == 0) v = cmake<V>(T(0), T(0));
      gst(cptr<T>(M, P.o_out) + id, v);
    } else if constexpr (OP == OP_GTERMS) {
      // G = F(J) + (1/eta) (i kx F(chi v) - i ky F(chi u)) + sigma F(chi_s omega);
      // stage != 0: minus the spectrum at o_in2
      const Wave<T> wv = wave<T>(M, mx, my);
      const T ie = T(M.pen_a / M.dt), sg = T(M.sponge_a / M.dt);
      const V pen = csub(mul_ia(at(2, w, iy), wv.kx), mul_ia(at(1, w, iy), wv.ky));
      V g = cadd(cadd(at(0, w, iy), cscale(pen, ie)), cscale(at(3, w, iy), sg));
      if (P.stage != 0) g = csub(g, gld(cptr<T>(M, P.o_in2) + id));
      if (mx == 0 && my == 0) g = cmake<V>(T(0), T(0));
      gst(cptr<T>(M, P.o_out) + id, g);
    } else if constexpr (OP == OP_ADJ_B) {
      // lambda_s = F(l_w) - (i ky F(l_u) - i kx F(l_v)) / |k|^2 -> LS, LW, LK = dt/6 LS
      const Wave<T> wv = wave<T>(M, mx, my);
      const V lpsi = csub(mul_ia(at(1, w, iy), wv.ky), mul_ia(at(2, w, iy), wv.kx));
      const V l = csub(at(0, w, iy), cscale(lpsi, wv.inv_k2));
      gst(cptr<T>(M, P.o_out) + id, l);
      gst(cptr<T>(M, P.o_aux) + id, l);
      gst(cptr<T>(M, P.o_in) + id, cscale(l, T(M.dt6)));
    } else if constexpr (OP == OP_ADJ_RHS) {
      const Wave<T> wv = wave<T>(M, mx, my);
      V lpsi = csub(mul_ia(at(0, w, iy), wv.ky), mul_ia(at(1, w, iy), wv.kx));
      if constexpr (CL == 1) {
        lpsi = cadd(lpsi, cscale(at(4, w, iy), wv.ky * wv.ky - wv.kx * wv.kx));
        lpsi = cadd(lpsi, cscale(at(5, w, iy), -wv.kx * wv.ky));
      }
      const V Lx = cadd(mul_ia(at(2, w, iy), -wv.kx), mul_ia(at(3, w, iy), -wv.ky));
      if (P.adj_mode != 0) {
        // transport pass at the test-filtered stage input: its term,
        // test-filtered, to o_e
        const V e = csub(Lx, cscale(lpsi, wv.inv_k2));
        gst(cptr<T>(M, P.o_e) + id, in_test(M, P.nx, P.ny, mx, my) ? e : cmake<V>(T(0), T(0)));
        continue;
      }
      V* lk = cptr<T>(M, P.o_in2);
      V l = gld(lk + id);
      if (mx == 0 && my == 0) l = cmake<V>(T(0), T(0));
      const V lp = cadd(lpsi, mul_ia(l, (T(M.beta) * wv.kx)));
      V lx = csub(Lx, cscale(l, (wv.k2 * T(M.inv_re) + T(M.mu))));
      lx = csub(lx, cscale(lp, wv.inv_k2));
      if (P.adj_dyn) lx = cadd(lx, gld(cptr<T>(M, P.o_e) + id));   // the dynamic coefficient's term
      V* lw = cptr<T>(M, P.o_aux);
      gst(lw + id, cadd(gld(lw + id), lx));
      if (P.stage > 1) {
        const double dt = M.dt;
        const double cs = P.stage == 4 ? M.dt3 : P.stage == 3 ? M.dt3 : M.dt6;
        const double ds = P.stage == 4 ? dt : M.dt2;
        gst(lk + id, cadd(cscale(gld(cptr<T>(M, P.o_out) + id), T(cs)), cscale(lx, T(ds))));
      }
    } else if constexpr (!dyn) {
      const Wave<T> wv = wave<T>(M, mx, my);
      if (P.stage == SGS_STAGE) {
        V cq = cmake<V>(T(0), T(0));
        if constexpr (CL != 0)
          cq = cscale(cadd(mul_ia(at(1, w, iy), wv.kx), mul_ia(at(2, w, iy), wv.ky)), T(M.coef_static));
        if (mx == 0 && my == 0) cq = cmake<V>(T(0), T(0));
        gst(cptr<T>(M, P.o_out) + id, cq);
        continue;
      }
      if (P.stage == AB2CN_STAGE) {
        const V j = at(0, w, iy);
        V N = cmake<V>(-j.x, -j.y);
        if constexpr (CL != 0) {
          const V Q = cadd(mul_ia(at(1, w, iy), wv.kx), mul_ia(at(2, w, iy), wv.ky));
          N = cadd(N, cscale(Q, T(M.coef_static)));
        }
        ab2cn_update<T>(M, P, id, mx, my, N);
        continue;
      }
      const V* xin = cptr<T>(M, P.stage == 1 ? P.o_in2 : P.o_in);
      const V x = gld(xin + id);
      const V j = at(0, w, iy);
      V r = cmake<V>(-j.x, -j.y);
      r = csub(r, cscale(x, (wv.k2 * T(M.inv_re) + T(M.mu))));
      r = csub(r, mul_ia(poisson<T>(M, x, wv, mx, my), (T(M.beta) * wv.kx)));
      if constexpr (CL != 0) {
        const V Q = cadd(mul_ia(at(1, w, iy), wv.kx), mul_ia(at(2, w, iy), wv.ky));
        r = cadd(r, cscale(Q, T(M.coef_static)));
      }
      if (mx == 0 && my == 0) r = cmake<V>(T(0), T(0));
      const V w0 = gld(cptr<T>(M, P.o_in2) + id);
      V* acc = cptr<T>(M, P.o_aux);
      V* xout = cptr<T>(M, P.o_in);
      const double dt = M.dt;
      if (P.stage == 1) {
        gst(acc + id, cadd(w0, cscale(r, T(M.dt6))));
        gst(xout + id, cadd(w0, cscale(r, T(M.dt2))));
      } else if (P.stage == 2) {
        gst(acc + id, cadd(gld(acc + id), cscale(r, T(M.dt3))));
        gst(xout + id, cadd(w0, cscale(r, T(M.dt2))));
      } else if (P.stage == 3) {
        gst(acc + id, cadd(gld(acc + id), cscale(r, T(M.dt3))));
        gst(xout + id, cadd(w0, cscale(r, T(dt))));
      } else {
        gst(xout + id, cadd(gld(acc + id), cscale(r, T(M.dt6))));
      }
    } else {
      const Wave<T> wv = wave<T>(M, mx, my);
      const bool t = mylim >= -1 ? (my <= mylim && -my <= mylim) : in_test(M, P.nx, P.ny, mx, my);
      const V j = at(0, w, iy);
      const V Q = cadd(mul_ia(at(1, w, iy), wv.kx), mul_ia(at(2, w, iy), wv.ky));
      gst(cptr<T>(M, P.o_out) + id, j);
      gst(cptr<T>(M, P.o_aux) + id, Q);
      const V h = t ? csub(at(3, w, iy), j) : at(3, w, iy);
      V g = cscale(cadd(mul_ia(at(4, w, iy), wv.kx), mul_ia(at(5, w, iy), wv.ky)), T(M.r_test));
      if (t) g = csub(g, Q);
      const double wt = mx == 0 ? 1.0 : 2.0;
      hm += wt * ((double)h.x * (double)g.x + (double)h.y * (double)g.y);
      mm += wt * ((double)g.x * (double)g.x + (double)g.y * (double)g.y);
      if (P.adj_dyn) {   // kept for the adjoint
        gst(cptr<T>(M, P.o_h) + id, h);
        gst(cptr<T>(M, P.o_m) + id, g);
      }
    }
  }
  if constexpr (OP == OP_RHS && dyn) {
    QG_STAMP_DRAIN(2, 3);
    double shm = hm, smm = mm;
    block_sum2(shm, smm, red);
    if (threadIdx.x == 0) {
      double* part = rptr<double>(M, P.o_part) + 2 * strip;
      part[0] = shm;
      part[1] = smm;
    }
    QG_STAMP_DRAIN(2, 4);
  }
}

// The dynamic closures' right-hand-side column pass in two halves: six
// 1024-point transforms in one block need 104 KB of LDS in FP64 (one block
// per compute unit, so that a single member's 342 column blocks run in two
// rounds) and 52 KB in FP32 (two blocks of 12 waves).  Here three thread
// groups (6 waves at 1024) transform the grid level's products (J and the
// two flux components), keep the column's modes of them in registers, then
// transform the test level's products in the same LDS (their loads went
// out before the first half's transform) and form what the one-pass kernel
// forms: J and Q stored, H, M and the block's partial sums of <HM> and
// <M^2> (H and M also stored when adj_dyn).  The same arithmetic per mode
// as k_colfwdp; each thread adds two modes into the partial sums.
template <typename T, int CL, int LOGN, int SCH, bool WV = false>
__global__ void __launch_bounds__(3 << (LOGN - (WV ? 4 : 3))) k_colfwdd(Phase P) {
  using V = cpx<T>;
  // WV: one wave per transform, 16 elements per thread, radix-16 schedule
  constexpr int EPT = WV ? 16 : 8, SC = WV ? 2 : SCH;
  constexpr int CPD = QG_COL_PADS;
  constexpr int N = 1 << LOGN, LG = LOGN - (WV ? 4 : 3), NT = 3 << LG;
  constexpr int n = N + (N >> CPD);
  constexpr int KYN = 2 * ((N - 1) / 3) + 1;   // the 2/3 set's m_y count
  constexpr int QM = (KYN + NT - 1) / NT;      // modes per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  lds_poison_all(smem_raw, P.lds_bytes);
  __shared__ double red[32];
  QG_STAMP(2, 0, 0.f);
  const MemberDev M = member_const(P, blockIdx.z);
  V* tile = reinterpret_cast<V*>(smem_raw);
  const int grp = threadIdx.x >> LG;
  const int lt = threadIdx.x & ((1 << LG) - 1);
  const int kx0 = xcd_order(blockIdx.x, gridDim.x);
  if (kx0 >= P.kxn) return;
  const long long pstride = (long long)P.ny * P.kxp;
  const V* src = cptr<T>(M, P.o_mp) + grp * pstride + (long long)kx0 * P.ny;
  const int mylim = test_mylim(M, P.nx, P.ny, kx0);
  const V* twc = reinterpret_cast<const V*>(SC == 2 ? P.twy2 : SC ? P.twy1 : P.twy);
  const auto tw1 = fft1c_first_tw<V, LOGN, SC, EPT>(twc, lt);
  V v[EPT], w[EPT];
#pragma unroll
  for (int t = 0; t < EPT; ++t) v[t] = gld(src + lt + (t << LG));
#pragma unroll
  for (int t = 0; t < EPT; ++t) w[t] = gld(src + 3 * pstride + lt + (t << LG));
  QG_STAMP(2, 1, v[EPT - 1].x);
  V* buf = tile + grp * n;
  fft1c_pass0<V, false, CPD, 0, EPT, WV, LOGN>(v, buf, lt, true);
  fft1c_rest<V, LOGN, false, CPD, SC, EPT, WV, true>(buf, twc, lt, true, tw1);
  if constexpr (WV) __syncthreads();   // every group's transform before the reads across groups
  // the grid level's products at this thread's modes
  auto pos = [&](int iy) {
    const int my = my_of_iy(iy, P.myh, P.kyn);
    return padp<CPD>(my >= 0 ? my : my + N);
  };
  V a0[QM], a1[QM], a2[QM];
#pragma unroll
  for (int k = 0; k < QM; ++k) {
    const int q = threadIdx.x + k * NT;
    if (q < P.kyn) {
      const int y = pos(q);
      a0[k] = tile[y];
      a1[k] = tile[n + y];
      a2[k] = tile[2 * n + y];
    }
  }
  __syncthreads();   // every read of the first half before the second half's writes
  fft1c_pass0<V, false, CPD, 0, EPT, WV, LOGN>(w, buf, lt, true);
  fft1c_rest<V, LOGN, false, CPD, SC, EPT, WV, true>(buf, twc, lt, true, tw1);
  if constexpr (WV) __syncthreads();
  QG_STAMP_LDS(2, 2);
  double hm = 0.0, mm = 0.0;
  const int mx = kx0;
#pragma unroll
  for (int k = 0; k < QM; ++k) {
    const int iy = threadIdx.x + k * NT;
    if (iy >= P.kyn) continue;
    const int my = my_of_iy(iy, P.myh, P.kyn);
    const int y = pos(iy);
    const int id = mx * P.kyn + iy;
    const Wave<T> wv = wave<T>(M, mx, my);
    const bool t = my <= mylim && -my <= mylim;
    const V j = a0[k];
    const V Q = cadd(mul_ia(a1[k], wv.kx), mul_ia(a2[k], wv.ky));
    gst(cptr<T>(M, P.o_out) + id, j);
    gst(cptr<T>(M, P.o_aux) + id, Q);
    const V b3 = tile[y], b4 = tile[n + y], b5 = tile[2 * n + y];
    const V h = t ? csub(b3, j) : b3;
    V g = cscale(cadd(mul_ia(b4, wv.kx), mul_ia(b5, wv.ky)), T(M.r_test));
    if (t) g = csub(g, Q);
    const double wt = mx == 0 ? 1.0 : 2.0;
    hm += wt * ((double)h.x * (double)g.x + (double)h.y * (double)g.y);
    mm += wt * ((double)g.x * (double)g.x + (double)g.y * (double)g.y);
    if (P.adj_dyn) {   // kept for the adjoint (or the pointwise clip)
      gst(cptr<T>(M, P.o_h) + id, h);
      gst(cptr<T>(M, P.o_m) + id, g);
    }
  }
  QG_STAMP_DRAIN(2, 3);
  block_sum2(hm, mm, red);
  if (threadIdx.x == 0) {
    double* part = rptr<double>(M, P.o_part) + 2 * kx0;
    part[0] = hm;
    part[1] = mm;
  }
  QG_STAMP_DRAIN(2, 4);
}

// ---------------------------------------------------------------- combine
// Dynamic closures: C = max(<HM>, 0)/<M^2> from the fixed-order sum of the
// strip partials (every block sums them identically), then the RHS
// R = -J + C Q - (k^2/Re + mu) x - i beta kx psi and the RK4 update.
// Every thread of the block (NT threads) loads its share of the partials at
// once; the 64-lane wave sums and then the wave sums are added in a fixed
// order, so every block of a launch forms the same C.  red: 2 doubles per
// wave.  The thread's first pair comes in as `first` (dyn_part_first), so
// that a caller can issue that load before it waits on loads of its own.
struct DynPart {
  double hm, mm;
};
__device__ __forceinline__ DynPart dyn_part_first(const double* part, int nparts) {
  // unconditional (the index clamped; dyn_coefficient adds it only below
  // nparts), so that no branch puts the load next to its first use
  const double* pv = part + 2 * min((int)threadIdx.x, nparts - 1);
  return DynPart{pv[0], pv[1]};
}
template <int NT>
__device__ __forceinline__ void dyn_coefficient(const DynPart& first, const double* part, int nparts, double* red,
                                                double& C, double& hm_out, double& mm_out, int clip_mode = 0) {
  double hm = 0.0, mm = 0.0;
  if ((int)threadIdx.x < nparts) {
    hm += first.hm;
    mm += first.mm;
  }
  for (int i = threadIdx.x + NT; i < nparts; i += NT) { hm += part[2 * i]; mm += part[2 * i + 1]; }
  for (int o = 32; o > 0; o >>= 1) { hm += __shfl_xor(hm, o, 64); mm += __shfl_xor(mm, o, 64); }
  constexpr int nw = (NT + 63) >> 6;
  if ((threadIdx.x & 63) == 0) { red[2 * (threadIdx.x >> 6)] = hm; red[2 * (threadIdx.x >> 6) + 1] = mm; }
  __syncthreads();
  hm = 0.0;
  mm = 0.0;
  for (int w = 0; w < nw; ++w) { hm += red[2 * w]; mm += red[2 * w + 1]; }
  hm_out = hm;
  mm_out = mm;
  // clip_mode 1: the numerator is already clipped at every grid point
  C = mm > 0.0 ? (clip_mode == 1 ? hm : fmax(hm, 0.0)) / mm : 0.0;
}

template <typename T>
__global__ void __launch_bounds__(COMBINE_THREADS) k_combine(Phase P) {
  using V = cpx<T>;
  __shared__ double red[2 * (COMBINE_THREADS / 64)];
  QG_STAMP(3, 0, 0.f);
  const MemberDev M = member_const(P, blockIdx.z);
  // the partial sums' first load goes out before the per-mode loads
  const DynPart pf = dyn_part_first(rptr<double>(M, P.o_part), P.nparts);
  const int q = blockIdx.x * COMBINE_THREADS + threadIdx.x;
  const bool in = q < P.kxn * P.kyn;
  const bool rk = P.stage >= 1 && P.stage <= 4;
  const V* jsp = cptr<T>(M, P.o_out);
  const V* qsp = cptr<T>(M, P.o_aux);
  V* acc = cptr<T>(M, P.o_mp);   // accumulator offset passed in o_mp for this kernel
  int mx = 0, my = 0;
  // RK stages: the operands and the part of the right-hand side that does
  // not depend on C are loaded and formed before the partial sums are
  // reduced, so that the two memory latencies overlap
  V r0 = cmake<V>(T(0), T(0)), qv = r0, w0 = r0, a = r0;
  if (in) {
    mx = div_kyn(q, P.kyn);
    my = my_of_iy(q - (int)__umul24((unsigned)mx, (unsigned)P.kyn), P.myh, P.kyn);
    if (rk) {
      const Wave<T> w = wave<T>(M, mx, my);
      const V x = gld(cptr<T>(M, P.stage == 1 ? P.o_in2 : P.o_in) + q);
      const V j = gld(jsp + q);
      qv = gld(qsp + q);
      w0 = gld(cptr<T>(M, P.o_in2) + q);
      if (P.stage > 1) a = gld(acc + q);
      r0 = cmake<V>(-j.x, -j.y);
      r0 = csub(r0, cscale(x, (w.k2 * T(M.inv_re) + T(M.mu))));
      r0 = csub(r0, mul_ia(poisson<T>(M, x, w, mx, my), (T(M.beta) * w.kx)));
    }
  }
  QG_STAMP(3, 1, r0.x);
  double C, hm, mm;
  dyn_coefficient<COMBINE_THREADS>(pf, rptr<double>(M, P.o_part), P.nparts, red, C, hm, mm, M.clip_mode);
  QG_STAMP(3, 2, C);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* c = rptr<double>(M, P.o_coef);
    if (P.stage == SGS_STAGE) {
      c[0] = C;
    } else {
      c[P.stage] = C;
      c[8 + 2 * P.stage] = hm;
      c[9 + 2 * P.stage] = mm;
    }
    if (P.adj_dyn) {   // kept for the adjoint
      double* k = rptr<double>(M, P.o_cs);
      k[0] = C;
      k[1] = hm;
      k[2] = mm;
    }
  }
  if (!in) return;
  if (P.stage == SGS_STAGE) {
    // the closure's term C Q alone, to o_in
    V cq = cscale(qsp[q], T(C));
    if (mx == 0 && my == 0) cq = cmake<V>(T(0), T(0));
    gst(cptr<T>(M, P.o_in) + q, cq);
    return;
  }
  if (P.stage == AB2CN_STAGE) {
    const V j = jsp[q];
    ab2cn_update<T>(M, P, q, mx, my, cadd(cmake<V>(-j.x, -j.y), cscale(qsp[q], T(C))));
    return;
  }
  V r = cadd(r0, cscale(qv, T(C)));
  if (mx == 0 && my == 0) r = cmake<V>(T(0), T(0));
  const double dt = M.dt;
  V* xout = cptr<T>(M, P.o_in);
  if (P.stage == 1) {
    gst(acc + q, cadd(w0, cscale(r, T(M.dt6))));
    gst(xout + q, cadd(w0, cscale(r, T(M.dt2))));
  } else if (P.stage == 2) {
    gst(acc + q, cadd(a, cscale(r, T(M.dt3))));
    gst(xout + q, cadd(w0, cscale(r, T(M.dt2))));
  } else if (P.stage == 3) {
    gst(acc + q, cadd(a, cscale(r, T(M.dt3))));
    gst(xout + q, cadd(w0, cscale(r, T(dt))));
  } else {
    gst(xout + q, cadd(a, cscale(r, T(M.dt6))));
  }
  QG_STAMP_DRAIN(3, 3);
}

// ---------------------------------------------------------------- dynamic-closure adjoint
// Per stage of the reverse sweep.  k_adj_dot: block partial sums of
// s = <lambda, Q> (Parseval weights 1 at m_x = 0 else 2) with lambda at
// o_in2 and the stage's Q at o_aux, to the member's dpart area.
template <typename T>
__global__ void __launch_bounds__(COMBINE_THREADS) k_adj_dot(Phase P) {
  using V = cpx<T>;
  __shared__ double red[COMBINE_THREADS / 64];
  const MemberDev M = member_const(P, blockIdx.z);
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (q < P.kxn * P.kyn) {
    const V l = gld(cptr<T>(M, P.o_in2) + q), Q = gld(cptr<T>(M, P.o_aux) + q);
    v = (q < P.kyn ? 1.0 : 2.0) * ((double)l.x * (double)Q.x + (double)l.y * (double)Q.y);
  }
  v = block_sum(v, red);
  if (threadIdx.x == 0) rptr<double>(M, P.o_dpart)[blockIdx.x] = v;
}

// k_adj_dyn_prep: the stage's C, <HM>, <M^2> as the forward step kept them
// (o_cs), s from the k_adj_dot partials in a fixed order, then the
// cotangents of H and M (kept at o_h, o_m)
//   a = (s/<M^2>) M,  b = (s/<M^2>)(H - 2 C M)   (zero where the clip holds),
// and C to ADJ_C_SLOT for the stage's own adjoint pass.
template <typename T>
__global__ void __launch_bounds__(COMBINE_THREADS) k_adj_dyn_prep(Phase P) {
  using V = cpx<T>;
  __shared__ double red[COMBINE_THREADS / 64];
  const MemberDev M = member_const(P, blockIdx.z);
  const double* ps = rptr<double>(M, P.o_dpart);
  const int nparts = (P.kxn * P.kyn + COMBINE_THREADS - 1) / COMBINE_THREADS;
  double sv = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) sv += ps[i];
  for (int o = 32; o > 0; o >>= 1) sv += __shfl_xor(sv, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sv;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)((blockDim.x + 63) >> 6); ++w) s += red[w];
  const double* k = rptr<double>(M, P.o_cs);
  const double C = k[0], hm = k[1], mm = k[2];
  if (blockIdx.x == 0 && threadIdx.x == 0) rptr<double>(M, P.o_coef)[ADJ_C_SLOT] = C;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.kxn * P.kyn) return;
  const double f = (hm > 0.0 && mm > 0.0) ? s / mm : 0.0;
  const V h = gld(cptr<T>(M, P.o_h) + q), g = gld(cptr<T>(M, P.o_m) + q);
  const double gx = g.x, gy = g.y;
  gst(cptr<T>(M, P.o_a) + q, cmake<V>(T(f * gx), T(f * gy)));
  gst(cptr<T>(M, P.o_b) + q, cmake<V>(T(f * ((double)h.x - 2.0 * C * gx)), T(f * ((double)h.y - 2.0 * C * gy))));
}

// ---------------------------------------------------------------- LES filter
// H_full of Sec. III on one member pair: the fully-resolved state (FR
// D-compact spectrum) times exp(-k^2 (delta Delta_FR)^2 / 6), cut off at
// |k| > pi / Delta_FF, rescaled by 1/delta^2 onto the coarse grid's
// full-set compact spectrum (Nyquist lines excluded).  Every retained mode
// lies inside the FR 2/3 set (delta >= 2).
template <typename T>
__global__ void __launch_bounds__(256) k_filter_les(FilterArgs A) {
  using V = cpx<T>;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= A.kxn_c * A.kyn_c) return;
  const int mx = q / A.kyn_c;
  const int iyc = q - mx * A.kyn_c;
  const int my = my_of_iy(iyc, A.myh_c, A.kyn_c);
  V v = cmake<V>(T(0), T(0));
  const double kx = A.two_pi_lx * mx, ky = A.two_pi_ly * my;
  const double k2 = kx * kx + ky * ky;
  if (k2 <= A.kc2 && mx < A.kxn_f && my <= A.myh_f && -my <= A.myh_f) {
    const int iyf = my >= 0 ? my : my + A.kyn_f;
    const V w = gld(reinterpret_cast<const V*>(A.src) + (mx * A.kyn_f + iyf));
    const double h = exp(-k2 * A.width2 / 6.0) * A.inv_d2;
    v = cmake<V>(T((double)w.x * h), T((double)w.y * h));
  }
  gst(reinterpret_cast<V*>(A.dst) + q, v);
}

// ---------------------------------------------------------------- PCC
// Pattern correlation of two fields per member, two-pass in double
// precision with fixed summation orders: (1) per-block sums of a and b,
// (2) the means from those partials, then per-block centred sums of
// (a - <a>)(b - <b>), (a - <a>)^2, (b - <b>)^2, (3) one block per member
// adds them up.  Partials live in the member's dpart area: 2 doubles per
// block, then 3 per block.
constexpr int PCC_THREADS = 256;

template <typename T>
__global__ void __launch_bounds__(PCC_THREADS) k_pcc_sums(Phase P, const void* a, const void* b) {
  __shared__ double red[PCC_THREADS / 64];
  const MemberDev M = member_const(P, blockIdx.z);
  const long long n = (long long)P.nx * P.ny;
  const T* x = reinterpret_cast<const T*>(reinterpret_cast<const char*>(a) + M.omega_off);
  const T* y = reinterpret_cast<const T*>(reinterpret_cast<const char*>(b) + M.omega_off);
  double sx = 0.0, sy = 0.0;
  for (long long i = (long long)blockIdx.x * PCC_THREADS + threadIdx.x; i < n; i += (long long)gridDim.x * PCC_THREADS) {
    sx += (double)x[i];
    sy += (double)y[i];
  }
  sx = block_sum(sx, red);
  sy = block_sum(sy, red);
  if (threadIdx.x == 0) {
    double* part = rptr<double>(M, P.o_dpart) + 2 * blockIdx.x;
    part[0] = sx;
    part[1] = sy;
  }
}

template <typename T>
__global__ void __launch_bounds__(PCC_THREADS) k_pcc_centred(Phase P, const void* a, const void* b) {
  __shared__ double red[PCC_THREADS / 64];
  __shared__ double mean[2];
  const MemberDev M = member_const(P, blockIdx.z);
  const long long n = (long long)P.nx * P.ny;
  double* part = rptr<double>(M, P.o_dpart);
  if (threadIdx.x < 64) {
    // the first wave: lane k takes block k's sums (at most 64 blocks), then
    // a fixed shuffle tree, so every block forms the same means
    double sx = 0.0, sy = 0.0;
    for (int k = threadIdx.x; k < (int)gridDim.x; k += 64) { sx += part[2 * k]; sy += part[2 * k + 1]; }
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_xor(sx, o, 64);
      sy += __shfl_xor(sy, o, 64);
    }
    if (threadIdx.x == 0) {
      mean[0] = sx / (double)n;
      mean[1] = sy / (double)n;
    }
  }
  __syncthreads();
  const double mx = mean[0], my = mean[1];
  const T* x = reinterpret_cast<const T*>(reinterpret_cast<const char*>(a) + M.omega_off);
  const T* y = reinterpret_cast<const T*>(reinterpret_cast<const char*>(b) + M.omega_off);
  double sxy = 0.0, sxx = 0.0, syy = 0.0;
  for (long long i = (long long)blockIdx.x * PCC_THREADS + threadIdx.x; i < n; i += (long long)gridDim.x * PCC_THREADS) {
    const double dx = (double)x[i] - mx, dy = (double)y[i] - my;
    sxy += dx * dy;
    sxx += dx * dx;
    syy += dy * dy;
  }
  sxy = block_sum(sxy, red);
  sxx = block_sum(sxx, red);
  syy = block_sum(syy, red);
  if (threadIdx.x == 0) {
    double* c = part + 2 * gridDim.x + 3 * blockIdx.x;
    c[0] = sxy;
    c[1] = sxx;
    c[2] = syy;
  }
}

#if QG_HAS(4)
__global__ void __launch_bounds__(64) k_pcc_final(Phase P, int nblk, double* out) {
  const MemberDev M = member_const(P, blockIdx.x);
  const double* c = rptr<double>(M, P.o_dpart) + 2 * nblk;
  // lane k < nblk (at most 64 blocks) loads block k's sums; fixed shuffle tree
  double sxy = 0.0, sxx = 0.0, syy = 0.0;
  for (int k = threadIdx.x; k < nblk; k += 64) { sxy += c[3 * k]; sxx += c[3 * k + 1]; syy += c[3 * k + 2]; }
  for (int o = 32; o > 0; o >>= 1) {
    sxy += __shfl_xor(sxy, o, 64);
    sxx += __shfl_xor(sxx, o, 64);
    syy += __shfl_xor(syy, o, 64);
  }
  if (threadIdx.x == 0) out[M.user_index] = sxy / sqrt(sxx * syy);
}
#endif

// C of the dynamic closures for diagnostics (slot 0 of the coef area).
#if QG_HAS(4)
__global__ void k_dyn_coef(Phase P, int slot) {
  __shared__ double red[2];   // one 64-thread wave
  const MemberDev M = member_const(P, blockIdx.z);
  double C, hm, mm;
  const double* part = rptr<double>(M, P.o_part);
  dyn_coefficient<64>(dyn_part_first(part, P.nparts), part, P.nparts, red, C, hm, mm, M.clip_mode);
  if (threadIdx.x == 0) rptr<double>(M, P.o_coef)[slot] = C;
}
#endif

// ---------------------------------------------------------------- diagnostics
// Parseval sums of energy sum w |k|^2 |psi|^2 and enstrophy sum w |omega|^2.
template <typename T>
__global__ void __launch_bounds__(256) k_diag_spectral(Phase P) {
  using V = cpx<T>;
  __shared__ double red[16];
  const MemberDev M = member_const(P, blockIdx.z);
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0, z = 0.0;
  if (q < P.kxn * P.kyn) {
    const int mx = div_kyn(q, P.kyn);
    const int iy = q - (int)__umul24((unsigned)mx, (unsigned)P.kyn);
    const int my = my_of_iy(iy, P.myh, P.kyn);
    const Wave<T> w = wave<T>(M, mx, my);
    const V x = cptr<T>(M, P.o_in)[q];
    const double a2 = (double)x.x * x.x + (double)x.y * x.y;
    const double wt = mx == 0 ? 1.0 : 2.0;
    const bool zm = (mx == 0 && my == 0);
    z = zm ? 0.0 : wt * a2;
    e = zm ? 0.0 : wt * a2 * w.inv_k2;   // |k|^2 |psi|^2 = |omega|^2 / |k|^2
  }
  double se = block_sum(e, red);
  double sz = block_sum(z, red);
  if (threadIdx.x == 0) {
    double* d = rptr<double>(M, P.o_aux) + 2 * blockIdx.x;
    d[0] = se;
    d[1] = sz;
  }
}

#if QG_HAS(4)
__global__ void __launch_bounds__(64) k_diag_final(Phase P, int nrow, int nspec, double* out, int) {
  const MemberDev& M = P.mem[P.m0 + blockIdx.x];
  const double* rp = rptr<double>(M, P.o_dpart);
  const double* sp = rptr<double>(M, P.o_aux);
  // one 64-lane wave per member: lane l takes partials l, l + 64, ... (all
  // loads in flight at once), then a fixed butterfly of shuffles
  double nus = 0.0, mn = INFINITY, mxv = -INFINITY, cf = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < nrow; i += 64) {
    nus += rp[5 * i]; mn = fmin(mn, rp[5 * i + 1]); mxv = fmax(mxv, rp[5 * i + 2]);
    cf = fmax(cf, rp[5 * i + 3]); bad = fmax(bad, rp[5 * i + 4]);
  }
  double e = 0.0, z = 0.0;
  for (int i = threadIdx.x; i < nspec; i += 64) { e += sp[2 * i]; z += sp[2 * i + 1]; }
  for (int o = 32; o > 0; o >>= 1) {
    nus += __shfl_xor(nus, o, 64);
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mxv = fmax(mxv, __shfl_xor(mxv, o, 64));
    cf = fmax(cf, __shfl_xor(cf, o, 64));
    bad = fmax(bad, __shfl_xor(bad, o, 64));
    e += __shfl_xor(e, o, 64);
    z += __shfl_xor(z, o, 64);
  }
  if (threadIdx.x != 0) return;
  const double n2 = M.inv_n * M.inv_n;
  double* o = out + 8 * M.user_index;
  o[0] = 0.5 * e * n2;
  o[1] = 0.5 * z * n2;
  o[2] = (M.closure == 3 || M.closure == 4) ? rptr<double>(M, P.o_coef)[0] : M.coef_static;
  o[3] = mn;
  o[4] = nus * M.inv_n;
  o[5] = mxv;
  o[6] = cf * M.dt * M.inv_delta;
  o[7] = (bad > 0.0 || !isfinite(e) || !isfinite(z)) ? 1.0 : 0.0;
}
#endif

// ---------------------------------------------------------------- adjoint misc
// dL/dc: the row blocks' partial sums of one adjoint stage, in a fixed
// order, accumulated into coef slot 24 of the member (mode 0); mode 1 zeroes
// the slot; mode 2 adds the slot to the caller's grad_c.  One 64-lane wave
// per member: lane l sums partials l, l + 64, ... (all loads in flight at
// once), then a fixed butterfly of shuffles adds the lanes.
#if QG_HAS(4)
__global__ void __launch_bounds__(64) k_adj_grad_c(Phase P, int nrow, double* grad_c, int mode) {
  const MemberDev& M = P.mem[P.m0 + blockIdx.x];
  double* slot = rptr<double>(M, P.o_coef) + 24;
  if (mode != 0) {
    if (threadIdx.x != 0) return;
    if (mode == 1) *slot = 0.0;
    else grad_c[M.user_index] += *slot;
    return;
  }
  const double* d = rptr<double>(M, P.o_dpart);
  double s = 0.0;
  for (int i = threadIdx.x; i < nrow; i += 64) s += d[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) *slot += s;
}
#endif

// dst = a * dst + src (zero_first: dst = src) over the D-compact state
template <typename T>
__global__ void k_spec_axpy(Phase P, long long o_dst, long long o_src, double a, int zero_first) {
  using V = cpx<T>;
  const MemberDev M = member_const(P, blockIdx.z);
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P.kxn * P.kyn) return;
  V* d = cptr<T>(M, o_dst);
  const V s = cptr<T>(M, o_src)[q];
  d[q] = zero_first ? s : cadd(cscale(d[q], T(a)), s);
}

#if QG_HAS(4)
// One member's constants into a device table (argument copied at launch, so
// the call needs no host buffer that outlives it).
__global__ void k_put_member(MemberDev* dst, MemberDev m) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = m;
}

// Per-pass twiddle table of length-n transforms under pass schedule sch (the
// layout of qg_fft.hpp), computed on the device: slot o of the pass with
// sub-length ns and radix r, o = (ns - 8) + k (r - 1) + (t - 1), holds
// exp(-2 pi i m / n) with m = t k n / (ns r), from the double-precision
// sincospi of the reduced angle.
template <typename T>
__global__ void k_twiddle_table(cpx<T>* dst, int logn, int sch) {
  const int n = 1 << logn;
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n - 8) return;
  int logns = 3;
  while (logns < logn) {
    const int lr = pass_log_radix(logn, logns, sch);
    if (o < (1 << (logns + lr)) - 8) break;
    logns += lr;
  }
  const int r = 1 << pass_log_radix(logn, logns, sch);
  const int idx = o - ((1 << logns) - 8);
  const int k = idx / (r - 1), t = idx % (r - 1) + 1;
  const long long m = ((long long)t * k << (logn - logns - pass_log_radix(logn, logns, sch))) & (n - 1);
  double sv, cv;
  sincospi(-2.0 * (double)m / (double)n, &sv, &cv);
  dst[o] = cmake<cpx<T>>(T(cv), T(sv));
}

__global__ void k_fill_zero(unsigned int* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0u;
}
#endif

// ---------------------------------------------------------------- launchers
// Launch of a phase kernel.  A profiling run sets P.ev0 / P.ev1: the launch
// then binds the two HIP events to the dispatch itself, so they carry its
// own begin and end times (no marker of their own in the stream).
#define QG_KLAUNCH(KERNEL, GRID, BLOCK, LDS, S, P)                                                    \
  do {                                                                                                \
    Phase P_ = (P);                                                                                   \
    P_.lds_bytes = (unsigned)(LDS);                                                                   \
    if (P_.ev0)                                                                                       \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, (std::uint32_t)(LDS), S, (hipEvent_t)P_.ev0,         \
                            (hipEvent_t)P_.ev1, 0u, P_);                                              \
    else                                                                                              \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, LDS, S, P_);                                            \
  } while (0)

// strips of a column pass, padded to a multiple of 8 (XCD-aware order)
static unsigned col_grid(const Phase& P) { return (unsigned)(((P.kxn + P.W - 1) / P.W + 7) / 8 * 8); }
static size_t col_tile(const Phase& P) { return (size_t)P.W * P.ny + (P.W == 1 ? P.ny / 8 : 0); }
static size_t col_smem(bool dbl, const Phase& P) { return (col_tile(P) + P.ny) * (dbl ? 16 : 8); }
static unsigned coli_grid(const Phase& P) { return (unsigned)(((P.kxn + P.Wi - 1) / P.Wi + 7) / 8 * 8); }
static size_t coli_smem(bool dbl, const Phase& P) {
  return ((size_t)P.Wi * P.ny + (P.Wi == 1 ? P.ny / 8 : 0) + P.ny) * (dbl ? 16 : 8);
}
static size_t row_smem(bool dbl, const Phase& P) { return ((size_t)P.RP * P.nx + P.nx) * (dbl ? 16 : 8); }
static int row_threads(const Phase& P) { return P.RP * P.nx / ROW_EPT; }

template <typename T, int OP, int CL>
static void launch_colinv_t(const Phase& P, int nmem, hipStream_t s) {
  dim3 grid(coli_grid(P), P.nf, nmem);
  const dim3 block(P.Wi * P.ny / COL_EPT);
  {
    // compile-time column lengths for the common sizes (every op: the
    // kernel's compile-time path is generic in the field formation)
    const size_t lds = (size_t)P.Wi * colinv_stride(P.ny) * sizeof(cpx<T>);
    // (their engines assume spectral fields on the 2/3 set)
    const int logny = P.myh == (P.ny - 1) / 3 && P.kxn == (P.nx - 1) / 3 + 1 ? P.logny : 0;
    // the step's passes take the tuned pass schedule
    const bool s1 = (OP == OP_RHS || OP == OP_B) && P.csch == 1;
    switch (logny) {
      case 8:
        if (s1) QG_KLAUNCH((k_colinv<T, OP, CL, 8, 1>), grid, block, lds, s, P);
        else QG_KLAUNCH((k_colinv<T, OP, CL, 8>), grid, block, lds, s, P);
        return;
      case 9:
        if (s1) QG_KLAUNCH((k_colinv<T, OP, CL, 9, 1>), grid, block, lds, s, P);
        else QG_KLAUNCH((k_colinv<T, OP, CL, 9>), grid, block, lds, s, P);
        return;
      case 10:
        if (s1) QG_KLAUNCH((k_colinv<T, OP, CL, 10, 1>), grid, block, lds, s, P);
        else QG_KLAUNCH((k_colinv<T, OP, CL, 10>), grid, block, lds, s, P);
        return;
      default: break;
    }
  }
  QG_KLAUNCH((k_colinv<T, OP, CL, 0>), grid, block, coli_smem(sizeof(T) == 8, P), s, P);
}
static int rowp_fields(int op, int cl) { return rowp_nb(op, cl); }
static size_t rowp_lds(bool dbl, int op, int cl, const Phase& P) {
  return (size_t)rowp_fields(op, cl) * (P.nx + (P.nx >> 3)) * (dbl ? 16 : 8);
}
static bool rowp_ok(bool dbl, int op, int cl, const Phase& P) {
  const int nb = rowp_fields(op, cl);
  return P.nx >= 64 && nb * P.nx / 8 <= 1024 && rowp_lds(dbl, op, cl, P) <= 128 * 1024;
}
// The compile-time row engines of length 2^LN; the step's passes take the
// tuned pass schedule (s1: schedule 1, or 2 where it applies) and
// wave-synchronous transforms (wv).  Schedule 2 (radix 16) needs 16
// elements per thread: the wave-synchronous 1024-point rows; elsewhere
// schedule 1 stands in for it.
template <typename T, int OP, int CL, int LN, int RPB>
static void launch_rowp_sched(const Phase& P, dim3 grid, dim3 block, size_t lds, hipStream_t s, bool s1, bool wv) {
  if (wv) {
    if constexpr (LN == 10) {
      if (P.rsch == 2) {
        QG_KLAUNCH((k_rowp<T, OP, CL, LN, 2, true, RPB>), grid, block, lds, s, P);
        return;
      }
    }
    if (s1) QG_KLAUNCH((k_rowp<T, OP, CL, LN, 1, true, RPB>), grid, block, lds, s, P);
    else QG_KLAUNCH((k_rowp<T, OP, CL, LN, 0, true, RPB>), grid, block, lds, s, P);
  } else {
    if (s1) QG_KLAUNCH((k_rowp<T, OP, CL, LN, 1, false, RPB>), grid, block, lds, s, P);
    else QG_KLAUNCH((k_rowp<T, OP, CL, LN, 0, false, RPB>), grid, block, lds, s, P);
  }
}
template <typename T, int OP, int CL, int LN>
static void launch_rowp_len(const Phase& P, dim3 grid, dim3 block, size_t lds, hipStream_t s, bool s1, bool wv,
                            int rpb) {
  if constexpr (OP == OP_RHS || OP == OP_B) {
    if (rpb == 2) launch_rowp_sched<T, OP, CL, LN, 2>(P, grid, block, lds, s, s1, wv);
    else launch_rowp_sched<T, OP, CL, LN, 1>(P, grid, block, lds, s, s1, wv);
    return;
  }
  QG_KLAUNCH((k_rowp<T, OP, CL, LN>), grid, block, lds, s, P);
}

template <typename T, int OP, int CL>
static void launch_rowp_t(const Phase& P, int nmem, hipStream_t s) {
  const int nb = rowp_fields(OP, CL);
  const int levels = (OP == OP_RHS && (CL == 3 || CL == 4)) || (OP == OP_ADJ_RHS && P.adj_mode == 2) ? 2 : 1;
  const size_t lds = rowp_lds(sizeof(T) == 8, OP, CL, P);
  // the step's passes take the tuned row pairs per block, pass schedule and
  // synchronisation (one wave per transform: 16 points per thread at 1024)
  const bool step = OP == OP_RHS || OP == OP_B;
  const int rpb = step && P.rpb == 2 ? 2 : 1;
  const bool s1 = step && P.rsch >= 1;
  const bool wv = step && P.rwv == 1;
  const dim3 block(nb * (wv && P.nx >= 1024 ? P.nx / 16 : P.nx / 8));
  dim3 grid(P.ny / (2 * rpb), levels, nmem);
  // compile-time transform lengths for the common row lengths (their
  // engines assume the mixed fields hold the 2/3 set: kxn columns)
  const int lognx = P.kxn == (P.nx - 1) / 3 + 1 ? P.lognx : 0;
  switch (lognx) {
    case 8: launch_rowp_len<T, OP, CL, 8>(P, grid, block, lds, s, s1, wv, rpb); return;
    case 9: launch_rowp_len<T, OP, CL, 9>(P, grid, block, lds, s, s1, wv, rpb); return;
    case 10: launch_rowp_len<T, OP, CL, 10>(P, grid, block, lds, s, s1, wv, rpb); return;
    default: break;
  }
  // the run-time-length engine: one row pair per block
  grid.x = P.ny / 2;
  QG_KLAUNCH((k_rowp<T, OP, CL, 0>), grid, dim3(nb * P.nx / 8), lds, s, P);
}

template <typename T, int OP, int CL>
static void launch_row_t(const Phase& P, int nmem, hipStream_t s) {
  if constexpr (OP == OP_PEN || OP == OP_SPONGE || OP == OP_GTERMS || OP == OP_CLIPF) {
    // field-parallel kernel only (the sizes it cannot take are refused before)
    if (rowp_ok(sizeof(T) == 8, OP, CL, P)) launch_rowp_t<T, OP, CL>(P, nmem, s);
    return;
  }
  if constexpr (OP == OP_RHS || OP == OP_B || OP == OP_ADJ_RHS || OP == OP_ADJ_B) {
    if (rowp_ok(sizeof(T) == 8, OP, CL, P)) { launch_rowp_t<T, OP, CL>(P, nmem, s); return; }
  }
  dim3 grid(P.ny / (2 * P.RP), 1, nmem);
  QG_KLAUNCH((k_row<T, OP, CL>), grid, dim3(row_threads(P)), row_smem(sizeof(T) == 8, P), s, P);
}
static int colfwdp_products(int op, int cl) {
  if (op == OP_RHS) return cl == 0 ? 1 : (cl == 3 || cl == 4) ? 6 : 3;
  if (op == OP_ADJ_B) return 3;
  if (op == OP_PEN) return 2;
  if (op == OP_GTERMS) return 4;
  if (op == OP_ADJ_RHS) return cl == 1 ? 6 : 4;
  return 1;
}
static bool colfwdp_ok(bool dbl, int op, int cl, const Phase& P) {
  const int np = colfwdp_products(op, cl);
  const size_t n = col_tile(P);
  return np * ((size_t)P.W * P.ny) / COL_EPT <= 1024 && (np * n + P.ny) * (dbl ? 16 : 8) <= 128 * 1024;
}
template <typename T, int OP, int CL>
static void launch_colfwdp_t(const Phase& P, int nmem, hipStream_t s) {
  const int np = colfwdp_products(OP, CL);
  dim3 grid(col_grid(P), 1, nmem);
  const size_t n = col_tile(P);
  const dim3 block(np * ((size_t)P.W * P.ny) / COL_EPT);
  {
    // compile-time column lengths for the common sizes (one column per
    // block; every op, as for the column-inverse pass)
    const size_t lds = np * n * sizeof(cpx<T>);
    const bool s1 = (OP == OP_RHS || OP == OP_B) && P.csch == 1;
    if constexpr (OP == OP_RHS && (CL == 3 || CL == 4)) {
      // dynamic closures: the pass in two halves (k_colfwdd), three
      // transforms' LDS per block
      if (P.W == 1 && P.logny >= 8 && P.logny <= 10) {
        const size_t lds2 = 3 * (size_t)(P.ny + (P.ny >> QG_COL_PADS)) * sizeof(cpx<T>);
        const dim3 block2(3 * P.ny / COL_EPT);
        // 1024-point columns with the wave-synchronous choice: one wave
        // per transform, radix-16 passes (FP32 only: the FP64 form would
        // hold about 260 registers per lane, one wave per SIMD)
        if constexpr (sizeof(T) == 4)
          if (P.logny == 10 && P.cwv) {
            QG_KLAUNCH((k_colfwdd<T, CL, 10, 0, true>), grid, dim3(3 * P.ny / 16), lds2, s, P);
            return;
          }
        switch (P.logny) {
          case 8:
            if (s1) QG_KLAUNCH((k_colfwdd<T, CL, 8, 1>), grid, block2, lds2, s, P);
            else QG_KLAUNCH((k_colfwdd<T, CL, 8, 0>), grid, block2, lds2, s, P);
            return;
          case 9:
            if (s1) QG_KLAUNCH((k_colfwdd<T, CL, 9, 1>), grid, block2, lds2, s, P);
            else QG_KLAUNCH((k_colfwdd<T, CL, 9, 0>), grid, block2, lds2, s, P);
            return;
          default:
            if (s1) QG_KLAUNCH((k_colfwdd<T, CL, 10, 1>), grid, block2, lds2, s, P);
            else QG_KLAUNCH((k_colfwdd<T, CL, 10, 0>), grid, block2, lds2, s, P);
            return;
        }
      }
    }
    if (P.W == 1) switch (P.logny) {
      case 8:
        if (s1) QG_KLAUNCH((k_colfwdp<T, OP, CL, 8, 1>), grid, block, lds, s, P);
        else QG_KLAUNCH((k_colfwdp<T, OP, CL, 8>), grid, block, lds, s, P);
        return;
      case 9:
        if (s1) QG_KLAUNCH((k_colfwdp<T, OP, CL, 9, 1>), grid, block, lds, s, P);
        else QG_KLAUNCH((k_colfwdp<T, OP, CL, 9>), grid, block, lds, s, P);
        return;
      case 10:
        if (s1) QG_KLAUNCH((k_colfwdp<T, OP, CL, 10, 1>), grid, block, lds, s, P);
        else QG_KLAUNCH((k_colfwdp<T, OP, CL, 10>), grid, block, lds, s, P);
        return;
      default: break;
    }
  }
  QG_KLAUNCH((k_colfwdp<T, OP, CL, 0>), grid, block, (np * n + P.ny) * sizeof(cpx<T>), s, P);
}

template <typename T, int OP, int CL>
static void launch_colfwd_t(const Phase& P, int nmem, hipStream_t s) {
  if constexpr (OP == OP_PEN || OP == OP_GTERMS) {
    // product-parallel kernel only (the sizes it cannot take are refused before)
    if (colfwdp_ok(sizeof(T) == 8, OP, CL, P)) launch_colfwdp_t<T, OP, CL>(P, nmem, s);
    return;
  }
  if constexpr (OP == OP_RHS || OP == OP_B || OP == OP_ENTRY || OP == OP_MASKFWD || OP == OP_ADJ_B ||
                OP == OP_ADJ_RHS) {
    if (colfwdp_ok(sizeof(T) == 8, OP, CL, P)) { launch_colfwdp_t<T, OP, CL>(P, nmem, s); return; }
  }
  dim3 grid(col_grid(P), 1, nmem);
  constexpr int EPT = COL_EPT;
  QG_KLAUNCH((k_colfwd<T, OP, CL, EPT>), grid, dim3(P.W * P.ny / COL_EPT), col_smem(sizeof(T) == 8, P), s, P);
}

#define QG_CL_SWITCH(FN, T, OP, cl, P, n, s)                 \
  switch (cl) {                                              \
    case 0: FN<T, OP, 0>(P, n, s); break;                    \
    case 1: FN<T, OP, 1>(P, n, s); break;                    \
    case 2: FN<T, OP, 2>(P, n, s); break;                    \
    case 3: FN<T, OP, 3>(P, n, s); break;                    \
    default: FN<T, OP, 4>(P, n, s); break;                   \
  }

#define QG_CL_SWITCH_STATIC(FN, T, OP, cl, P, n, s)          \
  switch (cl) {                                              \
    case 0: FN<T, OP, 0>(P, n, s); break;                    \
    case 1: FN<T, OP, 1>(P, n, s); break;                    \
    default: FN<T, OP, 2>(P, n, s); break;                   \
  }

template <typename T> void colinv_dispatch(int op, int cl, const Phase& P, int n, hipStream_t s) {
  switch (op) {
    case OP_RHS: QG_CL_SWITCH(launch_colinv_t, T, OP_RHS, cl, P, n, s); break;
    case OP_DIAG: QG_CL_SWITCH(launch_colinv_t, T, OP_DIAG, cl, P, n, s); break;
    case OP_B: launch_colinv_t<T, OP_B, 0>(P, n, s); break;
    case OP_EXIT: case OP_ADJ_ENTRY: launch_colinv_t<T, OP_EXIT, 0>(P, n, s); break;
    case OP_MASKGRAD: launch_colinv_t<T, OP_MASKGRAD, 0>(P, n, s); break;
    case OP_SPONGE: launch_colinv_t<T, OP_SPONGE, 0>(P, n, s); break;
    case OP_GTERMS: launch_colinv_t<T, OP_GTERMS, 0>(P, n, s); break;
    case OP_CLIPF: launch_colinv_t<T, OP_CLIPF, 0>(P, n, s); break;
    case OP_ADJ_B: launch_colinv_t<T, OP_ADJ_B, 0>(P, n, s); break;
    case OP_ADJ_RHS: QG_CL_SWITCH_STATIC(launch_colinv_t, T, OP_ADJ_RHS, cl, P, n, s); break;
    default: break;
  }
}
template <typename T> void row_dispatch(int op, int cl, const Phase& P, int n, hipStream_t s) {
  switch (op) {
    case OP_RHS: QG_CL_SWITCH(launch_row_t, T, OP_RHS, cl, P, n, s); break;
    case OP_DIAG: QG_CL_SWITCH(launch_row_t, T, OP_DIAG, cl, P, n, s); break;
    case OP_B: launch_row_t<T, OP_B, 0>(P, n, s); break;
    case OP_ENTRY: case OP_ADJ_EXIT: launch_row_t<T, OP_ENTRY, 0>(P, n, s); break;
    case OP_EXIT: case OP_ADJ_ENTRY: launch_row_t<T, OP_EXIT, 0>(P, n, s); break;
    case OP_MASKFWD: launch_row_t<T, OP_MASKFWD, 0>(P, n, s); break;
    case OP_PEN: launch_row_t<T, OP_PEN, 0>(P, n, s); break;
    case OP_SPONGE: launch_row_t<T, OP_SPONGE, 0>(P, n, s); break;
    case OP_GTERMS: launch_row_t<T, OP_GTERMS, 0>(P, n, s); break;
    case OP_CLIPF: launch_row_t<T, OP_CLIPF, 0>(P, n, s); break;
    case OP_MASKGRAD: launch_row_t<T, OP_MASKGRAD, 0>(P, n, s); break;
    case OP_ADJ_B: launch_row_t<T, OP_ADJ_B, 0>(P, n, s); break;
    case OP_ADJ_RHS: QG_CL_SWITCH_STATIC(launch_row_t, T, OP_ADJ_RHS, cl, P, n, s); break;
    default: break;
  }
}
template <typename T> void colfwd_dispatch(int op, int cl, const Phase& P, int n, hipStream_t s) {
  switch (op) {
    case OP_RHS: QG_CL_SWITCH(launch_colfwd_t, T, OP_RHS, cl, P, n, s); break;
    case OP_B: launch_colfwd_t<T, OP_B, 0>(P, n, s); break;
    case OP_ENTRY: case OP_ADJ_EXIT: launch_colfwd_t<T, OP_ENTRY, 0>(P, n, s); break;
    case OP_MASKFWD: launch_colfwd_t<T, OP_MASKFWD, 0>(P, n, s); break;
    case OP_PEN: launch_colfwd_t<T, OP_PEN, 0>(P, n, s); break;
    case OP_GTERMS: launch_colfwd_t<T, OP_GTERMS, 0>(P, n, s); break;
    case OP_ADJ_B: launch_colfwd_t<T, OP_ADJ_B, 0>(P, n, s); break;
    case OP_ADJ_RHS: QG_CL_SWITCH_STATIC(launch_colfwd_t, T, OP_ADJ_RHS, cl, P, n, s); break;
    default: break;
  }
}

// slices 0-3 instantiate the column and row launchers per precision; slice
// 4 uses them
#if QG_HAS(0)
template void colinv_dispatch<float>(int, int, const Phase&, int, hipStream_t);
template void colfwd_dispatch<float>(int, int, const Phase&, int, hipStream_t);
#endif
#if QG_HAS(1)
template void row_dispatch<float>(int, int, const Phase&, int, hipStream_t);
#endif
#if QG_HAS(2)
template void colinv_dispatch<double>(int, int, const Phase&, int, hipStream_t);
template void colfwd_dispatch<double>(int, int, const Phase&, int, hipStream_t);
#endif
#if QG_HAS(3)
template void row_dispatch<double>(int, int, const Phase&, int, hipStream_t);
#endif
#if QG_PART == 4
extern template void colinv_dispatch<float>(int, int, const Phase&, int, hipStream_t);
extern template void colfwd_dispatch<float>(int, int, const Phase&, int, hipStream_t);
extern template void row_dispatch<float>(int, int, const Phase&, int, hipStream_t);
extern template void colinv_dispatch<double>(int, int, const Phase&, int, hipStream_t);
extern template void colfwd_dispatch<double>(int, int, const Phase&, int, hipStream_t);
extern template void row_dispatch<double>(int, int, const Phase&, int, hipStream_t);
#endif

#if QG_HAS(4)
hipError_t launch_colinv(bool dbl, int op, int cl, const Phase& P, int n, hipStream_t s) {
  if (dbl) colinv_dispatch<double>(op, cl, P, n, s); else colinv_dispatch<float>(op, cl, P, n, s);
  return hipGetLastError();
}
bool gterms_ok(bool dbl, const Phase& P) {
  return P.W == 1 && rowp_ok(dbl, OP_GTERMS, 0, P) && colfwdp_ok(dbl, OP_GTERMS, 0, P);
}
bool row_two_levels_ok(bool dbl, int op, int cl, const Phase& P) { return rowp_ok(dbl, op, cl, P); }

int row_launch_blocks(bool dbl, int op, int cl, const Phase& P) {
  const bool par = (op == OP_RHS || op == OP_B || op == OP_ADJ_RHS) && rowp_ok(dbl, op, cl, P);
  return par ? P.ny / 2 : P.ny / (2 * P.RP);
}

hipError_t launch_row(bool dbl, int op, int cl, const Phase& P, int n, hipStream_t s) {
  if (dbl) row_dispatch<double>(op, cl, P, n, s); else row_dispatch<float>(op, cl, P, n, s);
  return hipGetLastError();
}
hipError_t launch_colfwd(bool dbl, int op, int cl, const Phase& P, int n, hipStream_t s) {
  if (dbl) colfwd_dispatch<double>(op, cl, P, n, s); else colfwd_dispatch<float>(op, cl, P, n, s);
  return hipGetLastError();
}
hipError_t launch_combine(bool dbl, int, const Phase& P, int n, hipStream_t s) {
  dim3 grid((P.kxn * P.kyn + COMBINE_THREADS - 1) / COMBINE_THREADS, 1, n);
  if (dbl) QG_KLAUNCH(k_combine<double>, grid, dim3(COMBINE_THREADS), 0, s, P);
  else QG_KLAUNCH(k_combine<float>, grid, dim3(COMBINE_THREADS), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_dyn_coef(const Phase& P, int n, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_dyn_coef, dim3(1, 1, n), dim3(64), 0, s, P, slot);
  return hipGetLastError();
}
hipError_t launch_diag_spectral(bool dbl, const Phase& P, int n, hipStream_t s) {
  dim3 grid((P.kxn * P.kyn + 255) / 256, 1, n);
  if (dbl) hipLaunchKernelGGL(k_diag_spectral<double>, grid, dim3(256), 0, s, P);
  else hipLaunchKernelGGL(k_diag_spectral<float>, grid, dim3(256), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_diag_final(const Phase& P, int n, int nrow, int nspec, double* out, int m0, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_final, dim3(n), dim3(64), 0, s, P, nrow, nspec, out, m0);
  return hipGetLastError();
}
hipError_t launch_adj_grad_c(const Phase& P, int n, int nrow, double* grad_c, int m0, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_grad_c, dim3(n), dim3(64), 0, s, P, nrow, grad_c, m0);
  return hipGetLastError();
}
hipError_t launch_spec_axpy(bool dbl, const Phase& P, int n, long long o_dst, long long o_src, double a,
                            int zero_first, hipStream_t s) {
  dim3 grid((P.kxn * P.kyn + 255) / 256, 1, n);
  if (dbl) hipLaunchKernelGGL(k_spec_axpy<double>, grid, dim3(256), 0, s, P, o_dst, o_src, a, zero_first);
  else hipLaunchKernelGGL(k_spec_axpy<float>, grid, dim3(256), 0, s, P, o_dst, o_src, a, zero_first);
  return hipGetLastError();
}
hipError_t launch_spec_copy(bool dbl, const Phase& P, int n, long long o_dst, long long o_src, hipStream_t s) {
  return launch_spec_axpy(dbl, P, n, o_dst, o_src, 0.0, 1, s);
}
hipError_t launch_filter_les(bool dbl, const FilterArgs& A, hipStream_t s) {
  dim3 grid((A.kxn_c * A.kyn_c + 255) / 256);
  if (dbl) hipLaunchKernelGGL(k_filter_les<double>, grid, dim3(256), 0, s, A);
  else hipLaunchKernelGGL(k_filter_les<float>, grid, dim3(256), 0, s, A);
  return hipGetLastError();
}
hipError_t launch_pcc(bool dbl, const Phase& P, int n, int nblk, const void* a, const void* b, double* out,
                      hipStream_t s) {
  const dim3 grid(nblk, 1, n);
  if (dbl) {
    hipLaunchKernelGGL(k_pcc_sums<double>, grid, dim3(PCC_THREADS), 0, s, P, a, b);
    hipLaunchKernelGGL(k_pcc_centred<double>, grid, dim3(PCC_THREADS), 0, s, P, a, b);
  } else {
    hipLaunchKernelGGL(k_pcc_sums<float>, grid, dim3(PCC_THREADS), 0, s, P, a, b);
    hipLaunchKernelGGL(k_pcc_centred<float>, grid, dim3(PCC_THREADS), 0, s, P, a, b);
  }
  hipLaunchKernelGGL(k_pcc_final, dim3(n), dim3(64), 0, s, P, nblk, out);
  return hipGetLastError();
}
hipError_t launch_adj_dyn_prep(bool dbl, const Phase& P, int n, hipStream_t s) {
  dim3 grid((P.kxn * P.kyn + COMBINE_THREADS - 1) / COMBINE_THREADS, 1, n);
  if (dbl) {
    hipLaunchKernelGGL(k_adj_dot<double>, grid, dim3(COMBINE_THREADS), 0, s, P);
    hipLaunchKernelGGL(k_adj_dyn_prep<double>, grid, dim3(COMBINE_THREADS), 0, s, P);
  } else {
    hipLaunchKernelGGL(k_adj_dot<float>, grid, dim3(COMBINE_THREADS), 0, s, P);
    hipLaunchKernelGGL(k_adj_dyn_prep<float>, grid, dim3(COMBINE_THREADS), 0, s, P);
  }
  return hipGetLastError();
}
hipError_t launch_ab2cn_finish(bool dbl, const Phase& P, int n, hipStream_t s) {
  dim3 grid((P.kxn * P.kyn + 255) / 256, 1, n);
  if (dbl) hipLaunchKernelGGL(k_ab2cn_finish<double>, grid, dim3(256), 0, s, P);
  else hipLaunchKernelGGL(k_ab2cn_finish<float>, grid, dim3(256), 0, s, P);
  return hipGetLastError();
}
hipError_t launch_put_member(MemberDev* dst, const MemberDev& m, hipStream_t s) {
  hipLaunchKernelGGL(k_put_member, dim3(1), dim3(64), 0, s, dst, m);
  return hipGetLastError();
}
hipError_t launch_twiddle_table(bool dbl, void* dst, int logn, int sch, hipStream_t s) {
  const int n = 1 << logn;
  const dim3 grid((n + 255) / 256);
  if (dbl) hipLaunchKernelGGL(k_twiddle_table<double>, grid, dim3(256), 0, s, (cpx<double>*)dst, logn, sch);
  else hipLaunchKernelGGL(k_twiddle_table<float>, grid, dim3(256), 0, s, (cpx<float>*)dst, logn, sch);
  return hipGetLastError();
}
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  unsigned int blocks = (unsigned int)((n + 255) / 256 > 4096 ? 4096 : (n + 255) / 256);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (unsigned int*)p, n);
  return hipGetLastError();
}
#endif  // QG_HAS(4)

}  // namespace qg
