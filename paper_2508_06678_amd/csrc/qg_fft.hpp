// Batched complex FFTs staged in LDS for gfx950.
//
// The pseudo-spectral method evaluates derivatives in Fourier space and
// products in physical space (Sec. II-C), so every right-hand-side
// evaluation is a sequence of 2-D transforms.  They are split into a column
// pass (complex, along y, over the retained kx modes only) and a row pass
// (real <-> half spectrum along x, two rows packed as one complex row).
// Both passes use the routine below: a self-sorting Stockham transform of
// power-of-two length N, mixed radix 8 / 4 / 2, in place in LDS, for a
// batch of nb independent vectors whose element n of vector b sits at
// buf[n * es + b * bs].
//
// Forward transforms use exp(-2 pi i m n / N) and are unnormalised; inverse
// transforms use the conjugate twiddles and are also unnormalised (callers
// fold 1/(nx ny) into the spectral data).
//
// The passes follow a schedule of radices (pass_log_radix below).  Twiddles
// come from a per-pass table (computed on the host in extended precision
// and rounded once), one per schedule: the pass with sub-transform length
// Ns >= 8 and radix R keeps exp(-2 pi i t k / (Ns R)) at
//     (Ns - 8) + k (R - 1) + (t - 1),   0 <= k < Ns,  1 <= t < R,
// so a butterfly reads its R - 1 twiddles from consecutive slots; the pass
// fills slots [Ns - 8, Ns R - 8), so the table of a length-N transform has
// N - 8 entries whatever the schedule (the first pass, Ns = 1, needs none).
#pragma once
#include <hip/hip_runtime.h>

namespace qg {

template <typename T> struct cpx_of;
template <> struct cpx_of<float> { using type = float2; };
template <> struct cpx_of<double> { using type = double2; };
template <typename T> using cpx = typename cpx_of<T>::type;

template <typename V> __device__ __forceinline__ V cmake(decltype(V{}.x) a, decltype(V{}.x) b) {
  V r; r.x = a; r.y = b; return r;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return cmake<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return cmake<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return cmake<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return cmake<V>(a.x, -a.y); }
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V{}.x) s) { return cmake<V>(a.x * s, a.y * s); }
// multiplication by +i and by -i
template <typename V> __device__ __forceinline__ V cmul_i(V a) { return cmake<V>(-a.y, a.x); }
template <typename V> __device__ __forceinline__ V cmul_mi(V a) { return cmake<V>(a.y, -a.x); }

// LDS poison (debug builds with QG_LDS_POISON): before a transform pass
// writes its outputs, the threads of the transform set every element of its
// LDS buffer to NaN (all bits set, a NaN in both precisions), so that a
// position the pass fails to write, or a read that runs ahead of the write
// it depends on, carries NaN into the result.  n: elements of the buffer,
// tid / nthreads: the thread's index in the transform and their number.
// Ordinary builds compile this to nothing.
template <typename V>
__device__ __forceinline__ void lds_poison(V* buf, int n, int tid, int nthreads, bool active) {
#ifdef QG_LDS_POISON
  if (active) {
    using S = decltype(V{}.x);
    S nan;
    __builtin_memset(&nan, 0xff, sizeof(S));
    for (int i = tid; i < n; i += nthreads) buf[i] = cmake<V>(nan, nan);
  }
#else
  (void)buf; (void)n; (void)tid; (void)nthreads; (void)active;
#endif
}
#ifdef QG_LDS_POISON
constexpr bool kLdsPoison = true;
#else
constexpr bool kLdsPoison = false;
#endif

// Pass schedules.  A transform of length 2^logn is a sequence of Stockham
// passes; the pass with sub-transform length 2^logns has radix
// 2^pass_log_radix(logn, logns, sch).  The first pass (logns = 0) is radix
// 8 in every schedule (its inputs come from registers).  Schedule 0: radix 8
// while three factors of two remain, then one radix-4 or radix-2 pass
// (1024 = 8 8 8 2); schedule 1: radix 4 while more than three factors
// remain, then the rest in one pass (1024 = 8 4 4 8, 512 = 8 4 4 4, 256 =
// 8 4 8); schedule 2: radix 16 while four factors of two remain, then the
// rest (1024 = 8 16 8): one LDS exchange fewer, for transforms with 16
// elements per thread (the wave-synchronous 1024-point rows).  The
// run-time engines use schedule 0; the compile-time ones take one of them
// (a tuning choice), each with its own twiddle table.
__host__ __device__ constexpr int pass_log_radix(int logn, int logns, int sch) {
  return logns == 0 ? 3
       : sch == 0 ? (logn - logns >= 3 ? 3 : logn - logns)
       : sch == 1 ? (logn - logns > 3 ? 2 : logn - logns)
                  : (logn - logns >= 4 ? 4 : logn - logns);
}
constexpr int NSCHED = 3;

// Radix-2/4/8 DFT kernels in registers.  INV selects exp(+2 pi i / R).
template <typename V, bool INV> __device__ __forceinline__ void dft2(V* v) {
  V a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename V, bool INV> __device__ __forceinline__ void dft4(V& v0, V& v1, V& v2, V& v3) {
  V a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = csub(v1, v3);
  a3 = INV ? cmul_i(a3) : cmul_mi(a3);
  v0 = cadd(a0, a2);
  v2 = csub(a0, a2);
  v1 = cadd(a1, a3);
  v3 = csub(a1, a3);
}

template <typename V, bool INV> __device__ __forceinline__ void dft4(V* v) { dft4<V, INV>(v[0], v[1], v[2], v[3]); }

// Length-8 DFT as one radix-2 split (decimation in frequency) into two
// length-4 DFTs: a_t = v_t + v_{t+4} gives the even outputs, (v_t - v_{t+4})
// times w8^t gives the odd outputs, w8 = exp(-+ 2 pi i / 8).
template <typename V, bool INV> __device__ __forceinline__ void dft8(V* v) {
  using T = decltype(V{}.x);
  const T h = T(0.70710678118654752440084436210485);
  V a0 = cadd(v[0], v[4]), a1 = cadd(v[1], v[5]), a2 = cadd(v[2], v[6]), a3 = cadd(v[3], v[7]);
  V b0 = csub(v[0], v[4]), b1 = csub(v[1], v[5]), b2 = csub(v[2], v[6]), b3 = csub(v[3], v[7]);
  if (!INV) {
    b1 = cmake<V>((b1.x + b1.y) * h, (b1.y - b1.x) * h);     // * (1 - i)/sqrt2
    b2 = cmul_mi(b2);                                        // * -i
    b3 = cmake<V>((b3.y - b3.x) * h, -(b3.x + b3.y) * h);    // * (-1 - i)/sqrt2
  } else {
    b1 = cmake<V>((b1.x - b1.y) * h, (b1.y + b1.x) * h);     // * (1 + i)/sqrt2
    b2 = cmul_i(b2);                                         // * i
    b3 = cmake<V>(-(b3.x + b3.y) * h, (b3.x - b3.y) * h);    // * (-1 + i)/sqrt2
  }
  dft4<V, INV>(a0, a1, a2, a3);
  dft4<V, INV>(b0, b1, b2, b3);
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

// Length-8 DFT whose inputs v_t with bit t of ZM set are known to be zero
// (band-limited data: the 2/3 rule and the test filter leave whole blocks of
// a transform's input empty).  The first layer of the split drops the
// additions with a zero operand; the rest is dft8.
template <typename V, bool INV, int ZM> __device__ __forceinline__ void dft8z(V* v) {
  using T = decltype(V{}.x);
  if constexpr (ZM == 0) {
    dft8<V, INV>(v);
  } else {
    const T h = T(0.70710678118654752440084436210485);
    V a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool z0 = (ZM >> t) & 1, z1 = (ZM >> (t + 4)) & 1;
      if (z0 && z1) { a[t] = cmake<V>(T(0), T(0)); b[t] = a[t]; }
      else if (z1) { a[t] = v[t]; b[t] = v[t]; }
      else if (z0) { a[t] = v[t + 4]; b[t] = cmake<V>(-v[t + 4].x, -v[t + 4].y); }
      else { a[t] = cadd(v[t], v[t + 4]); b[t] = csub(v[t], v[t + 4]); }
    }
    if (!INV) {
      b[1] = cmake<V>((b[1].x + b[1].y) * h, (b[1].y - b[1].x) * h);
      b[2] = cmul_mi(b[2]);
      b[3] = cmake<V>((b[3].y - b[3].x) * h, -(b[3].x + b[3].y) * h);
    } else {
      b[1] = cmake<V>((b[1].x - b[1].y) * h, (b[1].y + b[1].x) * h);
      b[2] = cmul_i(b[2]);
      b[3] = cmake<V>(-(b[3].x + b[3].y) * h, (b[3].x - b[3].y) * h);
    }
    dft4<V, INV>(a[0], a[1], a[2], a[3]);
    dft4<V, INV>(b[0], b[1], b[2], b[3]);
    v[0] = a[0]; v[2] = a[1]; v[4] = a[2]; v[6] = a[3];
    v[1] = b[0]; v[3] = b[1]; v[5] = b[2]; v[7] = b[3];
  }
}

// Length-16 DFT as 4 x 4 (Cooley-Tukey): length-4 DFTs over the stride-4
// subsequences x[4 n1 + n2], the twiddles w16^(n2 k1), then length-4 DFTs
// across n2; X[k1 + 4 k2] lands in v[k1 + 4 k2].  w16 = exp(-2 pi i / 16)
// (its conjugate for INV); with c = cos pi/8, s = sin pi/8:
// w16^1 = c - i s, w16^2 = (1 - i)/sqrt2, w16^3 = s - i c, w16^4 = -i,
// w16^6 = -(1 + i)/sqrt2, w16^9 = -c + i s.
template <typename V, bool INV> __device__ __forceinline__ void dft16(V* v) {
  using T = decltype(V{}.x);
  const T c = T(0.92387953251128675613), sn = T(0.38268343236508977173), h = T(0.70710678118654752440);
  V a[4][4];   // a[n2][k1]
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    a[n2][0] = v[n2];
    a[n2][1] = v[4 + n2];
    a[n2][2] = v[8 + n2];
    a[n2][3] = v[12 + n2];
    dft4<V, INV>(a[n2][0], a[n2][1], a[n2][2], a[n2][3]);
  }
  // multiplication by w = re + i im (forward) or its conjugate (inverse)
  auto mulw = [](V z, T re, T im) {
    const T i2 = INV ? -im : im;
    return cmake<V>(z.x * re - z.y * i2, z.x * i2 + z.y * re);
  };
  a[1][1] = mulw(a[1][1], c, -sn);     // w^1
  a[1][2] = mulw(a[1][2], h, -h);      // w^2
  a[1][3] = mulw(a[1][3], sn, -c);     // w^3
  a[2][1] = mulw(a[2][1], h, -h);      // w^2
  a[2][2] = INV ? cmul_i(a[2][2]) : cmul_mi(a[2][2]);   // w^4 = -i
  a[2][3] = mulw(a[2][3], -h, -h);     // w^6
  a[3][1] = mulw(a[3][1], sn, -c);     // w^3
  a[3][2] = mulw(a[3][2], -h, -h);     // w^6
  a[3][3] = mulw(a[3][3], -c, sn);     // w^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    dft4<V, INV>(a[0][k1], a[1][k1], a[2][k1], a[3][k1]);
    v[k1] = a[0][k1];
    v[k1 + 4] = a[1][k1];
    v[k1 + 8] = a[2][k1];
    v[k1 + 12] = a[3][k1];
  }
}

template <typename V, int R, bool INV> __device__ __forceinline__ void dftR(V* v) {
  if constexpr (R == 16) dft16<V, INV>(v);
  else if constexpr (R == 8) dft8<V, INV>(v);
  else if constexpr (R == 4) dft4<V, INV>(v);
  else dft2<V, INV>(v);
}

// Geometry of one batched transform inside a workgroup.
struct FftShape {
  int logN;       // transform length 2^logN
  int es, bs;     // element stride and batch stride in LDS (in elements)
  int lognb;      // 2^lognb vectors
  bool batch_fast;  // consecutive threads walk the batch index first
};

// Thread group that runs one batched transform: threads [0, nt) of the
// group (tid = rank in the group).  Inactive groups still reach every
// barrier, so several groups of a block can transform different vectors
// concurrently in lock-step.
struct FftGroup {
  int tid, nt;
  bool active;
};

// One Stockham pass of radix R with sub-transform length Ns = 2^logNs:
// butterfly j reads elements j + t N/R, multiplies element t by
// w_{Ns R}^{t (j mod Ns)}, transforms, and writes them to
// (j / Ns) Ns R + (j mod Ns) + t Ns.  In place: all reads, barrier, writes.
template <typename V, int R, bool INV, int MAXB>
__device__ __forceinline__ void stockham_pass(V* __restrict__ buf, const V* __restrict__ tw,
                                              const FftShape& s, int logNs, const FftGroup& g) {
  constexpr int logR = (R == 8) ? 3 : (R == 4) ? 2 : 1;
  const int logNR = s.logN - logR;
  const int total = g.active ? 1 << (s.lognb + logNR) : 0;
  V v[MAXB][R];
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int q = g.tid + i * g.nt;
    if (q < total) {
      int b, j;
      if (s.batch_fast) { b = q & ((1 << s.lognb) - 1); j = q >> s.lognb; }
      else { j = q & ((1 << logNR) - 1); b = q >> logNR; }
      const int k = j & ((1 << logNs) - 1);
      const V* src = buf + b * s.bs;
#pragma unroll
      for (int t = 0; t < R; ++t) v[i][t] = src[(j + (t << logNR)) * s.es];
      if (logNs > 0) {
        const V* w = tw + ((1 << logNs) - 8) + k * (R - 1);
#pragma unroll
        for (int t = 1; t < R; ++t) v[i][t] = cmul(v[i][t], INV ? cconj(w[t - 1]) : w[t - 1]);
      }
      dftR<V, R, INV>(v[i]);
    }
  }
  __syncthreads();
  if constexpr (kLdsPoison) {
    // the group's vectors span (nb - 1) bs + (N - 1) es + 1 elements
    lds_poison(buf, (((1 << s.lognb) - 1) * s.bs + ((1 << s.logN) - 1) * s.es) + 1, g.tid, g.nt, g.active);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MAXB; ++i) {
    const int q = g.tid + i * g.nt;
    if (q < total) {
      int b, j;
      if (s.batch_fast) { b = q & ((1 << s.lognb) - 1); j = q >> s.lognb; }
      else { j = q & ((1 << logNR) - 1); b = q >> logNR; }
      const int k = j & ((1 << logNs) - 1);
      const int base = ((j >> logNs) << (logNs + logR)) + k;
      V* dst = buf + b * s.bs;
#pragma unroll
      for (int t = 0; t < R; ++t) dst[(base + (t << logNs)) * s.es] = v[i][t];
    }
  }
  __syncthreads();
}

// Copy the per-pass twiddle table of length-N transforms from global memory
// to LDS (callers synchronise before the first pass).
template <typename V>
__device__ __forceinline__ void stage_twiddles(V* __restrict__ dst, const V* __restrict__ src, int logN) {
  const int n = (1 << logN) - 8;
  for (int m = threadIdx.x; m < n; m += blockDim.x) dst[m] = src[m];
}

// Full transform: radix-8 passes, then one radix-4 or radix-2 pass.
// EPT bounds the elements per thread: nb * N <= EPT * g.nt.
template <typename V, bool INV, int EPT>
__device__ __forceinline__ void fft_lds(V* __restrict__ buf, const V* __restrict__ tw, const FftShape& s,
                                        const FftGroup& g) {
  int logNs = 0;
  int rem = s.logN;
  while (rem >= 3) {
    stockham_pass<V, 8, INV, EPT / 8>(buf, tw, s, logNs, g);
    logNs += 3;
    rem -= 3;
  }
  if (rem == 2) stockham_pass<V, 4, INV, EPT / 4>(buf, tw, s, logNs, g);
  else if (rem == 1) stockham_pass<V, 2, INV, EPT / 2>(buf, tw, s, logNs, g);
}

// ---------------------------------------------------------------------------
// Single-vector transform of length N = 2^logN (32 <= N <= 4096) by a group
// of N/8 threads, one vector per group, in a padded LDS buffer: element i
// lives at pad8(i) = i + i/8, which spreads the stride-8 stores of the first
// Stockham pass over all banks.  The first pass takes its 8 inputs
// x[j + t N/8] (j = rank in the group) from registers, so callers that can
// form the input directly (c2r from the mixed layout, products formed
// pointwise) skip one LDS round trip.  Output: natural order, padded.
__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }

template <typename V, bool INV>
__device__ __forceinline__ void fft1_pass0(V (&v)[8], V* __restrict__ buf, int j, bool active, int logN) {
  if (active) dftR<V, 8, INV>(v);
  __syncthreads();
  if constexpr (kLdsPoison) {
    lds_poison(buf, 9 << (logN - 3), j, 1 << (logN - 3), active);
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int t = 0; t < 8; ++t) buf[9 * j + t] = v[t];
  }
  __syncthreads();
}

template <typename V, int R, bool INV>
__device__ __forceinline__ void fft1_pass(V* __restrict__ buf, const V* __restrict__ tw, int logN, int logNs, int j0,
                                          int nt, bool active) {
  constexpr int logR = (R == 8) ? 3 : (R == 4) ? 2 : 1;
  constexpr int NB = 8 / R;   // butterflies per thread
  const int logNR = logN - logR;
  V v[NB][R];
  if (active) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = j0 + b * nt;
      const int k = j & ((1 << logNs) - 1);
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = buf[pad8(j + (t << logNR))];
      const V* w = tw + ((1 << logNs) - 8) + k * (R - 1);
#pragma unroll
      for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], INV ? cconj(w[t - 1]) : w[t - 1]);
      dftR<V, R, INV>(v[b]);
    }
  }
  __syncthreads();
  if constexpr (kLdsPoison) {
    lds_poison(buf, pad8(1 << logN), j0, nt, active);
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = j0 + b * nt;
      const int k = j & ((1 << logNs) - 1);
      const int base = ((j >> logNs) << (logNs + logR)) + k;
#pragma unroll
      for (int t = 0; t < R; ++t) buf[pad8(base + (t << logNs))] = v[b][t];
    }
  }
  __syncthreads();
}

// Passes after the first (the first is fft1_pass0, radix 8).
template <typename V, bool INV>
__device__ __forceinline__ void fft1_rest(V* __restrict__ buf, const V* __restrict__ tw, int logN, int j, bool active) {
  const int nt = 1 << (logN - 3);
  int logNs = 3;
  int rem = logN - 3;
  while (rem >= 3) {
    fft1_pass<V, 8, INV>(buf, tw, logN, logNs, j, nt, active);
    logNs += 3;
    rem -= 3;
  }
  if (rem == 2) fft1_pass<V, 4, INV>(buf, tw, logN, logNs, j, nt, active);
  else if (rem == 1) fft1_pass<V, 2, INV>(buf, tw, logN, logNs, j, nt, active);
}

// ---------------------------------------------------------------------------
// The same single-vector transform with the length fixed at compile time
// (N = 2^LOGN >= 8 * 2^P) and a pad slot every 2^P elements
// (padp<P>(i) = i + i / 2^P): every pass is unrolled and every LDS address
// is one per-thread base plus constant offsets.  padp<P> is additive over
// multiples of 2^P, so the reads of all passes share the base padp(j); a
// write of a pass goes to padp(base + t Ns) = padp(base) + t Ns + (t Ns)/2^P
// (base = its butterfly's first output, whose offset below Ns is < 2^P when
// Ns < 2^P).
template <int P> __device__ __forceinline__ int padp(int i) { return i + (i >> P); }

// Synchronisation between the passes of a transform.  Block-wide by
// default; WAVE: every thread that exchanges data with this one belongs to
// its wave (a transform of at most 64 threads, aligned to the wave), whose
// LDS operations are performed in order, so waiting for the wave's own LDS
// traffic (and keeping the compiler from moving accesses across) suffices.
template <bool WAVE> __device__ __forceinline__ void fft_sync() {
  if constexpr (WAVE) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  } else {
    __syncthreads();
  }
}

// First pass (radix 8) from registers.  A thread holds EPT = 8 NB0
// elements: butterflies q = j + b N/EPT (b < NB0), butterfly q taking
// x[q + t N/8] from v[b + NB0 t] and writing x'[8 q + t].
// ZM: inputs known to be zero (bit t: x[q + t N/8]), see dft8z.
template <typename V, bool INV, int P, int ZM = 0, int EPT = 8, bool WAVE = false, int LOGN = 0>
__device__ __forceinline__ void fft1c_pass0(V (&v)[EPT], V* __restrict__ buf, int j, bool active) {
  static_assert(P >= 3, "pad period of at least 8");
  constexpr int NB0 = EPT / 8;
  static_assert(NB0 == 1 || LOGN > 0, "several butterflies per thread need the length");
  constexpr int nt = NB0 == 1 ? 0 : (1 << LOGN) / EPT;   // threads per transform
  V u[NB0][8];
#pragma unroll
  for (int b = 0; b < NB0; ++b) {
#pragma unroll
    for (int t = 0; t < 8; ++t) u[b][t] = v[b + NB0 * t];
    if (active) dft8z<V, INV, ZM>(u[b]);
  }
  fft_sync<WAVE>();
  if constexpr (kLdsPoison) {
    static_assert(LOGN > 0, "the poisoned extent needs the length");
    lds_poison(buf, padp<P>(1 << LOGN), j, (1 << LOGN) / EPT, active);
    fft_sync<WAVE>();
  }
  if (active) {
    V* wb = buf + 8 * j + (j >> (P - 3));
#pragma unroll
    for (int b = 0; b < NB0; ++b) {
#pragma unroll
      for (int t = 0; t < 8; ++t) wb[b * (8 * nt + ((8 * nt) >> P)) + t] = u[b][t];
    }
  }
  fft_sync<WAVE>();
}

// One pass of the compile-time engine, radix R = 2^pass_log_radix(LOGN,
// LOGNS, SCH), N/8 threads with 8 elements each (8/R butterflies per
// thread: j + b N/8).  A pass before the last has Ns dividing N/8, so the
// butterflies of a thread share their twiddles and their outputs lie N R/8
// apart; in the last pass (Ns R = N) every butterfly index is below Ns.
template <typename V, int LOGN, int LOGNS, bool INV, int P, int SCH, int EPT = 8, bool WAVE = false>
__device__ __forceinline__ void fft1c_pass(V* __restrict__ buf, const V* __restrict__ tw, int j, bool active) {
  constexpr int N = 1 << LOGN;
  constexpr int NS = 1 << LOGNS;
  constexpr int logR = pass_log_radix(LOGN, LOGNS, SCH);
  constexpr int R = 1 << logR;
  constexpr bool LAST = LOGNS + logR == LOGN;
  constexpr int NB = EPT / R;        // butterflies per thread
  constexpr int nt = N / EPT;        // threads per transform
  constexpr int NR = N / R;
  static_assert(LOGN >= P + 3 && LOGNS >= 3, "compile-time engine: N >= 8 * 2^P, passes after the first");
  static_assert(LAST || NB == 1 || nt % NS == 0, "a pass before the last has Ns dividing N/8");
  V v[NB][R];
  if (active) {
    const V* rb = buf + padp<P>(j);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = rb[b * (nt + (nt >> P)) + t * (NR + (NR >> P))];
      const int k = (NB > 1 && LAST) ? j + b * nt : (j & (NS - 1));
      const V* w = tw + (NS - 8) + k * (R - 1);
#pragma unroll
      for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], INV ? cconj(w[t - 1]) : w[t - 1]);
      dftR<V, R, INV>(v[b]);
    }
  }
  fft_sync<WAVE>();
  if constexpr (kLdsPoison) {
    lds_poison(buf, padp<P>(N), j, nt, active);
    fft_sync<WAVE>();
  }
  if (active) {
    if constexpr (NB > 1 && LAST) {
      V* wb = buf + padp<P>(j);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int t = 0; t < R; ++t) wb[b * (nt + (nt >> P)) + t * NS + ((t * NS) >> P)] = v[b][t];
      }
    } else {
      constexpr int BO = nt * R;   // output offset of the thread's next butterfly
      const int k = j & (NS - 1);
      V* wb = buf + padp<P>(((j >> LOGNS) << (LOGNS + logR)) + k);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int t = 0; t < R; ++t) wb[b * (BO + (BO >> P)) + t * NS + ((t * NS) >> P)] = v[b][t];
      }
    }
  }
  fft_sync<WAVE>();
  if constexpr (!LAST) fft1c_pass<V, LOGN, LOGNS + logR, INV, P, SCH, EPT, WAVE>(buf, tw, j, active);
}

// The twiddles of a thread's butterflies in the pass with sub-length
// 2^LOGNS (one set when they share them, NB sets in a last pass).
template <typename V, int LOGN, int LOGNS, int SCH, int EPT>
struct PassTw {
  static constexpr int logR = pass_log_radix(LOGN, LOGNS, SCH), R = 1 << logR, NS = 1 << LOGNS;
  static constexpr bool LAST = LOGNS + logR == LOGN;
  static constexpr int NB = EPT / R, nt = (1 << LOGN) / EPT;
  static constexpr int NK = (NB > 1 && LAST) ? NB : 1;
  V w[NK][R - 1];
  __device__ __forceinline__ void load(const V* __restrict__ tw, int j) {
#pragma unroll
    for (int b = 0; b < NK; ++b) {
      const int k = NK > 1 ? j + b * nt : (j & (NS - 1));
#pragma unroll
      for (int t = 0; t < R - 1; ++t) w[b][t] = tw[(NS - 8) + k * (R - 1) + t];
    }
  }
};

// fft1c_pass with the pass's twiddles given (cur) and the next pass's
// loaded while this one computes: their latency (an L2 round trip) is
// no longer exposed after every barrier.  TRUNC: the caller reads only the
// outputs of the 2/3 set, k < (N - 1)/3 + 1 and their mirrors N - k; the
// last pass then neither writes (nor forms) its output blocks that lie
// wholly between (at the 1024-point length and a last radix of 8, the
// blocks k in [384, 640)).
template <typename V, int LOGN, int LOGNS, bool INV, int P, int SCH, int EPT, bool WAVE, bool TRUNC = false>
__device__ __forceinline__ void fft1c_pass_pf(V* __restrict__ buf, const V* __restrict__ tw, int j, bool active,
                                              const PassTw<V, LOGN, LOGNS, SCH, EPT>& cur) {
  using TW = PassTw<V, LOGN, LOGNS, SCH, EPT>;
  constexpr int N = 1 << LOGN;
  constexpr int NS = TW::NS, logR = TW::logR, R = TW::R, NB = TW::NB, nt = TW::nt;
  constexpr bool LAST = TW::LAST;
  constexpr int NR = N / R;
  constexpr int NEXT = LAST ? LOGNS : LOGNS + logR;
  V v[NB][R];
  PassTw<V, LOGN, NEXT, SCH, EPT> nxt;
  if (active) {
    const V* rb = buf + padp<P>(j);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = rb[b * (nt + (nt >> P)) + t * (NR + (NR >> P))];
    }
    if constexpr (!LAST) nxt.load(tw, j);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const V* w = cur.w[TW::NK > 1 ? b : 0];
#pragma unroll
      for (int t = 1; t < R; ++t) v[b][t] = cmul(v[b][t], INV ? cconj(w[t - 1]) : w[t - 1]);
      dftR<V, R, INV>(v[b]);
    }
  }
  fft_sync<WAVE>();
  if constexpr (kLdsPoison) {
    lds_poison(buf, padp<P>(N), j, nt, active);
    fft_sync<WAVE>();
  }
  // the last pass's output block t holds k in [t NS, (t + 1) NS)
  constexpr int KX = (N - 1) / 3 + 1;
  auto skip = [&](int t) constexpr { return TRUNC && LAST && t * NS >= KX && (t + 1) * NS - 1 <= N - KX; };
  if (active) {
    if constexpr (NB > 1 && LAST) {
      V* wb = buf + padp<P>(j);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int t = 0; t < R; ++t)
          if (!skip(t)) wb[b * (nt + (nt >> P)) + t * NS + ((t * NS) >> P)] = v[b][t];
      }
    } else {
      constexpr int BO = nt * R;
      const int k = j & (NS - 1);
      V* wb = buf + padp<P>(((j >> LOGNS) << (LOGNS + logR)) + k);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int t = 0; t < R; ++t)
          if (!skip(t)) wb[b * (BO + (BO >> P)) + t * NS + ((t * NS) >> P)] = v[b][t];
      }
    }
  }
  fft_sync<WAVE>();
  if constexpr (!LAST) fft1c_pass_pf<V, LOGN, NEXT, INV, P, SCH, EPT, WAVE, TRUNC>(buf, tw, j, active, nxt);
}

// The twiddles of the first pass after fft1c_pass0 (sub-length 8), for a
// caller to load before the first pass so that their latency overlaps it.
template <typename V, int LOGN, int SCH = 0, int EPT = 8>
__device__ __forceinline__ PassTw<V, LOGN, 3, SCH, EPT> fft1c_first_tw(const V* __restrict__ tw, int j) {
  PassTw<V, LOGN, 3, SCH, EPT> t;
  t.load(tw, j);
  return t;
}

// Passes after the first (fft1c_pass0), compile-time length, schedule SCH,
// EPT elements per thread, wave- or block-wide synchronisation; the first
// of them takes the twiddles the caller loaded (fft1c_first_tw), each
// loads the next one's while it computes.
template <typename V, int LOGN, bool INV, int P, int SCH = 0, int EPT = 8, bool WAVE = false, bool TRUNC = false>
__device__ __forceinline__ void fft1c_rest(V* __restrict__ buf, const V* __restrict__ tw, int j, bool active,
                                           const PassTw<V, LOGN, 3, SCH, EPT>& first) {
  fft1c_pass_pf<V, LOGN, 3, INV, P, SCH, EPT, WAVE, TRUNC>(buf, tw, j, active, first);
}

// The whole block as one group.
template <typename V, bool INV, int EPT>
__device__ __forceinline__ void fft_lds(V* __restrict__ buf, const V* __restrict__ tw, const FftShape& s) {
  fft_lds<V, INV, EPT>(buf, tw, s, FftGroup{(int)threadIdx.x, (int)blockDim.x, true});
}

}  // namespace qg
