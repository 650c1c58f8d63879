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
// fold 1/(nx ny) into the spectral data).  Twiddles come from the table
// tw[m] = exp(-2 pi i m / N), m in [0, N), staged in LDS (computed on the
// host in extended precision and rounded once).
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

template <typename V, int R, bool INV> __device__ __forceinline__ void dftR(V* v) {
  if constexpr (R == 8) dft8<V, INV>(v);
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
  const int twshift = s.logN - logNs - logR;
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
        const int step = k << twshift;
        int idx = step;
#pragma unroll
        for (int t = 1; t < R; ++t, idx += step) {
          V w = tw[idx];
          if (INV) w = cconj(w);
          v[i][t] = cmul(v[i][t], w);
        }
      }
      dftR<V, R, INV>(v[i]);
    }
  }
  __syncthreads();
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

// Copy the twiddle table of length-N transforms from global memory to LDS
// (callers synchronise before the first pass).
template <typename V>
__device__ __forceinline__ void stage_twiddles(V* __restrict__ dst, const V* __restrict__ src, int logN) {
  const int n = 1 << logN;
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
__device__ __forceinline__ void fft1_pass0(V (&v)[8], V* __restrict__ buf, int j, bool active) {
  if (active) dftR<V, 8, INV>(v);
  __syncthreads();
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
  const int twshift = logN - logNs - logR;
  V v[NB][R];
  if (active) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = j0 + b * nt;
      const int k = j & ((1 << logNs) - 1);
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = buf[pad8(j + (t << logNR))];
      const int step = k << twshift;
      int idx = step;
#pragma unroll
      for (int t = 1; t < R; ++t, idx += step) {
        V w = tw[idx];
        if (INV) w = cconj(w);
        v[b][t] = cmul(v[b][t], w);
      }
      dftR<V, R, INV>(v[b]);
    }
  }
  __syncthreads();
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
// Radix-16 single-vector transform for N >= 256: a group of N/16 threads
// (one wave at N = 1024), 16 elements per thread, passes 16, 16, then 16/8/4/2
// for what remains; padded LDS (one slot per 16 elements).  The twiddles of
// every pass after the first depend only on the thread's rank, so they are
// read once per kernel into a Tw16 register set and reused by every
// transform of that length in the kernel.
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Length-16 DFT in registers as 4 x 4: inner length-4 DFTs over n1 of
// x[4 n1 + n2], twiddles w16^(n2 k1), outer length-4 DFTs over n2; output in
// natural order.
template <typename V, bool INV> __device__ __forceinline__ void dft16(V* v) {
  using T = decltype(V{}.x);
  const T c1 = T(0.92387953251128675612818318939678828682);   // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403039886676);   // sin(pi/8)
  const T h = T(0.70710678118654752440084436210484903928);
  V y[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    V a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
    dft4<V, INV>(a0, a1, a2, a3);
    y[n2 * 4 + 0] = a0; y[n2 * 4 + 1] = a1; y[n2 * 4 + 2] = a2; y[n2 * 4 + 3] = a3;
  }
  // twiddles w16^(n2 k1) (forward: exp(-2 pi i m/16); inverse: conjugate)
  const T sg = INV ? T(1) : T(-1);
  auto tw = [&](V a, T c, T s) { return cmake<V>(a.x * c - a.y * sg * s, a.x * sg * s + a.y * c); };
  y[1 * 4 + 1] = tw(y[5], c1, s1);          // m = 1
  y[1 * 4 + 2] = tw(y[6], h, h);            // m = 2
  y[1 * 4 + 3] = tw(y[7], s1, c1);          // m = 3
  y[2 * 4 + 1] = tw(y[9], h, h);            // m = 2
  y[2 * 4 + 2] = INV ? cmul_i(y[10]) : cmul_mi(y[10]);   // m = 4
  y[2 * 4 + 3] = tw(y[11], -h, h);          // m = 6
  y[3 * 4 + 1] = tw(y[13], s1, c1);         // m = 3
  y[3 * 4 + 2] = tw(y[14], -h, h);          // m = 6
  y[3 * 4 + 3] = tw(y[15], -c1, -s1);       // m = 9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    V b0 = y[k1], b1 = y[4 + k1], b2 = y[8 + k1], b3 = y[12 + k1];
    dft4<V, INV>(b0, b1, b2, b3);
    v[k1] = b0; v[k1 + 4] = b1; v[k1 + 8] = b2; v[k1 + 12] = b3;
  }
}

template <typename V, int R, bool INV> __device__ __forceinline__ void dftR16(V* v) {
  if constexpr (R == 16) dft16<V, INV>(v);
  else dftR<V, R, INV>(v);
}

// Compile-time schedule for length 2^LOGN (LOGN >= 8): after the first
// radix-16 pass, radix 16 while >= 4 bits remain, then one pass of 8/4/2.
template <int LOGN> struct Sched16 {
  static constexpr int rem(int p) { return LOGN - 4 - 4 * p; }             // bits left before pass p+1
  static constexpr int logR(int p) { return rem(p) >= 4 ? 4 : rem(p); }
  static constexpr int npass = (LOGN - 4 + 3) / 4;                           // passes after the first
  static constexpr int logNs(int p) { return 4 + 4 * p; }
};

// Twiddle registers of the passes after the first: 15 per pass (radix 16:
// one butterfly of 15 twiddles; radix R < 16: 16/R butterflies of R-1).
template <typename V, int LOGN> struct Tw16 {
  V w[Sched16<LOGN>::npass][15];
};

template <typename V, int LOGN>
__device__ __forceinline__ void tw16_load(Tw16<V, LOGN>& T16, const V* __restrict__ tw, int j) {
  using S = Sched16<LOGN>;
  constexpr int nt = 1 << (LOGN - 4);
#pragma unroll
  for (int p = 0; p < S::npass; ++p) {
    const int logR = S::logR(p);
    const int R = 1 << logR;
    const int nb = 16 / R;
    const int logNs = S::logNs(p);
    const int twshift = LOGN - logNs - logR;
#pragma unroll
    for (int b = 0; b < nb; ++b) {
      const int k = (j + b * nt) & ((1 << logNs) - 1);
#pragma unroll
      for (int t = 1; t < R; ++t) {
        T16.w[p][b * (R - 1) + (t - 1)] = tw[(t * k) << twshift];
      }
    }
  }
}

template <typename V, bool INV>
__device__ __forceinline__ void fft16_pass0(V (&v)[16], V* __restrict__ buf, int j, bool active) {
  if (active) dft16<V, INV>(v);
  __syncthreads();
  if (active) {
#pragma unroll
    for (int t = 0; t < 16; ++t) buf[17 * j + t] = v[t];
  }
  __syncthreads();
}

template <typename V, int LOGN, int P, bool INV>
__device__ __forceinline__ void fft16_pass(V* __restrict__ buf, const Tw16<V, LOGN>& T16, int j0, bool active) {
  using S = Sched16<LOGN>;
  constexpr int logR = S::logR(P);
  constexpr int R = 1 << logR;
  constexpr int NB = 16 / R;
  constexpr int nt = 1 << (LOGN - 4);
  constexpr int logNR = LOGN - logR;
  constexpr int logNs = S::logNs(P);
  V v[NB][R];
  if (active) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = j0 + b * nt;
#pragma unroll
      for (int t = 0; t < R; ++t) v[b][t] = buf[pad16(j + (t << logNR))];
#pragma unroll
      for (int t = 1; t < R; ++t) {
        V w = T16.w[P][b * (R - 1) + (t - 1)];
        if (INV) w = cconj(w);
        v[b][t] = cmul(v[b][t], w);
      }
      dftR16<V, R, INV>(v[b]);
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = j0 + b * nt;
      const int k = j & ((1 << logNs) - 1);
      const int base = ((j >> logNs) << (logNs + logR)) + k;
#pragma unroll
      for (int t = 0; t < R; ++t) buf[pad16(base + (t << logNs))] = v[b][t];
    }
  }
  __syncthreads();
}

template <typename V, int LOGN, bool INV, int P = 0>
__device__ __forceinline__ void fft16_rest(V* __restrict__ buf, const Tw16<V, LOGN>& T16, int j, bool active) {
  if constexpr (P < Sched16<LOGN>::npass) {
    fft16_pass<V, LOGN, P, INV>(buf, T16, j, active);
    fft16_rest<V, LOGN, INV, P + 1>(buf, T16, j, active);
  }
}

// The whole block as one group.
template <typename V, bool INV, int EPT>
__device__ __forceinline__ void fft_lds(V* __restrict__ buf, const V* __restrict__ tw, const FftShape& s) {
  fft_lds<V, INV, EPT>(buf, tw, s, FftGroup{(int)threadIdx.x, (int)blockDim.x, true});
}

}  // namespace qg
