// Radix-8/4/2 Stockham FFT of one line held in LDS, for wave64 gfx950.
//
// A line of L complex values (L a power of two) is transformed by TPL threads.
// Stage s with radix RAD and sub-transform size NS (1, RAD0, RAD0*RAD1, ...):
// butterfly j reads x[j + r L/RAD], applies the twiddles w^{r k}
// (k = j mod NS, w = exp(-+2 pi i / (NS RAD))), does a RAD-point DFT and
// writes y[(j - k) RAD + k + r NS].  After all stages the result is in natural
// order (the Stockham auto-sort formulation, Govindaraju et al. 2008).  Every
// stage keeps RAD values per butterfly in registers and is done in place with
// two workgroup barriers (read all, then write all).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace gofd_fft {

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {   // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__device__ __forceinline__ cplx<R> rot90(cplx<R> a) {
  if constexpr (INV)
    return {-a.y, a.x};
  else
    return {a.y, -a.x};
}

template <typename R, bool INV>
__device__ __forceinline__ void dft2(cplx<R>* a) {
  const cplx<R> t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cplx<R>& a0, cplx<R>& a1, cplx<R>& a2, cplx<R>& a3) {
  const cplx<R> s0 = cadd(a0, a2), d0 = csub(a0, a2);
  const cplx<R> s1 = cadd(a1, a3), d1 = rot90<R, INV>(csub(a1, a3));
  a0 = cadd(s0, s1);
  a2 = csub(s0, s1);
  a1 = cadd(d0, d1);
  a3 = csub(d0, d1);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cplx<R>* a) {
  // even / odd halves
  cplx<R> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  cplx<R> o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
  dft4<R, INV>(e0, e1, e2, e3);
  dft4<R, INV>(o0, o1, o2, o3);
  const R c = (R)0.70710678118654752440084436210484903928;
  // o_k *= w^k, w = exp(-+ 2 pi i / 8)
  if constexpr (!INV) {
    o1 = {(o1.x + o1.y) * c, (o1.y - o1.x) * c};
    o2 = {o2.y, -o2.x};
    o3 = {(o3.y - o3.x) * c, -(o3.x + o3.y) * c};
  } else {
    o1 = {(o1.x - o1.y) * c, (o1.x + o1.y) * c};
    o2 = {-o2.y, o2.x};
    o3 = {-(o3.x + o3.y) * c, (o3.x - o3.y) * c};
  }
  a[0] = cadd(e0, o0);
  a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1);
  a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2);
  a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3);
  a[7] = csub(e3, o3);
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cplx<R>* a) {
  if constexpr (RAD == 8)
    dft8<R, INV>(a);
  else if constexpr (RAD == 4)
    dft4<R, INV>(a[0], a[1], a[2], a[3]);
  else
    dft2<R, INV>(a);
}

// LDS index with padding against bank conflicts of strided stage stores
template <int L>
__device__ __forceinline__ int pidx(int i) {
  return i + (i >> 5);
}
template <int L>
constexpr int padded_len() {
  return L + L / 32 + 1;
}

template <typename R, int L, int TPL, bool INV, int NS>
__device__ __forceinline__ void stages(cplx<R>* buf, const cplx<R>* __restrict__ tw, int t) {
  if constexpr (NS < L) {
    constexpr int REM = L / NS;
    constexpr int RAD = (REM >= 8) ? 8 : REM;
    constexpr int NB = L / RAD;             // butterflies in this stage
    static_assert(NB % TPL == 0, "threads per line must divide the butterfly count");
    constexpr int PER = NB / TPL;
    constexpr int TWS = L / (NS * RAD);     // twiddle table stride
    cplx<R> a[PER][RAD];
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPL;
#pragma unroll
      for (int r = 0; r < RAD; ++r) a[p][r] = buf[pidx<L>(j + r * NB)];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int j = t + p * TPL;
      const int k = j & (NS - 1);
      if constexpr (NS > 1) {
        // w^r for r = 1..RAD-1 from the table entries w^1, w^2, w^4 (products
        // for the others: at most two roundings away from the table values)
        cplx<R> w[8];
        w[1] = tw[k * TWS];
        if constexpr (RAD >= 4) {
          w[2] = tw[2 * k * TWS];
          w[3] = cmul(w[1], w[2]);
        }
        if constexpr (RAD == 8) {
          w[4] = tw[4 * k * TWS];
          w[5] = cmul(w[4], w[1]);
          w[6] = cmul(w[4], w[2]);
          w[7] = cmul(w[4], w[3]);
        }
#pragma unroll
        for (int r = 1; r < RAD; ++r) a[p][r] = INV ? cmulc(a[p][r], w[r]) : cmul(a[p][r], w[r]);
      }
      dft<R, RAD, INV>(a[p]);
      const int base = (j - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[pidx<L>(base + r * NS)] = a[p][r];
    }
    __syncthreads();
    stages<R, L, TPL, INV, NS * RAD>(buf, tw, t);
  }
}

// Forward (INV = false, exponent -) or unnormalised inverse (exponent +)
// transform of buf[pidx(0..L)] by threads t = 0..TPL-1 of a line.  Callers
// must synchronise before (data ready); the routine ends with a barrier.
template <typename R, int L, int TPL, bool INV>
__device__ __forceinline__ void fft_line(cplx<R>* buf, const cplx<R>* __restrict__ tw, int t) {
  stages<R, L, TPL, INV, 1>(buf, tw, t);
}

}  // namespace gofd_fft
