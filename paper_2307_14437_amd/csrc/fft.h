// Radix-16/8/4/2 Stockham FFT of one line, for wave64 gfx950.
//
// A line of L complex values (L a power of two) is transformed by TPL = L/E
// threads that each hold E values in registers: thread t holds elements
// t + m TPL (m = 0..E-1) both before the first stage and after the last.
// Stage s with radix RAD and sub-transform size NS (1, RAD0, RAD0*RAD1, ...):
// butterfly j reads x[j + r L/RAD], applies the twiddles w^{r k}
// (k = j mod NS, w = exp(-+2 pi i / (NS RAD))), does a RAD-point DFT and
// writes y[(j - k) RAD + k + r NS]; after all stages the result is in natural
// order (the Stockham auto-sort formulation, Govindaraju et al. 2008).  The
// first stage takes its inputs from registers and the last stage leaves its
// outputs in registers, so a line needs one LDS exchange per stage boundary
// and none for loading or storing: callers load from and store to HBM
// directly with the element-to-thread map above.
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

// a * exp(-+ i theta) with c = cos theta, s = sin theta
template <typename R, bool INV>
__device__ __forceinline__ cplx<R> rotc(cplx<R> a, R c, R s) {
  if constexpr (!INV)
    return {a.x * c + a.y * s, a.y * c - a.x * s};
  else
    return {a.x * c - a.y * s, a.y * c + a.x * s};
}

// 16-point DFT as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <typename R, bool INV>
__device__ __forceinline__ void dft16(cplx<R>* a) {
  const R c1 = (R)0.92387953251128675612818318939678828682;   // cos(pi/8)
  const R s1 = (R)0.38268343236508977172845998403039886676;   // sin(pi/8)
  const R c2 = (R)0.70710678118654752440084436210484903928;   // cos(pi/4)
  cplx<R> b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cplx<R> x0 = a[n2], x1 = a[n2 + 4], x2 = a[n2 + 8], x3 = a[n2 + 12];
    dft4<R, INV>(x0, x1, x2, x3);
    b[n2][0] = x0;
    b[n2][1] = x1;
    b[n2][2] = x2;
    b[n2][3] = x3;
  }
  // b[n2][k1] *= w16^(n2 k1)
  b[1][1] = rotc<R, INV>(b[1][1], c1, s1);
  b[1][2] = rotc<R, INV>(b[1][2], c2, c2);
  b[1][3] = rotc<R, INV>(b[1][3], s1, c1);
  b[2][1] = rotc<R, INV>(b[2][1], c2, c2);
  b[2][2] = rot90<R, INV>(b[2][2]);
  b[2][3] = rotc<R, INV>(b[2][3], -c2, c2);
  b[3][1] = rotc<R, INV>(b[3][1], s1, c1);
  b[3][2] = rotc<R, INV>(b[3][2], -c2, c2);
  b[3][3] = rotc<R, INV>(b[3][3], -c1, -s1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cplx<R> y0 = b[0][k1], y1 = b[1][k1], y2 = b[2][k1], y3 = b[3][k1];
    dft4<R, INV>(y0, y1, y2, y3);
    a[k1] = y0;
    a[k1 + 4] = y1;
    a[k1 + 8] = y2;
    a[k1 + 12] = y3;
  }
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cplx<R>* a) {
  if constexpr (RAD == 16)
    dft16<R, INV>(a);
  else if constexpr (RAD == 8)
    dft8<R, INV>(a);
  else if constexpr (RAD == 4)
    dft4<R, INV>(a[0], a[1], a[2], a[3]);
  else
    dft2<R, INV>(a);
}

// LDS index of element i: one pad entry after every E entries, so that the
// stride-E writes of the first stage hit distinct banks.
template <int E>
__device__ __forceinline__ int pidx(int i) {
  return i + i / E;
}
template <int L, int E>
constexpr int padded_len() {
  return L + L / E;
}

// w^r for r = 1..RAD-1 from the table entries w^1, w^2, w^4, w^8 (products for
// the others: at most three roundings away from the table values)
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void twiddle(cplx<R>* a, const cplx<R>* wb) {
  cplx<R> w[16];
  w[1] = wb[0];
  if constexpr (RAD >= 4) {
    w[2] = wb[1];
    w[3] = cmul(w[1], w[2]);
  }
  if constexpr (RAD >= 8) {
    w[4] = wb[2];
    w[5] = cmul(w[4], w[1]);
    w[6] = cmul(w[4], w[2]);
    w[7] = cmul(w[4], w[3]);
  }
  if constexpr (RAD >= 16) {
    w[8] = wb[3];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
  }
#pragma unroll
  for (int r = 1; r < RAD; ++r) a[r] = INV ? cmulc(a[r], w[r]) : cmul(a[r], w[r]);
}

// Base twiddles of one thread: for every stage after the first and every
// butterfly of the thread, the table entries w^1, w^2, w^4, w^8 (up to the
// stage's radix) at its k.  They depend on the thread position only, so a
// kernel loads them once at its start, where their latency overlaps the data
// loads, and the forward and inverse transforms of a line share them.
constexpr int ilog2c(int x) {
  int n = 0;
  while (x > 1) {
    x >>= 1;
    ++n;
  }
  return n;
}
template <int L, int E>
constexpr int stage_radix(int NS) {
  return (L / NS >= E) ? E : L / NS;
}
// slots used by the stages after the first and before the one of size NS
template <int L, int E>
constexpr int tw_slots_before(int NS_end) {
  int n = 0;
  for (int NS = stage_radix<L, E>(1); NS < NS_end && NS < L; NS *= stage_radix<L, E>(NS))
    n += (E / stage_radix<L, E>(NS)) * ilog2c(stage_radix<L, E>(NS));
  return n;
}

template <typename R, int L, int E>
struct Twiddles {
  static constexpr int N = tw_slots_before<L, E>(L);
  cplx<R> w[N > 0 ? N : 1];

  template <int NS>
  __device__ __forceinline__ void load_from(const cplx<R>* __restrict__ tw, int t) {
    if constexpr (NS < L) {
      constexpr int RAD = stage_radix<L, E>(NS);
      constexpr int PER = E / RAD, NB = ilog2c(RAD), TPL = L / E, TWS = L / (NS * RAD);
      constexpr int OFF = tw_slots_before<L, E>(NS);
#pragma unroll
      for (int p = 0; p < PER; ++p) {
        const int k = (t + p * TPL) & (NS - 1);
#pragma unroll
        for (int q = 0; q < NB; ++q) w[OFF + p * NB + q] = tw[(k << q) * TWS];
      }
      load_from<NS * RAD>(tw, t);
    }
  }
  // tw: the table exp(-2 pi i j / L), j = 0..L-1
  __device__ __forceinline__ void load(const cplx<R>* __restrict__ tw, int t) {
    load_from<stage_radix<L, E>(1)>(tw, t);
  }
  // Between two transforms of one kernel (double precision): the compiler may
  // no longer assume the values unchanged, so it derives the twiddle products
  // of the second transform again instead of keeping those of the first in
  // registers, which would not fit.  In single precision they fit and are kept.
  __device__ __forceinline__ void opaque() {
    if constexpr (sizeof(R) == 8) {
#pragma unroll
      for (int i = 0; i < N; ++i) asm volatile("" : "+v"(w[i].x), "+v"(w[i].y));
    }
  }
};

// One Stockham stage and, recursively, the ones after it.  LDS protocol: the
// first stage writes the buffer (callers guarantee no thread still reads
// it), every later stage waits for the previous writes, reads, and (unless
// it is the last) waits again before overwriting the buffer.
template <typename R, int L, int E, bool INV, int NS>
__device__ __forceinline__ void rstage(cplx<R> (&v)[E], cplx<R>* buf, const Twiddles<R, L, E>& tws, int t) {
  constexpr int TPL = L / E;
  constexpr int REM = L / NS;
  constexpr int RAD = (REM >= E) ? E : REM;
  constexpr int PER = E / RAD;                  // butterflies per thread
  constexpr bool FIRST = (NS == 1);
  constexpr bool LAST = (NS * RAD == L);
  constexpr int NB = ilog2c(RAD);
  static_assert(RAD >= 2 && PER * RAD == E, "radix plan");
  cplx<R> a[PER][RAD];
  if constexpr (!FIRST) __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p)
#pragma unroll
    for (int r = 0; r < RAD; ++r) {
      const int m = p + r * PER;                // element t + m TPL = j + r L/RAD
      if constexpr (FIRST)
        a[p][r] = v[m];
      else
        a[p][r] = buf[pidx<E>(t + m * TPL)];
    }
  if constexpr (!FIRST && !LAST) __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    if constexpr (!FIRST) {
      constexpr int OFF = tw_slots_before<L, E>(NS);
      twiddle<R, RAD, INV>(a[p], &tws.w[OFF + p * NB]);
    }
    dft<R, RAD, INV>(a[p]);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[p + r * PER] = a[p][r];
    } else {
      const int j = t + p * TPL;
      const int k = j & (NS - 1);
      const int base = (j - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[pidx<E>(base + r * NS)] = a[p][r];
    }
  }
  if constexpr (!LAST) rstage<R, L, E, INV, NS * RAD>(v, buf, tws, t);
}

// Forward (INV = false, exponent -) or unnormalised inverse (exponent +)
// transform of the line held in v by threads t = 0..L/E-1, with buf (padded
// length) as exchange space and the thread's base twiddles tws.  On entry no
// thread may still read buf; on exit other threads may still read it
// (synchronise before writing it again).
template <typename R, int L, int E, bool INV>
__device__ __forceinline__ void fft_regs(cplx<R> (&v)[E], cplx<R>* buf, const Twiddles<R, L, E>& tws, int t) {
  rstage<R, L, E, INV, 1>(v, buf, tws, t);
}

}  // namespace gofd_fft
