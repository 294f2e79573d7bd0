// Device-side state of the conjugate-gradient iteration and its scalar step,
// shared by the solver kernels and the FFT pass that finishes the reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace gofd_cg {

// Per-rhs CG scalars.  alpha and beta of the last decided step, gamma = (r, u)
// of the current iterate, rr = (r, r), bb = (b, b), tol2 = tol^2 bb.
struct Scal {
  double alpha, beta, gamma, rr, bb, tol2, rrn, pad0;
  int done, iters, status, pad;
};

enum { ST_OK = 0, ST_BREAKDOWN = 1 };

// LDS doubles that block_sum_n<NT, NQ> needs
template <int NT, int NQ>
constexpr int block_sum_lds() {
  return NQ * (NT >= 64 ? NT / 64 : NT);
}

// Fixed-order block sum of NQ quantities with wave shuffles and one barrier:
// every lane of a wave gets the same bits (the butterfly adds the same pairs)
// and every thread adds the per-wave sums in the same order.  Blocks of fewer
// than 64 threads add the values through LDS in thread order.
template <int NT, int NQ>
__device__ __forceinline__ void block_sum_n(double* v, double* sh) {
  if constexpr (NT < 64) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q * NT + threadIdx.x] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double t = 0.0;
      for (int k = 0; k < NT; ++k) t += sh[q * NT + k];
      v[q] = t;
    }
    __syncthreads();
    return;
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
  const int wid = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) sh[q * (NT / 64) + wid] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) t += sh[q * (NT / 64) + k];
    v[q] = t;
  }
  __syncthreads();
}

// Scalar step from gamma = (r, u), rr = (r, r) and delta = (K u, u) in the
// single-reduction form of CG (Chronopoulos and Gear, 1989):
//   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev).
// Tests convergence of the current iterate first (rr against tol2).  Writes
// the new state to O; returns true when the iteration stops (converged or
// broken down).
__device__ __forceinline__ bool cg_decide(const Scal& S, double g, double rr, double d, Scal& O, double& alpha,
                                          double& beta) {
  O = S;
  O.rr = rr;
  bool stop = false;
  if (!isfinite(rr)) {
    O.status = ST_BREAKDOWN;
    stop = true;
  } else if (rr <= S.tol2) {
    stop = true;
  } else {
    beta = g / S.gamma;
    double den = d - beta * g / S.alpha;
    if (!(den > 0.0) && d > 0.0) {
      // (p, K p) lost to cancellation (possible with single-precision
      // products): restart along u, i.e. beta = 0 and (p, K p) = delta
      beta = 0.0;
      den = d;
    }
    if (!(g > 0.0) || !(den > 0.0) || !isfinite(den)) {
      O.status = ST_BREAKDOWN;
      stop = true;
    } else {
      alpha = g / den;
      O.alpha = alpha;
      O.beta = beta;
      O.gamma = g;
      O.iters = S.iters + 1;
    }
  }
  if (stop) O.done = 1;
  return stop;
}

// Partial sums handed from the scatter (or the start kernel, or the upper
// triangular solve) to the column pass: n1 partials of gamma and of (r, r).
struct Level1 {
  const double* partG = nullptr;
  const double* partR = nullptr;
  int n1 = 0;
};

// The state of one item into page-locked host memory for the host to read
// while the device runs on: the fields first, then (after a system-scope
// fence) pad = 1 as the mark that they are complete.  The host clears the
// mark before it issues the launch that writes the slot.
__device__ __forceinline__ void state_to_host(Scal* h, const Scal& S) {
  h->alpha = S.alpha;
  h->beta = S.beta;
  h->gamma = S.gamma;
  h->rr = S.rr;
  h->bb = S.bb;
  h->tol2 = S.tol2;
  h->rrn = S.rrn;
  h->done = S.done;
  h->iters = S.iters;
  h->status = S.status;
  __threadfence_system();
  __hip_atomic_store(&h->pad, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
}

// Finishing step run by one block of NT threads: sums the three arrays of nb
// partials left by the column pass (gamma, (r, r), delta; layout
// part[rhs][3][nb]) in a fixed order and writes the decided state.  Inactive
// when sc is null.  With host given (page-locked host memory, one Scal per
// item), the state also goes there (state_to_host).
struct Finish {
  Scal* sc = nullptr;
  const double* part = nullptr;
  int nb = 0;
  Scal* host = nullptr;

  template <int NT>
  __device__ __forceinline__ void run(int rhs, double* sh) const {
    double t[3] = {0.0, 0.0, 0.0};
    const double* pr = part + (long long)rhs * 3 * nb;
    // all loads of a thread first (independent), then the adds in index order
    constexpr int MAXL = 8;
    for (int i0 = threadIdx.x; i0 < nb; i0 += MAXL * NT) {
      double v[3][MAXL];
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
          const int i = i0 + j * NT;
          v[q][j] = i < nb ? pr[q * nb + i] : 0.0;
        }
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int j = 0; j < MAXL; ++j) t[q] += v[q][j];
    }
    block_sum_n<NT, 3>(t, sh);
    if (threadIdx.x == 0) {
      const Scal S = sc[rhs];
      Scal O = S;
      if (!S.done) {
        double alpha = 0.0, beta = 0.0;
        cg_decide(S, t[0], t[1], t[2], O, alpha, beta);
        sc[rhs] = O;
      }
      if (host) state_to_host(host + rhs, O);
    }
  }
};

}  // namespace gofd_cg
