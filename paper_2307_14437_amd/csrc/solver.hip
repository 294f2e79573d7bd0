// Preconditioned conjugate gradients for eq. GoFD-2 on the device.
//
//   K u = b,  K = I_J^T A_FD I_J,  b = h^{2s} I_J^T f_FD   (eq. GoFD-2, interior block)
//
// All vectors have N_v entries in the mesh's numbering; Dirichlet entries are
// kept at zero, which is the interior block of the remark after eq. GoFD-2.
//
// CG runs in the single-reduction form of Chronopoulos and Gear (1989), whose
// iterates equal those of preconditioned CG in exact arithmetic.  One
// iteration is five kernels: the gather I u, the three FFT passes of A_FD
// (the column pass also leaves the partial sums of delta = (K u, u) by
// Parseval, and block 0 of the last pass finishes every reduction and decides
// alpha, beta and convergence), and the I^T scatter, which applies the step
// to the vertex vectors as it forms w = K u and leaves the partial sums of
// the next gamma = (r, u) and (r, r).  All sums are fixed-order, so results
// do not depend on scheduling; the host reads the convergence flags every
// few iterations, and those iterations are captured once in a hipGraph and
// replayed.
//
// Preconditioners: none; D_h (CG on the symmetric form of eq. Ah-3); the IC(1)
// factor of A_h^(5/9/27) (Section 3.3), applied with two level-scheduled
// triangular solves.
//
// FP32 mode: the grid-side arrays and FFTs of every K product inside CG run
// in single precision; an outer loop in double precision recomputes the true
// residual r = b - K x with a double-precision product, solves K d = r to a
// modest relative tolerance and updates x += d (iterative refinement).
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <vector>

#include "bary.h"
#include "internal.h"
#include "precond_host.h"

namespace {

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

constexpr int NB_DOT = 256;      // blocks of the residual kernel (fixed: deterministic sums)
#ifndef GOFD_BS
#define GOFD_BS 128
#endif
constexpr int BS = GOFD_BS;       // threads per block of the CG vector kernels (build-time knob)
constexpr int MAX_SC = 16384;    // most blocks of the CG scatter (one partial sum each)
#ifndef GOFD_SCAT_G
#define GOFD_SCAT_G 16
#endif
constexpr int SCAT_G = GOFD_SCAT_G;   // lanes per vertex in the I^T scatter (build-time knob: 8, 16, 32)

using gofd_cg::block_sum_n;
using gofd_cg::Scal;
using gofd_cg::ST_BREAKDOWN;
using gofd_cg::ST_OK;

// fixed-order block reduction of one double per thread (NT threads)
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Sum of n partials in a fixed order (strided per thread, then the block
// tree): every block that calls it gets the same bits.
__device__ __forceinline__ double sum_fixed(const double* __restrict__ part, int n, double* sh) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += BS) s += part[i];
  return block_sum<BS>(s, sh);
}

// ---------------------------------------------------------------- kernels

// b = c * mask * I^T f (grid f), or c * mask * D * f (vertex f); one rhs per blockIdx.y
template <int G>
__global__ __launch_bounds__(BS) void k_rhs_grid(const int* __restrict__ off, const int* __restrict__ node,
                                                 const double* __restrict__ w, const double* __restrict__ f,
                                                 long long nv, long long n_nodes, const double* __restrict__ mask,
                                                 double c, double* __restrict__ b) {
  const long long v = ((long long)blockIdx.x * BS + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  const int rhs = blockIdx.y;
  if (v >= nv) return;
  const double* fr = f + rhs * n_nodes;
  double acc = 0.0;
  for (int i = off[v] + lane; i < off[v + 1]; i += G) acc += w[i] * fr[node[i]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (lane == 0) b[rhs * nv + v] = c * mask[v] * acc;
}

__global__ void k_rhs_vertex(const double* __restrict__ f, const double* __restrict__ D, const double* __restrict__ mask,
                             long long nv, double c, double* __restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i < nv) b[rhs * nv + i] = c * mask[i] * D[i] * f[rhs * nv + i];
}

// CG step in the form of Chronopoulos and Gear: with u = M r and w = K u,
//   gamma = (r, u), delta = (w, u), beta = gamma / gamma_prev,
//   alpha = gamma / (delta - beta gamma / alpha_prev),
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s.
// The vector kernels below run nbs blocks of BS threads, each over a
// contiguous range of vertices, and leave one partial sum per block.

// start from x = 0: r = b, u = M_diag b (or u given), p = s = 0; partials of
// gamma = (r, u) and (r, r).  Item blockIdx.y, vectors at off.
__global__ __launch_bounds__(BS) void k_cg_start(const CgItem* __restrict__ items, const double* __restrict__ b,
                                                 double* __restrict__ x, double* __restrict__ r,
                                                 double* __restrict__ u, double* __restrict__ p,
                                                 double* __restrict__ s, double* __restrict__ partG,
                                                 double* __restrict__ partR) {
  __shared__ double sh[gofd_cg::block_sum_lds<BS, 2>()];
  const int it = blockIdx.y;
  const CgItem& I = items[it];
  const long long o = I.off, nv = I.nv;
  const bool ufilled = I.dk < 0;              // IC(1): u = M^{-1} b was formed before
  const double* dinv = I.dk == 1 ? I.dscale : nullptr;
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < nv; i += (long long)gridDim.x * BS) {
    const double bi = b[o + i];
    x[o + i] = 0.0;
    r[o + i] = bi;
    double ui = ufilled ? u[o + i] : (dinv ? bi * dinv[i] : bi);
    if (!ufilled) u[o + i] = ui;
    p[o + i] = 0.0;
    s[o + i] = 0.0;
    acc[0] += bi * ui;
    acc[1] += bi * bi;
  }
  block_sum_n<BS, 2>(acc, sh);
  if (threadIdx.x == 0) {
    partG[(long long)it * gridDim.x + blockIdx.x] = acc[0];
    partR[(long long)it * gridDim.x + blockIdx.x] = acc[1];
  }
}

// one block per rhs: initial state (gamma_prev = inf, alpha_prev = 1 make the
// first beta zero and the first alpha gamma / delta)
// bref (nullable): per item, the (b, b) the tolerance refers to when the
// system being solved is the correction K d = b - K x0 of a warm start
__global__ __launch_bounds__(BS) void k_cg_init(const double* __restrict__ partG, const double* __restrict__ partR,
                                                int nb, Scal* __restrict__ sc, double tol,
                                                const double* __restrict__ bref) {
  __shared__ double sh[BS];
  const int rhs = blockIdx.x;
  const double g = sum_fixed(partG + (long long)rhs * nb, nb, sh);
  const double bb = sum_fixed(partR + (long long)rhs * nb, nb, sh);
  if (threadIdx.x != 0) return;
  Scal S{};
  S.alpha = 1.0;
  S.beta = 0.0;
  S.gamma = HUGE_VAL;
  S.rr = bb;
  S.bb = bref ? bref[rhs] : bb;
  S.tol2 = tol * tol * S.bb;
  S.done = (bb == 0.0) ? 1 : 0;
  S.status = ST_OK;
  if (!(g > 0.0) && bb > 0.0) {
    S.status = ST_BREAKDOWN;
    S.done = 1;
  }
  sc[rhs] = S;
}

// Residual replacement (reliable updating): r = b - q with q = K x from a
// double-precision product, u = M_diag r; partials of gamma and (r, r).
__global__ __launch_bounds__(BS) void k_cg_replace(const CgItem* __restrict__ items, const double* __restrict__ b,
                                                   const double* __restrict__ q, double* __restrict__ r,
                                                   double* __restrict__ u, const Scal* __restrict__ sc,
                                                   double* __restrict__ partG, double* __restrict__ partR,
                                                   const int* __restrict__ map) {
  __shared__ double sh[gofd_cg::block_sum_lds<BS, 2>()];
  const int it = map ? map[blockIdx.y] : blockIdx.y;
  const CgItem& I = items[it];
  if (sc[it].status != ST_OK) return;
  const long long o = I.off, nv = I.nv;
  const int dk = I.dk;
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < nv; i += (long long)gridDim.x * BS) {
    const double ri = b[o + i] - q[o + i];
    r[o + i] = ri;
    acc[1] += ri * ri;
    if (dk >= 0) {
      const double ui = dk ? ri * I.dscale[i] : ri;
      u[o + i] = ui;
      acc[0] += ri * ui;
    }
  }
  block_sum_n<BS, 2>(acc, sh);
  if (threadIdx.x == 0) {
    if (dk >= 0) partG[(long long)it * gridDim.x + blockIdx.x] = acc[0];
    partR[(long long)it * gridDim.x + blockIdx.x] = acc[1];
  }
}

// one block per rhs: after a replacement the true (r, r) decides whether the
// rhs has converged; a rhs that had stopped on its recursive residual resumes
// when the true one is still above the tolerance.  With host given, every
// rhs's state also goes there (state_to_host).
__global__ __launch_bounds__(BS) void k_cg_reopen(const double* __restrict__ partR, int nb, Scal* __restrict__ sc,
                                                  Scal* __restrict__ host, const int* __restrict__ map) {
  __shared__ double sh[BS];
  const int rhs = map ? map[blockIdx.x] : blockIdx.x;
  const double rr = sum_fixed(partR + (long long)rhs * nb, nb, sh);
  if (threadIdx.x != 0) return;
  Scal S = sc[rhs];
  if (S.status == ST_OK) {
    S.rr = rr;
    S.done = (rr <= S.tol2) ? 1 : 0;
    sc[rhs] = S;
  }
  if (host) state_to_host(host + rhs, S);
}

// w = mask * I^T y (the product K u, G lanes per vertex) and, in the same
// pass, the step decided by the last FFT pass: s = w + beta s, p = u + beta p,
// x += alpha p, r -= alpha s and, for a diagonal (or no) preconditioner,
// u = M r; partials of the next (r, r) and gamma = (r, u).  Item blockIdx.y;
// block b takes the vertex groups [b*per, (b+1)*per) in XCD-contiguous order
// (blocks past the item's vertices leave zero partials).
template <typename Y, typename WT, int G>
__global__ __launch_bounds__(BS) void k_scatter_cg(const CgItem* __restrict__ items, const Y* __restrict__ y,
                                                   long long n_nodes, const Scal* __restrict__ sc,
                                                   double* __restrict__ x, double* __restrict__ p,
                                                   double* __restrict__ s, double* __restrict__ r,
                                                   double* __restrict__ u, int per, double* __restrict__ partG,
                                                   double* __restrict__ partR, const int* __restrict__ amap) {
  constexpr int VPB = BS / G;                 // vertices per block pass
  constexpr int U = G >= 16 ? 4 : 64 / G;     // entries per lane loaded together (64 per vertex)
  __shared__ double sh[gofd_cg::block_sum_lds<BS, 2>()];
  const int it = amap ? amap[blockIdx.y] : blockIdx.y;
  const CgItem& I = items[it];
  const long long o = I.off, nv = I.nv;
  const int dk = I.dk;
  const auto off = gmem(I.csc_off);
  const auto node = gmem(I.csc_node);
  const auto imask = gmem(I.imask);
  const auto dscale = gmem(I.dscale);
  const __attribute__((address_space(1))) WT* wts;
  if constexpr (sizeof(WT) == 4)
    wts = gmem(reinterpret_cast<const WT*>(I.csc_w32));
  else
    wts = gmem(reinterpret_cast<const WT*>(I.csc_w));
  const int lane = threadIdx.x % G;
  const long long g0 = (long long)xcd_remap(blockIdx.x, gridDim.x) * per;
  const Y* yr = y + it * n_nodes;
  const Scal& S = sc[it];
  const bool done = S.done;                   // block-uniform
  const double alpha = S.alpha, beta = S.beta;
  double acc2[2] = {0.0, 0.0};                // (r, r), (r, u)
  for (int q = 0; q < per && !done; ++q) {
    // Every load below is unconditional, from clamped in-range indices (a
    // vertex past the end reads the last vertex, an entry past its vertex
    // reads entry 0 with weight zero), so that all of them can be in flight
    // together; every lane of a vertex group reads the vertex's own vectors.
    const long long v = (g0 + q) * VPB + threadIdx.x / G;
    const bool valid = v < nv;
    const long long vc = valid ? v : nv - 1;
    const int i0 = off[vc], i1r = off[vc + 1];
    const int i1 = valid ? i1r : i0;
    const double vm = imask[vc], vs = s[o + vc], vp = p[o + vc], vu = u[o + vc], vr = r[o + vc],
                 vx = x[o + vc], vd = dscale[vc];
    int nd[U];
    WT wt[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int i = i0 + lane + k * G;
      const int ic = i < i1 ? i : 0;
      nd[k] = node[ic];
      wt[k] = wts[ic];
      if (i >= i1) wt[k] = (WT)0;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k) acc += (double)wt[k] * (double)yr[nd[k]];
    for (int i = i0 + lane + U * G; i < i1; i += G) acc += (double)wts[i] * (double)yr[node[i]];
#pragma unroll
    for (int k = G / 2; k > 0; k >>= 1) acc += __shfl_xor(acc, k, G);
    if (lane == 0 && valid) {
      const double wv = vm * acc;
      const double sn = fma(beta, vs, wv);
      const double pn = fma(beta, vp, vu);
      const double rn = fma(-alpha, sn, vr);
      s[o + v] = sn;
      p[o + v] = pn;
      x[o + v] = fma(alpha, pn, vx);
      r[o + v] = rn;
      acc2[0] += rn * rn;
      if (dk >= 0) {
        const double un = dk ? rn * vd : rn;
        u[o + v] = un;
        acc2[1] += rn * un;
      }
    }
  }
  if (done) return;
  block_sum_n<BS, 2>(acc2, sh);
  if (threadIdx.x == 0) {
    partR[(long long)it * gridDim.x + blockIdx.x] = acc2[0];
    if (dk >= 0) partG[(long long)it * gridDim.x + blockIdx.x] = acc2[1];
  }
}

// The same step with w = mask * I^T y from the partial slots of the row-pair
// form (pass C left the sum of each vertex's entries in each row pair): one
// vertex per thread adds its slots in order.  Item blockIdx.y.
__global__ __launch_bounds__(BS) void k_vertex_cg(const CgItem* __restrict__ items, const double* __restrict__ P,
                                                  long long pstride, const Scal* __restrict__ sc,
                                                  double* __restrict__ x, double* __restrict__ p,
                                                  double* __restrict__ s, double* __restrict__ r,
                                                  double* __restrict__ u, double* __restrict__ partG,
                                                  double* __restrict__ partR, const int* __restrict__ amap,
                                                  float* __restrict__ us) {
  constexpr int PU = 8;                       // slots loaded together
  __shared__ double sh[gofd_cg::block_sum_lds<BS, 2>()];
  const int it = amap ? amap[blockIdx.y] : blockIdx.y;
  const CgItem& I = items[it];
  const long long o = I.off, nv = I.nv;
  const int dk = I.dk;
  const auto pv = gmem(I.pv_off);
  const auto imask = gmem(I.imask);
  const auto dscale = gmem(I.dscale);
  const auto Pi = gmem(P + it * pstride);
  const Scal& S = sc[it];
  if (S.done) return;                         // block-uniform
  const double alpha = S.alpha, beta = S.beta;
  // loads from clamped in-range positions (all in flight together)
  const long long v = (long long)xcd_remap(blockIdx.x, gridDim.x) * BS + threadIdx.x;
  const bool valid = v < nv;
  const long long vc = valid ? v : nv - 1;
  const int a = pv[vc], br = pv[vc + 1];
  const int b = valid ? br : a;
  const double vm = imask[vc], vs = s[o + vc], vp = p[o + vc], vu = u[o + vc], vr = r[o + vc], vx = x[o + vc],
               vd = dscale[vc];
  double pp[PU];
  int ps[PU];
  const auto pos = gmem(I.rp_pos);
#pragma unroll
  for (int k = 0; k < PU; ++k) pp[k] = Pi[a + k < b ? a + k : 0];
  if (us)
#pragma unroll
    for (int k = 0; k < PU; ++k) ps[k] = pos[a + k < b ? a + k : 0];
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < PU; ++k)
    if (a + k < b) acc += pp[k];
  for (int i = a + PU; i < b; ++i) acc += Pi[i];
  double acc2[2] = {0.0, 0.0};                // (r, r), (r, u)
  if (valid) {
    const double wv = vm * acc;
    const double sn = fma(beta, vs, wv);
    const double pn = fma(beta, vp, vu);
    const double rn = fma(-alpha, sn, vr);
    s[o + v] = sn;
    p[o + v] = pn;
    x[o + v] = fma(alpha, pn, vx);
    r[o + v] = rn;
    acc2[0] = rn * rn;
    if (dk >= 0) {
      const double un = dk ? rn * vd : rn;
      u[o + v] = un;
      acc2[1] = rn * un;
      if (us) {                               // u at the vertex's slots for the next gather
        float* ui = us + it * pstride;
        const float uf = (float)un;
#pragma unroll
        for (int k = 0; k < PU; ++k)
          if (a + k < b) ui[ps[k]] = uf;
        for (int i = a + PU; i < b; ++i) ui[pos[i]] = uf;
      }
    }
  }
  block_sum_n<BS, 2>(acc2, sh);
  if (threadIdx.x == 0) {
    partR[(long long)it * gridDim.x + blockIdx.x] = acc2[0];
    if (dk >= 0) partG[(long long)it * gridDim.x + blockIdx.x] = acc2[1];
  }
}

// u at every slot of each vertex (row-pair-major positions), for the FP32
// gather through the slots: after the start and after a residual replacement
// (the vertex kernel keeps it current in between).  Item blockIdx.y.
__global__ __launch_bounds__(BS) void k_u_to_slots(const CgItem* __restrict__ items, const double* __restrict__ u,
                                                   float* __restrict__ us, long long ustride,
                                                   const int* __restrict__ map) {
  const int it = map ? map[blockIdx.y] : blockIdx.y;
  const CgItem& I = items[it];
  float* ui = us + it * ustride;
  for (long long v = (long long)blockIdx.x * BS + threadIdx.x; v < I.nv; v += (long long)gridDim.x * BS) {
    const float uf = (float)u[I.off + v];
    for (int i = I.pv_off[v]; i < I.pv_off[v + 1]; ++i) ui[I.rp_pos[i]] = uf;
  }
}

// Residual replacement from the row-pair form: q = mask * (sum of each
// vertex's partial slots, left by the last row pass of an FP64 product of x),
// r = b - q, u = M_diag r, u at the vertex's slots (us, if given) and the
// partials of gamma and (r, r), as k_cg_replace.  Item map[blockIdx.y] (or
// blockIdx.y).
__global__ __launch_bounds__(BS) void k_cg_replace_rp(const CgItem* __restrict__ items,
                                                      const double* __restrict__ P, long long pstride,
                                                      const double* __restrict__ b, double* __restrict__ r,
                                                      double* __restrict__ u, const Scal* __restrict__ sc,
                                                      double* __restrict__ partG, double* __restrict__ partR,
                                                      const int* __restrict__ map, float* __restrict__ us) {
  __shared__ double sh[gofd_cg::block_sum_lds<BS, 2>()];
  const int it = map ? map[blockIdx.y] : blockIdx.y;
  const CgItem& I = items[it];
  if (sc[it].status != ST_OK) return;
  const long long o = I.off, nv = I.nv;
  const int dk = I.dk;
  const double* Pi = P + it * pstride;
  double acc[2] = {0.0, 0.0};
  for (long long v = (long long)blockIdx.x * BS + threadIdx.x; v < nv; v += (long long)gridDim.x * BS) {
    double w = 0.0;
    for (int i = I.pv_off[v]; i < I.pv_off[v + 1]; ++i) w += Pi[i];
    const double ri = b[o + v] - I.imask[v] * w;
    r[o + v] = ri;
    acc[1] += ri * ri;
    if (dk >= 0) {
      const double ui = dk ? ri * I.dscale[v] : ri;
      u[o + v] = ui;
      acc[0] += ri * ui;
      if (us) {
        float* ui32 = us + it * pstride;
        for (int i = I.pv_off[v]; i < I.pv_off[v + 1]; ++i) ui32[I.rp_pos[i]] = (float)ui;
      }
    }
  }
  block_sum_n<BS, 2>(acc, sh);
  if (threadIdx.x == 0) {
    if (dk >= 0) partG[(long long)it * gridDim.x + blockIdx.x] = acc[0];
    partR[(long long)it * gridDim.x + blockIdx.x] = acc[1];
  }
}

// r = b - q (q = K x), partials of (r, r) and (b, b); used by the refinement
// loop (FP64 residual).  Item blockIdx.y.
__global__ __launch_bounds__(BS) void k_residual(const CgItem* __restrict__ items, const double* __restrict__ b,
                                                 const double* __restrict__ q, double* __restrict__ r,
                                                 double* __restrict__ partials) {
  __shared__ double sh[BS];
  const int it = blockIdx.y;
  const CgItem& I = items[it];
  const long long o = I.off, nv = I.nv;
  double s_rr = 0.0, s_bb = 0.0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < nv; i += (long long)gridDim.x * BS) {
    const double ri = b[o + i] - q[o + i];
    r[o + i] = ri;
    s_rr += ri * ri;
    s_bb += b[o + i] * b[o + i];
  }
  s_rr = block_sum<BS>(s_rr, sh);
  s_bb = block_sum<BS>(s_bb, sh);
  double* part = partials + (long long)it * 2 * NB_DOT;
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_rr;
    part[NB_DOT + blockIdx.x] = s_bb;
  }
}

__global__ __launch_bounds__(BS) void k_residual_finish(const double* __restrict__ partials, double* __restrict__ out2) {
  __shared__ double sh[BS];
  const int rhs = blockIdx.x;
  const double* part = partials + (long long)rhs * 2 * NB_DOT;
  const double rr = sum_fixed(part, NB_DOT, sh);
  const double bb = sum_fixed(part + NB_DOT, NB_DOT, sh);
  if (threadIdx.x == 0) {
    out2[2 * rhs] = rr;
    out2[2 * rhs + 1] = bb;
  }
}

__global__ void k_axpy_mask(double* __restrict__ x, const double* __restrict__ d, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

// plain scatter q = mask * I^T y (no dot), item blockIdx.y
template <int G>
__global__ __launch_bounds__(BS) void k_scatter_plain(const CgItem* __restrict__ items, const double* __restrict__ y,
                                                      long long n_nodes, double* __restrict__ q,
                                                      const int* __restrict__ map) {
  const int it = map ? map[blockIdx.y] : blockIdx.y;
  const CgItem& I = items[it];
  const long long v = ((long long)xcd_remap(blockIdx.x, gridDim.x) * BS + threadIdx.x) / G;
  const int lane = threadIdx.x % G;
  if (v >= I.nv) return;
  const double* yr = y + it * n_nodes;
  double acc = 0.0;
  for (int i = I.csc_off[v] + lane; i < I.csc_off[v + 1]; i += G) acc += I.csc_w[i] * yr[I.csc_node[i]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (lane == 0) q[I.off + v] = I.imask[v] * acc;
}

// ---------------------------------------------------------------- triangular solves
//
// Level-scheduled inside one workgroup per right-hand side: the rows of a
// dependency level are independent, so the block's threads take them in
// parallel, and a workgroup barrier separates consecutive levels.  No
// workgroup ever waits on another, so the solve cannot stall on memory
// visibility between XCDs; the cost is one barrier plus one dependent read
// round trip per level.

// The upper solve also forms gamma = (r, u) for CG (fixed-order block sum,
// written as partial 0 of nbu with the others zero).
template <bool LOWER>
__global__ __launch_bounds__(1024) void k_trsv_levels(const int* __restrict__ ptr, const int* __restrict__ col,
                                                      const double* __restrict__ val, const int* __restrict__ lvl_ptr,
                                                      const int* __restrict__ lvl_rows, int nlev,
                                                      const double* __restrict__ rhs_in, double* __restrict__ out,
                                                      long long stride, const Scal* __restrict__ sc,
                                                      const double* __restrict__ rvec, double* __restrict__ partG,
                                                      int nbu) {
  __shared__ double sh[1024 / 64];
  const int k = blockIdx.x;
  if (sc && sc[k].done) return;
  const double* b = rhs_in + k * stride;
  double* y = out + k * stride;
  for (int l = 0; l < nlev; ++l) {
    const int r0 = lvl_ptr[l], r1 = lvl_ptr[l + 1];
    for (int t = r0 + (int)threadIdx.x; t < r1; t += (int)blockDim.x) {
      const int row = lvl_rows[t];
      const int e0 = ptr[row], e1 = ptr[row + 1];
      // lower: diagonal last; upper: diagonal first
      const int dpos = LOWER ? e1 - 1 : e0;
      const int lo = LOWER ? e0 : e0 + 1, hi = LOWER ? e1 - 1 : e1;
      double s = 0.0;
      for (int i = lo; i < hi; ++i) s += val[i] * y[col[i]];
      y[row] = (b[row] - s) / val[dpos];
    }
    __syncthreads();
  }
  if (!LOWER && partG) {
    const double* rv = rvec + k * stride;
    double s = 0.0;
    for (long long i = threadIdx.x; i < stride; i += 1024) s += rv[i] * y[i];
    block_sum_n<1024, 1>(&s, sh);
    for (int i = threadIdx.x; i < nbu; i += 1024) partG[(long long)k * nbu + i] = (i == 0) ? s : 0.0;
  }
}

// One dependency level of a triangular solve with its rows spread over the
// grid (blockIdx.x) and one right-hand side per blockIdx.y: used when the
// factor has few levels (multicolour order), one launch per level, so that
// no workgroup waits on another.
// TRSV_LANES lanes share a row: each takes every TRSV_LANES-th entry, so the
// row's loads are in flight together, and a fixed butterfly adds the lanes'
// sums (the same order every time).
constexpr int TRSV_LANES = 16;
template <bool LOWER>
__global__ __launch_bounds__(256) void k_trsv_level(const int* __restrict__ ptr, const int* __restrict__ col,
                                                    const double* __restrict__ val, const int* __restrict__ rows,
                                                    int r0, int r1, const double* __restrict__ rhs_in,
                                                    double* __restrict__ out, long long stride,
                                                    const Scal* __restrict__ sc) {
  const int k = blockIdx.y;
  if (sc && sc[k].done) return;
  const int lane = threadIdx.x % TRSV_LANES;
  const int t = r0 + (int)((blockIdx.x * blockDim.x + threadIdx.x) / TRSV_LANES);
  const bool ok = t < r1;
  const double* b = rhs_in + k * stride;
  double* y = out + k * stride;
  const int row = rows[ok ? t : r0];
  const int e0 = ptr[row], e1 = ptr[row + 1];
  const int dpos = LOWER ? e1 - 1 : e0;
  const int lo = LOWER ? e0 : e0 + 1, hi = LOWER ? e1 - 1 : e1;
  double s = 0.0;
  for (int i = lo + lane; i < hi; i += TRSV_LANES) s += val[i] * y[col[i]];
#pragma unroll
  for (int o = TRSV_LANES / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, TRSV_LANES);
  if (ok && lane == 0) y[row] = (b[row] - s) / val[dpos];
}

// One colour of the triangular solves in multicolour order: the factor's rows
// r0..r1-1 (row t is vertex perm[t]) depend only on rows of colours that
// earlier launches solved, so the colour is solved in one launch, its rows
// contiguous.  TRSV_LANES lanes share a row and each reads its first two
// entries without waiting (the index clamped into the row, the product masked),
// any further ones in a loop.
//   LOWER:  y_t = (r[perm t] - sum_{j<t} L_tj y_j) / L_tt.  With TAIL (the last
//           colour) the row of U = L^T is solved as well: no row of a later
//           colour exists, so u_t = y_t / L_tt.
//   upper:  u_t = (y_t - sum_{j>t} U_tj u_j) / U_tt.
// A solved u_t goes to pu (factor order, read by later colours) and to
// u[perm t] (vertex order).  With part given (gamma of CG), block b of the
// grid-stride launch adds r[perm t] u_t of its rows to part[b]; the TAIL
// launch, the first of the upper solves, stores instead, so after colour 0
// part holds the partials of (r, u) in a fixed order.
template <bool LOWER, bool TAIL>
__global__ __launch_bounds__(256) void k_trsv_colour(const int* __restrict__ ptr, const int* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     const int* __restrict__ perm, int r0, int r1,
                                                     const double* __restrict__ r, double* __restrict__ y,
                                                     double* __restrict__ pu, double* __restrict__ u,
                                                     long long stride, const Scal* __restrict__ sc,
                                                     double* __restrict__ part, int nbu) {
  constexpr int RPB = 256 / TRSV_LANES;   // rows per block and pass
  __shared__ double sh[gofd_cg::block_sum_lds<256, 1>()];
  const int k = blockIdx.y;
  if (sc && sc[k].done) return;
  const int lane = threadIdx.x % TRSV_LANES;
  const double* rk = r + k * stride;
  double* yk = y + k * stride;
  double* puk = pu + k * stride;
  const double* dep = LOWER ? yk : puk;
  const int nrows = r1 - r0;
  double acc = 0.0;
  for (int base = blockIdx.x * RPB; base < nrows; base += gridDim.x * RPB) {
    const int tt = base + (int)threadIdx.x / TRSV_LANES;
    const bool ok = tt < nrows;
    const int t = r0 + (ok ? tt : 0);
    const int e0 = ptr[t], e1 = ptr[t + 1];
    const int v = perm[t];
    const int dpos = LOWER ? e1 - 1 : e0;
    const int lo = LOWER ? e0 : e0 + 1, hi = LOWER ? e1 - 1 : e1;
    const int ia = lo + lane, ib = ia + TRSV_LANES;
    const int ca = ia < hi ? ia : dpos, cb = ib < hi ? ib : dpos;
    const double rv = rk[v];
    const double rhs = LOWER ? rv : yk[t];
    const double d = val[dpos];
    const double va = val[ca], vb = val[cb];
    const int ja = col[ca], jb = col[cb];
    // past the row's end the load re-reads the entry's own value (never a
    // location this launch writes) and the product is masked
    const double xa = *(ia < hi ? dep + ja : val + ca);
    const double xb = *(ib < hi ? dep + jb : val + cb);
    double s = (ia < hi ? va * xa : 0.0) + (ib < hi ? vb * xb : 0.0);
    for (int i = ib + TRSV_LANES; i < hi; i += TRSV_LANES) s += val[i] * dep[col[i]];
#pragma unroll
    for (int o = TRSV_LANES / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, TRSV_LANES);
    if (ok && lane == 0) {
      const double yt = (rhs - s) / d;
      if (LOWER && !TAIL) {
        yk[t] = yt;
      } else {
        const double ut = TAIL ? yt / d : yt;
        puk[t] = ut;
        u[k * stride + v] = ut;
        acc += rv * ut;
      }
    }
  }
  if (LOWER && !TAIL) return;
  if (part) {
    double s1[1] = {acc};
    gofd_cg::block_sum_n<256, 1>(s1, sh);
    if (threadIdx.x == 0) {
      double* p = part + (long long)k * nbu + blockIdx.x;
      *p = TAIL ? s1[0] : *p + s1[0];
    }
  }
}

// Block multicolour order: at most BMC_BLOCK rows per block, one wave per
// block, four lanes per row; lane (i, q) of a wave holds row i's entries
// (i, q + 4m), m = 0..3, of the block's own matrix (layout of the block
// arrays: (j / 4) * 64 + i * 4 + j % 4).
constexpr int BMC_BLOCK = 16;

// x + x from the lane given by a quad permutation (DPP, no LDS): quad_perm
// [1,0,3,2] (0xB1) adds the neighbour at xor 1, [2,3,0,1] (0x4E) at xor 2
template <int CTRL>
__device__ __forceinline__ double quad_add(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return x + __hiloint2double(hi, lo);
}

// x_i = sum_j m_ij b_j over the block (m the inverse of the block's own
// triangle): lane (i, q) fetches b of rows q + 4m from their lanes, adds its
// four products, and the row's four lanes add their sums
__device__ __forceinline__ double block_product(const double (&m4)[4], double b, int q) {
  double p = 0.0;
#pragma unroll
  for (int m = 0; m < 4; ++m) p = fma(m4[m], __shfl(b, 4 * (q + 4 * m)), p);
  return quad_add<0x4E>(quad_add<0xB1>(p));
}

// Sum over slabs a < min(NS, ns) of a block's entries to other blocks, in slab
// order, added to s0: lane i * 4 + q adds entry q + 4a of row i, w * dep[col]
// (col -1 marks padding).  All NS column and value loads are issued before any
// value of dep is read; slabs past ns re-read slab ns - 1 (cached) and padding
// re-reads `pad` (the row's value of r, never a location the launch writes),
// their products masked.
template <int NS, class IP, class FP>
__device__ __forceinline__ double slab_sum(IP ecol, FP eval, int e0, int ns, int lane, const double* dep,
                                           const double* pad, double s0 = 0.0) {
  int cc[NS];
  float w[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    const int idx = e0 + min(a, ns - 1) * 64 + lane;
    cc[a] = ecol[idx];
    w[a] = eval[idx];
  }
  double x[NS];
#pragma unroll
  for (int a = 0; a < NS; ++a) x[a] = *(a < ns && cc[a] >= 0 ? dep + cc[a] : pad);
  double s = s0;
#pragma unroll
  for (int a = 0; a < NS; ++a) s += (a < ns && cc[a] >= 0) ? (double)w[a] * x[a] : 0.0;
  return s;
}

// One item (problem, right-hand side) of the block multicolour solves: its
// factor's arrays (see gofd_precond_s), its colour table (colour c is blocks
// cbeg[c]..cbeg[c+1]-1, ncol colours) and its vectors at off.
struct BmcItem {
  const int* bs;
  const int* cbeg;
  const int* eoffL;
  const int* ecolL;
  const float* evalL;
  const int* eoffU;
  const int* ecolU;
  const float* evalU;
  const float* binvL;
  const float* binvU;
  const int* perm;
  long long off;
  int item, ncol;
};

// One colour of the triangular solves in block multicolour order, for every
// item of the launch (blockIdx.y): the item's blocks of colour c (rows
// bs[b]..bs[b+1]-1 of its factor's order, row t is vertex perm[t]) depend only
// on blocks of colours that earlier launches solved.  A wave takes one block
// at a time (four per workgroup, grid-stride): the lanes of a row add the
// row's entries to other blocks (the block's slabs of 64 entries,
// eoff[b]..eoff[b+1]-1, lane i * 4 + q of slab a holding entry q + 4a of row i
// or -1; all of them or four at a time in flight, see WIDE below), giving b_t,
// and the block's rows then follow from the inverse of its own triangle
// (formed on the host; values in single precision, arithmetic in double):
//   LOWER:  y = L_bb^{-1} (r[perm] - L_b,other y_other).  On the item's last
//           colour the wave goes on to the block's rows of U = L^T, which need
//           no other block: u = U_bb^{-1} y.
//   upper:  u = U_bb^{-1} (y - U_b,other u_other)   (colours below the last).
// A solved u goes to pu (factor order, read by later colours) and to u[perm]
// (vertex order); with part given, workgroup w adds r[perm t] u_t of its rows
// to the item's partial w of gamma (part + item * nbu), the last colour's
// launch storing instead and clearing the partials past its grid, so that
// after colour 0 the item's nbu partials hold (r, u) in a fixed order.
//
// trsv_block_item: the work of one workgroup on one item, blocks b0..b1-1 of
// the item's colour, the last colour's upper rows too when tail.  WIDE: all
// slabs of a block in flight at once (launches of one problem, bound by the
// latency of their few rounds of loads); otherwise four at a time, in fewer
// registers (launches over many items, bound by how many waves fit).
template <bool LOWER, bool WIDE>
__device__ __forceinline__ void trsv_block_item(const int* __restrict__ bs_, const int* __restrict__ eoff_,
                                                const int* __restrict__ ecol_, const float* __restrict__ eval_,
                                                const float* __restrict__ binv_, const float* __restrict__ binvU_,
                                                const int* __restrict__ perm_, long long off, int item, bool tail,
                                                int b0, int b1, const double* __restrict__ r, double* __restrict__ y,
                                                double* __restrict__ pu, double* __restrict__ u,
                                                double* __restrict__ part, int nbu, const Scal* __restrict__ sc,
                                                double* sh) {
  // A finished item stores nothing (with sc given; callers that test the flag
  // themselves pass none); its flag, the upper block inverse of the last
  // colour and the partial this workgroup adds to are all read up front and
  // waited for only where used, so that each launch waits for three rounds
  // of loads (block ranges, then indices and inverses, then values).
  const bool done = sc && sc[item].done;              // block-uniform
  const bool accum = part && !tail && !LOWER;         // upper colours below the last add to their partial
  double pprev = 0.0;
  if (accum && threadIdx.x == 0) pprev = part[(long long)item * nbu + blockIdx.x];
  // the pointers as global ones (loads through them are global, not flat)
  const auto bs = gmem(bs_);
  const auto eoff = gmem(eoff_);
  const auto ecol = gmem(ecol_);
  const auto eval = gmem(eval_);
  const auto binv = gmem(binv_);
  const auto perm = gmem(perm_);
  const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
  const int i = lane >> 2, q = lane & 3;
  const double* rk = r + off;
  double* yk = y + off;
  double* puk = pu + off;
  const double* dep = LOWER ? yk : puk;
  double acc = 0.0;
  for (int kb = b0 + (int)blockIdx.x * 4 + wave; kb < b1; kb += (int)gridDim.x * 4) {
    const int t0 = bs[kb], nb = bs[kb + 1] - t0;
    const int e0 = eoff[kb], ns = (eoff[kb + 1] - e0) >> 6;
    const bool ok = i < nb;
    const int t = t0 + (ok ? i : 0);
    const int v = perm[t];
    const double rv = rk[v];
    const double rhs = LOWER ? rv : yk[t];
    double m4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) m4[a] = (double)binv[(long long)kb * (BMC_BLOCK * BMC_BLOCK) + a * 64 + lane];
    double m4u[4] = {0.0, 0.0, 0.0, 0.0};
    if (tail) {
      const auto binvU = gmem(binvU_);
#pragma unroll
      for (int a = 0; a < 4; ++a) m4u[a] = (double)binvU[(long long)kb * (BMC_BLOCK * BMC_BLOCK) + a * 64 + lane];
    }
    // WIDE: the block's slabs all in flight at once (up to 16; a block with more goes on four at a time), so
    // that a launch waits for one round of column loads and one of values whatever the block's slab count
    double s = 0.0;
    int a0 = 0;
    if constexpr (WIDE) {
      if (ns > 8) s = slab_sum<16>(ecol, eval, e0, ns, lane, dep, rk + v);
      else if (ns > 4) s = slab_sum<8>(ecol, eval, e0, ns, lane, dep, rk + v);
      else if (ns > 0) s = slab_sum<4>(ecol, eval, e0, ns, lane, dep, rk + v);
      a0 = 16;
    }
    for (; a0 < ns; a0 += 4) s = slab_sum<4>(ecol, eval, e0 + a0 * 64, ns - a0, lane, dep, rk + v, s);
    s = quad_add<0x4E>(quad_add<0xB1>(s));
    double xi = block_product(m4, ok ? rhs - s : 0.0, q);
    if (tail) xi = block_product(m4u, ok ? xi : 0.0, q);
    if (done) break;
    if (ok && q == 0) {
      if (LOWER && !tail) {
        yk[t] = xi;
      } else {
        puk[t] = xi;
        u[off + v] = xi;
        acc += rv * xi;
      }
    }
  }
  if (done || !part || (LOWER && !tail)) return;      // block-uniform
  double s1[1] = {acc};
  gofd_cg::block_sum_n<256, 1>(s1, sh);
  if (threadIdx.x == 0) {
    double* p = part + (long long)item * nbu;
    p[blockIdx.x] = accum ? pprev + s1[0] : s1[0];
    if (tail && blockIdx.x == 0)
      for (int w = gridDim.x; w < nbu; ++w) p[w] = 0.0;
  }
}

// One problem's items (blockIdx.y = right-hand side k, item i0 + k, vectors
// at off0 + k * stride), its factor's arrays and the colour's block range as
// arguments; TAIL on the problem's last colour.
template <bool LOWER, bool TAIL>
__global__ __launch_bounds__(256) void k_trsv_block(const int* __restrict__ bs, int b0, int b1,
                                                    const int* __restrict__ eoff, const int* __restrict__ ecol,
                                                    const float* __restrict__ eval, const float* __restrict__ binv,
                                                    const float* __restrict__ binvU, const int* __restrict__ perm,
                                                    const double* __restrict__ r, double* __restrict__ y,
                                                    double* __restrict__ pu, double* __restrict__ u, long long off0,
                                                    long long stride, int i0, const Scal* __restrict__ sc,
                                                    double* __restrict__ part, int nbu) {
  __shared__ double sh[gofd_cg::block_sum_lds<256, 1>()];
  const int item = i0 + (int)blockIdx.y;
  trsv_block_item<LOWER, true>(bs, eoff, ecol, eval, binv, binvU, perm, off0 + blockIdx.y * stride, item, TAIL, b0,
                               b1, r, y, pu, u, part, nbu, sc, sh);
}

// Every item of the table (blockIdx.y) in one launch per colour c; an item
// without that colour in this direction returns at once.
template <bool LOWER>
__global__ __launch_bounds__(256) void k_trsv_block_items(const BmcItem* __restrict__ items, int c,
                                                          const double* __restrict__ r, double* __restrict__ y,
                                                          double* __restrict__ pu, double* __restrict__ u,
                                                          const Scal* __restrict__ sc, double* __restrict__ part,
                                                          int nbu) {
  __shared__ double sh[gofd_cg::block_sum_lds<256, 1>()];
  const BmcItem I = items[blockIdx.y];                // a kernel argument: global, scalar loads
  // most workgroups of a launch over many items belong to items that have
  // finished: those return before any other load
  if (sc && sc[I.item].done) return;                  // block-uniform
  if (LOWER ? c >= I.ncol : c > I.ncol - 2) return;   // the item has no such colour in this direction
  const int b0 = gmem(I.cbeg)[c], b1 = gmem(I.cbeg)[c + 1];
  trsv_block_item<LOWER, false>(I.bs, LOWER ? I.eoffL : I.eoffU, LOWER ? I.ecolL : I.ecolU,
                                LOWER ? I.evalL : I.evalU, LOWER ? I.binvL : I.binvU, I.binvU, I.perm, I.off, I.item,
                                LOWER && c == I.ncol - 1, b0, b1, r, y, pu, u, part, nbu, nullptr, sh);
}

// out[i] = in[perm[i]] (to = true) or out[perm[i]] = in[i], per right-hand side blockIdx.y
template <bool TO>
__global__ void k_permute(const double* __restrict__ in, const int* __restrict__ perm, long long n,
                          long long stride, const Scal* __restrict__ sc, double* __restrict__ out) {
  const int k = blockIdx.y;
  if (sc && sc[k].done) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (TO) out[k * stride + i] = in[k * stride + perm[i]];
  else out[k * stride + perm[i]] = in[k * stride + i];
}

// gamma = (r, u): nbu partials per right-hand side (blockIdx.y), block b over a grid-stride slice
__global__ __launch_bounds__(BS) void k_dot_rhs(const double* __restrict__ r, const double* __restrict__ u,
                                                long long n, long long stride, const Scal* __restrict__ sc,
                                                double* __restrict__ partG, int nbu) {
  __shared__ double sh[gofd_cg::block_sum_lds<BS, 1>()];
  const int k = blockIdx.y;
  if (sc && sc[k].done) return;
  double s[1] = {0.0};
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < n; i += (long long)nbu * BS)
    s[0] += r[k * stride + i] * u[k * stride + i];
  block_sum_n<BS, 1>(s, sh);
  if (threadIdx.x == 0) partG[(long long)k * nbu + blockIdx.x] = s[0];
}

__global__ void k_fill_d(double* __restrict__ p, long long n, double v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------- preconditioner handle

struct gofd_precond_s {
  int kind = 0;
  int64_t nv = 0;
  DevBuf Lptr, Lcol, Lval, Uptr, Ucol, Uval;
  DevBuf Llev_ptr, Llev_rows, Ulev_ptr, Ulev_rows;   // rows grouped by dependency level
  int Lnlev = 0, Unlev = 0;
  std::vector<int32_t> hLptr, hLcol;
  std::vector<double> hLval;
  // multicolour order: factor row i is vertex perm[i] (vectors are permuted
  // around the solves); few levels, so each level is its own launch
  DevBuf perm;
  std::vector<int32_t> hperm;
  std::vector<int32_t> hLlp, hUlp;   // level boundaries (host copies for the per-level launches)
  std::vector<int32_t> hcp;          // multicolour order: rows of colour c are hcp[c]..hcp[c+1]-1
  // block multicolour order: block b is rows hbs[b]..hbs[b+1]-1, colour c is
  // blocks hbc[c]..hbc[c+1]-1; on the device the block starts, each block's
  // entries to other blocks in slabs of 64 (offsets Leptr / Ueptr per block,
  // Lecol / Uecol and values: rows of L, resp. of U = L^T) and the inverse of
  // each block's own triangle, dense (bL: L_bb^{-1}, bU: U_bb^{-1}; 256 per
  // block, value (i, j) at ((j / 4) * 64 + i * 4 + j % 4), the register layout
  // of the solve); values stored in single precision, the solves in double
  std::vector<int32_t> hbs, hbc;
  DevBuf bs, cbeg, Leptr, Lecol, Leval, Ueptr, Uecol, Ueval, bL, bU;
  gofd_precond_info info{};
};

// levels at most this many: one launch per level over the whole device; more:
// one workgroup per right-hand side with a barrier per level
constexpr int TRSV_LEVEL_LAUNCH_MAX = 64;

// the block factor's device arrays (see gofd_precond_s); synchronises the
// stream before the host copies go out of scope
static int upload_block_factor(gofd_ctx_s* ctx, gofd_precond_s* pc, const std::vector<int64_t>& Lptr,
                               const std::vector<int32_t>& Lcol, const std::vector<double>& Lval,
                               const std::vector<int32_t>& Uptr, const std::vector<int32_t>& Ucol,
                               const std::vector<double>& Uval) {
  const int64_t n = (int64_t)Lptr.size() - 1;
  const int nb = (int)pc->hbs.size() - 1;
  constexpr int BS_ = BMC_BLOCK, BB = BMC_BLOCK * BMC_BLOCK;
  static_assert(BMC_BLOCK == 16, "a wave holds a block: sixteen rows of four lanes");
  std::vector<int32_t> fb(n);
  for (int b = 0; b < nb; ++b)
    for (int t = pc->hbs[b]; t < pc->hbs[b + 1]; ++t) fb[t] = b;
  auto slot = [](int i, int j) { return (j / 4) * 64 + i * 4 + (j % 4); };
  std::vector<float> binv((size_t)nb * BB, 0.0f), binvU((size_t)nb * BB, 0.0f);
  std::vector<int32_t> eoffL(nb + 1, 0), eoffU(nb + 1, 0), ecL, ecU;
  std::vector<float> evL, evU;
  std::vector<std::vector<std::pair<int32_t, double>>> extL(BS_), extU(BS_);
  for (int b = 0; b < nb; ++b) {
    const int t0 = pc->hbs[b], m = pc->hbs[b + 1] - t0;
    // the block's own triangle (rows of L inside the block, diagonal included) and the entries to other blocks
    double Lb[BS_][BS_] = {};
    for (int i = 0; i < m; ++i) {
      const int64_t t = t0 + i;
      extL[i].clear();
      extU[i].clear();
      for (int64_t e = Lptr[t]; e < Lptr[t + 1]; ++e) {
        const int32_t j = Lcol[e];
        if (fb[j] == b) Lb[i][j - t0] = Lval[e];
        else extL[i].push_back({j, Lval[e]});
      }
      for (int64_t e = Uptr[t] + 1; e < Uptr[t + 1]; ++e)
        if (fb[Ucol[e]] != b) extU[i].push_back({Ucol[e], Uval[e]});
    }
    // its inverse, column by column by forward substitution (lower triangular); that of U_bb = L_bb^T is the
    // transpose
    for (int c = 0; c < m; ++c) {
      double x[BS_] = {};
      for (int i = c; i < m; ++i) {
        double acc = (i == c) ? 1.0 : 0.0;
        for (int j = c; j < i; ++j) acc -= Lb[i][j] * x[j];
        x[i] = acc / Lb[i][i];
      }
      for (int i = c; i < m; ++i) {
        binv[(size_t)b * BB + slot(i, c)] = (float)x[i];
        binvU[(size_t)b * BB + slot(c, i)] = (float)x[i];
      }
    }
    // slabs of 64: lane i * 4 + q of slab a holds entry q + 4a of row i (col -1: none)
    auto slabs = [&](std::vector<std::vector<std::pair<int32_t, double>>>& ext, std::vector<int32_t>& off,
                     std::vector<int32_t>& ec, std::vector<float>& ev) {
      size_t mx = 0;
      for (int i = 0; i < m; ++i) mx = std::max(mx, ext[i].size());
      const int ns = (int)((mx + 3) / 4);
      for (int a = 0; a < ns; ++a)
        for (int lane = 0; lane < 64; ++lane) {
          const int i = lane / 4, e = lane % 4 + 4 * a;
          const bool has = i < m && e < (int)ext[i].size();
          ec.push_back(has ? ext[i][e].first : -1);
          ev.push_back(has ? (float)ext[i][e].second : 0.0f);
        }
      off[b + 1] = (int32_t)ec.size();
    };
    slabs(extL, eoffL, ecL, evL);
    slabs(extU, eoffU, ecU, evU);
  }
  if (ecL.size() >= (size_t)1 << 31 || ecU.size() >= (size_t)1 << 31)
    return gofd_fail(ctx, GOFD_E_OOM, "block factor too large");
  // algorithmic bytes of one application (the layout's padding left out)
  int64_t ext = 0;
  for (int32_t c : ecL) ext += c >= 0;
  for (int32_t c : ecU) ext += c >= 0;
  pc->info.apply_bytes = 8 * ext + 2 * (int64_t)nb * BB * (int64_t)sizeof(float) + 3 * 4 * (int64_t)(nb + 1) +
                         2 * 4 * n + 7 * 8 * n;
  hipStream_t st = ctx->stream;
  auto up = [&](DevBuf& d, const void* h, size_t bytes) -> int {
    GOFD_TRY(dev_reserve(ctx, d, std::max<size_t>(bytes, 8)));
    if (bytes) HIP_TRY(ctx, hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, st));
    return GOFD_OK;
  };
  GOFD_TRY(up(pc->bs, pc->hbs.data(), sizeof(int32_t) * pc->hbs.size()));
  GOFD_TRY(up(pc->cbeg, pc->hbc.data(), sizeof(int32_t) * pc->hbc.size()));
  GOFD_TRY(up(pc->Leptr, eoffL.data(), sizeof(int32_t) * eoffL.size()));
  GOFD_TRY(up(pc->Lecol, ecL.data(), sizeof(int32_t) * ecL.size()));
  GOFD_TRY(up(pc->Leval, evL.data(), sizeof(float) * evL.size()));
  GOFD_TRY(up(pc->Ueptr, eoffU.data(), sizeof(int32_t) * eoffU.size()));
  GOFD_TRY(up(pc->Uecol, ecU.data(), sizeof(int32_t) * ecU.size()));
  GOFD_TRY(up(pc->Ueval, evU.data(), sizeof(float) * evU.size()));
  GOFD_TRY(up(pc->bL, binv.data(), sizeof(float) * binv.size()));
  GOFD_TRY(up(pc->bU, binvU.data(), sizeof(float) * binvU.size()));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return GOFD_OK;
}

static int host_transfer(gofd_ctx_s* ctx, gofd_transfer_s* tr, HostTransfer& h) {
  hipStream_t st = ctx->stream;
  h.d = tr->d;
  h.W = tr->W;
  h.nv = tr->nv;
  h.n_nodes = tr->n_nodes;
  h.elem.resize(tr->n_nodes);
  h.elems = tr->elems_host;
  h.bnd = tr->bmask_host;
  h.csc_off.resize(tr->nv + 1);
  h.csc_node.resize(tr->nnz);
  h.csc_w.resize(tr->nnz);
  h.node_w.resize(tr->n_nodes * (tr->d + 1));
  DevBuf tmp;
  GOFD_TRY(dev_reserve(ctx, tmp, sizeof(double) * tr->n_nodes * (tr->d + 1)));
  GOFD_TRY(gofd_transfer_export(ctx, tr, GOFD_TR_ELL_WEIGHTS, tmp.p));
  HIP_TRY(ctx, hipMemcpyAsync(h.node_w.data(), tmp.p, sizeof(double) * h.node_w.size(), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(h.elem.data(), tr->elem.p, sizeof(int32_t) * tr->n_nodes, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(h.csc_off.data(), tr->csc_off.p, sizeof(int32_t) * (tr->nv + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(h.csc_node.data(), tr->csc_node.p, sizeof(int32_t) * tr->nnz, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(h.csc_w.data(), tr->csc_w.p, sizeof(double) * tr->nnz, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return GOFD_OK;
}

extern "C" int gofd_precond_create(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int kind, gofd_precond* out,
                                   gofd_precond_info* info) {
  if (!ctx || !tr || !op || !out) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  const auto t0 = std::chrono::steady_clock::now();
  auto* pc = new (std::nothrow) gofd_precond_s();
  if (!pc) return GOFD_E_OOM;
  std::unique_ptr<gofd_precond_s> guard(pc);
  pc->kind = kind;
  pc->nv = tr->nv;
  if (kind == GOFD_PC_NONE || kind == GOFD_PC_DIAG) {
    *out = guard.release();
    if (info) *info = pc->info;
    return GOFD_OK;
  }
  const bool mc = (kind & GOFD_PC_MULTICOLOR) != 0;
  const bool bmc = (kind & GOFD_PC_BLOCK_MULTICOLOR) != 0;
  const bool lap = (kind & GOFD_PC_LAPLACIAN) != 0;
  const int base = kind & ~(GOFD_PC_MULTICOLOR | GOFD_PC_BLOCK_MULTICOLOR | GOFD_PC_LAPLACIAN);
  if (mc && bmc) return gofd_fail(ctx, GOFD_E_ARG, "multicolour and block multicolour orders exclude each other");
  int npts = 0;
  if (base == GOFD_PC_IC1_5 && tr->d == 2) npts = 5;
  if (base == GOFD_PC_IC1_9 && tr->d == 2) npts = 9;
  if (base == GOFD_PC_IC1_27 && tr->d == 3) npts = 27;
  if (!npts) return gofd_fail(ctx, GOFD_E_ARG, "preconditioner kind does not match the dimension");
  HostTransfer ht;
  GOFD_TRY(host_transfer(ctx, tr, ht));
  HostCsr A;
  // the stencil values: A_FD's entries on the pattern, or (Laplacian kinds)
  // the discrete Laplacian on the same pattern, npts - 1 at the centre and -1
  // at every other point (5-point: the standard one; 9- and 27-point: the
  // isotropic compact ones, up to a factor)
  std::vector<double> lapT;
  if (lap) {
    lapT.assign(tr->d == 3 ? 8 : 4, -1.0);
    lapT[0] = npts - 1;
  }
  if (!assemble_pattern_matrix(ht, lap ? lapT.data() : op->T_host.data(), lap ? 2 : op->W, npts, A))
    return gofd_fail(ctx, GOFD_E_ARG, "pattern assembly failed");
  std::vector<int64_t> Lptr;
  std::vector<int32_t> Lcol;
  if (mc) {
    // greedy colouring of A's graph, vertices ordered by (colour, index); the
    // factor is computed for P A P^T with level-1 fill kept only between
    // vertices of different colours, so a colour's rows never depend on each other
    std::vector<int32_t> colour;
    pc->info.colours = greedy_colouring(A, colour);
    if (pc->info.colours > TRSV_LEVEL_LAUNCH_MAX)
      return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "multicolour order needs more than 64 colours");
    pc->hperm.resize(A.n);
    for (int64_t i = 0; i < A.n; ++i) pc->hperm[i] = (int32_t)i;
    std::stable_sort(pc->hperm.begin(), pc->hperm.end(),
                     [&](int32_t a, int32_t b) { return colour[a] < colour[b]; });
    HostCsr B;
    permute_symmetric(A, pc->hperm, B);
    A.rowptr.swap(B.rowptr);
    A.col.swap(B.col);
    A.val.swap(B.val);
    std::vector<int32_t> pcol(A.n);
    for (int64_t i = 0; i < A.n; ++i) pcol[i] = colour[pc->hperm[i]];
    colour.swap(pcol);
    pc->hcp.assign(pc->info.colours + 1, 0);
    for (int64_t i = 0; i < A.n; ++i) pc->hcp[colour[i] + 1]++;
    for (int c = 0; c < pc->info.colours; ++c) pc->hcp[c + 1] += pc->hcp[c];
    ic_symbolic(A, 1, Lptr, Lcol);
    drop_same_colour(colour, Lptr, Lcol);
  } else if (bmc) {
    // blocks of at most BMC_BLOCK vertices grown breadth first, the graph of
    // the blocks coloured in smallest-last order, vertices ordered by (block colour, block,
    // vertex); the level-1 fill is kept inside a block and between colours,
    // so the blocks of one colour are never coupled in the factor
    std::vector<int32_t> blk;
    const int nb = grow_blocks(A, BMC_BLOCK, blk);
    HostCsr G;
    block_graph(A, blk, nb, G);
    std::vector<int32_t> bcol;
    pc->info.colours = smallest_last_colouring(G, bcol);
    if (pc->info.colours > TRSV_LEVEL_LAUNCH_MAX)
      return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "block multicolour order needs more than 64 colours");
    pc->hperm.resize(A.n);
    for (int64_t i = 0; i < A.n; ++i) pc->hperm[i] = (int32_t)i;
    std::stable_sort(pc->hperm.begin(), pc->hperm.end(), [&](int32_t a, int32_t b) {
      return bcol[blk[a]] != bcol[blk[b]] ? bcol[blk[a]] < bcol[blk[b]] : blk[a] < blk[b];
    });
    HostCsr B;
    permute_symmetric(A, pc->hperm, B);
    A.rowptr.swap(B.rowptr);
    A.col.swap(B.col);
    A.val.swap(B.val);
    std::vector<int32_t> pblk(A.n), pcol(A.n);
    for (int64_t i = 0; i < A.n; ++i) {
      pblk[i] = blk[pc->hperm[i]];
      pcol[i] = bcol[pblk[i]];
    }
    // blocks in the factor's order (contiguous runs) and each colour's blocks
    pc->hbs.assign(1, 0);
    pc->hbc.assign(1, 0);
    for (int64_t i = 1; i <= A.n; ++i)
      if (i == A.n || pblk[i] != pblk[i - 1]) {
        if (i < A.n && pcol[i] != pcol[i - 1]) pc->hbc.push_back((int32_t)pc->hbs.size());
        pc->hbs.push_back((int32_t)i);
      }
    pc->hbc.push_back((int32_t)pc->hbs.size() - 1);
    ic_symbolic(A, 1, Lptr, Lcol);
    drop_same_colour(pcol, Lptr, Lcol, &pblk);
  } else {
    ic_symbolic(A, 1, Lptr, Lcol);
  }
  std::vector<double> Lval;
  double alpha = 0.0;
  while (!ic_numeric(A, alpha, Lptr, Lcol, Lval)) {
    alpha = alpha == 0.0 ? 1e-3 : 2.0 * alpha;
    if (alpha > 1e3) return gofd_fail(ctx, GOFD_E_BREAKDOWN, "incomplete Cholesky failed for every shift");
  }
  const int64_t n = tr->nv, nnz = (int64_t)Lcol.size();
  if (nnz >= (1LL << 31)) return gofd_fail(ctx, GOFD_E_OOM, "factor too large");
  pc->hLptr.assign(Lptr.begin(), Lptr.end());
  pc->hLcol = Lcol;
  pc->hLval = Lval;
  // transpose: U = L^T in CSR (diagonal first in every row)
  std::vector<int32_t> Uptr(n + 1, 0), Ucol(nnz);
  std::vector<double> Uval(nnz);
  for (int64_t e = 0; e < nnz; ++e) Uptr[Lcol[e] + 1]++;
  for (int64_t i = 0; i < n; ++i) Uptr[i + 1] += Uptr[i];
  {
    std::vector<int32_t> cur(Uptr.begin(), Uptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t e = Lptr[i]; e < Lptr[i + 1]; ++e) {
        const int32_t c = Lcol[e];
        Ucol[cur[c]] = (int32_t)i;
        Uval[cur[c]++] = Lval[e];
      }
  }
  // dependency levels: forward solve on L (rows depend on smaller columns),
  // backward solve on U = L^T (rows depend on larger columns)
  std::vector<int32_t> Llp, Llr, Ulp, Ulr;
  {
    std::vector<int> lev(n, 0);
    int depth = 0;
    for (int64_t i = 0; i < n; ++i) {
      int l = 0;
      for (int64_t e = Lptr[i]; e < Lptr[i + 1] - 1; ++e) l = std::max(l, lev[Lcol[e]] + 1);
      lev[i] = l;
      depth = std::max(depth, l + 1);
    }
    Llp.assign(depth + 1, 0);
    for (int64_t i = 0; i < n; ++i) Llp[lev[i] + 1]++;
    for (int l = 0; l < depth; ++l) Llp[l + 1] += Llp[l];
    Llr.resize(n);
    std::vector<int32_t> cur(Llp.begin(), Llp.end() - 1);
    for (int64_t i = 0; i < n; ++i) Llr[cur[lev[i]]++] = (int32_t)i;
    pc->Lnlev = depth;
    pc->info.levels = depth;
    std::fill(lev.begin(), lev.end(), 0);
    depth = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
      int l = 0;
      for (int64_t e = Uptr[i] + 1; e < Uptr[i + 1]; ++e) l = std::max(l, lev[Ucol[e]] + 1);
      lev[i] = l;
      depth = std::max(depth, l + 1);
    }
    Ulp.assign(depth + 1, 0);
    for (int64_t i = 0; i < n; ++i) Ulp[lev[i] + 1]++;
    for (int l = 0; l < depth; ++l) Ulp[l + 1] += Ulp[l];
    Ulr.resize(n);
    std::vector<int32_t> cur2(Ulp.begin(), Ulp.end() - 1);
    for (int64_t i = 0; i < n; ++i) Ulr[cur2[lev[i]]++] = (int32_t)i;
    pc->Unlev = depth;
    pc->hLlp = Llp;
    pc->hUlp = Ulp;
  }
  hipStream_t st = ctx->stream;
  if (bmc) GOFD_TRY(upload_block_factor(ctx, pc, Lptr, Lcol, Lval, Uptr, Ucol, Uval));
  if (mc || bmc) {
    GOFD_TRY(dev_reserve(ctx, pc->perm, sizeof(int32_t) * n));
    HIP_TRY(ctx, hipMemcpyAsync(pc->perm.p, pc->hperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  }
  GOFD_TRY(dev_reserve(ctx, pc->Lptr, sizeof(int32_t) * (n + 1)));
  GOFD_TRY(dev_reserve(ctx, pc->Lcol, sizeof(int32_t) * nnz));
  GOFD_TRY(dev_reserve(ctx, pc->Lval, sizeof(double) * nnz));
  GOFD_TRY(dev_reserve(ctx, pc->Uptr, sizeof(int32_t) * (n + 1)));
  GOFD_TRY(dev_reserve(ctx, pc->Ucol, sizeof(int32_t) * nnz));
  GOFD_TRY(dev_reserve(ctx, pc->Uval, sizeof(double) * nnz));
  GOFD_TRY(dev_reserve(ctx, pc->Llev_ptr, sizeof(int32_t) * Llp.size()));
  GOFD_TRY(dev_reserve(ctx, pc->Llev_rows, sizeof(int32_t) * n));
  GOFD_TRY(dev_reserve(ctx, pc->Ulev_ptr, sizeof(int32_t) * Ulp.size()));
  GOFD_TRY(dev_reserve(ctx, pc->Ulev_rows, sizeof(int32_t) * n));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Lptr.p, pc->hLptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Lcol.p, Lcol.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Lval.p, Lval.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Uptr.p, Uptr.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Ucol.p, Ucol.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Uval.p, Uval.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Llev_ptr.p, Llp.data(), sizeof(int32_t) * Llp.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Llev_rows.p, Llr.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Ulev_ptr.p, Ulp.data(), sizeof(int32_t) * Ulp.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(pc->Ulev_rows.p, Ulr.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  pc->info.shift = alpha;
  pc->info.nnz_L = nnz;
  pc->info.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = pc->info;
  *out = guard.release();
  return GOFD_OK;
}

extern "C" int gofd_precond_free(gofd_precond pc) {
  if (!pc) return GOFD_E_ARG;
  (void)hipDeviceSynchronize();
  delete pc;
  return GOFD_OK;
}

extern "C" int gofd_precond_export_order(gofd_ctx ctx, gofd_precond pc, int32_t* perm) {
  if (!ctx || !pc || !perm) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  if (pc->hLptr.empty()) return gofd_fail(ctx, GOFD_E_ARG, "preconditioner has no factor");
  for (int64_t i = 0; i < pc->nv; ++i) perm[i] = pc->hperm.empty() ? (int32_t)i : pc->hperm[i];
  return GOFD_OK;
}

extern "C" int gofd_precond_export(gofd_ctx ctx, gofd_precond pc, int32_t* rowptr, int32_t* cols, double* vals) {
  if (!ctx || !pc || !rowptr || !cols || !vals) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  if (pc->hLptr.empty()) return gofd_fail(ctx, GOFD_E_ARG, "preconditioner has no factor");
  std::memcpy(rowptr, pc->hLptr.data(), sizeof(int32_t) * pc->hLptr.size());
  std::memcpy(cols, pc->hLcol.data(), sizeof(int32_t) * pc->hLcol.size());
  std::memcpy(vals, pc->hLval.data(), sizeof(double) * pc->hLval.size());
  return GOFD_OK;
}

// ---------------------------------------------------------------- solve driver

namespace {

struct Problem {
  gofd_transfer_s* tr;
  gofd_fdop_s* op;
  gofd_precond_s* pc;   // may be null
  int nrhs;
};

bool is_ic(const gofd_precond_s* pc) {
  const int base = pc ? (pc->kind & ~(GOFD_PC_MULTICOLOR | GOFD_PC_BLOCK_MULTICOLOR | GOFD_PC_LAPLACIAN)) : 0;
  return pc && (base == GOFD_PC_IC1_5 || base == GOFD_PC_IC1_9 || base == GOFD_PC_IC1_27);
}

// 1: diagonal (D_h), 0: none, -1: IC(1) factor
int diag_kind_of(const gofd_precond_s* pc) {
  return is_ic(pc) ? -1 : ((pc && pc->kind == GOFD_PC_DIAG) ? 1 : 0);
}

// A batch: problems of one grid shape (d, W, L), solved together.  Items are
// (problem, rhs) pairs in problem order; the vectors of all items are laid
// end to end (item i at off[i], N_v of its mesh entries each).
// a non-owning view of device memory
struct DevView {
  void* p = nullptr;
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// the batch descriptors (CgItem array and spectrum pointer tables) on the
// device, and their page-locked staging copy; kept in the context
struct BatchBufs {
  DevBuf desc;
  void* stage = nullptr;
  size_t stage_bytes = 0;
  ~BatchBufs() {
    if (stage) (void)hipHostFree(stage);
  }
};
static BatchBufs& ctx_batch(gofd_ctx_s* ctx);

struct Batch {
  std::vector<Problem> probs;
  std::vector<long long> poff;     // offset of problem q's first vector
  std::vector<int> pitem;          // first item of problem q
  std::vector<long long> ioff;     // offset of item i
  std::vector<long long> inv;      // N_v of item i
  int nitems = 0;
  long long ntot = 0, nv_max = 0;
  bool any_ic = false;
  bool rp = true;                  // every transfer has the row-pair form of I^T
  bool seg = true;                 // ... and the per-node segment rows (FP32 gather through the slots)
  long long slots_max = 0;         // most partial slots of an item
  int rp_ent_ahead = 0;            // entries of a thread the last row pass reads ahead (largest of the items)
  gofd_fdop_s* op0 = nullptr;      // shape and FFT workspaces of the batch
  DevView items, tab64, tab32;     // CgItem[nitems]; spectrum pointer tables (in the context's buffers)
  // items preconditioned in block multicolour order: their descriptors, the
  // most colours among them and, per colour, the most blocks of one item
  DevView bmc;
  int nbmc = 0, bmc_cols = 0;
  std::vector<int> bmc_blocks;
  int nbmc_probs = 0, bmc_prob = -1;  // problems with such items; the (last) one of them
};

int batch_init(gofd_ctx_s* ctx, Batch& B, const std::vector<Problem>& probs) {
  B.probs = probs;
  B.op0 = probs[0].op;
  std::vector<CgItem> h;
  std::vector<const void*> t64, t32;
  long long off = 0;
  for (const Problem& P : probs) {
    gofd_transfer_s* tr = P.tr;
    if (P.op->d != B.op0->d || P.op->W != B.op0->W || P.op->L != B.op0->L)
      return gofd_fail(ctx, GOFD_E_ARG, "internal: batch with different grid shapes");
    B.poff.push_back(off);
    B.pitem.push_back((int)h.size());
    B.any_ic = B.any_ic || is_ic(P.pc);
    B.nv_max = std::max<long long>(B.nv_max, tr->nv);
    B.rp = B.rp && tr->rp_ok;
    B.seg = B.seg && tr->rp_ok && tr->seg_rows_ok;
    B.slots_max = std::max<long long>(B.slots_max, tr->n_slots);
    B.rp_ent_ahead = std::max(B.rp_ent_ahead, tr->rp_ent_ahead);
    for (int k = 0; k < P.nrhs; ++k) {
      CgItem I{};
      I.csc_off = tr->csc_off.as<int>();
      I.csc_node = tr->csc_node.as<int>();
      I.csc_w = tr->csc_w.as<double>();
      I.csc_w32 = tr->csc_w32.as<float>();
      I.imask = tr->imask.as<double>();
      I.dscale = tr->dscale.as<double>();
      I.recs = tr->rec.p;
      I.elem = tr->elem.as<int>();
      I.ell_idx = tr->ell_idx.as<int>();
      I.ell_v = tr->ell_v.as<int4>();
      I.ell_w = tr->ell_w.as<double2>();
      I.row32_v = tr->row32_v.as<int4>();
      I.row32_w = tr->row32_w.as<float2>();
      if (tr->rp_ok) {
        I.rp_meta = tr->rp_meta.as<int>();
        I.rp_tseg = tr->rp_tseg.as<int>();
        I.rp_code = tr->rp_code.as<unsigned short>();
        I.rp_w32 = tr->rp_w32.as<float>();
        I.rp_w64 = tr->rp_w64.as<double>();
        I.rp_dest = tr->rp_dest.as<int>();
        I.pv_off = tr->pv_off.as<int>();
        if (tr->seg_rows_ok) {
          I.rp_pos = tr->rp_pos.as<int>();
          I.seg_row = tr->seg_row.as<int4>();
          I.seg_row_w2 = tr->seg_row_w2.as<float>();
        }
      }
      I.g.d = tr->d;
      I.g.W = tr->W;
      I.g.h = tr->h;
      for (int a = 0; a < 3; ++a) I.g.lo[a] = tr->lo[a];
      I.nv = tr->nv;
      I.off = off;
      I.dk = diag_kind_of(P.pc);
      h.push_back(I);
      t64.push_back(P.op->That64.p);
      t32.push_back(P.op->That32.p);
      B.ioff.push_back(off);
      B.inv.push_back(tr->nv);
      off += tr->nv;
    }
  }
  B.nitems = (int)h.size();
  B.ntot = off;
  std::vector<BmcItem> hb;
  for (size_t q = 0; q < probs.size(); ++q) {
    const gofd_precond_s* pc = probs[q].pc;
    if (!is_ic(pc) || pc->hbc.empty()) continue;
    const int C = (int)pc->hbc.size() - 1;
    B.bmc_cols = std::max(B.bmc_cols, C);
    if ((int)B.bmc_blocks.size() < C) B.bmc_blocks.resize(C, 0);
    for (int c = 0; c < C; ++c) B.bmc_blocks[c] = std::max(B.bmc_blocks[c], pc->hbc[c + 1] - pc->hbc[c]);
    for (int k = 0; k < probs[q].nrhs; ++k) {
      BmcItem e{};
      e.bs = pc->bs.as<int>();
      e.cbeg = pc->cbeg.as<int>();
      e.eoffL = pc->Leptr.as<int>();
      e.ecolL = pc->Lecol.as<int>();
      e.evalL = pc->Leval.as<float>();
      e.eoffU = pc->Ueptr.as<int>();
      e.ecolU = pc->Uecol.as<int>();
      e.evalU = pc->Ueval.as<float>();
      e.binvL = pc->bL.as<float>();
      e.binvU = pc->bU.as<float>();
      e.perm = pc->perm.as<int>();
      e.item = B.pitem[q] + k;
      e.off = B.ioff[e.item];
      e.ncol = C;
      hb.push_back(e);
    }
  }
  B.nbmc = (int)hb.size();
  for (size_t q = 0; q < probs.size(); ++q)
    if (is_ic(probs[q].pc) && !probs[q].pc->hbc.empty()) {
      ++B.nbmc_probs;
      B.bmc_prob = (int)q;
    }
  B.seg = B.seg && B.rp && !B.any_ic;        // IC(1) makes u in its own kernels
  // one block [CgItem x n | void* x n | void* x n | BmcItem x nbmc], staged in
  // page-locked memory (the previous solve on the context has finished with
  // it) and copied in one transfer, without waiting for it
  const size_t n = h.size(), o64 = sizeof(CgItem) * n, o32 = o64 + sizeof(void*) * n, ob = o32 + sizeof(void*) * n,
               bytes = ob + sizeof(BmcItem) * hb.size();
  BatchBufs& bb = ctx_batch(ctx);
  if (bb.stage_bytes < bytes) {
    if (bb.stage) (void)hipHostFree(bb.stage);
    bb.stage = nullptr;
    bb.stage_bytes = 0;
    HIP_TRY(ctx, hipHostMalloc(&bb.stage, bytes, hipHostMallocDefault));
    bb.stage_bytes = bytes;
  }
  char* sp = static_cast<char*>(bb.stage);
  std::memcpy(sp, h.data(), o64);
  std::memcpy(sp + o64, t64.data(), o32 - o64);
  std::memcpy(sp + o32, t32.data(), ob - o32);
  if (!hb.empty()) std::memcpy(sp + ob, hb.data(), bytes - ob);
  GOFD_TRY(dev_reserve(ctx, bb.desc, bytes));
  HIP_TRY(ctx, hipMemcpyAsync(bb.desc.p, bb.stage, bytes, hipMemcpyHostToDevice, ctx->stream));
  B.items.p = bb.desc.p;
  B.tab64.p = static_cast<char*>(bb.desc.p) + o64;
  B.tab32.p = static_cast<char*>(bb.desc.p) + o32;
  B.bmc.p = hb.empty() ? nullptr : static_cast<char*>(bb.desc.p) + ob;
  return GOFD_OK;
}

struct Work {
  DevBuf x, r, u, p, s, b, xr, dvec, q, grid;
  DevBuf pr, pu;                // r and u in a preconditioner's multicolour order
  DevBuf P;                     // row-pair form: partial slots, double[nitems][slots_max]
  DevBuf us;                    // with the segment rows: u per slot, float[nitems][slots_max] (row-pair-major)
  DevBuf amap;                  // int[nitems]: the items still iterating (first nact entries)
  DevBuf rmap;                  // int[nitems]: the items of a residual replacement
  int nact = 0;                 // items the iteration's launches cover
  DevBuf scal;                  // Scal[nitems]
  DevBuf partG, partR;          // double[nitems][nbs]: gamma and (r, r) partials
  DevBuf partD;                 // double[nitems][3][pass-B blocks]: partials summed by the column pass
  DevBuf partials, out2;        // residual partials, ||r||^2 and ||b||^2
  int nbs = 1;                  // blocks of the CG vector kernels (scatter, start) per item
  int per = 1;                  // vertex groups per scatter block
  // warm start (gofd_solve with an initial guess): w.b holds b - K x0 and the
  // tolerance refers to (b, b) of the original right-hand sides, per item
  DevBuf bref;
  const double* bref_on = nullptr;   // device copy while a warm-started solve runs, else null
  std::vector<double> bref_host;
};

// the context's solver workspace and batch descriptors (made on first use,
// freed with the context; one solve at a time uses them)
struct SolverCache {
  Work w;
  BatchBufs b;
};
static SolverCache& ctx_cache(gofd_ctx_s* ctx) {
  if (!ctx->solver_ws) {
    ctx->solver_ws = new SolverCache();
    ctx->solver_ws_free = [](void* p) { delete static_cast<SolverCache*>(p); };
  }
  return *static_cast<SolverCache*>(ctx->solver_ws);
}
static Work& ctx_work(gofd_ctx_s* ctx) { return ctx_cache(ctx).w; }
static BatchBufs& ctx_batch(gofd_ctx_s* ctx) { return ctx_cache(ctx).b; }

int reserve_work(gofd_ctx_s* ctx, Work& w, const Batch& B) {
  const size_t vb = sizeof(double) * std::max<long long>(B.ntot, 1);
  for (DevBuf* b : {&w.x, &w.r, &w.u, &w.p, &w.s, &w.b, &w.xr, &w.dvec, &w.q}) GOFD_TRY(dev_reserve(ctx, *b, vb));
  if (B.any_ic)
    for (DevBuf* b : {&w.pr, &w.pu}) GOFD_TRY(dev_reserve(ctx, *b, vb));
  long long nn = 1;
  for (int a = 0; a < B.op0->d; ++a) nn *= B.op0->W;
  const int ni = B.nitems;
  GOFD_TRY(dev_reserve(ctx, w.grid, sizeof(double) * nn * ni));
  GOFD_TRY(dev_reserve(ctx, w.scal, sizeof(Scal) * ni));
  if (B.rp) {
    // vertex kernel: one vertex per thread
    GOFD_TRY(dev_reserve(ctx, w.P, sizeof(double) * std::max<long long>(B.slots_max, 1) * ni));
    if (B.seg) GOFD_TRY(dev_reserve(ctx, w.us, sizeof(float) * std::max<long long>(B.slots_max, 1) * ni));
    w.per = 1;
    w.nbs = (int)std::max<long long>(1, (B.nv_max + BS - 1) / BS);
  } else {
    const long long groups = (B.nv_max + BS / SCAT_G - 1) / (BS / SCAT_G);
    w.per = (int)std::max<long long>(1, (groups + MAX_SC - 1) / MAX_SC);
    w.nbs = (int)std::max<long long>(1, (groups + w.per - 1) / w.per);
  }
  GOFD_TRY(dev_reserve(ctx, w.partG, sizeof(double) * w.nbs * ni));
  GOFD_TRY(dev_reserve(ctx, w.partR, sizeof(double) * w.nbs * ni));
  GOFD_TRY(dev_reserve(ctx, w.partials, sizeof(double) * 2 * NB_DOT * ni));
  GOFD_TRY(dev_reserve(ctx, w.amap, sizeof(int) * ni));
  GOFD_TRY(dev_reserve(ctx, w.rmap, sizeof(int) * ni));
  w.nact = ni;
  GOFD_TRY(dev_reserve(ctx, w.out2, sizeof(double) * 2 * ni));
  return GOFD_OK;
}

long long grid_nodes(const gofd_fdop_s* op) {
  long long nn = 1;
  for (int a = 0; a < op->d; ++a) nn *= op->W;
  return nn;
}

// FP64 product of x through the row-pair form into the partial slots (the
// last row pass sums each vertex's entries per row pair), for replacements
// (with map given: only the n items map[0..n) of the batch)
int apply_K_slots(gofd_ctx_s* ctx, const Batch& B, Work& w, const double* v, const int* map, int n) {
  GatherSpec g;
  g.items = B.items.as<CgItem>();
  g.ubase = v;
  g.items_mask = true;
  g.amap = map;
  g.that64_tab = static_cast<const void* const*>(B.tab64.p);
  g.that32_tab = static_cast<const void* const*>(B.tab32.p);
  g.rp_P = w.P.as<double>();
  g.rp_pstride = std::max<long long>(B.slots_max, 1);
  g.rp_ent_ahead = B.rp_ent_ahead;
  return conv_apply(ctx, B.op0, n, nullptr, &g, w.grid.p, false);
}

// q = K v for every item in double precision (masked), for true residuals;
// v and q are batch vectors
// (with map given: only the n items map[0..n) of the batch)
int apply_K_plain(gofd_ctx_s* ctx, const Batch& B, Work& w, const double* v, double* q, const int* map = nullptr,
                  int n = -1) {
  if (n < 0) n = B.nitems;
  GatherSpec g;
  g.items = B.items.as<CgItem>();
  g.ubase = v;
  g.items_mask = true;
  g.amap = map;
  g.that64_tab = static_cast<const void* const*>(B.tab64.p);
  g.that32_tab = static_cast<const void* const*>(B.tab32.p);
  GOFD_TRY(conv_apply(ctx, B.op0, n, nullptr, &g, w.grid.p, false));
  dim3 gs(grid1(B.nv_max * SCAT_G, BS), n);
  hipLaunchKernelGGL((k_scatter_plain<SCAT_G>), gs, dim3(BS), 0, ctx->stream, B.items.as<CgItem>(),
                     w.grid.as<double>(), grid_nodes(B.op0), q, map);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

// u = M^{-1} r with the IC(1) factor of every IC problem; the upper solve also
// writes the partials of gamma = (r, u) into partG (if given)
int precond_apply(gofd_ctx_s* ctx, const Batch& B, Work& w, const Scal* sc, double* partG) {
  hipStream_t st = ctx->stream;
  if (B.nbmc) {
    // the items in block multicolour order: one launch per colour and direction for all of them (an item's
    // last colour solves its lower and upper rows in one launch); grids of at most nbs workgroups, the
    // partials' count
    auto grid = [&](int c) {
      return dim3((unsigned)std::max(1, std::min(w.nbs, (B.bmc_blocks[c] + 3) / 4)), (unsigned)B.nbmc);
    };
    if (B.nbmc_probs == 1) {
      // one problem: its arrays and block ranges as arguments (no descriptor loads)
      const Problem& P = B.probs[B.bmc_prob];
      const gofd_precond_s* pc = P.pc;
      const int C = (int)pc->hbc.size() - 1;
      const long long o = B.poff[B.bmc_prob], n = P.tr->nv;
      const int i0 = B.pitem[B.bmc_prob];
      // (a launch that writes the partials covers all nbs of them)
      auto g1 = [&](int c, bool partials) {
        return dim3(partials ? (unsigned)w.nbs : (unsigned)std::max(1, (pc->hbc[c + 1] - pc->hbc[c] + 3) / 4),
                    P.nrhs);
      };
      for (int c = 0; c < C; ++c) {
        const int b0 = pc->hbc[c], b1 = pc->hbc[c + 1];
        if (c + 1 < C)
          hipLaunchKernelGGL((k_trsv_block<true, false>), g1(c, false), dim3(256), 0, st, pc->bs.as<int>(), b0, b1,
                             pc->Leptr.as<int>(), pc->Lecol.as<int>(), pc->Leval.as<float>(), pc->bL.as<float>(),
                             nullptr, pc->perm.as<int>(), w.r.as<double>(), w.dvec.as<double>(), w.pu.as<double>(),
                             w.u.as<double>(), o, n, i0, sc, nullptr, w.nbs);
        else
          hipLaunchKernelGGL((k_trsv_block<true, true>), g1(c, partG != nullptr), dim3(256), 0, st, pc->bs.as<int>(),
                             b0, b1,
                             pc->Leptr.as<int>(), pc->Lecol.as<int>(), pc->Leval.as<float>(), pc->bL.as<float>(),
                             pc->bU.as<float>(), pc->perm.as<int>(), w.r.as<double>(), w.dvec.as<double>(),
                             w.pu.as<double>(), w.u.as<double>(), o, n, i0, sc, partG, w.nbs);
      }
      for (int c = C - 2; c >= 0; --c)
        hipLaunchKernelGGL((k_trsv_block<false, false>), g1(c, partG != nullptr), dim3(256), 0, st, pc->bs.as<int>(),
                           pc->hbc[c],
                           pc->hbc[c + 1], pc->Ueptr.as<int>(), pc->Uecol.as<int>(), pc->Ueval.as<float>(),
                           pc->bU.as<float>(), nullptr, pc->perm.as<int>(), w.r.as<double>(), w.dvec.as<double>(),
                           w.pu.as<double>(), w.u.as<double>(), o, n, i0, sc, partG, w.nbs);
    } else {
      const BmcItem* items = B.bmc.as<BmcItem>();
      for (int c = 0; c < B.bmc_cols; ++c)
        hipLaunchKernelGGL(k_trsv_block_items<true>, grid(c), dim3(256), 0, st, items, c, w.r.as<double>(),
                           w.dvec.as<double>(), w.pu.as<double>(), w.u.as<double>(), sc, partG, w.nbs);
      for (int c = B.bmc_cols - 2; c >= 0; --c)
        hipLaunchKernelGGL(k_trsv_block_items<false>, grid(c), dim3(256), 0, st, items, c, w.r.as<double>(),
                           w.dvec.as<double>(), w.pu.as<double>(), w.u.as<double>(), sc, partG, w.nbs);
    }
  }
  for (size_t q = 0; q < B.probs.size(); ++q) {
    const Problem& P = B.probs[q];
    if (!is_ic(P.pc)) continue;
    gofd_precond_s* pc = P.pc;
    const long long n = P.tr->nv, o = B.poff[q];
    const int i0 = B.pitem[q];
    const Scal* scq = sc ? sc + i0 : nullptr;
    if (!pc->hbc.empty()) continue;                   // block multicolour: all items together above
    if (!pc->hcp.empty() && (int)pc->hcp.size() - 1 <= TRSV_LEVEL_LAUNCH_MAX) {
      // multicolour order: one launch per colour and direction, the last
      // colour's upper rows solved in the last lower launch; the permutation
      // and gamma's partials are part of the launches
      const int C = (int)pc->hcp.size() - 1;
      const double* rin = w.r.as<double>() + o;
      double* y = w.dvec.as<double>() + o;
      double* pu = w.pu.as<double>() + o;
      double* u = w.u.as<double>() + o;
      double* part = partG ? partG + (long long)i0 * w.nbs : nullptr;
      const int* perm_d = pc->perm.as<int>();
      auto grid_rows = [&](int rows) {
        return dim3(part ? w.nbs : grid1((long long)std::max(rows, 1) * TRSV_LANES, 256), P.nrhs);
      };
      for (int c = 0; c + 1 < C; ++c) {
        const int r0 = pc->hcp[c], r1 = pc->hcp[c + 1];
        hipLaunchKernelGGL((k_trsv_colour<true, false>), dim3(grid1((long long)std::max(r1 - r0, 1) * TRSV_LANES, 256), P.nrhs),
                           dim3(256), 0, st, pc->Lptr.as<int>(), pc->Lcol.as<int>(), pc->Lval.as<double>(), perm_d, r0,
                           r1, rin, y, pu, u, n, scq, nullptr, 0);
      }
      hipLaunchKernelGGL((k_trsv_colour<true, true>), grid_rows(pc->hcp[C] - pc->hcp[C - 1]), dim3(256), 0, st,
                         pc->Lptr.as<int>(), pc->Lcol.as<int>(), pc->Lval.as<double>(), perm_d, pc->hcp[C - 1],
                         pc->hcp[C], rin, y, pu, u, n, scq, part, w.nbs);
      for (int c = C - 2; c >= 0; --c) {
        const int r0 = pc->hcp[c], r1 = pc->hcp[c + 1];
        hipLaunchKernelGGL((k_trsv_colour<false, false>), grid_rows(r1 - r0), dim3(256), 0, st, pc->Uptr.as<int>(),
                           pc->Ucol.as<int>(), pc->Uval.as<double>(), perm_d, r0, r1, rin, y, pu, u, n, scq, part,
                           w.nbs);
      }
      continue;
    }
    if (pc->Lnlev <= TRSV_LEVEL_LAUNCH_MAX && pc->Unlev <= TRSV_LEVEL_LAUNCH_MAX) {
      // few levels: one launch per level over the device; vectors in the
      // factor's order when it has one (pr, pu: permuted r and u)
      const bool perm = !pc->hperm.empty();
      const double* rin = w.r.as<double>() + o;
      double* uout = w.u.as<double>() + o;
      const dim3 gp(grid1(n, 256), P.nrhs);
      if (perm) {
        hipLaunchKernelGGL(k_permute<true>, gp, dim3(256), 0, st, rin, pc->perm.as<int>(), n, n, scq,
                           w.pr.as<double>() + o);
        rin = w.pr.as<double>() + o;
        uout = w.pu.as<double>() + o;
      }
      for (int l = 0; l < pc->Lnlev; ++l) {
        const int r0 = pc->hLlp[l], r1 = pc->hLlp[l + 1];
        hipLaunchKernelGGL(k_trsv_level<true>, dim3(grid1((long long)(r1 - r0) * TRSV_LANES, 256), P.nrhs), dim3(256), 0, st,
                           pc->Lptr.as<int>(), pc->Lcol.as<int>(), pc->Lval.as<double>(), pc->Llev_rows.as<int>(), r0,
                           r1, rin, w.dvec.as<double>() + o, n, scq);
      }
      for (int l = 0; l < pc->Unlev; ++l) {
        const int r0 = pc->hUlp[l], r1 = pc->hUlp[l + 1];
        hipLaunchKernelGGL(k_trsv_level<false>, dim3(grid1((long long)(r1 - r0) * TRSV_LANES, 256), P.nrhs), dim3(256), 0, st,
                           pc->Uptr.as<int>(), pc->Ucol.as<int>(), pc->Uval.as<double>(), pc->Ulev_rows.as<int>(), r0,
                           r1, w.dvec.as<double>() + o, uout, n, scq);
      }
      if (perm)
        hipLaunchKernelGGL(k_permute<false>, gp, dim3(256), 0, st, uout, pc->perm.as<int>(), n, n, scq,
                           w.u.as<double>() + o);
      if (partG)
        hipLaunchKernelGGL(k_dot_rhs, dim3(w.nbs, P.nrhs), dim3(BS), 0, st, w.r.as<double>() + o,
                           w.u.as<double>() + o, n, n, scq, partG + (long long)i0 * w.nbs, w.nbs);
      continue;
    }
    hipLaunchKernelGGL((k_trsv_levels<true>), dim3(P.nrhs), dim3(1024), 0, st, pc->Lptr.as<int>(),
                       pc->Lcol.as<int>(), pc->Lval.as<double>(), pc->Llev_ptr.as<int>(), pc->Llev_rows.as<int>(),
                       pc->Lnlev, w.r.as<double>() + o, w.dvec.as<double>() + o, n, scq, nullptr, nullptr, w.nbs);
    hipLaunchKernelGGL((k_trsv_levels<false>), dim3(P.nrhs), dim3(1024), 0, st, pc->Uptr.as<int>(),
                       pc->Ucol.as<int>(), pc->Uval.as<double>(), pc->Ulev_ptr.as<int>(), pc->Ulev_rows.as<int>(),
                       pc->Unlev, w.dvec.as<double>() + o, w.u.as<double>() + o, n, scq, w.r.as<double>() + o,
                       partG ? partG + (long long)i0 * w.nbs : nullptr, w.nbs);
  }
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

// Per-stage timing of the iterations (no graph): every stage's kernel is
// launched with the extended launch that records a start and an end event on
// the library's stream at the kernel's own start and end; the two
// triangular solves of IC(1) are bracketed by ordinary events.
struct StageProf {
  hipEvent_t ev[2 * GOFD_N_STAGES] = {};      // start and end of each stage
  double sum[GOFD_N_STAGES] = {};
  int cnt[GOFD_N_STAGES] = {};
  bool ok = false;
  explicit StageProf(bool on) {
    if (!on) return;
    ok = true;
    for (auto& e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
  }
  ~StageProf() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void write(double* out) const {
    for (int i = 0; i < GOFD_N_STAGES; ++i) out[i] = cnt[i] ? sum[i] / cnt[i] : 0.0;
  }
};

// One CG iteration of the whole batch: product w = K u (gather, FFT passes
// with the delta partials and the step decision, scatter with the vector
// update), then for IC(1) problems the triangular solves u = M^{-1} r with
// the next gamma.
// whether the FP32 gather of the iterations reads u per slot
static bool seg_gather(const Batch& B, bool fp32) { return B.rp && B.seg && fp32 && conv_gather_fused(B.op0, fp32); }

// u per slot from u (before the first iteration and after a replacement;
// with map given only the n items map[0..n))
static void refresh_slots(gofd_ctx_s* ctx, const Batch& B, Work& w, bool fp32, const int* map = nullptr,
                          int n = -1) {
  if (!seg_gather(B, fp32)) return;
  hipLaunchKernelGGL(k_u_to_slots, dim3(w.nbs, n < 0 ? B.nitems : n), dim3(BS), 0, ctx->stream,
                     B.items.as<CgItem>(), w.u.as<double>(), w.us.as<float>(), std::max<long long>(B.slots_max, 1),
                     map);
}

// With host_out given, the step decision also stores the state there.
int cg_iteration(gofd_ctx_s* ctx, const Batch& B, Work& w, bool fp32, StageProf* prof = nullptr,
                 Scal* host_out = nullptr) {
  hipStream_t st = ctx->stream;
  GatherSpec g;
  g.items = B.items.as<CgItem>();
  g.ubase = w.u.as<double>();
  g.items_mask = false;             // CG keeps every Dirichlet entry of u at zero
  g.that64_tab = static_cast<const void* const*>(B.tab64.p);
  g.that32_tab = static_cast<const void* const*>(B.tab32.p);
  g.skip = &w.scal.as<Scal>()->done;
  g.skip_stride = (int)(sizeof(Scal) / sizeof(int));
  const int* amap = w.nact < B.nitems ? w.amap.as<int>() : nullptr;   // the items still iterating
  g.amap = amap;
  g.dpart = w.partD.as<double>();
  g.lv1.partG = w.partG.as<double>();
  g.lv1.partR = w.partR.as<double>();
  g.lv1.n1 = w.nbs;
  g.fin.sc = w.scal.as<Scal>();
  g.fin.part = w.partD.as<double>();
  g.fin.nb = conv_passB_blocks(B.op0, fp32);
  g.fin.host = host_out;
  if (B.rp) {
    g.rp_P = w.P.as<double>();
    g.rp_pstride = std::max<long long>(B.slots_max, 1);
    g.rp_ent_ahead = B.rp_ent_ahead;
    if (seg_gather(B, fp32)) g.rp_us = w.us.as<float>();
  }
  if (prof) {
    // the same launches one stage at a time, each kernel recording its own
    // start and end events
    // (a gather that runs inside the first row pass is timed with it)
    static const int stage_passes[4] = {8, 1, 2, 4};
    const bool fused = conv_gather_fused(B.op0, fp32);
    for (int k = 0; k < 4; ++k) {
      if (k == GOFD_ST_GATHER && fused) continue;
      ctx->timer_start = prof->ev[2 * k];
      ctx->timer_stop = prof->ev[2 * k + 1];
      GOFD_TRY(conv_apply(ctx, B.op0, w.nact, nullptr, &g, w.grid.p, fp32,
                          stage_passes[k] | (k == GOFD_ST_PASS_A && fused ? 8 : 0)));
      ctx->timer_start = ctx->timer_stop = nullptr;
    }
    ctx->timer_start = prof->ev[8];
    ctx->timer_stop = prof->ev[9];
  } else {
    GOFD_TRY(conv_apply(ctx, B.op0, w.nact, nullptr, &g, w.grid.p, fp32));
  }
  const dim3 gs(w.nbs, w.nact);
  const long long nn = grid_nodes(B.op0);
#define GOFD_SCATTER_ARGS(Y)                                                                                     \
  B.items.as<CgItem>(), Y, nn, w.scal.as<Scal>(), w.x.as<double>(), w.p.as<double>(), w.s.as<double>(),          \
      w.r.as<double>(), w.u.as<double>(), w.per, w.partG.as<double>(), w.partR.as<double>(), amap
  if (B.rp)
    GOFD_LAUNCH(ctx, k_vertex_cg, gs, dim3(BS), 0, st, B.items.as<CgItem>(), w.P.as<double>(), g.rp_pstride,
                w.scal.as<Scal>(), w.x.as<double>(), w.p.as<double>(), w.s.as<double>(), w.r.as<double>(),
                w.u.as<double>(), w.partG.as<double>(), w.partR.as<double>(), amap, g.rp_us ? w.us.as<float>() : nullptr);
  else if (fp32)
    GOFD_LAUNCH(ctx, (k_scatter_cg<float, float, SCAT_G>), gs, dim3(BS), 0, st, GOFD_SCATTER_ARGS(w.grid.as<float>()));
  else
    GOFD_LAUNCH(ctx, (k_scatter_cg<double, double, SCAT_G>), gs, dim3(BS), 0, st,
                GOFD_SCATTER_ARGS(w.grid.as<double>()));
#undef GOFD_SCATTER_ARGS
  HIP_TRY(ctx, hipGetLastError());
  if (prof) {
    ctx->timer_start = ctx->timer_stop = nullptr;
    if (B.any_ic) HIP_TRY(ctx, hipEventRecord(prof->ev[10], st));
  }
  if (B.any_ic) GOFD_TRY(precond_apply(ctx, B, w, w.scal.as<Scal>(), w.partG.as<double>()));
  if (prof) {
    if (B.any_ic) HIP_TRY(ctx, hipEventRecord(prof->ev[11], st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int k = 0; k < GOFD_N_STAGES; ++k) {
      if (k == GOFD_ST_PRECOND && !B.any_ic) continue;
      if (k == GOFD_ST_GATHER && conv_gather_fused(B.op0, fp32)) continue;
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, prof->ev[2 * k], prof->ev[2 * k + 1]));
      prof->sum[k] += ms;
      prof->cnt[k] += 1;
    }
  }
  return GOFD_OK;
}

// CG from x = 0 on the batch right-hand sides w.b; result in w.x.  Returns
// per-item iterations and status through hs (host Scal copies).
//
// With replace_drop > 0 the recursively updated residual is replaced by the
// true one, r = b - K x with a double-precision product, whenever (r, r) has
// dropped by replace_drop^2 since its last replacement and whenever it stops
// on its recursive residual (reliable updating), item by item; each item's
// count goes to n_replace[item].
int pcg_run(gofd_ctx_s* ctx, const Batch& B, Work& w, double tol, bool fp32, int max_iter, int check_every,
            bool use_graph, std::vector<Scal>& hs, double* history, double replace_drop = 0.0,
            int* n_replace = nullptr, StageProf* prof = nullptr) {
  hipStream_t st = ctx->stream;
  const int ni = B.nitems;
  if (n_replace) std::fill(n_replace, n_replace + ni, 0);
  GOFD_TRY(conv_prepare(ctx, B.op0, ni));
  GOFD_TRY(dev_reserve(ctx, w.partD, sizeof(double) * 3 * conv_passB_blocks(B.op0, fp32) * ni));
  if (B.any_ic) {
    // u = M^{-1} b before the start kernel (no state is read: pass none)
    HIP_TRY(ctx, hipMemcpyAsync(w.r.p, w.b.p, sizeof(double) * B.ntot, hipMemcpyDeviceToDevice, st));
    GOFD_TRY(precond_apply(ctx, B, w, nullptr, nullptr));
  }
  hipLaunchKernelGGL(k_cg_start, dim3(w.nbs, ni), dim3(BS), 0, st, B.items.as<CgItem>(), w.b.as<double>(),
                     w.x.as<double>(), w.r.as<double>(), w.u.as<double>(), w.p.as<double>(), w.s.as<double>(),
                     w.partG.as<double>(), w.partR.as<double>());
  hipLaunchKernelGGL(k_cg_init, dim3(ni), dim3(BS), 0, st, w.partG.as<double>(), w.partR.as<double>(), w.nbs,
                     w.scal.as<Scal>(), tol, w.bref_on);
  refresh_slots(ctx, B, w, fp32);
  HIP_TRY(ctx, hipGetLastError());
  hs.resize(ni);
  check_every = std::max(1, check_every);
  if (prof) {
    use_graph = false;                // stages timed one by one, state read every iteration
    check_every = 1;
  }
  w.nact = ni;                          // every item iterates at the start
  // Page-locked state slots for the pipelined checks: chunk slots 0 and 1
  // (the last iteration of a chunk stores its state there) and slot 2 for a
  // residual replacement.
  const bool piped = !history && !prof;
  Scal* hb = nullptr;       // host view
  Scal* hd = nullptr;       // device view of the same memory
  if (piped) {
    const size_t need_bytes = sizeof(Scal) * 3 * (size_t)ni + sizeof(int) * (size_t)ni;
    if (ctx->host_state_bytes < need_bytes) {
      if (ctx->host_state) (void)hipHostFree(ctx->host_state);
      ctx->host_state = nullptr;
      ctx->host_state_bytes = 0;
      // coherent: the kernels' stores bypass the device caches
      HIP_TRY(ctx, hipHostMalloc(&ctx->host_state, need_bytes, hipHostMallocCoherent));
      ctx->host_state_bytes = need_bytes;
    }
    hb = static_cast<Scal*>(ctx->host_state);
    HIP_TRY(ctx, hipHostGetDevicePointer((void**)&hd, ctx->host_state, 0));
  }
  // one chunk of n iterations whose last iteration stores the state into
  // chunk slot `slot` (none without the pipelined checks)
  auto chunk_launches = [&](int slot, int n) -> int {
    for (int j = 0; j < n; ++j)
      GOFD_TRY(cg_iteration(ctx, B, w, fp32, nullptr, (hd && j == n - 1) ? hd + (size_t)slot * ni : nullptr));
    return GOFD_OK;
  };
  // one graph executable per chunk slot, captured over the current item list
  // (graph replays keep its launch shapes); two chunks in flight use both
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  auto drop_graphs = [&]() {
    for (int k = 0; k < 2; ++k) {
      if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
      if (graph[k]) (void)hipGraphDestroy(graph[k]);
      exec[k] = nullptr;
      graph[k] = nullptr;
    }
  };
  auto capture = [&]() -> int {
    drop_graphs();
    for (int k = 0; k < 2; ++k) {
      if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        use_graph = false;
        drop_graphs();
        return GOFD_OK;
      }
      const int rc = chunk_launches(k, check_every);
      hipError_t e = hipStreamEndCapture(st, &graph[k]);
      if (rc != GOFD_OK) {
        drop_graphs();
        return rc;
      }
      if (e != hipSuccess || hipGraphInstantiate(&exec[k], graph[k], nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        drop_graphs();
        use_graph = false;
        return GOFD_OK;
      }
    }
    return GOFD_OK;
  };
  if (use_graph && piped) GOFD_TRY(capture());
  // Active items: once at most 7/8 of the items the launches cover still
  // iterate (or a replacement reopened one outside them), the launches are
  // narrowed to those items (block rows map to them) and the graph captured
  // again.  Stopped items would otherwise still occupy launch slots (narrowing
  // drains the stream once; at 1/2 the stopped items' blocks cost more).
  std::vector<char> in_map(ni, 1);
  std::vector<int> act_h;
  auto compact = [&](const std::vector<Scal>& st_) -> int {
    act_h.clear();
    bool missing = false;
    for (int k = 0; k < ni; ++k)
      if (st_[k].status == ST_OK && !st_[k].done) {
        act_h.push_back(k);
        missing = missing || !in_map[k];
      }
    if (act_h.empty() || (!missing && 8 * (int)act_h.size() > 7 * w.nact)) return GOFD_OK;
    HIP_TRY(ctx, hipStreamSynchronize(st));          // nothing in flight reads the old list
    HIP_TRY(ctx, hipMemcpyAsync(w.amap.p, act_h.data(), sizeof(int) * act_h.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    w.nact = (int)act_h.size();
    std::fill(in_map.begin(), in_map.end(), 0);
    for (int k : act_h) in_map[k] = 1;
    if (hb)                 // no launch stores the state of the items left out
      for (int k = 0; k < ni; ++k)
        if (!in_map[k]) hb[k] = hb[ni + k] = st_[k];
    if (use_graph) GOFD_TRY(capture());
    return GOFD_OK;
  };
  // residual replacement: true residual of x in double precision, then the
  // state's flags from it (reads the state back into tmp)
  std::vector<double> rr_ref(ni, HUGE_VAL);
  // items whose stop a replacement has confirmed with the true residual: they
  // trigger no further replacement
  std::vector<char> settled(ni, 0);
  // the launches of a replacement for the n items of map (every item with map
  // null): r = b - K x with an FP64 product (through the row-pair slots when
  // the batch has them), u = M r, the partials, u at the slots, and the
  // states (also into host, if given)
  auto replace_launch = [&](const int* map, int n, Scal* host) -> int {
    if (B.rp) {
      GOFD_TRY(apply_K_slots(ctx, B, w, w.x.as<double>(), map, n));
      hipLaunchKernelGGL(k_cg_replace_rp, dim3(w.nbs, n), dim3(BS), 0, st, B.items.as<CgItem>(), w.P.as<double>(),
                         std::max<long long>(B.slots_max, 1), w.b.as<double>(), w.r.as<double>(),
                         w.u.as<double>(), w.scal.as<Scal>(), w.partG.as<double>(), w.partR.as<double>(), map,
                         seg_gather(B, fp32) ? w.us.as<float>() : nullptr);
    } else {
      GOFD_TRY(apply_K_plain(ctx, B, w, w.x.as<double>(), w.q.as<double>(), map, n));
      hipLaunchKernelGGL(k_cg_replace, dim3(w.nbs, n), dim3(BS), 0, st, B.items.as<CgItem>(), w.b.as<double>(),
                         w.q.as<double>(), w.r.as<double>(), w.u.as<double>(), w.scal.as<Scal>(),
                         w.partG.as<double>(), w.partR.as<double>(), map);
      refresh_slots(ctx, B, w, fp32, map, n);
    }
    hipLaunchKernelGGL(k_cg_reopen, dim3(n), dim3(BS), 0, st, w.partR.as<double>(), w.nbs, w.scal.as<Scal>(), host,
                       map);
    HIP_TRY(ctx, hipGetLastError());
    if (B.any_ic) GOFD_TRY(precond_apply(ctx, B, w, w.scal.as<Scal>(), w.partG.as<double>()));
    return GOFD_OK;
  };
  auto replace_residual = [&](std::vector<Scal>& tmp) -> int {
    GOFD_TRY(replace_launch(nullptr, ni, nullptr));
    HIP_TRY(ctx, hipMemcpyAsync(tmp.data(), w.scal.p, sizeof(Scal) * ni, hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    for (int k = 0; k < ni; ++k) {
      rr_ref[k] = tmp[k].rr;
      settled[k] = tmp[k].done ? 1 : 0;
    }
    return GOFD_OK;
  };
  // Iteration j tests x_j (its last pass) and then applies step j, so after
  // `it` iterations `it` steps are applied unless the solve stopped earlier.
  int it = 0;
  int rc = GOFD_OK;
  std::vector<Scal> tmp(ni);
  if (history) history[0] = 1.0;
  // (until the first replacement the reference is the starting residual,
  // (r, r) = (b, b) from x = 0)
  // When one item needs a replacement, every item that has not had its stop
  // confirmed gets one (rsel): more frequent replacements keep each item's
  // recursive residual closer to its true one (an item replaced only at its
  // own triggers needed up to 70% more iterations in a batch).  Confirmed
  // items are left out of the FP64 product.
  std::vector<char> rsel(ni, 0);
  auto wants = [&](int k, const Scal& s) {
    if (rr_ref[k] == HUGE_VAL) rr_ref[k] = s.bb;
    return s.status == ST_OK && !settled[k] && (s.done || s.rr < replace_drop * replace_drop * rr_ref[k]);
  };
  auto need_replace = [&](const std::vector<Scal>& st_) {
    bool need = false;
    for (int k = 0; k < ni; ++k) need = wants(k, st_[k]) || need;
    for (int k = 0; k < ni; ++k) rsel[k] = need && st_[k].status == ST_OK && !settled[k];
    return need;
  };
  if (piped) {
    // Pipelined checks: up to two chunks of iterations in flight, the last
    // iteration of each storing the state into the chunk's page-locked slot
    // (with a mark per item that the host clears before the issue and polls
    // for); the host decides on the older chunk's state while the newer one
    // runs.  Items that stopped skip their work in the chunk run past their
    // stop.  A residual replacement (of the items whose stop is not yet
    // confirmed) is queued behind the chunks in flight and writes their states
    // into slot 2; the states of chunks issued before it are superseded and
    // not acted on.  Chunks issued after it run on, unless every item had
    // stopped or is close to its tolerance (the replacement may confirm the
    // stop).  Without a graph, chunks shrink to two iterations once every item
    // is within 100x of its tolerance in the residual norm, so that fewer
    // iterations run past a stop.

    // items whose state a launch into the slot writes: the items the chunk's
    // launches cover, or the items of the pending replacement
    auto expect = [&](int slot, int k) { return slot == 2 ? rsel[k] != 0 : in_map[k] != 0; };
    auto clear_marks = [&](int slot) {
      for (int k = 0; k < ni; ++k)
        if (expect(slot, k)) hb[(size_t)slot * ni + k].pad = 0;
    };
    // wait until every expected item of the slot carries its mark; a stream
    // that has gone idle (or failed) without them is an error
    auto wait_marks = [&](int slot) -> int {
      const volatile Scal* v = hb + (size_t)slot * ni;
      for (long long spin = 0;; ++spin) {
        bool ready = true;
        for (int k = 0; k < ni && ready; ++k)
          if (expect(slot, k)) ready = v[k].pad == 1;
        if (ready) break;
        if ((spin & 1023) == 1023) {
          const hipError_t q = hipStreamQuery(st);
          if (q == hipErrorNotReady) continue;
          if (q != hipSuccess) return gofd_fail(ctx, GOFD_E_HIP, "solver iterations failed");
          bool late = true;        // the stream is idle: the marks must be there now
          for (int k = 0; k < ni && late; ++k)
            if (expect(slot, k)) late = v[k].pad == 1;
          if (!late) return gofd_fail(ctx, GOFD_E_HIP, "solver state not written");
          break;
        }
        __builtin_ia32_pause();
      }
      std::atomic_thread_fence(std::memory_order_acquire);
      return GOFD_OK;
    };
    auto issue = [&](int slot, int n) -> int {
      clear_marks(slot);
      if (use_graph) {
        if (hipGraphLaunch(exec[slot], st) != hipSuccess) return gofd_fail(ctx, GOFD_E_HIP, "graph launch failed");
      } else {
        GOFD_TRY(chunk_launches(slot, n));
      }
      it += n;
      return GOFD_OK;
    };
    // the selected items' list goes to the device through page-locked memory
    // (read by the copy when the stream reaches it; one replacement at a time)
    int* hmap = reinterpret_cast<int*>(hb + 3 * (size_t)ni);
    auto issue_replace = [&]() -> int {
      clear_marks(2);
      int nr = 0;
      for (int k = 0; k < ni; ++k)
        if (rsel[k]) hmap[nr++] = k;
      const int* map = nullptr;
      if (nr < ni) {
        HIP_TRY(ctx, hipMemcpyAsync(w.rmap.p, hmap, sizeof(int) * nr, hipMemcpyHostToDevice, st));
        map = w.rmap.as<int>();
      }
      return replace_launch(map, nr, hd + 2 * (size_t)ni);
    };
    // every item stopped or within 100x of its tolerance (residual norm)
    auto near_stop = [&](const std::vector<Scal>& st_) {
      bool near = true;
      for (int k = 0; k < ni; ++k) near = near && (st_[k].done || st_[k].rr <= 1e4 * st_[k].tol2);
      return near;
    };
    std::deque<int> fl;      // slots of the launches in flight, in stream order
    int next = 0;            // chunk slot of the next chunk
    int nch = 0;             // chunks in flight
    int chunk = check_every; // iterations per chunk
    bool superseded = false; // a replacement is in flight
    bool hold = false;       // issue no chunk until the replacement's state is read
    while (rc == GOFD_OK) {
      while (!hold && nch < 2 && it < max_iter && rc == GOFD_OK) {
        rc = issue(next, use_graph ? check_every : chunk);
        fl.push_back(next);
        ++nch;
        next ^= 1;
      }
      if (rc != GOFD_OK || fl.empty()) break;
      const int slot = fl.front();
      fl.pop_front();
      if ((rc = wait_marks(slot)) != GOFD_OK) break;
      if (slot == 2) {
        // tmp keeps the other items' last chunk state
        for (int k = 0; k < ni; ++k)
          if (rsel[k]) {
            tmp[k] = hb[2 * (size_t)ni + k];
            rr_ref[k] = tmp[k].rr;
            settled[k] = tmp[k].done ? 1 : 0;
          }
        superseded = hold = false;
      } else {
        --nch;
        if (superseded) continue;
        std::copy(hb + (size_t)slot * ni, hb + (size_t)(slot + 1) * ni, tmp.begin());
        if (near_stop(tmp)) chunk = std::min(chunk, 2);
        if (replace_drop > 0.0 && need_replace(tmp)) {
          if ((rc = issue_replace()) != GOFD_OK) break;
          fl.push_back(2);
          superseded = true;
          if (n_replace)
            for (int k = 0; k < ni; ++k) n_replace[k] += rsel[k];
          hold = near_stop(tmp);
          continue;
        }
      }
      bool all = true;
      for (int k = 0; k < ni; ++k) all = all && tmp[k].done;
      if (all) break;
      const int before = w.nact;
      if ((rc = compact(tmp)) != GOFD_OK) break;
      if (w.nact != before) {                          // compact drained the stream
        fl.clear();
        nch = 0;
      }
    }
  }
  // residual history or stage timing: no graph, the state read after every
  // iteration (stage timing: every check_every, which it set to one)
  while (it < max_iter && !piped && rc == GOFD_OK) {
    const int chunk = history ? 1 : check_every;
    for (int j = 0; j < chunk && rc == GOFD_OK; ++j) rc = cg_iteration(ctx, B, w, fp32, prof);
    if (rc != GOFD_OK) break;
    it += chunk;
    if (hipMemcpyAsync(tmp.data(), w.scal.p, sizeof(Scal) * ni, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = gofd_fail(ctx, GOFD_E_HIP, "reading solver state failed");
      break;
    }
    // the state's rr is that of the iterate tested last: x_{it-1}
    if (history && it - 1 <= max_iter) history[it - 1] = tmp[0].bb > 0 ? std::sqrt(tmp[0].rr / tmp[0].bb) : 0.0;
    if (replace_drop > 0.0 && need_replace(tmp)) {
      if ((rc = replace_residual(tmp)) != GOFD_OK) break;
      if (n_replace)
        for (int k = 0; k < ni; ++k) n_replace[k] += (tmp[k].status == ST_OK) ? 1 : 0;
    }
    bool all = true;
    for (int k = 0; k < ni; ++k) all = all && tmp[k].done;
    if (all) break;
  }
  (void)hipStreamSynchronize(st);       // a chunk may still run: finish it before the graphs go
  drop_graphs();
  if (rc != GOFD_OK) return rc;
  // the final states (through the page-locked replacement slot when there is one)
  Scal* dst = hb ? hb + 2 * (size_t)ni : hs.data();
  HIP_TRY(ctx, hipMemcpyAsync(dst, w.scal.p, sizeof(Scal) * ni, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (hb) std::copy(dst, dst + ni, hs.begin());
  return GOFD_OK;
}

// true residual r = b - K x in double precision (batch vectors); returns
// ||r||^2 and ||b||^2 per item
int true_residual(gofd_ctx_s* ctx, const Batch& B, Work& w, const double* x, const double* b, double* r,
                  std::vector<double>& rr, std::vector<double>& bb) {
  const int ni = B.nitems;
  GOFD_TRY(conv_prepare(ctx, B.op0, ni));
  GOFD_TRY(apply_K_plain(ctx, B, w, x, w.q.as<double>()));
  dim3 gd(NB_DOT, ni);
  hipLaunchKernelGGL(k_residual, gd, dim3(BS), 0, ctx->stream, B.items.as<CgItem>(), b, w.q.as<double>(), r,
                     w.partials.as<double>());
  hipLaunchKernelGGL(k_residual_finish, dim3(ni), dim3(BS), 0, ctx->stream, w.partials.as<double>(),
                     w.out2.as<double>());
  std::vector<double> h(2 * ni);
  HIP_TRY(ctx, hipMemcpyAsync(h.data(), w.out2.p, sizeof(double) * 2 * ni, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  rr.resize(ni);
  bb.resize(ni);
  for (int k = 0; k < ni; ++k) {
    rr[k] = h[2 * k];
    bb[k] = h[2 * k + 1];
  }
  return GOFD_OK;
}

__global__ void k_mask_copy(const double* __restrict__ a, const double* __restrict__ mask, long long n,
                            double* __restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] * mask[i];
}

// b += mask a
__global__ void k_add_masked(const double* __restrict__ a, const double* __restrict__ mask, long long n,
                             double* __restrict__ b) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] += a[i] * mask[i];
}

// right-hand sides of problem q into the batch vector b
int form_rhs(gofd_ctx_s* ctx, const Problem& P, const double* f, int f_loc, double* b) {
  gofd_transfer_s* tr = P.tr;
  hipStream_t st = ctx->stream;
  if (f_loc == GOFD_F_GRID) {
    dim3 gs(grid1(tr->nv * SCAT_G, BS), P.nrhs);
    hipLaunchKernelGGL((k_rhs_grid<SCAT_G>), gs, dim3(BS), 0, st, tr->csc_off.as<int>(), tr->csc_node.as<int>(),
                       tr->csc_w.as<double>(), f, (long long)tr->nv, (long long)tr->n_nodes, tr->imask.as<double>(),
                       P.op->h2s, b);
  } else if (f_loc == GOFD_F_VERTEX) {
    dim3 gs(grid1(tr->nv, BS), P.nrhs);
    hipLaunchKernelGGL(k_rhs_vertex, gs, dim3(BS), 0, st, f, tr->D.as<double>(), tr->imask.as<double>(),
                       (long long)tr->nv, P.op->h2s, b);
  } else {
    return gofd_fail(ctx, GOFD_E_ARG, "f_loc must be GOFD_F_GRID or GOFD_F_VERTEX");
  }
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

}  // namespace

// Solve K u = b for the batch right-hand sides already formed in w.b; the
// solution of problem q goes to u_out[q] (nrhs_q * N_v doubles).
static int solve_system(gofd_ctx_s* ctx, const Batch& B, Work& w, double tol, const gofd_solve_opts* o,
                        double* const* u_out, gofd_solve_info* info) {
  const auto t0 = std::chrono::steady_clock::now();
  const int mode = o ? o->mode : GOFD_MODE_FP64;
  const int max_iter = (o && o->max_iter > 0) ? o->max_iter : 20000;
  const int check = (o && o->check_every > 0) ? o->check_every : 8;
  const bool graph = o ? o->use_graph != 0 : false;
  double* history = o ? o->history : nullptr;
  StageProf profobj(o && o->stage_ms);
  StageProf* prof = (o && o->stage_ms) ? &profobj : nullptr;
  if (prof && !prof->ok) return gofd_fail(ctx, GOFD_E_HIP, "event creation failed");
  const int ni = B.nitems;
  const long long ntot = B.ntot;
  hipStream_t st = ctx->stream;
  std::vector<Scal> hs;
  std::vector<int> iters(ni, 0), refs(ni, 0), status(ni, GOFD_OK);
  std::vector<double> rel(ni, 0.0);
  auto copy_out = [&](const double* src) -> int {
    for (size_t q = 0; q < B.probs.size(); ++q)
      HIP_TRY(ctx, hipMemcpyAsync(u_out[q], src + B.poff[q],
                                  sizeof(double) * B.probs[q].tr->nv * B.probs[q].nrhs, hipMemcpyDeviceToDevice, st));
    return GOFD_OK;
  };
  int rc = GOFD_OK;
  bool confirmed = false;         // final residuals known from the last replacements
  if (mode == GOFD_MODE_FP64 || mode == GOFD_MODE_FP32_RELIABLE) {
    const bool rel32 = mode == GOFD_MODE_FP32_RELIABLE;
    const double drop = rel32 ? ((o && o->inner_tol > 0) ? o->inner_tol : 1e-2) : 0.0;
    std::vector<int> nrep(ni, 0);
    rc = pcg_run(ctx, B, w, tol, rel32, max_iter, check, graph, hs, history, drop, nrep.data(), prof);
    if (rc != GOFD_OK) return rc;
    GOFD_TRY(copy_out(w.x.as<double>()));
    for (int k = 0; k < ni; ++k) {
      iters[k] = hs[k].iters;
      refs[k] = nrep[k];
      if (hs[k].status == ST_BREAKDOWN) status[k] = GOFD_E_BREAKDOWN;
      else if (!hs[k].done) status[k] = GOFD_E_NOT_CONVERGED;
    }
    // with reliable updating every stop was confirmed by a replacement, whose
    // (r, r) is that of b - K x in double precision for the x copied out (a
    // stopped item's x no longer changes)
    confirmed = rel32 && nrep.size() == (size_t)ni;
    for (int k = 0; k < ni && confirmed; ++k) confirmed = status[k] == GOFD_OK && nrep[k] > 0;
  } else if (mode == GOFD_MODE_FP32_REFINE) {
    const double inner = (o && o->inner_tol > 0) ? o->inner_tol : 1e-5;
    const int max_ref = (o && o->max_refine > 0) ? o->max_refine : 30;
    // xr = 0; r = b; loop
    DevBuf bsave;
    GOFD_TRY(dev_reserve(ctx, bsave, sizeof(double) * ntot));
    HIP_TRY(ctx, hipMemcpyAsync(bsave.p, w.b.p, sizeof(double) * ntot, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_fill_d, dim3(grid1(ntot, 256)), dim3(256), 0, st, w.xr.as<double>(), ntot, 0.0);
    std::vector<double> rr, bb;
    std::vector<char> conv(ni, 0);
    int total_it = 0;
    for (int ref = 0; ref <= max_ref; ++ref) {
      // true residual of the current iterate (b - K xr); first pass has xr = 0
      GOFD_TRY(true_residual(ctx, B, w, w.xr.as<double>(), bsave.as<double>(), w.b.as<double>(), rr, bb));
      if (w.bref_on) bb = w.bref_host;
      bool all = true;
      for (int k = 0; k < ni; ++k) {
        rel[k] = bb[k] > 0 ? std::sqrt(rr[k] / bb[k]) : 0.0;
        if (rel[k] <= tol) conv[k] = 1;
        all = all && conv[k];
      }
      if (all || ref == max_ref || total_it >= max_iter) break;
      // items already within the tolerance take no further correction: a zero right-hand side stops their
      // CG before the first iteration, so d = 0 and their x stays as it is
      for (int k = 0; k < ni; ++k)
        if (conv[k])
          hipLaunchKernelGGL(k_fill_d, dim3(grid1(B.inv[k], 256)), dim3(256), 0, st, w.b.as<double>() + B.ioff[k],
                             B.inv[k], 0.0);
      // correction: K d = r with single-precision grid products (tolerance relative to this r)
      const double* bref_keep = w.bref_on;
      w.bref_on = nullptr;
      rc = pcg_run(ctx, B, w, inner, true, max_iter - total_it, check, graph, hs, nullptr, 0.0, nullptr, prof);
      w.bref_on = bref_keep;
      if (rc != GOFD_OK) return rc;
      int mx = 0;
      for (int k = 0; k < ni; ++k) {
        if (conv[k]) continue;
        iters[k] += hs[k].iters;
        refs[k] += 1;
        mx = std::max(mx, hs[k].iters);
        if (hs[k].status == ST_BREAKDOWN) status[k] = GOFD_E_BREAKDOWN;
      }
      total_it += mx;
      hipLaunchKernelGGL(k_axpy_mask, dim3(grid1(ntot, 256)), dim3(256), 0, st, w.xr.as<double>(), w.x.as<double>(),
                         ntot);
    }
    GOFD_TRY(copy_out(w.xr.as<double>()));
    for (int k = 0; k < ni; ++k)
      if (!conv[k] && status[k] == GOFD_OK) status[k] = GOFD_E_NOT_CONVERGED;
    // restore b for the final residual
    HIP_TRY(ctx, hipMemcpyAsync(w.b.p, bsave.p, sizeof(double) * ntot, hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
  } else {
    return gofd_fail(ctx, GOFD_E_ARG, "unknown solve mode");
  }
  // final relative residual in double precision (of the solution just copied out)
  std::vector<double> rr(ni), bb(ni);
  if (confirmed) {
    for (int k = 0; k < ni; ++k) {
      rr[k] = hs[k].rr;
      bb[k] = hs[k].bb;
    }
  } else {
    const double* xfin = (mode == GOFD_MODE_FP32_REFINE) ? w.xr.as<double>() : w.x.as<double>();
    GOFD_TRY(true_residual(ctx, B, w, xfin, w.b.as<double>(), w.r.as<double>(), rr, bb));
    if (w.bref_on) bb = w.bref_host;
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  int worst = GOFD_OK;
  for (int k = 0; k < ni; ++k) {
    rel[k] = bb[k] > 0 ? std::sqrt(rr[k] / bb[k]) : 0.0;
    if (info) {
      info[k].iterations = iters[k];
      info[k].refinements = refs[k];
      info[k].rel_residual = rel[k];
      info[k].time_ms = ms;
      info[k].status = status[k];
    }
    if (status[k] != GOFD_OK && worst == GOFD_OK) worst = status[k];
  }
  if (prof) prof->write(o->stage_ms);
  if (worst != GOFD_OK) return gofd_fail(ctx, worst, "solve did not reach the tolerance for every right-hand side");
  return GOFD_OK;
}

static int check_problem(gofd_ctx_s* ctx, gofd_transfer tr, gofd_fdop op, gofd_precond pc, int nrhs) {
  if (!tr || !op || nrhs < 1) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  if (pc && pc->nv != tr->nv) return gofd_fail(ctx, GOFD_E_ARG, "preconditioner built for another mesh");
  return GOFD_OK;
}

extern "C" int gofd_solve(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, gofd_precond pc, int nrhs, const double* f,
                          int f_loc, double tol, const gofd_solve_opts* opts, double* u, gofd_solve_info* info) {
  if (!ctx || !f || !u) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  GOFD_TRY(check_problem(ctx, tr, op, pc, nrhs));
  if (!(tol > 0.0)) return gofd_fail(ctx, GOFD_E_ARG, "tol must be positive");
  WorkStream ws(ctx);
  Batch B;
  GOFD_TRY(batch_init(ctx, B, {Problem{tr, op, pc, nrhs}}));
  Work& w = ctx_work(ctx);
  GOFD_TRY(reserve_work(ctx, w, B));
  GOFD_TRY(form_rhs(ctx, B.probs[0], f, f_loc, w.b.as<double>()));
  double* outs[1] = {u};
  const double* x0 = opts ? opts->x0 : nullptr;
  if (!x0) return solve_system(ctx, B, w, tol, opts, outs, info);
  // warm start: CG from x0 is CG from 0 on the correction K d = b - K x0,
  // stopped at ||b - K x0 - K d|| <= tol ||b||; then u = x0 + d
  hipStream_t st = ctx->stream;
  const long long nv = tr->nv, ntot = nv * nrhs;
  for (int k = 0; k < nrhs; ++k)
    hipLaunchKernelGGL(k_mask_copy, dim3(grid1(nv, 256)), dim3(256), 0, st, x0 + k * nv, tr->imask.as<double>(), nv,
                       w.xr.as<double>() + k * nv);
  std::vector<double> rr, bb;
  GOFD_TRY(true_residual(ctx, B, w, w.xr.as<double>(), w.b.as<double>(), w.r.as<double>(), rr, bb));
  HIP_TRY(ctx, hipMemcpyAsync(w.b.p, w.r.p, sizeof(double) * ntot, hipMemcpyDeviceToDevice, st));
  GOFD_TRY(dev_reserve(ctx, w.bref, sizeof(double) * nrhs));
  HIP_TRY(ctx, hipMemcpyAsync(w.bref.p, bb.data(), sizeof(double) * nrhs, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  w.bref_host = bb;
  w.bref_on = w.bref.as<double>();
  const int rc = solve_system(ctx, B, w, tol, opts, outs, info);
  w.bref_on = nullptr;
  // u = d + x0 (interior) also when the solve reports an error: u then holds its last iterate
  for (int k = 0; k < nrhs; ++k)
    hipLaunchKernelGGL(k_add_masked, dim3(grid1(nv, 256)), dim3(256), 0, st, x0 + k * nv, tr->imask.as<double>(), nv,
                       u + k * nv);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return rc;
}

// Problems are grouped by grid shape (d, W, L); each group is one batch whose
// CG iterations advance together, every stage one launch for the group.
// One shape group of a batched call: its problems' items advance together.
// Fills inf (one entry per item of the group, problem order) and returns the
// solve's status.
static int solve_group(gofd_ctx_s* ctx, const std::vector<int>& members, const gofd_transfer* trs,
                       const gofd_fdop* ops, const gofd_precond* pcs, const int* nrhs, const double* const* f,
                       int f_loc, double tol, const gofd_solve_opts* opts, double* const* u,
                       std::vector<gofd_solve_info>& inf) {
  std::vector<Problem> probs;
  for (int q : members) probs.push_back(Problem{trs[q], ops[q], pcs ? pcs[q] : nullptr, nrhs[q]});
  Batch B;
  GOFD_TRY(batch_init(ctx, B, probs));
  Work& w = ctx_work(ctx);
  GOFD_TRY(reserve_work(ctx, w, B));
  std::vector<double*> outs;
  for (size_t j = 0; j < members.size(); ++j) {
    GOFD_TRY(form_rhs(ctx, B.probs[j], f[members[j]], f_loc, w.b.as<double>() + B.poff[j]));
    outs.push_back(u[members[j]]);
  }
  inf.assign(B.nitems, gofd_solve_info{});
  return solve_system(ctx, B, w, tol, opts, outs.data(), inf.data());
}

// Problems are grouped by grid shape (d, W, L); each group is one batch whose
// CG iterations advance together, every stage one launch for the group.
// Several groups run concurrently, each from a host thread on a child context
// (own streams and workspaces), ordered after the caller's stream on entry
// and before it on exit.
extern "C" int gofd_solve_batched(gofd_ctx ctx, int nprob, const gofd_transfer* trs, const gofd_fdop* ops,
                                  const gofd_precond* pcs, const int* nrhs, const double* const* f, int f_loc,
                                  double tol, const gofd_solve_opts* opts, double* const* u, gofd_solve_info* info) {
  if (!ctx || nprob < 1 || !trs || !ops || !nrhs || !f || !u) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!(tol > 0.0)) return gofd_fail(ctx, GOFD_E_ARG, "tol must be positive");
  if (opts && opts->x0) return gofd_fail(ctx, GOFD_E_ARG, "an initial guess is taken by gofd_solve only");
  std::vector<int> item0(nprob + 1, 0);
  for (int q = 0; q < nprob; ++q) {
    GOFD_TRY(check_problem(ctx, trs[q], ops[q], pcs ? pcs[q] : nullptr, nrhs[q]));
    if (!f[q] || !u[q]) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
    item0[q + 1] = item0[q] + nrhs[q];
  }
  std::vector<std::vector<int>> groups;
  {
    std::vector<char> done(nprob, 0);
    for (int q0 = 0; q0 < nprob; ++q0) {
      if (done[q0]) continue;
      std::vector<int> members;
      for (int q = q0; q < nprob; ++q)
        if (!done[q] && ops[q]->d == ops[q0]->d && ops[q]->W == ops[q0]->W && ops[q]->L == ops[q0]->L) {
          members.push_back(q);
          done[q] = 1;
        }
      groups.push_back(members);
    }
  }
  const size_t ng = groups.size();
  std::vector<std::vector<gofd_solve_info>> infs(ng);
  std::vector<int> rcs(ng, GOFD_OK);
  WorkStream ws(ctx);
  // host-side outputs of stage timing and residual history are single arrays: groups one after another then
  const bool concurrent = ng > 1 && !(opts && (opts->stage_ms || opts->history));
  if (!concurrent) {
    for (size_t g = 0; g < ng; ++g) {
      rcs[g] = solve_group(ctx, groups[g], trs, ops, pcs, nrhs, f, f_loc, tol, opts, u, infs[g]);
      if (rcs[g] != GOFD_OK && rcs[g] != GOFD_E_NOT_CONVERGED && rcs[g] != GOFD_E_BREAKDOWN) return rcs[g];
    }
  } else {
    std::vector<gofd_ctx_s*> kids(ng);
    for (size_t g = 0; g < ng; ++g)
      if (!(kids[g] = ctx_child(ctx, g))) return gofd_fail(ctx, GOFD_E_HIP, "could not create a stream context");
    hipEvent_t start;
    HIP_TRY(ctx, hipEventCreateWithFlags(&start, hipEventDisableTiming));
    HIP_TRY(ctx, hipEventRecord(start, ctx->stream));
    for (size_t g = 0; g < ng; ++g) HIP_TRY(ctx, hipStreamWaitEvent(kids[g]->stream, start, 0));
    std::vector<std::thread> th;
    for (size_t g = 0; g < ng; ++g)
      th.emplace_back([&, g]() {
        (void)hipSetDevice(ctx->device);
        WorkStream wsg(kids[g]);
        rcs[g] = solve_group(kids[g], groups[g], trs, ops, pcs, nrhs, f, f_loc, tol, opts, u, infs[g]);
      });
    for (auto& t : th) t.join();
    // the caller's work continues once every group has finished
    for (size_t g = 0; g < ng; ++g) HIP_TRY(ctx, hipStreamWaitEvent(ctx->stream, kids[g]->ev_out, 0));
    (void)hipEventDestroy(start);
    for (size_t g = 0; g < ng; ++g)
      if (rcs[g] != GOFD_OK && rcs[g] != GOFD_E_NOT_CONVERGED && rcs[g] != GOFD_E_BREAKDOWN)
        return gofd_fail(ctx, rcs[g], kids[g]->last_error);
  }
  int worst = GOFD_OK;
  for (size_t g = 0; g < ng; ++g) {
    if (rcs[g] != GOFD_OK && worst == GOFD_OK) worst = rcs[g];
    if (!info) continue;
    int it = 0;
    for (int q : groups[g])
      for (int k = 0; k < nrhs[q]; ++k) info[item0[q] + k] = infs[g][it++];
  }
  if (worst != GOFD_OK) return gofd_fail(ctx, worst, "solve did not reach the tolerance for every right-hand side");
  return GOFD_OK;
}

// ---------------------------------------------------------------- adjoint

namespace {

// grid field v = c * I (mask * x): gather of vertex values at every node
template <int D>
__global__ void k_gather_grid(GridGeom g, const ElemRec<D>* __restrict__ recs,
                              const int* __restrict__ elem, const double* __restrict__ x,
                              const double* __restrict__ mask, long long n_nodes, double c, double* __restrict__ v) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_nodes) return;
  const int e = elem[k];
  if (e < 0) {
    v[k] = 0.0;
    return;
  }
  int vid[D + 1];
  double lam[D + 1];
  node_weights<D>(g, recs, e, k, vid, lam);
  double s = 0.0;
  for (int r = 0; r <= D; ++r) s += lam[r] * mask[vid[r]] * x[vid[r]];
  v[k] = c * s;
}

// dL/dX_{j,a} = sum over nodes k touching vertex j (as vertex i of elem(k)) of
//   sum_r G_r(k) * (-(E^{-1})_{r,a} phi_i(x_k)),  G_r = lam_{v_r} r_k - (A I lam)_k u_{v_r}
// One thread per vertex, nodes in ascending order: deterministic.
template <int D>
__global__ void k_grad_X(GridGeom g, const double* __restrict__ X, const ElemRec<D>* __restrict__ recs,
                         const int* __restrict__ elem, const int* __restrict__ off, const int* __restrict__ node,
                         long long nv, const double* __restrict__ u, const double* __restrict__ lam_v,
                         const double* __restrict__ mask, const double* __restrict__ rgrid,
                         const double* __restrict__ ylam, double* __restrict__ gX) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  double acc[D] = {};
  for (int q = off[j]; q < off[j + 1]; ++q) {
    const long long k = node[q];
    const int e = elem[k];
    int vid[D + 1];
    double phi[D + 1];
    node_weights<D>(g, recs, e, k, vid, phi);
    int i = 0;
    for (int r = 0; r <= D; ++r)
      if (vid[r] == (int)j) i = r;
    double V[(D + 1) * D];
    for (int r = 0; r <= D; ++r)
      for (int a = 0; a < D; ++a) V[r * D + a] = X[(long long)vid[r] * D + a];
    double Ei[(D + 1) * (D + 1)];
    inverse_E<D>(V, Ei);
    const double rk = rgrid[k], yk = ylam[k];
    for (int r = 0; r <= D; ++r) {
      const double mr = mask[vid[r]];
      const double G = mr * (lam_v[vid[r]] * rk - yk * u[vid[r]]);
      for (int a = 0; a < D; ++a) acc[a] += G * (-Ei[r * (D + 1) + a] * phi[i]);
    }
  }
  for (int a = 0; a < D; ++a) gX[j * D + a] = acc[a];
}

__global__ void k_rgrid(const double* __restrict__ f, const double* __restrict__ yu, const int* __restrict__ elem,
                        long long n, double h2s, double* __restrict__ r) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) r[k] = elem[k] >= 0 ? h2s * f[k] - yu[k] : 0.0;
}


}  // namespace

extern "C" int gofd_solve_adjoint(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, gofd_precond pc, const double* dLdu,
                                  const double* u, const double* f, double tol, const gofd_solve_opts* opts,
                                  double* grad_f, double* grad_X, double* lambda, gofd_solve_info* info) {
  if (!ctx || !tr || !op || !dLdu || !u || !f) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  if (!(tol > 0.0)) return gofd_fail(ctx, GOFD_E_ARG, "tol must be positive");
  WorkStream ws(ctx);
  hipStream_t st = ctx->stream;
  GOFD_TRY(check_problem(ctx, tr, op, pc, 1));
  Batch B;
  GOFD_TRY(batch_init(ctx, B, {Problem{tr, op, pc, 1}}));
  Work& w = ctx_work(ctx);
  GOFD_TRY(reserve_work(ctx, w, B));
  const long long nv = tr->nv, nn = tr->n_nodes;
  // adjoint right-hand side: dL/du on the interior block (K is symmetric)
  hipLaunchKernelGGL(k_mask_copy, dim3(grid1(nv, 256)), dim3(256), 0, st, dLdu, tr->imask.as<double>(), nv,
                     w.b.as<double>());
  DevBuf lam;
  GOFD_TRY(dev_reserve(ctx, lam, sizeof(double) * nv));
  double* outs[1] = {lam.as<double>()};
  GOFD_TRY(solve_system(ctx, B, w, tol, opts, outs, info));
  if (lambda) HIP_TRY(ctx, hipMemcpyAsync(lambda, lam.p, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
  GridGeom g;
  g.d = tr->d;
  g.W = tr->W;
  g.h = tr->h;
  for (int a = 0; a < 3; ++a) g.lo[a] = tr->lo[a];
  if (grad_f) {
    if (tr->d == 2)
      hipLaunchKernelGGL(k_gather_grid<2>, dim3(grid1(nn, 256)), dim3(256), 0, st, g, tr->rec.as<ElemRec2>(),
                         tr->elem.as<int>(), lam.as<double>(), tr->imask.as<double>(), nn, op->h2s, grad_f);
    else
      hipLaunchKernelGGL(k_gather_grid<3>, dim3(grid1(nn, 256)), dim3(256), 0, st, g, tr->rec.as<ElemRec3>(),
                         tr->elem.as<int>(), lam.as<double>(), tr->imask.as<double>(), nn, op->h2s, grad_f);
  }
  if (grad_X) {
    DevBuf yu, yl, rg;
    GOFD_TRY(dev_reserve(ctx, yu, sizeof(double) * nn));
    GOFD_TRY(dev_reserve(ctx, yl, sizeof(double) * nn));
    GOFD_TRY(dev_reserve(ctx, rg, sizeof(double) * nn));
    GOFD_TRY(conv_prepare(ctx, op, 1));
    GatherSpec gs;
    gs.tr = tr;
    gs.mask = tr->imask.as<double>();
    gs.u = u;
    GOFD_TRY(conv_apply(ctx, op, 1, nullptr, &gs, yu.p, false));        // A I u
    gs.u = lam.as<double>();
    GOFD_TRY(conv_apply(ctx, op, 1, nullptr, &gs, yl.p, false));        // A I lambda
    hipLaunchKernelGGL(k_rgrid, dim3(grid1(nn, 256)), dim3(256), 0, st, f, yu.as<double>(), tr->elem.as<int>(), nn,
                       op->h2s, rg.as<double>());
    // u restricted to the interior (the solve's unknowns)
    hipLaunchKernelGGL(k_mask_copy, dim3(grid1(nv, 256)), dim3(256), 0, st, u, tr->imask.as<double>(), nv,
                       w.x.as<double>());
    if (tr->d == 2)
      hipLaunchKernelGGL(k_grad_X<2>, dim3(grid1(nv, 128)), dim3(128), 0, st, g, tr->X.as<double>(),
                         tr->rec.as<ElemRec2>(), tr->elem.as<int>(), tr->csc_off.as<int>(), tr->csc_node.as<int>(),
                         nv, w.x.as<double>(), lam.as<double>(), tr->imask.as<double>(), rg.as<double>(),
                         yl.as<double>(), grad_X);
    else
      hipLaunchKernelGGL(k_grad_X<3>, dim3(grid1(nv, 128)), dim3(128), 0, st, g, tr->X.as<double>(),
                         tr->rec.as<ElemRec3>(), tr->elem.as<int>(), tr->csc_off.as<int>(), tr->csc_node.as<int>(),
                         nv, w.x.as<double>(), lam.as<double>(), tr->imask.as<double>(), rg.as<double>(),
                         yl.as<double>(), grad_X);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return GOFD_OK;
}
