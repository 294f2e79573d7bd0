// Truncated conjugate gradients on eq. GoFD-2 with checkpointed iterates, and
// the reverse-mode gradient of that truncated solve.
//
// Forward (textbook CG from x_0, double precision throughout):
//   r_0 = b - K x_0, p_0 = r_0, gamma_0 = (r_0, r_0);  for i = 0, 1, ...:
//   q_i = K p_i, delta_i = (p_i, q_i), alpha_i = gamma_i / delta_i,
//   x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i q_i,
//   gamma_{i+1} = (r_{i+1}, r_{i+1}), beta_i = gamma_{i+1} / gamma_i,
//   p_{i+1} = r_{i+1} + beta_i p_i,
// with K = I_J^T A_FD I_J and b = h^{2s} I_J^T f (eq. GoFD-2 on the interior
// block).  It stops after max_iter iterations or once gamma <= tol^2 (b, b).
// The scalars of every iteration are kept on the device, and (x, r, p) every
// c iterations (checkpoints).
//
// Backward: the adjoint of x_n is given; the adjoints of r, p and gamma are
// carried from iteration n-1 down to 0.  Step i needs p_i, q_i and r_{i+1},
// which are recomputed from the checkpoint that opens their segment of c
// iterations (one product each), using the stored alpha_i and beta_i.  Per
// step (bars are adjoints, primes the values after the step's updates):
//   beta-bar  = (p-bar, p_i),    gamma-bar' = gamma-bar + beta-bar / gamma_i,
//   r-bar'    = r-bar + p-bar + 2 gamma-bar' r_{i+1},
//   alpha-bar = (x-bar, p_i) - (r-bar', q_i),
//   delta-bar = -alpha-bar gamma_i / delta_i^2,
//   q-bar     = -alpha_i r-bar' + delta-bar p_i,
//   p-bar'    = beta_i p-bar + alpha_i x-bar + delta-bar q_i + K q-bar,
//   gamma-bar (of gamma_i) = -beta-bar gamma_{i+1} / gamma_i^2 + alpha-bar / delta_i.
// At the start, r-bar_0 = r-bar + p-bar + 2 gamma-bar r_0, which is the
// adjoint of b; that of x_0 is x-bar - K r-bar_0.  K is symmetric, and its
// adjoint is the sum of the rank-one terms q-bar_i p_i^T - r-bar_0 x_0^T;
// through K = I^T A I and b = h^{2s} I^T f every term a b^T gives
// dL/dI_kj += a_j (A I b)_k + (A I a)_k b_j, and b gives h^{2s} f_k r-bar_0,j.
// Those are summed per (grid node, element corner) and chained to the vertex
// coordinates through the barycentric weights, with point location held
// fixed, as in the adjoint of the converged solve.
#include <algorithm>
#include <memory>
#include <vector>

#include "bary.h"
#include "internal.h"

struct gofd_cg_tape_s {
  gofd_ctx_s* ctx = nullptr;
  gofd_transfer_s* tr = nullptr;
  gofd_fdop_s* op = nullptr;
  int n = 0;                 // iterations run
  int c = 1;                 // checkpoint interval
  int cap = 0;               // max_iter (scalar capacity)
  bool has_x0 = false;
  DevBuf f;                  // copy of f (grid)
  DevBuf x0;                 // copy of x_0 on the interior (if given)
  DevBuf ck;                 // checkpoints j = 0 .. cap / c: x, r, p (3 N_v doubles each)
  DevBuf sc;                 // scalars: gamma[cap+1], delta[cap+1], alpha[cap+1], beta[cap+1]
  DevBuf state;              // UState
};

namespace {

constexpr int UB = 256;      // threads per block of the vector kernels
constexpr int UNB = 256;     // blocks of the dot-product kernels (fixed: sums in a fixed order)

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

struct UState {
  double gamma, bb, tol2;    // forward: gamma of the current iterate, (b, b), tol^2 (b, b)
  double gbar, gbarp, dbar;  // backward: adjoint of gamma carried, and gamma-bar', delta-bar of a step
  int n, done, status, pad;
};

// scalar tape: four arrays of cap + 1 doubles (gamma_i, delta_i, alpha_i, beta_i)
enum { GAM = 0, DEL = 1, ALP = 2, BET = 3 };
template <typename P>
__device__ __forceinline__ P* sc_arr(P* s, int cap, int which) {
  return s + (long long)which * (cap + 1);
}

template <int NQ>
__device__ __forceinline__ void block_reduce(double* v, double* sh) {
  gofd_cg::block_sum_n<UB, NQ>(v, sh);
}

// sum of partials part[0..nb) by one block in a fixed order
__device__ double sum_parts(const double* __restrict__ part, int nb, double* sh) {
  double v[1] = {0.0};
  for (int i = threadIdx.x; i < nb; i += UB) v[0] += part[i];
  block_reduce<1>(v, sh);
  return v[0];
}

struct Dots {
  const double* a[4];
  const double* a2[4];   // optional second term added to a
  const double* b[4];
};

// partial sums of NQ dot products (a_q + a2_q, b_q) over n entries, one per block
template <int NQ>
__global__ __launch_bounds__(UB) void k_dots(Dots d, long long n, double* __restrict__ part) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, NQ>()];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (long long i = (long long)blockIdx.x * UB + threadIdx.x; i < n; i += (long long)gridDim.x * UB) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double a = d.a2[q] ? d.a[q][i] + d.a2[q][i] : d.a[q][i];
      acc[q] += a * d.b[q][i];
    }
  }
  block_reduce<NQ>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NQ; ++q) part[q * gridDim.x + blockIdx.x] = acc[q];
}

// b = h^{2s} mask I^T f over the vertex-major structure (entries in a fixed order)
__global__ void k_rhs(const int* __restrict__ off, const int* __restrict__ node, const double* __restrict__ w,
                      const double* __restrict__ f, const double* __restrict__ mask, long long nv, double c,
                      double* __restrict__ b) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double acc = 0.0;
  for (int q = off[v]; q < off[v + 1]; ++q) acc += w[q] * f[node[q]];
  b[v] = c * mask[v] * acc;
}

// x = mask x_0 (or 0), r = mask (b - K x_0), p = r; partials of (r, r) and (b, b)
__global__ __launch_bounds__(UB) void k_u_init(const double* __restrict__ b, const double* __restrict__ kx0,
                                               const double* __restrict__ x0, const double* __restrict__ mask,
                                               long long n, double* __restrict__ x, double* __restrict__ r,
                                               double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, 2>()];
  double acc[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * UB + threadIdx.x; i < n; i += (long long)gridDim.x * UB) {
    const double m = mask[i];
    const double ri = kx0 ? m * (b[i] - kx0[i]) : b[i];
    x[i] = x0 ? m * x0[i] : 0.0;
    r[i] = ri;
    p[i] = ri;
    acc[0] += ri * ri;
    acc[1] += b[i] * b[i];
  }
  block_reduce<2>(acc, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = acc[0];
    part[gridDim.x + blockIdx.x] = acc[1];
  }
}

__global__ __launch_bounds__(UB) void k_u_start(const double* __restrict__ part, int nb, UState* __restrict__ S,
                                                double* __restrict__ sc, int cap, double tol) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, 1>()];
  const double g = sum_parts(part, nb, sh);
  const double bb = sum_parts(part + nb, nb, sh);
  if (threadIdx.x != 0) return;
  UState s{};
  s.gamma = g;
  s.bb = bb;
  s.tol2 = tol * tol * bb;
  s.n = 0;
  s.done = (g <= s.tol2) ? 1 : 0;
  s.status = 0;
  sc_arr(sc, cap, GAM)[0] = g;
  *S = s;
}

// delta_i = (p_i, q_i) -> alpha_i; a non-positive or non-finite delta is a breakdown
__global__ __launch_bounds__(UB) void k_u_alpha(const double* __restrict__ part, int nb, UState* __restrict__ S,
                                                double* __restrict__ sc, int cap, int i) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, 1>()];
  if (S->n != i || S->done) return;
  const double d = sum_parts(part, nb, sh);
  if (threadIdx.x != 0) return;
  if (!(d > 0.0) || !isfinite(d)) {
    S->status = 1;
    S->done = 1;
    return;
  }
  sc_arr(sc, cap, DEL)[i] = d;
  sc_arr(sc, cap, ALP)[i] = S->gamma / d;
}

// x += alpha p, r -= alpha q; partials of (r, r)
__global__ __launch_bounds__(UB) void k_u_update(const UState* __restrict__ S, const double* __restrict__ sc,
                                                 int cap, int i, double* __restrict__ x, double* __restrict__ r,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 long long n, double* __restrict__ part) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, 1>()];
  if (S->n != i || S->done) return;
  const double a = sc_arr(sc, cap, ALP)[i];
  double acc[1] = {0.0};
  for (long long k = (long long)blockIdx.x * UB + threadIdx.x; k < n; k += (long long)gridDim.x * UB) {
    x[k] = x[k] + a * p[k];
    const double rk = r[k] - a * q[k];
    r[k] = rk;
    acc[0] += rk * rk;
  }
  block_reduce<1>(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

__global__ __launch_bounds__(UB) void k_u_beta(const double* __restrict__ part, int nb, UState* __restrict__ S,
                                               double* __restrict__ sc, int cap, int i) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, 1>()];
  if (S->n != i || S->done) return;
  const double g1 = sum_parts(part, nb, sh);
  if (threadIdx.x != 0) return;
  if (!isfinite(g1)) {
    S->status = 1;
    S->done = 1;
    return;
  }
  sc_arr(sc, cap, GAM)[i + 1] = g1;
  sc_arr(sc, cap, BET)[i] = g1 / S->gamma;
  S->gamma = g1;
  S->n = i + 1;
  if (g1 <= S->tol2) S->done = 1;
}

// p = r + beta p; every c iterations the iterate (x, r, p) goes to its checkpoint
__global__ void k_u_p(const UState* __restrict__ S, const double* __restrict__ sc, int cap, int i,
                      const double* __restrict__ x, const double* __restrict__ r, double* __restrict__ p, long long n,
                      int c, double* __restrict__ ck) {
  if (S->n != i + 1) return;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double bt = sc_arr(sc, cap, BET)[i];
  const double pk = r[k] + bt * p[k];
  p[k] = pk;
  if ((i + 1) % c == 0) {
    double* C = ck + (long long)((i + 1) / c) * 3 * n;
    C[k] = x[k];
    C[n + k] = r[k];
    C[2 * n + k] = pk;
  }
}

__global__ void k_copy3(const double* __restrict__ x, const double* __restrict__ r, const double* __restrict__ p,
                        long long n, double* __restrict__ C) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  C[k] = x[k];
  C[n + k] = r[k];
  C[2 * n + k] = p[k];
}

// recomputation inside a segment: r_{i+1} = r_i - alpha_i q_i, p_{i+1} = r_{i+1} + beta_i p_i
__global__ void k_u_rec(const double* __restrict__ sc, int cap, int i, const double* __restrict__ r,
                        const double* __restrict__ p, const double* __restrict__ q, double* __restrict__ r1,
                        double* __restrict__ p1, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double a = sc_arr(sc, cap, ALP)[i];
  const double bt = sc_arr(sc, cap, BET)[i];
  const double rk = r[k] - a * q[k];
  r1[k] = rk;
  p1[k] = rk + bt * p[k];
}

__global__ void k_ub_seed(const double* __restrict__ xbar, const double* __restrict__ mask, long long n,
                          double* __restrict__ xb, double* __restrict__ rb, double* __restrict__ pb,
                          UState* __restrict__ S) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    S->gbar = 0.0;
    S->gbarp = 0.0;
    S->dbar = 0.0;
  }
  if (k >= n) return;
  xb[k] = mask[k] * xbar[k];
  rb[k] = 0.0;
  pb[k] = 0.0;
}

// scalars of backward step i from d1 = (p-bar, p_i), d2 = (r-bar + p-bar, q_i),
// d3 = (r_{i+1}, q_i), d4 = (x-bar, p_i)
__global__ __launch_bounds__(UB) void k_ub_scal(const double* __restrict__ part, int nb, UState* __restrict__ S,
                                                const double* __restrict__ sc, int cap, int i) {
  __shared__ double sh[gofd_cg::block_sum_lds<UB, 1>()];
  const double d1 = sum_parts(part, nb, sh);
  const double d2 = sum_parts(part + nb, nb, sh);
  const double d3 = sum_parts(part + 2 * nb, nb, sh);
  const double d4 = sum_parts(part + 3 * nb, nb, sh);
  if (threadIdx.x != 0) return;
  const double gi = sc_arr(sc, cap, GAM)[i], gi1 = sc_arr(sc, cap, GAM)[i + 1], di = sc_arr(sc, cap, DEL)[i];
  const double bbar = d1;
  const double gbarp = S->gbar + bbar / gi;
  const double abar = d4 - (d2 + 2.0 * gbarp * d3);
  S->gbarp = gbarp;
  S->dbar = -abar * gi / (di * di);
  S->gbar = -bbar * gi1 / (gi * gi) + abar / di;
}

__global__ void k_ub_vec(const UState* __restrict__ S, const double* __restrict__ sc, int cap, int i,
                         double* __restrict__ rb, double* __restrict__ pb, double* __restrict__ qb,
                         const double* __restrict__ r1, const double* __restrict__ p, const double* __restrict__ q,
                         const double* __restrict__ xb, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double a = sc_arr(sc, cap, ALP)[i], bt = sc_arr(sc, cap, BET)[i];
  const double gp = S->gbarp, db = S->dbar;
  const double rnew = rb[k] + pb[k] + 2.0 * gp * r1[k];
  rb[k] = rnew;
  qb[k] = -a * rnew + db * p[k];
  pb[k] = bt * pb[k] + a * xb[k] + db * q[k];
}

__global__ void k_add(double* __restrict__ a, const double* __restrict__ b, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] += b[k];
}

// r-bar_0 = r-bar + p-bar + 2 gamma-bar r_0 (p_0 = r_0 and gamma_0 = (r_0, r_0))
__global__ void k_ub_final(const UState* __restrict__ S, double* __restrict__ rb, const double* __restrict__ pb,
                           const double* __restrict__ r0, long long n) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) rb[k] = rb[k] + pb[k] + 2.0 * S->gbar * r0[k];
}

__global__ void k_ub_gx0(const double* __restrict__ xb, const double* __restrict__ t, const double* __restrict__ mask,
                         long long n, double* __restrict__ g) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) g[k] = mask[k] * (xb[k] - t[k]);
}

__global__ void k_mask(const double* __restrict__ a, const double* __restrict__ mask, long long n,
                       double* __restrict__ b) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) b[k] = mask[k] * a[k];
}

__global__ void k_fill(double* __restrict__ a, long long n, double v) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = v;
}

// G[k][r] += mask_j (c1 Ya_k vb_j + c2 Yb_k va_j), j = vertex r of node k's element
template <int D>
__global__ void k_accum_G(GridGeom g, const ElemRec<D>* __restrict__ recs, const int* __restrict__ elem,
                          long long nn, const double* __restrict__ mask, double c1, const double* __restrict__ Ya,
                          const double* __restrict__ vb, double c2, const double* __restrict__ Yb,
                          const double* __restrict__ va, double* __restrict__ G) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
  const int e = elem[k];
  if (e < 0) return;
  int vid[D + 1];
  double lam[D + 1];
  node_weights<D>(g, recs, e, k, vid, lam);
  const double ya = Ya[k], yb = Yb ? Yb[k] : 0.0;
  for (int r = 0; r <= D; ++r) {
    const int j = vid[r];
    double add = c1 * ya * vb[j];
    if (Yb) add += c2 * yb * va[j];
    G[k * (D + 1) + r] += mask[j] * add;
  }
}

// dL/dX_{j,a} = sum over the nodes k of vertex j (as corner i of elem(k)) of
// sum_r G[k][r] (-(E^{-1})_{r,a} lambda_i(x_k)); one thread per vertex, nodes in
// ascending order
template <int D>
__global__ void k_grad_X_nodes(GridGeom g, const double* __restrict__ X, const ElemRec<D>* __restrict__ recs,
                               const int* __restrict__ elem, const int* __restrict__ off,
                               const int* __restrict__ node, long long nv, const double* __restrict__ G,
                               double* __restrict__ gX) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  double acc[D] = {};
  for (int q = off[j]; q < off[j + 1]; ++q) {
    const long long k = node[q];
    const int e = elem[k];
    int vid[D + 1];
    double lam[D + 1];
    node_weights<D>(g, recs, e, k, vid, lam);
    int i = 0;
    for (int r = 0; r <= D; ++r)
      if (vid[r] == (int)j) i = r;
    double V[(D + 1) * D];
    for (int r = 0; r <= D; ++r)
      for (int a = 0; a < D; ++a) V[r * D + a] = X[(long long)vid[r] * D + a];
    double Ei[(D + 1) * (D + 1)];
    inverse_E<D>(V, Ei);
    for (int r = 0; r <= D; ++r) {
      const double Gr = G[k * (D + 1) + r];
      for (int a = 0; a < D; ++a) acc[a] += Gr * (-Ei[r * (D + 1) + a] * lam[i]);
    }
  }
  for (int a = 0; a < D; ++a) gX[j * D + a] = acc[a];
}

// grid field c * I (mask x)
template <int D>
__global__ void k_interp(GridGeom g, const ElemRec<D>* __restrict__ recs, const int* __restrict__ elem,
                         const double* __restrict__ x, const double* __restrict__ mask, long long nn, double c,
                         double* __restrict__ v) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nn) return;
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

GridGeom geom_of(const gofd_transfer_s* tr) {
  GridGeom g;
  g.d = tr->d;
  g.W = tr->W;
  g.h = tr->h;
  for (int a = 0; a < 3; ++a) g.lo[a] = tr->lo[a];
  return g;
}

// q = K v = I_J^T A_FD I_J v (double precision; the grid field A_FD I_J v is
// left in ygrid when given)
int apply_K(gofd_ctx_s* ctx, gofd_transfer_s* tr, gofd_fdop_s* op, const double* v, double* q, double* ygrid) {
  return apply_Ah_impl(ctx, tr, op, 1, v, q, GOFD_UNSCALED | GOFD_INTERIOR, ygrid);
}

Dots dots1(const double* a, const double* b) {
  Dots d{};
  d.a[0] = a;
  d.b[0] = b;
  return d;
}

}  // namespace

extern "C" int gofd_cg_checkpointed(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, const double* f_dev,
                                    const double* x0_dev, int max_iter, double tol, int ckpt_every, double* x_dev,
                                    gofd_cg_tape* tape_out, gofd_cg_tape_info* info) {
  if (!ctx || !tr || !op || !f_dev || !x_dev || !tape_out || max_iter < 0 || ckpt_every < 1 || !(tol >= 0.0))
    return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  *tape_out = nullptr;
  auto tp = std::unique_ptr<gofd_cg_tape_s>(new (std::nothrow) gofd_cg_tape_s());
  if (!tp) return gofd_fail(ctx, GOFD_E_OOM, "tape");
  gofd_cg_tape_s& T = *tp;
  T.ctx = ctx;
  T.tr = tr;
  T.op = op;
  T.c = ckpt_every;
  T.cap = max_iter;
  T.has_x0 = x0_dev != nullptr;
  const long long nv = tr->nv, nn = tr->n_nodes;
  const long long nck = max_iter / ckpt_every + 1;
  hipStream_t st = ctx->stream;
  GOFD_TRY(dev_reserve(ctx, T.f, sizeof(double) * nn));
  GOFD_TRY(dev_reserve(ctx, T.ck, sizeof(double) * 3 * nv * nck));
  GOFD_TRY(dev_reserve(ctx, T.sc, sizeof(double) * 4 * (max_iter + 1)));
  GOFD_TRY(dev_reserve(ctx, T.state, sizeof(UState)));
  DevBuf b, x, r, p, q, part;
  GOFD_TRY(dev_reserve(ctx, b, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, x, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, r, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, p, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, q, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, part, sizeof(double) * 4 * UNB));
  HIP_TRY(ctx, hipMemcpyAsync(T.f.p, f_dev, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
  const double* mask = tr->imask.as<double>();
  const unsigned gv = grid1(nv, UB);
  hipLaunchKernelGGL(k_rhs, dim3(gv), dim3(UB), 0, st, tr->csc_off.as<int>(), tr->csc_node.as<int>(),
                     tr->csc_w.as<double>(), T.f.as<double>(), mask, nv, op->h2s, b.as<double>());
  if (T.has_x0) {
    GOFD_TRY(dev_reserve(ctx, T.x0, sizeof(double) * nv));
    hipLaunchKernelGGL(k_mask, dim3(gv), dim3(UB), 0, st, x0_dev, mask, nv, T.x0.as<double>());
    GOFD_TRY(apply_K(ctx, tr, op, T.x0.as<double>(), q.as<double>(), nullptr));
  }
  UState* S = T.state.as<UState>();
  hipLaunchKernelGGL(k_u_init, dim3(UNB), dim3(UB), 0, st, b.as<double>(), T.has_x0 ? q.as<double>() : nullptr,
                     T.has_x0 ? T.x0.as<double>() : nullptr, mask, nv, x.as<double>(), r.as<double>(),
                     p.as<double>(), part.as<double>());
  hipLaunchKernelGGL(k_u_start, dim3(1), dim3(UB), 0, st, part.as<double>(), UNB, S, T.sc.as<double>(), max_iter,
                     tol);
  hipLaunchKernelGGL(k_copy3, dim3(gv), dim3(UB), 0, st, x.as<double>(), r.as<double>(), p.as<double>(), nv,
                     T.ck.as<double>());
  HIP_TRY(ctx, hipGetLastError());
  UState hs{};
  HIP_TRY(ctx, hipMemcpyAsync(&hs, S, sizeof(UState), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  constexpr int CHUNK = 16;   // iterations launched between two reads of the state
  for (int i0 = 0; i0 < max_iter && !hs.done; i0 += CHUNK) {
    for (int i = i0; i < std::min(max_iter, i0 + CHUNK); ++i) {
      GOFD_TRY(apply_K(ctx, tr, op, p.as<double>(), q.as<double>(), nullptr));
      hipLaunchKernelGGL(k_dots<1>, dim3(UNB), dim3(UB), 0, st, dots1(p.as<double>(), q.as<double>()), nv,
                         part.as<double>());
      hipLaunchKernelGGL(k_u_alpha, dim3(1), dim3(UB), 0, st, part.as<double>(), UNB, S, T.sc.as<double>(),
                         max_iter, i);
      hipLaunchKernelGGL(k_u_update, dim3(UNB), dim3(UB), 0, st, S, T.sc.as<double>(), max_iter, i, x.as<double>(),
                         r.as<double>(), p.as<double>(), q.as<double>(), nv, part.as<double>());
      hipLaunchKernelGGL(k_u_beta, dim3(1), dim3(UB), 0, st, part.as<double>(), UNB, S, T.sc.as<double>(),
                         max_iter, i);
      hipLaunchKernelGGL(k_u_p, dim3(gv), dim3(UB), 0, st, S, T.sc.as<double>(), max_iter, i, x.as<double>(),
                         r.as<double>(), p.as<double>(), nv, ckpt_every, T.ck.as<double>());
    }
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(&hs, S, sizeof(UState), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }
  HIP_TRY(ctx, hipMemcpyAsync(x_dev, x.p, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  T.n = hs.n;
  if (info) {
    info->iterations = hs.n;
    info->checkpoints = (int)(hs.n / ckpt_every + 1);
    info->rel_residual = hs.bb > 0.0 ? std::sqrt(hs.gamma / hs.bb) : 0.0;
    info->converged = (hs.gamma <= hs.tol2) ? 1 : 0;
  }
  if (hs.status) return gofd_fail(ctx, GOFD_E_BREAKDOWN, "CG breakdown (p^T K p <= 0 or a non-finite value)");
  *tape_out = tp.release();
  return GOFD_OK;
}

extern "C" int gofd_cg_tape_read(gofd_ctx ctx, gofd_cg_tape tape, int j, double* x_dev, double* r_dev,
                                 double* p_dev, double* scalars_host) {
  if (!ctx || !tape || j < 0 || j > tape->n / tape->c) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  hipStream_t st = ctx->stream;
  const long long nv = tape->tr->nv;
  const double* C = tape->ck.as<double>() + (long long)j * 3 * nv;
  if (x_dev) HIP_TRY(ctx, hipMemcpyAsync(x_dev, C, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
  if (r_dev) HIP_TRY(ctx, hipMemcpyAsync(r_dev, C + nv, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
  if (p_dev) HIP_TRY(ctx, hipMemcpyAsync(p_dev, C + 2 * nv, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
  if (scalars_host)
    HIP_TRY(ctx, hipMemcpyAsync(scalars_host, tape->sc.p, sizeof(double) * 4 * (tape->cap + 1),
                                hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return GOFD_OK;
}

extern "C" int gofd_cg_unrolled_grad(gofd_ctx ctx, gofd_cg_tape tape, const double* xbar_dev, double* grad_f_dev,
                                     double* grad_X_dev, double* grad_x0_dev) {
  if (!ctx || !tape || !xbar_dev || tape->ctx != ctx) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  gofd_transfer_s* tr = tape->tr;
  gofd_fdop_s* op = tape->op;
  const int d = tr->d, n = tape->n, c = tape->c, cap = tape->cap;
  const long long nv = tr->nv, nn = tr->n_nodes;
  const bool gX = grad_X_dev != nullptr;
  hipStream_t st = ctx->stream;
  const double* mask = tr->imask.as<double>();
  const unsigned gv = grid1(nv, UB), gn = grid1(nn, UB);
  double* sc = tape->sc.as<double>();
  UState* S = tape->state.as<UState>();
  const int seg = std::min(c, std::max(n, 1));
  DevBuf xb, rb, pb, qb, t, R, P, Q, part, Yp, Yq, Gn, Y2;
  GOFD_TRY(dev_reserve(ctx, xb, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, rb, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, pb, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, qb, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, t, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, R, sizeof(double) * nv * (seg + 1)));
  GOFD_TRY(dev_reserve(ctx, P, sizeof(double) * nv * (seg + 1)));
  GOFD_TRY(dev_reserve(ctx, Q, sizeof(double) * nv * seg));
  GOFD_TRY(dev_reserve(ctx, part, sizeof(double) * 4 * UNB));
  if (gX) {
    GOFD_TRY(dev_reserve(ctx, Yp, sizeof(double) * nn * seg));
    GOFD_TRY(dev_reserve(ctx, Yq, sizeof(double) * nn));
    GOFD_TRY(dev_reserve(ctx, Y2, sizeof(double) * nn));
    GOFD_TRY(dev_reserve(ctx, Gn, sizeof(double) * nn * (d + 1)));
    hipLaunchKernelGGL(k_fill, dim3(grid1(nn * (d + 1), UB)), dim3(UB), 0, st, Gn.as<double>(), nn * (d + 1), 0.0);
  }
  const GridGeom geom = geom_of(tr);
  auto accum = [&](double c1, const double* Ya, const double* vb, double c2, const double* Yb, const double* va) {
    if (d == 2)
      hipLaunchKernelGGL(k_accum_G<2>, dim3(gn), dim3(UB), 0, st, geom, tr->rec.as<ElemRec2>(), tr->elem.as<int>(),
                         nn, mask, c1, Ya, vb, c2, Yb, va, Gn.as<double>());
    else
      hipLaunchKernelGGL(k_accum_G<3>, dim3(gn), dim3(UB), 0, st, geom, tr->rec.as<ElemRec3>(), tr->elem.as<int>(),
                         nn, mask, c1, Ya, vb, c2, Yb, va, Gn.as<double>());
  };
  hipLaunchKernelGGL(k_ub_seed, dim3(gv), dim3(UB), 0, st, xbar_dev, mask, nv, xb.as<double>(), rb.as<double>(),
                     pb.as<double>(), S);
  const double* ck = tape->ck.as<double>();
  for (int s = (n - 1) / c; n > 0 && s >= 0; --s) {
    const int i0 = s * c, m = std::min(c, n - i0);
    const double* C = ck + (long long)s * 3 * nv;
    HIP_TRY(ctx, hipMemcpyAsync(R.p, C + nv, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(P.p, C + 2 * nv, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
    // recompute p_i, q_i = K p_i, r_{i+1} of the segment from its checkpoint
    for (int j = 0; j < m; ++j) {
      double* Pj = P.as<double>() + (long long)j * nv;
      double* Rj = R.as<double>() + (long long)j * nv;
      double* Qj = Q.as<double>() + (long long)j * nv;
      GOFD_TRY(apply_K(ctx, tr, op, Pj, Qj, gX ? Yp.as<double>() + (long long)j * nn : nullptr));
      hipLaunchKernelGGL(k_u_rec, dim3(gv), dim3(UB), 0, st, sc, cap, i0 + j, Rj, Pj, Qj, Rj + nv, Pj + nv, nv);
    }
    for (int j = m - 1; j >= 0; --j) {
      const int i = i0 + j;
      const double* Pj = P.as<double>() + (long long)j * nv;
      const double* Qj = Q.as<double>() + (long long)j * nv;
      const double* R1 = R.as<double>() + (long long)(j + 1) * nv;
      Dots dd{};
      dd.a[0] = pb.as<double>(); dd.b[0] = Pj;
      dd.a[1] = rb.as<double>(); dd.a2[1] = pb.as<double>(); dd.b[1] = Qj;
      dd.a[2] = R1; dd.b[2] = Qj;
      dd.a[3] = xb.as<double>(); dd.b[3] = Pj;
      hipLaunchKernelGGL(k_dots<4>, dim3(UNB), dim3(UB), 0, st, dd, nv, part.as<double>());
      hipLaunchKernelGGL(k_ub_scal, dim3(1), dim3(UB), 0, st, part.as<double>(), UNB, S, sc, cap, i);
      hipLaunchKernelGGL(k_ub_vec, dim3(gv), dim3(UB), 0, st, S, sc, cap, i, rb.as<double>(), pb.as<double>(),
                         qb.as<double>(), R1, Pj, Qj, xb.as<double>(), nv);
      GOFD_TRY(apply_K(ctx, tr, op, qb.as<double>(), t.as<double>(), gX ? Yq.as<double>() : nullptr));
      hipLaunchKernelGGL(k_add, dim3(gv), dim3(UB), 0, st, pb.as<double>(), t.as<double>(), nv);
      // dL/dI from the term q-bar_i p_i^T of K's adjoint
      if (gX) accum(1.0, Yp.as<double>() + (long long)j * nn, qb.as<double>(), 1.0, Yq.as<double>(), Pj);
    }
    HIP_TRY(ctx, hipGetLastError());
  }
  // adjoint of b: r-bar_0
  hipLaunchKernelGGL(k_ub_final, dim3(gv), dim3(UB), 0, st, S, rb.as<double>(), pb.as<double>(), ck + nv, nv);
  const bool need_kr = grad_x0_dev || (gX && tape->has_x0);
  if (need_kr) GOFD_TRY(apply_K(ctx, tr, op, rb.as<double>(), t.as<double>(), gX ? Yq.as<double>() : nullptr));
  if (grad_x0_dev)
    hipLaunchKernelGGL(k_ub_gx0, dim3(gv), dim3(UB), 0, st, xb.as<double>(), t.as<double>(), mask, nv, grad_x0_dev);
  if (gX) {
    if (tape->has_x0) {
      // the term -r-bar_0 x_0^T of K's adjoint (r_0 = b - K x_0)
      GOFD_TRY(apply_K(ctx, tr, op, tape->x0.as<double>(), qb.as<double>(), Y2.as<double>()));
      accum(-1.0, Y2.as<double>(), rb.as<double>(), -1.0, Yq.as<double>(), tape->x0.as<double>());
    }
    // b = h^{2s} I^T f
    accum(op->h2s, tape->f.as<double>(), rb.as<double>(), 0.0, nullptr, nullptr);
    if (d == 2)
      hipLaunchKernelGGL(k_grad_X_nodes<2>, dim3(grid1(nv, 128)), dim3(128), 0, st, geom, tr->X.as<double>(),
                         tr->rec.as<ElemRec2>(), tr->elem.as<int>(), tr->csc_off.as<int>(), tr->csc_node.as<int>(),
                         nv, Gn.as<double>(), grad_X_dev);
    else
      hipLaunchKernelGGL(k_grad_X_nodes<3>, dim3(grid1(nv, 128)), dim3(128), 0, st, geom, tr->X.as<double>(),
                         tr->rec.as<ElemRec3>(), tr->elem.as<int>(), tr->csc_off.as<int>(), tr->csc_node.as<int>(),
                         nv, Gn.as<double>(), grad_X_dev);
  }
  if (grad_f_dev) {
    if (d == 2)
      hipLaunchKernelGGL(k_interp<2>, dim3(gn), dim3(UB), 0, st, geom, tr->rec.as<ElemRec2>(), tr->elem.as<int>(),
                         rb.as<double>(), mask, nn, op->h2s, grad_f_dev);
    else
      hipLaunchKernelGGL(k_interp<3>, dim3(gn), dim3(UB), 0, st, geom, tr->rec.as<ElemRec3>(), tr->elem.as<int>(),
                         rb.as<double>(), mask, nn, op->h2s, grad_f_dev);
  }
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return GOFD_OK;
}

extern "C" int gofd_cg_tape_free(gofd_cg_tape tape) {
  delete tape;
  return GOFD_OK;
}
