// GoFD in one dimension (the 1D example of Section 5): a mesh of an interval
// (vertices x_0 < x_1 < .. < x_n, element e = [x_e, x_{e+1}]), the overlay
// grid of W = 2N+1 nodes on (c - R, c + R), T by the closed form eq. T-1D-0,
// A_FD by its circulant embedding of length L (eq. AU-1), the system eq. GoFD-2
// on the interior vertices.  A problem of FFT length L <= 4096 is held by one
// workgroup: the gathered line, its transform and the product stay in LDS and
// registers, and a whole CG solve runs inside one launch (one workgroup per
// right-hand side), so a solve costs no launches per iteration.
//
//  - Location: node k at z_k = (c - R) + k h (each operation rounded
//    separately); a node belongs to the element of smallest id whose closed
//    interval holds it (a node on vertex x_e, e >= 1, to element e - 1),
//    decided by exact comparisons; nodes outside [x_0, x_n] have no element.
//    Each element's nodes are a contiguous range found by binary search.
//  - Weights: lambda_0 = (x_{e+1} - z) / (x_{e+1} - x_e), lambda_1 = 1 - lambda_0.
//  - T_p by the recurrence T_{p+1} = T_p (p - s) / (p + s + 1) from
//    T_0 = Gamma(2s+1) / Gamma(s+1)^2 (the ratio of consecutive terms of eq.
//    T-1D-0); the spectrum of the embedding c_r = T_|r| is taken by the same
//    FFT on the device and stored with the 1/L of the inverse transform.
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "fft.h"
#include "internal.h"

struct gofd1d_s {
  gofd_ctx_s* ctx = nullptr;
  int64_t nv = 0;
  int N = 0, W = 0, L = 0;
  double R = 0, c = 0, h = 0, s = 0, lo = 0;
  DevBuf x;        // double[nv]
  DevBuf kfirst;   // int32[ne]: first node of each element (ne = nv - 1); kfirst > klast for none
  DevBuf klast;    // int32[ne]
  DevBuf elem;     // int32[W]: element of each node, -1 outside
  DevBuf lam;      // double[2W]: lambda_0, lambda_1 of each node (0 outside)
  DevBuf D;        // double[nv]: column sums
  DevBuf That;     // double[L]: spectrum of the embedding / L
  DevBuf T;        // double[2N+1]: T_0..T_2N
  DevBuf work;     // per right-hand side: x, r, p, q, z (5 nv doubles each) and the state
  gofd1d_info info{};
};

namespace {

// values per thread of the line transform
template <int L>
constexpr int e1() {
  return 8;
}

__device__ __forceinline__ double node_z(double lo, double h, int k) { return __dadd_rn(lo, __dmul_rn((double)k, h)); }

// node range of every element: kfirst = the first node with z > x_e (z >= x_0 for element 0),
// klast = the last node with z <= x_{e+1}
__global__ void k1_ranges(const double* __restrict__ x, long long ne, double lo, double h, int W,
                          int* __restrict__ kfirst, int* __restrict__ klast) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double a = x[e], b = x[e + 1];
  int lo_k = 0, hi_k = W;      // first k in [0, W) with z_k > a (>= a for e = 0)
  while (lo_k < hi_k) {
    const int mid = (lo_k + hi_k) / 2;
    const double z = node_z(lo, h, mid);
    const bool after = e == 0 ? (z >= a) : (z > a);
    if (after) hi_k = mid;
    else lo_k = mid + 1;
  }
  kfirst[e] = lo_k;
  lo_k = 0;
  hi_k = W;                    // first k with z_k > b
  while (lo_k < hi_k) {
    const int mid = (lo_k + hi_k) / 2;
    if (node_z(lo, h, mid) > b) hi_k = mid;
    else lo_k = mid + 1;
  }
  klast[e] = lo_k - 1;
}

__global__ void k1_fill(const double* __restrict__ x, long long ne, double lo, double h,
                        const int* __restrict__ kfirst, const int* __restrict__ klast, int* __restrict__ elem,
                        double* __restrict__ lam) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double a = x[e], b = x[e + 1];
  for (int k = kfirst[e]; k <= klast[e]; ++k) {
    const double z = node_z(lo, h, k);
    const double l0 = (b - z) / (b - a);
    elem[k] = (int)e;
    lam[2 * k] = l0;
    lam[2 * k + 1] = 1.0 - l0;
  }
}

__global__ void k1_colsum(const int* __restrict__ kfirst, const int* __restrict__ klast,
                          const double* __restrict__ lam, long long nv, double* __restrict__ D) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nv) return;
  double d = 0.0;
  if (j >= 1)
    for (int k = kfirst[j - 1]; k <= klast[j - 1]; ++k) d += lam[2 * k + 1];
  if (j + 1 < nv)
    for (int k = kfirst[j]; k <= klast[j]; ++k) d += lam[2 * k];
  D[j] = d;
}

__global__ void k1_fill_i32(int* a, long long n, int v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// spectrum of the embedding c_r = T_|r| (r = -2N..2N, wrapped mod L), times 1/L
template <int L>
__global__ __launch_bounds__(L / e1<L>()) void k1_spectrum(const double* __restrict__ T, int P,
                                                      const cplx<double>* __restrict__ tw,
                                                      double* __restrict__ That) {
  constexpr int PL = gofd_fft::padded_len<L, e1<L>()>();
  __shared__ cplx<double> buf[PL];
  const int t = threadIdx.x;
  cplx<double> v[e1<L>()];
#pragma unroll
  for (int m = 0; m < e1<L>(); ++m) {
    const int r = t + m * (L / e1<L>());
    const int a = r <= L / 2 ? r : L - r;      // |r| on the circle
    v[m] = {a <= P ? T[a] : 0.0, 0.0};
  }
  gofd_fft::Twiddles<double, L, e1<L>()> tws;
  tws.load(tw, t);
  gofd_fft::fft_regs<double, L, e1<L>(), false>(v, buf, tws, t);
#pragma unroll
  for (int m = 0; m < e1<L>(); ++m) That[t + m * (L / e1<L>())] = v[m].x / (double)L;
}

struct Prob1 {
  const int* elem;
  const double* lam;
  const int* kfirst;
  const int* klast;
  const double* That;
  const double* D;
  long long nv;
  int W;
};

// y = I^T A_FD I u on every vertex (u given at every vertex; the line's values in LDS as doubles in ybuf)
// (the thread's base twiddles are loaded here, next to the gather, so that they hold registers only
// during the transforms)
template <int L>
__device__ void product(const Prob1& P, const double* u, double* out, cplx<double>* buf, double* ybuf,
                        const cplx<double>* __restrict__ tw) {
  constexpr int TPL = L / e1<L>();
  const int t = threadIdx.x;
  gofd_fft::Twiddles<double, L, e1<L>()> tws;
  tws.load(tw, t);
  cplx<double> v[e1<L>()];
#pragma unroll
  for (int m = 0; m < e1<L>(); ++m) {
    const int k = t + m * TPL;
    const int kc = k < P.W ? k : P.W - 1;          // clamped, masked after
    const int e = P.elem[kc];
    const int ec = e >= 0 ? e : 0;
    double g = P.lam[2 * kc] * u[ec] + P.lam[2 * kc + 1] * u[ec + 1];
    if (k >= P.W || e < 0) g = 0.0;
    v[m] = {g, 0.0};
  }
  __syncthreads();                                  // buf and ybuf free
  gofd_fft::fft_regs<double, L, e1<L>(), false>(v, buf, tws, t);
#pragma unroll
  for (int m = 0; m < e1<L>(); ++m) {
    const double th = P.That[t + m * TPL];
    v[m] = {v[m].x * th, v[m].y * th};
  }
  __syncthreads();
  tws.opaque();
  gofd_fft::fft_regs<double, L, e1<L>(), true>(v, buf, tws, t);
  __syncthreads();                                  // every thread has left the transform
#pragma unroll
  for (int m = 0; m < e1<L>(); ++m) {
    const int k = t + m * TPL;
    if (k < P.W) ybuf[k] = v[m].x;
  }
  __syncthreads();
  for (long long j = t; j < P.nv; j += TPL) {
    double acc = 0.0;
    if (j >= 1)
      for (int k = P.kfirst[j - 1]; k <= P.klast[j - 1]; ++k) acc += P.lam[2 * k + 1] * ybuf[k];
    if (j + 1 < P.nv)
      for (int k = P.kfirst[j]; k <= P.klast[j]; ++k) acc += P.lam[2 * k] * ybuf[k];
    out[j] = acc;
  }
  __syncthreads();
}

// fixed-order block sum of NQ values (every thread gets the same bits)
template <int L, int NQ>
__device__ __forceinline__ void bsum(double* v, double* sh) {
  gofd_cg::block_sum_n<L / e1<L>(), NQ>(v, sh);
}

// y = D^{-1} I^T A_FD I u (0 where D = 0); one workgroup per field
template <int L>
__global__ __launch_bounds__(L / e1<L>()) void k1_apply(Prob1 P, const cplx<double>* __restrict__ tw,
                                                   const double* __restrict__ u, double* __restrict__ y) {
  constexpr int PL = gofd_fft::padded_len<L, e1<L>()>();
  __shared__ cplx<double> buf[PL];
  const int f = blockIdx.x;
  double* ybuf = reinterpret_cast<double*>(buf);
  product<L>(P, u + (long long)f * P.nv, y + (long long)f * P.nv, buf, ybuf, tw);
  for (long long j = threadIdx.x; j < P.nv; j += L / e1<L>()) {
    const double d = P.D[j];
    y[(long long)f * P.nv + j] = d > 0.0 ? y[(long long)f * P.nv + j] / d : 0.0;
  }
}

// CG on eq. GoFD-2 for right-hand side f (the grid values of f), one workgroup: b = h^{2s} I^T f on the
// interior vertices, x = 0, plain or D-preconditioned CG to ||r|| <= tol ||b||.  ws: x, r, p, q, z of this
// right-hand side; res: iterations, relative recursive residual, status (0 converged, 1 iteration limit,
// 2 breakdown).
template <int L>
__global__ __launch_bounds__(L / e1<L>()) void k1_cg(Prob1 P, const cplx<double>* __restrict__ tw,
                                                const double* __restrict__ f, double h2s, double tol, int max_iter,
                                                int diag, double* __restrict__ ws, double* __restrict__ xout,
                                                double* __restrict__ res) {
  constexpr int TPL = L / e1<L>();
  constexpr int PL = gofd_fft::padded_len<L, e1<L>()>();
  __shared__ cplx<double> buf[PL];
  __shared__ double sh[gofd_cg::block_sum_lds<TPL, 2>()];
  const int b = blockIdx.x, t = threadIdx.x;
  const long long nv = P.nv;
  double* x = ws + (long long)b * 5 * nv;
  double* r = x + nv;
  double* p = r + nv;
  double* q = p + nv;
  double* z = q + nv;
  double* ybuf = reinterpret_cast<double*>(buf);
  const double* fb = f + (long long)b * P.W;
  // b = h^{2s} I^T f (f on the grid, in LDS), interior vertices only
  for (int k = t; k < P.W; k += TPL) ybuf[k] = fb[k];
  __syncthreads();
  for (long long j = t; j < nv; j += TPL) {
    double acc = 0.0;
    if (j >= 1)
      for (int k = P.kfirst[j - 1]; k <= P.klast[j - 1]; ++k) acc += P.lam[2 * k + 1] * ybuf[k];
    if (j + 1 < nv)
      for (int k = P.kfirst[j]; k <= P.klast[j]; ++k) acc += P.lam[2 * k] * ybuf[k];
    const bool inner = j >= 1 && j + 1 < nv;
    r[j] = inner ? h2s * acc : 0.0;
    x[j] = 0.0;
  }
  __syncthreads();
  auto prec = [&](long long j, double rj) {
    const bool inner = j >= 1 && j + 1 < nv;
    return !inner ? 0.0 : (diag ? rj / P.D[j] : rj);
  };
  double s2[2] = {0.0, 0.0};
  for (long long j = t; j < nv; j += TPL) {
    const double zj = prec(j, r[j]);
    z[j] = zj;
    p[j] = zj;
    s2[0] += r[j] * zj;
    s2[1] += r[j] * r[j];
  }
  bsum<L, 2>(s2, sh);
  double rz = s2[0];
  const double bb = s2[1];
  double rr = bb;
  int it = 0, status = 1;
  if (bb == 0.0) status = 0;
  while (status == 1 && it < max_iter) {
    if (rr <= tol * tol * bb) {
      status = 0;
      break;
    }
    product<L>(P, p, q, buf, ybuf, tw);
    double pq[1] = {0.0};
    for (long long j = t; j < nv; j += TPL) {
      const bool inner = j >= 1 && j + 1 < nv;
      if (!inner) q[j] = 0.0;
      pq[0] += p[j] * (inner ? q[j] : 0.0);
    }
    bsum<L, 1>(pq, sh);
    if (!(pq[0] > 0.0)) {
      status = 2;
      break;
    }
    const double alpha = rz / pq[0];
    double nr[2] = {0.0, 0.0};
    for (long long j = t; j < nv; j += TPL) {
      x[j] += alpha * p[j];
      const double rj = r[j] - alpha * q[j];
      r[j] = rj;
      const double zj = prec(j, rj);
      z[j] = zj;
      nr[0] += rj * zj;
      nr[1] += rj * rj;
    }
    bsum<L, 2>(nr, sh);
    const double beta = nr[0] / rz;
    rz = nr[0];
    rr = nr[1];
    for (long long j = t; j < nv; j += TPL) p[j] = z[j] + beta * p[j];
    __syncthreads();
    ++it;
  }
  if (status == 1 && rr <= tol * tol * bb) status = 0;
  for (long long j = t; j < nv; j += TPL) xout[(long long)b * nv + j] = x[j];
  if (t == 0) {
    res[3 * b] = it;
    res[3 * b + 1] = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    res[3 * b + 2] = status;
  }
}

inline unsigned g1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

template <int L>
void launch_spectrum(gofd1d_s* P, hipStream_t st, const cplx<double>* tw) {
  hipLaunchKernelGGL((k1_spectrum<L>), dim3(1), dim3(L / e1<L>()), 0, st, P->T.as<double>(), 2 * P->N, tw,
                     P->That.as<double>());
}

Prob1 prob(gofd1d_s* P) {
  return Prob1{P->elem.as<int>(), P->lam.as<double>(), P->kfirst.as<int>(), P->klast.as<int>(),
               P->That.as<double>(), P->D.as<double>(), (long long)P->nv, P->W};
}

// dispatch on the FFT length
template <template <int> class F, typename... A>
bool by_length(int L, A&&... a) {
  switch (L) {
    case 512: F<512>::run(a...); return true;
    case 1024: F<1024>::run(a...); return true;
    case 2048: F<2048>::run(a...); return true;
    case 4096: F<4096>::run(a...); return true;
    default: return false;
  }
}
template <int L>
struct RunSpectrum {
  static void run(gofd1d_s* P, hipStream_t st, const cplx<double>* tw) { launch_spectrum<L>(P, st, tw); }
};
template <int L>
struct RunApply {
  static void run(gofd1d_s* P, hipStream_t st, const cplx<double>* tw, int nf, const double* u, double* y) {
    hipLaunchKernelGGL((k1_apply<L>), dim3(nf), dim3(L / e1<L>()), 0, st, prob(P), tw, u, y);
  }
};
template <int L>
struct RunCg {
  static void run(gofd1d_s* P, hipStream_t st, const cplx<double>* tw, int nrhs, const double* f, double h2s,
                  double tol, int max_iter, int diag, double* ws, double* x, double* res) {
    hipLaunchKernelGGL((k1_cg<L>), dim3(nrhs), dim3(L / e1<L>()), 0, st, prob(P), tw, f, h2s, tol, max_iter, diag, ws,
                       x, res);
  }
};

}  // namespace

extern "C" int gofd1d_create(gofd_ctx ctx, int64_t nv, const double* x_dev, int N, double R, double center,
                             double s, gofd1d* out, gofd1d_info* info) {
  if (!ctx || !x_dev || !out || nv < 3 || N < 1 || !(R > 0) || !(s > 0 && s < 1))
    return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  int L = 512;
  while (L < 4 * N) L *= 2;
  if (L > 4096) return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "1D FFT length above 4096 (N > 1024)");
  auto P = std::unique_ptr<gofd1d_s>(new (std::nothrow) gofd1d_s());
  if (!P) return gofd_fail(ctx, GOFD_E_OOM, "1D handle");
  P->ctx = ctx;
  P->nv = nv;
  P->N = N;
  P->W = 2 * N + 1;
  P->L = L;
  P->R = R;
  P->c = center;
  P->h = R / (double)N;
  P->lo = center - R;
  P->s = s;
  if (P->W < nv) return gofd_fail(ctx, GOFD_E_RANK, "2N+1 < N_v: I_h^FD cannot have full column rank");
  hipStream_t st = ctx->stream;
  std::vector<double> xh(nv);
  HIP_TRY(ctx, hipMemcpyAsync(xh.data(), x_dev, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  for (int64_t i = 0; i + 1 < nv; ++i)
    if (!(xh[i] < xh[i + 1])) return gofd_fail(ctx, GOFD_E_ARG, "vertices must be strictly increasing");
  double amin = INFINITY;
  for (int64_t i = 0; i + 1 < nv; ++i) amin = std::min(amin, xh[i + 1] - xh[i]);
  // T_0..T_2N by the ratio of consecutive terms of eq. T-1D-0
  std::vector<double> T(2 * (size_t)N + 1);
  T[0] = std::exp(std::lgamma(2 * s + 1) - 2 * std::lgamma(s + 1));
  for (int p = 0; p < 2 * N; ++p) T[p + 1] = T[p] * ((double)p - s) / ((double)p + s + 1.0);
  const long long ne = nv - 1;
  GOFD_TRY(dev_reserve(ctx, P->x, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, P->kfirst, sizeof(int) * ne));
  GOFD_TRY(dev_reserve(ctx, P->klast, sizeof(int) * ne));
  GOFD_TRY(dev_reserve(ctx, P->elem, sizeof(int) * P->W));
  GOFD_TRY(dev_reserve(ctx, P->lam, sizeof(double) * 2 * P->W));
  GOFD_TRY(dev_reserve(ctx, P->D, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, P->That, sizeof(double) * L));
  GOFD_TRY(dev_reserve(ctx, P->T, sizeof(double) * T.size()));
  HIP_TRY(ctx, hipMemcpyAsync(P->x.p, x_dev, sizeof(double) * nv, hipMemcpyDeviceToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(P->T.p, T.data(), sizeof(double) * T.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k1_fill_i32, dim3(g1(P->W, 256)), dim3(256), 0, st, P->elem.as<int>(), (long long)P->W, -1);
  HIP_TRY(ctx, hipMemsetAsync(P->lam.p, 0, sizeof(double) * 2 * P->W, st));
  hipLaunchKernelGGL(k1_ranges, dim3(g1(ne, 256)), dim3(256), 0, st, P->x.as<double>(), ne, P->lo, P->h, P->W,
                     P->kfirst.as<int>(), P->klast.as<int>());
  hipLaunchKernelGGL(k1_fill, dim3(g1(ne, 256)), dim3(256), 0, st, P->x.as<double>(), ne, P->lo, P->h,
                     P->kfirst.as<int>(), P->klast.as<int>(), P->elem.as<int>(), P->lam.as<double>());
  hipLaunchKernelGGL(k1_colsum, dim3(g1(nv, 256)), dim3(256), 0, st, P->kfirst.as<int>(), P->klast.as<int>(),
                     P->lam.as<double>(), (long long)nv, P->D.as<double>());
  const cplx<double>* tw = twiddles64(ctx, L);
  if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddles");
  by_length<RunSpectrum>(L, P.get(), st, tw);
  HIP_TRY(ctx, hipGetLastError());
  std::vector<double> Dh(nv);
  std::vector<int> eh(P->W);
  HIP_TRY(ctx, hipMemcpyAsync(Dh.data(), P->D.p, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(eh.data(), P->elem.p, sizeof(int) * P->W, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  gofd1d_info inf{};
  inf.W = P->W;
  inf.L = L;
  inf.h = P->h;
  inf.a_h = amin;
  double dmin = INFINITY;
  for (int64_t j = 1; j + 1 < nv; ++j) dmin = std::min(dmin, Dh[j]);
  inf.dmin_interior = dmin;
  for (int k = 0; k < P->W; ++k) inf.n_inside += eh[k] >= 0;
  P->info = inf;
  if (info) *info = inf;
  if (!(dmin > 0.0)) return gofd_fail(ctx, GOFD_E_ZERO_COLSUM, "an interior vertex has zero column sum D_j");
  *out = P.release();
  return GOFD_OK;
}

extern "C" int gofd1d_free(gofd1d h) {
  delete h;
  return GOFD_OK;
}

extern "C" int gofd1d_export(gofd_ctx ctx, gofd1d h, int part, void* out_dev) {
  if (!ctx || !h || !out_dev) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  hipStream_t st = ctx->stream;
  switch (part) {
    case GOFD1D_ELEM:
      HIP_TRY(ctx, hipMemcpyAsync(out_dev, h->elem.p, sizeof(int) * h->W, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD1D_WEIGHTS:
      HIP_TRY(ctx, hipMemcpyAsync(out_dev, h->lam.p, sizeof(double) * 2 * h->W, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD1D_D:
      HIP_TRY(ctx, hipMemcpyAsync(out_dev, h->D.p, sizeof(double) * h->nv, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD1D_T:
      HIP_TRY(ctx, hipMemcpyAsync(out_dev, h->T.p, sizeof(double) * (2 * h->N + 1), hipMemcpyDeviceToDevice, st));
      break;
    default:
      return gofd_fail(ctx, GOFD_E_ARG, "unknown part");
  }
  return GOFD_OK;
}

extern "C" int gofd1d_apply_Ah(gofd_ctx ctx, gofd1d h, int nfields, const double* u_dev, double* y_dev) {
  if (!ctx || !h || !u_dev || !y_dev || nfields < 1) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  const cplx<double>* tw = twiddles64(ctx, h->L);
  if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddles");
  by_length<RunApply>(h->L, h, ctx->stream, tw, nfields, u_dev, y_dev);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

extern "C" int gofd1d_solve(gofd_ctx ctx, gofd1d h, int nrhs, const double* f_dev, double tol, int max_iter,
                            int precond, double* u_dev, gofd1d_solve_info* info) {
  if (!ctx || !h || !f_dev || !u_dev || nrhs < 1 || !(tol >= 0) || (precond != 0 && precond != 1))
    return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (max_iter <= 0) max_iter = (int)std::min<int64_t>(10 * h->nv + 100, 1 << 20);
  GOFD_TRY(dev_reserve(ctx, h->work, sizeof(double) * (5 * (size_t)h->nv * nrhs + 3 * (size_t)nrhs)));
  double* ws = h->work.as<double>();
  double* res = ws + 5 * (size_t)h->nv * nrhs;
  const cplx<double>* tw = twiddles64(ctx, h->L);
  if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddles");
  const double h2s = std::pow(h->h, 2 * h->s);
  by_length<RunCg>(h->L, h, ctx->stream, tw, nrhs, f_dev, h2s, tol, max_iter, precond, ws, u_dev, res);
  HIP_TRY(ctx, hipGetLastError());
  std::vector<double> rh(3 * (size_t)nrhs);
  HIP_TRY(ctx, hipMemcpyAsync(rh.data(), res, sizeof(double) * rh.size(), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  int worst = GOFD_OK;
  for (int b = 0; b < nrhs; ++b) {
    if (info) {
      info[b].iterations = (int)rh[3 * b];
      info[b].rel_residual = rh[3 * b + 1];
      info[b].converged = rh[3 * b + 2] == 0.0;
    }
    if (rh[3 * b + 2] == 2.0) worst = GOFD_E_BREAKDOWN;
    else if (rh[3 * b + 2] == 1.0 && worst == GOFD_OK) worst = GOFD_E_NOT_CONVERGED;
  }
  if (worst != GOFD_OK)
    return gofd_fail(ctx, worst, worst == GOFD_E_BREAKDOWN ? "CG breakdown" : "iteration limit reached");
  return GOFD_OK;
}
