// Toeplitz coefficients T of the FD fractional Laplacian (Section 2.3).
//
// T_p = (-1)^{|p|} int_{[0,1]^d} psi~(xi) e^{i 2 pi p.xi} dxi   (eq. T-0),
// psi~(xi) = (sum_a 4 cos^2(pi xi_a))^s                          (eq. psi-2).
// Filon's rule with a piecewise-linear interpolant of psi~ (eq. Tp-1D-2),
// applied along every axis, is summed exactly by parts: along an axis its
// weights are the trapezoid weights times sigma_M(p) = (sin(pi p/M)/(pi p/M))^2.
// So the level-M value is
//   T^(M)_p = (-1)^{|p|} prod_a sigma_M(p_a) S^(M)_p,
//   S^(M)_p = M^{-d} sum_{j in [0,M)^d} psi~(j/M) prod_a cos(2 pi p_a j_a / M),
// and psi~ is even about 0 and 1/2 in every variable, so each axis sum folds
// onto j = 0..M/2 with weights 1, 2, ..., 2, 1.  Level M/2 uses the even
// samples of the same grid.  Richardson: T = (4 T^(M) - T^(M/2)) / 3 (the
// Filon error is O(M^-2)).  The axis sums are dense contractions of the sample
// array with a cosine matrix, done by a tiled FP64 kernel axis by axis.
#include <cmath>
#include <cstring>
#include <memory>

#include "internal.h"

namespace {

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_psi_samples(double* __restrict__ F, int d, long long Mh, long long M, double s) {
  long long n = 1;
  for (int a = 0; a < d; ++a) n *= Mh;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  long long rem = gid;
  double acc = 0.0;
  for (int a = 0; a < d; ++a) {
    const long long j = rem % Mh;
    rem /= Mh;
    const double c = cospi((double)j / (double)M);
    acc += 4.0 * c * c;
  }
  F[gid] = acc > 0.0 ? pow(acc, s) : 0.0;
}

// C[j][p] for j = 0..M/2, p = 0..P: folded trapezoid weight * cos(2 pi p j / M) / M
// at level M (coarse = 0), or the level-M/2 rule on the even samples (coarse = 1).
__global__ void k_cos_matrix(double* __restrict__ C, long long Mh, int P, long long M, int coarse) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Mh * (P + 1)) return;
  const long long j = gid / (P + 1);
  const long long p = gid % (P + 1);
  double v;
  if (!coarse) {
    const double w = (j == 0 || 2 * j == M) ? 1.0 : 2.0;
    const long long t = (p * j) % M;
    v = w * cospi(2.0 * (double)t / (double)M) / (double)M;
  } else {
    if (j & 1) {
      v = 0.0;
    } else {
      const long long jc = j / 2, Mc = M / 2;
      const double w = (jc == 0 || 2 * jc == Mc) ? 1.0 : 2.0;
      const long long t = (p * jc) % Mc;
      v = w * cospi(2.0 * (double)t / (double)Mc) / (double)Mc;
    }
  }
  C[gid] = v;
}

// Batched strided FP64 GEMM: Cm[b][m][n] = sum_k A[b][m][k] * B[b][k][n] with
// arbitrary element strides.  64x64 output tile per block, 4x4 per thread.
struct GemmArgs {
  const double* A;
  long long sAb, sAm, sAk;
  const double* B;
  long long sBb, sBk, sBn;
  double* C;
  long long sCb, sCm, sCn;
  long long Mm, Nn, Kk;
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const long long b = blockIdx.z;
  const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)blockIdx.x * BN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  const double* A = g.A + b * g.sAb;
  const double* B = g.B + b * g.sBb;
  for (long long k0 = 0; k0 < g.Kk; k0 += BK) {
    for (int i = threadIdx.x; i < BM * BK; i += 256) {
      const int kk = i / BM, mm = i % BM;
      const long long m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.Mm && k < g.Kk) ? A[m * g.sAm + k * g.sAk] : 0.0;
    }
    for (int i = threadIdx.x; i < BN * BK; i += 256) {
      const int kk = i / BN, nn = i % BN;
      const long long n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < g.Nn && k < g.Kk) ? B[k * g.sBk + n * g.sBn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double a[4], bb[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) bb[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * bb[c];
    }
    __syncthreads();
  }
  double* C = g.C + b * g.sCb;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long m = m0 + ty + 16 * r, n = n0 + tx + 16 * c;
      if (m < g.Mm && n < g.Nn) C[m * g.sCm + n * g.sCn] = acc[r][c];
    }
}

void gemm(hipStream_t st, const GemmArgs& a, long long batch) {
  dim3 grid(grid1(a.Nn, 64), grid1(a.Mm, 64), (unsigned)batch);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, a);
}

// T_p = (-1)^{|p|} [4 prod sigma_M S^M - prod sigma_{M/2} S^{M/2}] / 3  (or level M only)
__global__ void k_finalize(const double* __restrict__ SM, const double* __restrict__ SC, double* __restrict__ T,
                           int d, int P, long long M, int richardson) {
  long long n = 1;
  for (int a = 0; a < d; ++a) n *= (P + 1);
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n) return;
  long long rem = gid;
  double sigf = 1.0, sigc = 1.0;
  int parity = 0;
  for (int a = 0; a < d; ++a) {
    const long long p = rem % (P + 1);
    rem /= (P + 1);
    parity += (int)(p & 1);
    if (p > 0) {
      const double xf = M_PI * (double)p / (double)M;
      const double sf = sinpi((double)p / (double)M) / xf;
      sigf *= sf * sf;
      const double xc = M_PI * (double)p / (double)(M / 2);
      const double sc = sinpi((double)p / (double)(M / 2)) / xc;
      sigc *= sc * sc;
    }
  }
  const double sg = (parity & 1) ? -1.0 : 1.0;
  const double tf = sg * sigf * SM[gid];
  if (!richardson) {
    T[gid] = tf;
    return;
  }
  const double tc = sg * sigc * SC[gid];
  T[gid] = (4.0 * tf - tc) / 3.0;
}

// Contract the d-dimensional sample array (extent Mh per axis) with the cosine
// matrix along every axis: result S (extent P+1 per axis), layout fastest axis 0.
int transform_all_axes(gofd_ctx_s* ctx, int d, long long Mh, int P, const double* F, const double* C, DevBuf& w1,
                       DevBuf& w2, double* S) {
  hipStream_t st = ctx->stream;
  long long ext[3] = {Mh, Mh, Mh};
  const double* in = F;
  for (int ax = 0; ax < d; ++ax) {
    long long inner = 1, outer = 1;
    for (int q = 0; q < ax; ++q) inner *= ext[q];
    for (int q = ax + 1; q < d; ++q) outer *= ext[q];
    double* out = (ax == d - 1) ? S : ((ax % 2 == 0) ? w1.as<double>() : w2.as<double>());
    GemmArgs g{};
    if (ax == 0) {
      // rows of the array: out[o][p] = sum_j in[o][j] C[j][p]
      g.A = in; g.sAb = 0; g.sAm = Mh; g.sAk = 1;
      g.B = C; g.sBb = 0; g.sBk = P + 1; g.sBn = 1;
      g.C = out; g.sCb = 0; g.sCm = P + 1; g.sCn = 1;
      g.Mm = outer; g.Nn = P + 1; g.Kk = Mh;
      gemm(st, g, 1);
    } else {
      // for each outer block: out[o][p][i] = sum_j C[j][p] in[o][j][i]
      g.A = C; g.sAb = 0; g.sAm = 1; g.sAk = P + 1;
      g.B = in; g.sBb = Mh * inner; g.sBk = inner; g.sBn = 1;
      g.C = out; g.sCb = (long long)(P + 1) * inner; g.sCm = inner; g.sCn = 1;
      g.Mm = P + 1; g.Nn = inner; g.Kk = Mh;
      gemm(st, g, outer);
    }
    ext[ax] = P + 1;
    in = out;
  }
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

}  // namespace

extern "C" int gofd_fd_weights(gofd_ctx ctx, double s, const gofd_grid* grid, const gofd_fdw_opts* opts,
                               gofd_fdop* out) {
  if (!ctx || !out) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  auto* op = new (std::nothrow) gofd_fdop_s();
  if (!op) return GOFD_E_OOM;
  std::unique_ptr<gofd_fdop_s> guard(op);
  GOFD_TRY(fdop_init_geometry(ctx, op, s, grid));
  const int d = op->d;
  const int P = 2 * op->N;
  long long M = opts && opts->M > 0 ? opts->M : (d == 2 ? (1LL << 14) : (1LL << 11));
  const int rich = opts ? opts->richardson : 1;
  if (M & (M - 1)) return gofd_fail(ctx, GOFD_E_ARG, "M must be a power of two");
  while (M / 2 < 2LL * P + 1) M *= 2;    // both levels need M_level >= 2P + 1
  const long long Mh = M / 2 + 1;
  long long nF = 1, nS = 1, nW = 1;
  for (int a = 0; a < d; ++a) {
    nF *= Mh;
    nS *= (P + 1);
  }
  nW = (d == 2) ? Mh * (P + 1) : Mh * Mh * (P + 1);
  DevBuf F, C0, C1, w1, w2, SM, SC;
  GOFD_TRY(dev_reserve(ctx, F, sizeof(double) * nF));
  GOFD_TRY(dev_reserve(ctx, C0, sizeof(double) * Mh * (P + 1)));
  GOFD_TRY(dev_reserve(ctx, C1, sizeof(double) * Mh * (P + 1)));
  GOFD_TRY(dev_reserve(ctx, w1, sizeof(double) * nW));
  GOFD_TRY(dev_reserve(ctx, w2, sizeof(double) * (d == 3 ? Mh * (P + 1) * (P + 1) : 1)));
  GOFD_TRY(dev_reserve(ctx, SM, sizeof(double) * nS));
  GOFD_TRY(dev_reserve(ctx, SC, sizeof(double) * nS));
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_psi_samples, dim3(grid1(nF, 256)), dim3(256), 0, st, F.as<double>(), d, Mh, M, s);
  hipLaunchKernelGGL(k_cos_matrix, dim3(grid1(Mh * (P + 1), 256)), dim3(256), 0, st, C0.as<double>(), Mh, P, M, 0);
  hipLaunchKernelGGL(k_cos_matrix, dim3(grid1(Mh * (P + 1), 256)), dim3(256), 0, st, C1.as<double>(), Mh, P, M, 1);
  GOFD_TRY(transform_all_axes(ctx, d, Mh, P, F.as<double>(), C0.as<double>(), w1, w2, SM.as<double>()));
  if (rich) GOFD_TRY(transform_all_axes(ctx, d, Mh, P, F.as<double>(), C1.as<double>(), w1, w2, SC.as<double>()));
  GOFD_TRY(dev_reserve(ctx, op->T, sizeof(double) * nS));
  hipLaunchKernelGGL(k_finalize, dim3(grid1(nS, 256)), dim3(256), 0, st, SM.as<double>(), SC.as<double>(),
                     op->T.as<double>(), d, P, M, rich);
  HIP_TRY(ctx, hipGetLastError());
  op->T_host.resize(nS);
  HIP_TRY(ctx, hipMemcpyAsync(op->T_host.data(), op->T.p, sizeof(double) * nS, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  GOFD_TRY(fdop_finish(ctx, op));
  *out = guard.release();
  return GOFD_OK;
}
