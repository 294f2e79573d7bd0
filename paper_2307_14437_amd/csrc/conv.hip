// A_FD products by circulant embedding (Section 2.2, eq. AU-1), and A_h.
//
// The (2N+1)^d window is embedded in a grid of period L (the smallest power
// of two >= 4N) with the even kernel c_r = T_{|r|} for |r| <= 2N (wrapped
// modulo L, zero elsewhere).  For L = 4N the wrap puts T_{2N} at r = 2N, which
// is exact because T is even (eq. T-2).  The DFT of c is real and even, so
// only (L/2+1)^d values are stored, with the 1/L^d of the inverse folded in.
//
// 2D schedule (three passes over HBM, each line transformed in LDS):
//   A  row pairs: gather v = I u (or read a grid field), pack two real rows as
//      one complex line, forward FFT, split into the two half spectra,
//      write Z[row][k0] (k0 = 0..L/2);
//   B  groups of adjacent k0 columns: forward FFT along rows (W nonzero of
//      L), multiply by the real spectrum, inverse FFT, keep the W window
//      rows, in place;
//   C  row pairs: rebuild the Hermitian spectra of two real rows as one
//      complex line, inverse FFT, write the W window values.
#include <cmath>
#include <cstring>
#include <memory>

#include "bary.h"
#include "fft.h"
#include "internal.h"

using gofd_fft::fft_line;
using gofd_fft::padded_len;
using gofd_fft::pidx;

namespace {

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); renumber them so that logically adjacent blocks share an XCD.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int per = n / 8, rem = n % 8;
  const int x = b % 8, i = b / 8;
  const int start = (x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  return start + i;
}

// ---------------------------------------------------------------- sources

struct SrcGrid {
  const double* v;
  long long n_nodes;
  __device__ __forceinline__ double operator()(int rhs, long long k) const { return v[rhs * n_nodes + k]; }
};

template <int D>
struct SrcGather {
  GridGeom g;
  const ElemRec<D>* recs;
  const int* elem;
  const double* u;
  const double* scale;
  const double* mask;
  long long nv;
  __device__ __forceinline__ double operator()(int rhs, long long k) const {
    const int e = elem[k];
    if (e < 0) return 0.0;
    int vid[D + 1];
    double lam[D + 1];
    node_weights<D>(g, recs, e, k, vid, lam);
    const double* ur = u + rhs * nv;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r <= D; ++r) {
      double uv = ur[vid[r]];
      if (scale) uv *= scale[vid[r]];
      if (mask) uv *= mask[vid[r]];
      s += lam[r] * uv;
    }
    return s;
  }
};

// ---------------------------------------------------------------- pass A
// LINES row pairs per block, TPL threads per row pair.
template <typename R, int L, int LINES, int TPL, class Src>
__global__ __launch_bounds__(LINES* TPL) void k_passA(Src src, cplx<R>* __restrict__ Z, int W, int half,
                                                      const cplx<R>* __restrict__ tw, long long zs) {
  constexpr int PL = padded_len<L>();
  __shared__ cplx<R> sbuf[LINES * PL];
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* buf = sbuf + line * PL;
  const int row0 = (blockIdx.x * LINES + line) * 2;
  const int rhs = blockIdx.y;
  const bool has0 = row0 < W;
  const bool has1 = row0 + 1 < W;
#pragma unroll
  for (int m = t; m < L; m += TPL) {
    R a = 0, b = 0;
    if (m < W) {
      if (has0) a = (R)src(rhs, (long long)row0 * W + m);
      if (has1) b = (R)src(rhs, (long long)(row0 + 1) * W + m);
    }
    buf[pidx<L>(m)] = {a, b};
  }
  __syncthreads();
  fft_line<R, L, TPL, false>(buf, tw, t);
  if (!has0) return;
  cplx<R>* z0 = Z + rhs * zs + (long long)row0 * half;
  for (int k = t; k < half; k += TPL) {
    const cplx<R> zk = buf[pidx<L>(k)];
    const cplx<R> zm = buf[pidx<L>((L - k) & (L - 1))];
    z0[k] = {(zk.x + zm.x) * (R)0.5, (zk.y - zm.y) * (R)0.5};
    if (has1) z0[half + k] = {(zk.y + zm.y) * (R)0.5, (zm.x - zk.x) * (R)0.5};
  }
}

// ---------------------------------------------------------------- pass B
// Column slots 0..L/2-1: slot c > 0 is spectrum column k0 = c; slot 0 carries
// the two real columns k0 = 0 and k0 = L/2 packed as one complex column
// (after pass A both are exactly real), so the slots divide evenly into blocks.
// For the packed slot, with C = FFT(a + i b) and m = L - k:
//   A_k = (C_k + conj C_m)/2,  i B_k = (C_k - conj C_m)/2, and the product
//   D = T0 A + i T1 B gives D_k = (T0+T1)/2 C_k + (T0-T1)/2 conj C_m;
// the inverse FFT of D is (T0 * a) + i (T1 * b) with both parts real.
template <typename R, int L, int LINES, int NT>
__global__ __launch_bounds__(NT) void k_passB(cplx<R>* __restrict__ Z, int W, int half, const R* __restrict__ That,
                                              const cplx<R>* __restrict__ tw, long long zs) {
  constexpr int TPL = NT / LINES;
  constexpr int PL = padded_len<L>();
  constexpr int NQ = L / 2;                 // Nyquist column
  __shared__ cplx<R> buf[LINES * PL];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int rhs = blockIdx.y;
  const int k0 = b * LINES;
  cplx<R>* Zr = Z + rhs * zs;
#pragma unroll
  for (int idx = threadIdx.x; idx < L * LINES; idx += NT) {
    const int c = idx % LINES, i = idx / LINES;
    const int col = k0 + c;
    cplx<R> v = {0, 0};
    if (i < W) {
      if (col == 0)
        v = {Zr[(long long)i * half].x, Zr[(long long)i * half + NQ].x};
      else
        v = Zr[(long long)i * half + col];
    }
    buf[c * PL + pidx<L>(i)] = v;
  }
  __syncthreads();
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* lb = buf + line * PL;
  fft_line<R, L, TPL, false>(lb, tw, t);
  {
    const int col = k0 + line;
    if (col == 0) {
      for (int k1 = t; k1 <= L / 2; k1 += TPL) {
        const int m = (L - k1) & (L - 1);
        const R t0 = That[k1];                            // multiplier column k0 = 0
        const R t1 = That[(long long)NQ * half + k1];     // multiplier column k0 = L/2
        const R p = (t0 + t1) * (R)0.5, q = (t0 - t1) * (R)0.5;
        const cplx<R> ck = lb[pidx<L>(k1)], cm = lb[pidx<L>(m)];
        lb[pidx<L>(k1)] = {p * ck.x + q * cm.x, p * ck.y - q * cm.y};
        if (m != k1) lb[pidx<L>(m)] = {p * cm.x + q * ck.x, p * cm.y - q * ck.y};
      }
    } else {
      const R* Tc = That + (long long)col * half;
      for (int k1 = t; k1 < L; k1 += TPL) {
        const int kk = (k1 <= L / 2) ? k1 : L - k1;
        const R mlt = Tc[kk];
        cplx<R> v = lb[pidx<L>(k1)];
        lb[pidx<L>(k1)] = {v.x * mlt, v.y * mlt};
      }
    }
  }
  __syncthreads();
  fft_line<R, L, TPL, true>(lb, tw, t);
#pragma unroll 4
  for (int idx = threadIdx.x; idx < W * LINES; idx += NT) {
    const int c = idx % LINES, i = idx / LINES;
    const int col = k0 + c;
    const cplx<R> v = buf[c * PL + pidx<L>(i)];
    if (col == 0) {
      Zr[(long long)i * half] = {v.x, (R)0};
      Zr[(long long)i * half + NQ] = {v.y, (R)0};
    } else {
      Zr[(long long)i * half + col] = v;
    }
  }
}

// ---------------------------------------------------------------- pass C
template <typename R, typename Y, int L, int LINES, int TPL>
__global__ __launch_bounds__(LINES* TPL) void k_passC(const cplx<R>* __restrict__ Z, int W, int half,
                                                      const cplx<R>* __restrict__ tw, long long zs,
                                                      Y* __restrict__ y, long long n_nodes) {
  constexpr int PL = padded_len<L>();
  __shared__ cplx<R> sbuf[LINES * PL];
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* buf = sbuf + line * PL;
  const int row0 = (blockIdx.x * LINES + line) * 2;
  const int rhs = blockIdx.y;
  const bool has0 = row0 < W;
  const bool has1 = row0 + 1 < W;
  const cplx<R>* z0 = Z + rhs * zs + (long long)row0 * half;
#pragma unroll 4
  for (int k = t; k < half; k += TPL) {
    cplx<R> a = has0 ? z0[k] : cplx<R>{0, 0};
    cplx<R> b = has1 ? z0[half + k] : cplx<R>{0, 0};
    if (k == 0 || k == L / 2) {
      a.y = 0;
      b.y = 0;
    }
    buf[pidx<L>(k)] = {a.x - b.y, a.y + b.x};                                 // a + i b
    if (k > 0 && k < L / 2) buf[pidx<L>(L - k)] = {a.x + b.y, b.x - a.y};     // conj(a) + i conj(b)
  }
  __syncthreads();
  fft_line<R, L, TPL, true>(buf, tw, t);
  if (!has0) return;
  Y* yr = y + rhs * n_nodes + (long long)row0 * W;
  for (int m = t; m < W; m += TPL) {
    const cplx<R> v = buf[pidx<L>(m)];
    yr[m] = (Y)v.x;
    if (has1) yr[W + m] = (Y)v.y;
  }
}

// ---------------------------------------------------------------- launch

template <int L>
struct Cfg {
  static constexpr int TPL = (L / 8 < 512) ? L / 8 : 512;                  // threads per line
  static constexpr int LINES_A = (TPL >= 64) ? 1 : 64 / TPL;               // row pairs per block
  static constexpr int LINES_B = (L <= 256) ? ((L / 2 >= 8) ? 8 : L / 2) : (L <= 2048 ? 4 : 2);   // columns per block
  static constexpr int NT_A = LINES_A * TPL;
  static constexpr int NT_B = LINES_B * TPL;
};

template <typename R, int L, class Src, typename Y>
int run_2d(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes = 7) {
  const int W = op->W, half = op->half;
  const long long zs = (long long)W * half;
  const cplx<R>* tw;
  const R* That;
  if constexpr (sizeof(R) == 8) {
    tw = twiddles64(ctx, L);
    That = op->That64.as<R>();
  } else {
    tw = twiddles32(ctx, L);
    That = op->That32.as<R>();
  }
  if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddle table");
  GOFD_TRY(dev_reserve(ctx, op->Z, sizeof(cplx<R>) * zs * nrhs));
  cplx<R>* Z = op->Z.as<cplx<R>>();
  using C = Cfg<L>;
  const int pairs = (W + 1) / 2;
  const int nbA = (pairs + C::LINES_A - 1) / C::LINES_A;
  hipStream_t st = ctx->stream;
  if (passes & 1)
    hipLaunchKernelGGL((k_passA<R, L, C::LINES_A, C::TPL, Src>), dim3(nbA, nrhs), dim3(C::NT_A), 0, st, src, Z, W,
                       half, tw, zs);
  const int nb = (L / 2) / Cfg<L>::LINES_B;     // column slots 0..L/2-1 (DC and Nyquist share slot 0)
  if (passes & 2)
    hipLaunchKernelGGL((k_passB<R, L, Cfg<L>::LINES_B, Cfg<L>::NT_B>), dim3(nb, nrhs), dim3(Cfg<L>::NT_B), 0, st,
                       Z, W, half, That, tw, zs);
  if (passes & 4)
    hipLaunchKernelGGL((k_passC<R, Y, L, C::LINES_A, C::TPL>), dim3(nbA, nrhs), dim3(C::NT_A), 0, st, Z, W, half,
                       tw, zs, y, (long long)W * W);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

template <typename R, class Src, typename Y>
int dispatch_2d(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes = 7) {
  switch (op->L) {
    case 8: return run_2d<R, 8>(ctx, op, nrhs, src, y, passes);
    case 16: return run_2d<R, 16>(ctx, op, nrhs, src, y, passes);
    case 32: return run_2d<R, 32>(ctx, op, nrhs, src, y, passes);
    case 64: return run_2d<R, 64>(ctx, op, nrhs, src, y, passes);
    case 128: return run_2d<R, 128>(ctx, op, nrhs, src, y, passes);
    case 256: return run_2d<R, 256>(ctx, op, nrhs, src, y, passes);
    case 512: return run_2d<R, 512>(ctx, op, nrhs, src, y, passes);
    case 1024: return run_2d<R, 1024>(ctx, op, nrhs, src, y, passes);
    case 2048: return run_2d<R, 2048>(ctx, op, nrhs, src, y, passes);
    case 4096: return run_2d<R, 4096>(ctx, op, nrhs, src, y, passes);
    default: return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "FFT length " + std::to_string(op->L) + " not built");
  }
}

// ---------------------------------------------------------------- spectrum of the embedding
//
// Tc = DFT of the even kernel, one axis at a time: along an axis the kernel is
// real and even with period L, so its DFT is the cosine sum
//   sum_r c_r cos(2 pi k r / L) = c_0 + 2 sum_{0<r<L/2} c_r cos(2 pi k r/L) + c_{L/2} cos(pi k)
// with c_r = T_r for r <= 2N and 0 beyond.  Direct sums in double precision.
__global__ void k_cos_axis(const double* __restrict__ in, double* __restrict__ out, int n_in, int n_out,
                           long long inner, long long outer, int L, int nmax, const cplx<double>* __restrict__ tw,
                           double scale) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = outer * n_out * inner;
  if (gid >= total) return;
  const long long i = gid % inner;
  const long long k = (gid / inner) % n_out;
  const long long o = gid / (inner * n_out);
  double s = 0.0;
  for (int r = 0; r <= nmax && r <= L / 2; ++r) {
    const double w = (r == 0 || 2 * r == L) ? 1.0 : 2.0;
    const long long t = (k * (long long)r) % L;
    s += w * in[(o * n_in + r) * inner + i] * tw[t].x;
  }
  out[gid] = s * scale;
}

__global__ void k_widen(const float* __restrict__ a, double* __restrict__ b, long long m) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) b[i] = (double)a[i];
}

__global__ void k_scale(double* __restrict__ a, long long m, double c) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) a[i] *= c;
}

__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

}  // namespace

int fdop_finish(gofd_ctx_s* ctx, gofd_fdop_s* op) {
  const int d = op->d, W = op->W, L = op->L, half = op->half;
  const cplx<double>* tw = twiddles64(ctx, L);
  if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddle table");
  long long n_out = 1;
  for (int a = 0; a < d; ++a) n_out *= half;
  GOFD_TRY(dev_reserve(ctx, op->That64, sizeof(double) * n_out));
  GOFD_TRY(dev_reserve(ctx, op->That32, sizeof(float) * n_out));
  // transform axis by axis: shapes go from W^d to half^d, fastest axis first
  DevBuf a, b;
  long long cap = 1;
  for (int q = 0; q < d; ++q) cap *= std::max(W, half);
  GOFD_TRY(dev_reserve(ctx, a, sizeof(double) * cap));
  GOFD_TRY(dev_reserve(ctx, b, sizeof(double) * cap));
  HIP_TRY(ctx, hipMemcpyAsync(a.p, op->T.p, sizeof(double) * (long long)std::pow(W, d), hipMemcpyDeviceToDevice,
                              ctx->stream));
  int dims[3] = {W, W, W};   // current extent per axis (axis 0 fastest)
  const double scale = 1.0 / (double)L;
  for (int ax = 0; ax < d; ++ax) {
    long long inner = 1, outer = 1;
    for (int q = 0; q < ax; ++q) inner *= dims[q];
    for (int q = ax + 1; q < d; ++q) outer *= dims[q];
    const long long total = outer * half * inner;
    hipLaunchKernelGGL(k_cos_axis, dim3(grid1(total, 256)), dim3(256), 0, ctx->stream, a.as<double>(),
                       b.as<double>(), dims[ax], half, inner, outer, L, 2 * op->N, tw, scale);
    dims[ax] = half;
    std::swap(a.p, b.p);
    std::swap(a.bytes, b.bytes);
  }
  HIP_TRY(ctx, hipMemcpyAsync(op->That64.p, a.p, sizeof(double) * n_out, hipMemcpyDeviceToDevice, ctx->stream));
  hipLaunchKernelGGL(k_to_f32, dim3(grid1(n_out, 256)), dim3(256), 0, ctx->stream, op->That64.as<double>(),
                     op->That32.as<float>(), n_out);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return GOFD_OK;
}

int conv_prepare(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs) {
  if (!twiddles64(ctx, op->L) || !twiddles32(ctx, op->L)) return gofd_fail(ctx, GOFD_E_OOM, "twiddle table");
  long long zs = 1;
  for (int a = 0; a < op->d; ++a) zs *= (a == 0 ? op->half : op->W);
  return dev_reserve(ctx, op->Z, sizeof(cplx<double>) * zs * nrhs);
}

int conv_apply(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const double* v, const GatherSpec* g, void* y,
               bool fp32, int passes) {
  if (op->d != 2) return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "3D product not built yet");
  if (v) {
    SrcGrid src{v, (long long)op->W * op->W};
    return fp32 ? dispatch_2d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes)
                : dispatch_2d<double>(ctx, op, nrhs, src, static_cast<double*>(y), passes);
  }
  const gofd_transfer_s* tr = g->tr;
  SrcGather<2> src;
  src.g.d = 2;
  src.g.W = tr->W;
  src.g.h = tr->h;
  for (int a = 0; a < 3; ++a) src.g.lo[a] = tr->lo[a];
  src.recs = tr->rec.as<ElemRec2>();
  src.elem = tr->elem.as<int>();
  src.u = g->u;
  src.scale = g->col_scale;
  src.mask = g->mask;
  src.nv = tr->nv;
  return fp32 ? dispatch_2d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes)
              : dispatch_2d<double>(ctx, op, nrhs, src, static_cast<double*>(y), passes);
}

// ---------------------------------------------------------------- ABI

bool same_grid(const gofd_transfer_s* tr, const gofd_fdop_s* op) {
  return tr->d == op->d && tr->N == op->N && tr->R == op->R && tr->center[0] == op->center[0] &&
         tr->center[1] == op->center[1] && tr->center[2] == op->center[2];
}

extern "C" int gofd_apply_afd(gofd_ctx ctx, gofd_fdop op, int nrhs, const double* v, double* y, int flags) {
  if (!ctx || !op || !v || !y || nrhs < 1) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  const bool fp32 = flags & GOFD_FP32_GRID;
  if (!fp32) return conv_apply(ctx, op, nrhs, v, nullptr, y, false);
  long long n = (long long)std::pow(op->W, op->d) * nrhs;
  GOFD_TRY(dev_reserve(ctx, op->Y, sizeof(float) * n));
  GOFD_TRY(conv_apply(ctx, op, nrhs, v, nullptr, op->Y.p, true));
  // widen to the double output
  hipLaunchKernelGGL(k_widen, dim3(grid1(n, 256)), dim3(256), 0, ctx->stream, op->Y.as<float>(), y, n);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

extern "C" int gofd_apply_Ah(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int nrhs, const double* u, double* y,
                             int flags) {
  if (!ctx || !tr || !op || !u || !y || nrhs < 1) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  const bool fp32 = flags & GOFD_FP32_GRID;
  const bool sym = flags & GOFD_SYMMETRIC;
  const bool unscaled = flags & GOFD_UNSCALED;
  const bool interior = flags & GOFD_INTERIOR;
  if (sym && unscaled) return gofd_fail(ctx, GOFD_E_ARG, "SYMMETRIC and UNSCALED are exclusive");
  const long long n_nodes = tr->n_nodes;
  GOFD_TRY(dev_reserve(ctx, op->Y, (fp32 ? sizeof(float) : sizeof(double)) * n_nodes * nrhs));
  GatherSpec g;
  g.tr = tr;
  g.u = u;
  g.col_scale = sym ? tr->dsqrt.as<double>() : nullptr;
  g.mask = interior ? tr->imask.as<double>() : nullptr;
  GOFD_TRY(conv_apply(ctx, op, nrhs, nullptr, &g, op->Y.p, fp32));
  const double* scale = unscaled ? nullptr : (sym ? tr->dsqrt.as<double>() : tr->dscale.as<double>());
  GOFD_TRY(scatter_apply(ctx, tr, nrhs, op->Y.p, fp32, scale, interior ? tr->imask.as<double>() : nullptr, y));
  if (flags & GOFD_SCALE_H2S) {
    const double f = 1.0 / op->h2s;
    long long n = tr->nv * nrhs;
    hipLaunchKernelGGL(k_scale, dim3(grid1(n, 256)), dim3(256), 0, ctx->stream, y, n, f);
  }
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

// ---------------------------------------------------------------- operator from a table

static int next_pow2(long long x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

int fdop_init_geometry(gofd_ctx_s* ctx, gofd_fdop_s* op, double s, const gofd_grid* grid) {
  if (!grid || (grid->d != 2 && grid->d != 3) || grid->N < 1 || !(grid->R > 0))
    return gofd_fail(ctx, GOFD_E_ARG, "bad grid");
  if (!(s > 0.0 && s < 1.0)) return gofd_fail(ctx, GOFD_E_ARG, "s must lie in (0, 1)");
  op->ctx = ctx;
  op->d = grid->d;
  op->N = grid->N;
  op->W = 2 * grid->N + 1;
  op->L = next_pow2(4LL * grid->N);
  op->half = op->L / 2 + 1;
  op->s = s;
  op->R = grid->R;
  for (int a = 0; a < 3; ++a) op->center[a] = a < grid->d ? grid->center[a] : 0.0;
  op->h = grid->R / (double)grid->N;
  op->h2s = std::pow(op->h, 2.0 * s);
  return GOFD_OK;
}

extern "C" int gofd_fdop_from_table(gofd_ctx ctx, double s, const gofd_grid* grid, const double* T_host,
                                    gofd_fdop* out) {
  if (!ctx || !out || !T_host) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  auto* op = new (std::nothrow) gofd_fdop_s();
  if (!op) return GOFD_E_OOM;
  std::unique_ptr<gofd_fdop_s> guard(op);
  GOFD_TRY(fdop_init_geometry(ctx, op, s, grid));
  long long n = 1;
  for (int a = 0; a < op->d; ++a) n *= op->W;
  op->T_host.assign(T_host, T_host + n);
  GOFD_TRY(dev_reserve(ctx, op->T, sizeof(double) * n));
  HIP_TRY(ctx, hipMemcpyAsync(op->T.p, op->T_host.data(), sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
  GOFD_TRY(fdop_finish(ctx, op));
  *out = guard.release();
  return GOFD_OK;
}

extern "C" int gofd_fdop_get_table(gofd_ctx ctx, gofd_fdop op, double* T_host) {
  if (!ctx || !op || !T_host) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  std::memcpy(T_host, op->T_host.data(), sizeof(double) * op->T_host.size());
  return GOFD_OK;
}

extern "C" int gofd_fdop_free(gofd_fdop op) {
  if (!op) return GOFD_E_ARG;
  (void)hipDeviceSynchronize();
  delete op;
  return GOFD_OK;
}

extern "C" int gofd_time_kernel(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int which, int nrhs, const double* u,
                                int flags, int reps, double* avg_ms) {
  if (!ctx || !tr || !op || !u || !avg_ms || nrhs < 1 || reps < 1 || which < 0 || which > 3)
    return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  const bool fp32 = flags & GOFD_FP32_GRID;
  WorkStream ws(ctx);
  GOFD_TRY(conv_prepare(ctx, op, nrhs));
  GOFD_TRY(dev_reserve(ctx, op->Y, sizeof(double) * tr->n_nodes * nrhs));
  DevBuf z;
  GOFD_TRY(dev_reserve(ctx, z, sizeof(double) * tr->nv * nrhs));
  GatherSpec g;
  g.tr = tr;
  g.u = u;
  g.mask = tr->imask.as<double>();
  // fill the workspaces once with a full product
  GOFD_TRY(conv_apply(ctx, op, nrhs, nullptr, &g, op->Y.p, fp32, 7));
  auto launch = [&]() -> int {
    if (which == GOFD_K_SCATTER)
      return scatter_apply(ctx, tr, nrhs, op->Y.p, fp32, nullptr, tr->imask.as<double>(), z.as<double>());
    return conv_apply(ctx, op, nrhs, nullptr, &g, op->Y.p, fp32, 1 << which);
  };
  GOFD_TRY(launch());
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  HIP_TRY(ctx, hipEventRecord(e0, ctx->stream));
  int rc = GOFD_OK;
  for (int i = 0; i < reps && rc == GOFD_OK; ++i) rc = launch();
  HIP_TRY(ctx, hipEventRecord(e1, ctx->stream));
  HIP_TRY(ctx, hipEventSynchronize(e1));
  float ms = 0.f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  GOFD_TRY(rc);
  *avg_ms = ms / reps;
  return GOFD_OK;
}
