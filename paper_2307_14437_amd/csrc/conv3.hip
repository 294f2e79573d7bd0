// 3D A_FD products by circulant embedding (Section 2.2, eq. AU-1 in three
// dimensions), five passes over HBM, each line transformed by one group of
// threads with values in registers and LDS exchanges between the Stockham
// stages:
//   A  x-row pairs: pack two real rows as one complex line, forward FFT,
//      split into the two half spectra k0 = 0..L/2, write Z1;
//   B  y-lines (slot k0, plane i2): forward FFT over i1 (W nonzero of L),
//      write all L values to Z2;
//   C  z-lines (slot k0, k1): forward FFT over i2, multiply by the real
//      spectrum of the embedded kernel, inverse FFT, keep the W rows, in place;
//   D  y-lines: inverse FFT over k1, keep the W rows, write Z1;
//   E  x-row pairs: rebuild the Hermitian spectra of two real rows as one
//      complex line, inverse FFT, write the W window values of both rows.
// Layouts per rhs (slots in tiles of four, like the 2D product):
//   Z1[slot/4][row][slot%4], row = i1 + W i2 (W^2 rows), slots 0..L/2;
//   Z2[slot/4][i2][k1][slot%4], k1 = 0..L-1.
// Unlike the 2D product, the real columns k0 = 0 and L/2 are kept as their
// own slots (one extra slot out of L/2 + 1), which keeps every line
// independent in the later passes.
#include <cmath>

#include "cg_state.h"
#include "conv_common.h"
#include "fft.h"
#include "internal.h"

using gofd_fft::fft_regs;
using gofd_fft::padded_len;
using gofd_fft::pidx;

namespace {

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ long long z1idx(int slot, long long row, long long nrow) {
  return ((long long)(slot >> 2) * nrow + row) * 4 + (slot & 3);
}
__device__ __forceinline__ long long z2idx(int slot, int i2, int k1, int W, int L) {
  return (((long long)(slot >> 2) * W + i2) * L + k1) * 4 + (slot & 3);
}

// ---------------------------------------------------------------- pass A
template <typename R, int L, int E, int LINES, class Src>
__global__ __launch_bounds__(LINES*(L / E)) void k_p3A(Src src, cplx<R>* __restrict__ Z1, int W,
                                                       const cplx<R>* __restrict__ tw, long long z1s, Skip skip) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int H = L / 2;
  __shared__ cplx<R> sbuf[LINES * PL];
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* buf = sbuf + line * PL;
  const long long nrow = (long long)W * W;
  const long long row0 = ((long long)xcd_remap(blockIdx.x, gridDim.x) * LINES + line) * 2;
  const int rhs = skip.item(blockIdx.y);
  const bool has0 = row0 < nrow;
  const bool has1 = row0 + 1 < nrow;
  const long long r0c = has0 ? row0 : nrow - 1, r1c = has1 ? row0 + 1 : r0c;
  cplx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int col = t + m * TPL;
    R x = 0, y = 0;
    if (m <= E / 2) {                  // loads from clamped positions, masked after
      const int cc = col < W ? col : W - 1;
      x = (R)src(rhs, r0c * W + cc);
      y = (R)src(rhs, r1c * W + cc);
      if (!has0 || col >= W) x = 0;
      if (!has1 || col >= W) y = 0;
    }
    v[m] = {x, y};
  }
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  if (skip(rhs)) return;
  fft_regs<R, L, E, false>(v, buf, tws, t);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) buf[pidx<E>(t + m * TPL)] = v[m];
  __syncthreads();
  if (!has0) return;
  cplx<R>* Zr = Z1 + rhs * z1s;
#pragma unroll
  for (int q = 0; q <= E / 2; ++q) {
    const int k = t + q * TPL;
    if (q == E / 2 && t != 0) break;                       // k = L/2 once
    const cplx<R> zk = buf[pidx<E>(k)], zm = buf[pidx<E>((L - k) & (L - 1))];
    const cplx<R> z0 = {(zk.x + zm.x) * (R)0.5, (zk.y - zm.y) * (R)0.5};
    const cplx<R> z1 = {(zk.y + zm.y) * (R)0.5, (zm.x - zk.x) * (R)0.5};
    cplx<R>* dst = Zr + z1idx(k, row0, nrow);
    dst[0] = z0;
    if (has1) dst[4] = z1;
    (void)H;
  }
}

// ---------------------------------------------------------------- passes B and D (y lines)
// Block: LB slots of one plane i2.  INV = false: Z1 -> forward FFT -> Z2 (all
// L values); INV = true: Z2 -> inverse FFT -> Z1 (the W window rows).
template <typename R, int L, int E, int LB, bool INV>
__global__ __launch_bounds__(LB*(L / E)) void k_p3BD(cplx<R>* __restrict__ Z1, cplx<R>* __restrict__ Z2, int W,
                                                      int nsb, const cplx<R>* __restrict__ tw, long long z1s,
                                                      long long z2s, Skip skip) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int H = L / 2;
  __shared__ cplx<R> sbuf[LB * PL];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int sb = b % nsb, i2 = b / nsb;
  const int c = threadIdx.x % LB, t = threadIdx.x / LB;
  cplx<R>* buf = sbuf + c * PL;
  const int slot = sb * LB + c;
  const bool act = slot <= H;
  const long long nrow = (long long)W * W;
  const int rhs = skip.item(blockIdx.y);
  cplx<R>* Z1r = Z1 + rhs * z1s;
  cplx<R>* Z2r = Z2 + rhs * z2s;
  // loads from clamped in-range positions, masked after (all in flight together)
  const int sc = act ? slot : H;
  cplx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TPL;
    if constexpr (!INV) {
      if (m <= E / 2) {
        v[m] = Z1r[z1idx(sc, (long long)i2 * W + (i < W ? i : W - 1), nrow)];
        if (!act || i >= W) v[m] = cplx<R>{0, 0};
      } else {
        v[m] = cplx<R>{0, 0};
      }
    } else {
      v[m] = Z2r[z2idx(sc, i2, i, W, L)];
      if (!act) v[m] = cplx<R>{0, 0};
    }
  }
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  if (skip(rhs)) return;
  fft_regs<R, L, E, INV>(v, buf, tws, t);
  if (!act) return;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TPL;
    if constexpr (!INV)
      Z2r[z2idx(slot, i2, i, W, L)] = v[m];
    else if (m <= E / 2 && i < W)
      Z1r[z1idx(slot, (long long)i2 * W + i, nrow)] = v[m];
  }
}

// ---------------------------------------------------------------- pass C (z lines)
// Block: LB slots of one k1.  Forward FFT over i2, multiply by That at
// (k0, |k1|, |k2|) folded to 0..L/2, inverse FFT, keep the W rows.  With DOT,
// the block also leaves (A v, v) of its lines by Parseval (columns
// 0 < k0 < L/2 count twice) and the sums of its slice of the level-1
// partials: dpart[rhs][q][block], q = gamma, (r, r), delta.
template <typename R, int L, int E, int LB, bool DOT>
__global__ __launch_bounds__(LB*(L / E), (LB * (L / E) >= 256) ? 2 : 1) void k_p3C(cplx<R>* __restrict__ Z2, int W, int half, int nsb,
                                                     const R* That, const cplx<R>* __restrict__ tw,
                                                     long long z2s, Skip skip, double* __restrict__ dpart,
                                                     gofd_cg::Level1 lv1, const void* const* __restrict__ that_tab) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int H = L / 2;
  constexpr int NT = LB * TPL;
  __shared__ cplx<R> sbuf[LB * PL];
  __shared__ double shd[gofd_cg::block_sum_lds<NT, 3>()];
  // consecutive blocks take consecutive k1 of one slot group: a block reads
  // 4 slots (32 or 64 bytes) per z row, and the blocks that share those rows'
  // cache lines (the next k1) run next to it on the same XCD
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int sb = b / L, k1 = b % L;
  (void)nsb;
  const int c = threadIdx.x % LB, t = threadIdx.x / LB;
  cplx<R>* buf = sbuf + c * PL;
  const int slot = sb * LB + c;
  const bool act = slot <= H;
  const int rhs = skip.item(blockIdx.y);
  cplx<R>* Zr = Z2 + rhs * z2s;
  cplx<R> v[E];
  R pm[E];
  const int kk1 = (k1 <= H) ? k1 : L - k1;
  if (that_tab) That = static_cast<const R*>(that_tab[rhs]);     // per-item spectrum (batched solves)
  // That is half^3 with axis 0 fastest; by symmetry of the kernel the axes
  // may take k0, k1, k2 in any order: index (k0 half + k1) half + k2, so
  // that a thread's z frequencies are consecutive entries
  const int sc = act ? slot : H;
  const R* Tc = That + ((long long)sc * half + kk1) * half;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TPL;
    if (m <= E / 2) {
      v[m] = Zr[z2idx(sc, i < W ? i : W - 1, k1, W, L)];
      if (!act || i >= W) v[m] = cplx<R>{0, 0};
    } else {
      v[m] = cplx<R>{0, 0};
    }
    const int kk2 = (i <= H) ? i : L - i;
    pm[m] = Tc[kk2];
    if (!act) pm[m] = (R)0;
  }
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  double red[3] = {0.0, 0.0, 0.0};
  if constexpr (DOT) {
    const int chunk = (lv1.n1 + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * chunk, hi = min(lo + chunk, lv1.n1);
    for (int i = lo + threadIdx.x; i < hi; i += NT) {
      red[0] += lv1.partG[(long long)rhs * lv1.n1 + i];
      red[1] += lv1.partR[(long long)rhs * lv1.n1 + i];
    }
  }
  if (skip(rhs)) return;
  fft_regs<R, L, E, false>(v, buf, tws, t);
  const double wgt = (slot == 0 || slot == H) ? 1.0 : 2.0;
  // terms That_k |V_k|^2 in the grid precision, summed in double
  double dsum = 0.0;
#pragma unroll
  for (int m = 0; m < E; ++m) {
    if constexpr (DOT) dsum += (double)(pm[m] * (v[m].x * v[m].x + v[m].y * v[m].y));
    v[m] = {v[m].x * pm[m], v[m].y * pm[m]};
  }
  red[2] += wgt * dsum;
  if constexpr (DOT) {
    gofd_cg::block_sum_n<NT, 3>(red, shd);
    if (threadIdx.x == 0) {
      double* d = dpart + (long long)rhs * 3 * gridDim.x;
      d[blockIdx.x] = red[0];
      d[gridDim.x + blockIdx.x] = red[1];
      d[2 * gridDim.x + blockIdx.x] = red[2];
    }
  }
  __syncthreads();
  tws.opaque();
  fft_regs<R, L, E, true>(v, buf, tws, t);
  if (!act) return;
#pragma unroll
  for (int m = 0; m <= E / 2; ++m) {
    const int i = t + m * TPL;
    if (i < W) Zr[z2idx(slot, i, k1, W, L)] = v[m];
  }
}

// ---------------------------------------------------------------- pass E
// With fin active, one extra block (the last) finishes the CG reductions.
template <typename R, typename Y, int L, int E, int LINES>
__global__ __launch_bounds__(LINES*(L / E)) void k_p3E(const cplx<R>* __restrict__ Z1, int W,
                                                       const cplx<R>* __restrict__ tw, long long z1s,
                                                       Y* __restrict__ y, long long n_nodes, Skip skip,
                                                       gofd_cg::Finish fin) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int H = L / 2;
  constexpr int NT = LINES * TPL;
  __shared__ cplx<R> sbuf[LINES * PL];
  __shared__ double shf[gofd_cg::block_sum_lds<NT, 3>()];
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* buf = sbuf + line * PL;
  const int rhs = skip.item(blockIdx.y);
  if (fin.sc && blockIdx.x == gridDim.x - 1) {     // block-uniform: the finishing block
    fin.run<NT>(rhs, shf);
    return;
  }
  const int nrb = gridDim.x - (fin.sc ? 1 : 0);
  const long long nrow = (long long)W * W;
  const long long row0 = ((long long)xcd_remap(blockIdx.x, nrb) * LINES + line) * 2;
  const bool has0 = row0 < nrow;
  const bool has1 = row0 + 1 < nrow;
  const cplx<R>* Zr = Z1 + rhs * z1s;
  // rows past the end read row nrow - 1 (loads in flight together) and count as zero
  const long long r0c = has0 ? row0 : nrow - 1, r1c = has1 ? row0 + 1 : r0c;
  cplx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + m * TPL;
    const bool mirror = k > H;
    const int sl = mirror ? L - k : k;
    cplx<R> a = Zr[z1idx(sl, r0c, nrow)];
    cplx<R> bb = Zr[z1idx(sl, r1c, nrow)];
    if (!has0) a = cplx<R>{0, 0};
    if (!has1) bb = cplx<R>{0, 0};
    if (k == 0 || k == H) {                          // exactly real for real rows
      a.y = 0;
      bb.y = 0;
    }
    v[m] = mirror ? cplx<R>{a.x + bb.y, bb.x - a.y} : cplx<R>{a.x - bb.y, a.y + bb.x};
  }
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  if (skip(rhs)) return;
  fft_regs<R, L, E, true>(v, buf, tws, t);
  if (!has0) return;
  Y* yr = y + rhs * n_nodes + row0 * W;
#pragma unroll
  for (int m = 0; m <= E / 2; ++m) {
    const int col = t + m * TPL;
    if (col < W) {
      yr[col] = (Y)v[m].x;
      if (has1) yr[W + col] = (Y)v[m].y;
    }
  }
}

// ---------------------------------------------------------------- launch

// ALT = 1 selects the alternative schedule of the y/z/y passes: two slots per
// block where four are the default (more, smaller blocks)
template <typename R, int L, int ALT = 0>
struct Cfg3 {
  static constexpr int E = (L >= 16) ? 16 : L;
  static constexpr int TPL = L / E;
  static constexpr int LINES = (TPL >= 64) ? 1 : 64 / TPL;          // row pairs per block (A, E)
  static constexpr int LINE_BYTES = padded_len<L, E>() * (int)sizeof(cplx<R>);
  static constexpr int LB_DEF = (4 * TPL <= 1024 && 4 * LINE_BYTES <= 150 * 1024) ? 4 : 2;
  static constexpr bool HAS_ALT = LB_DEF == 4;
  static constexpr int LB = (ALT && HAS_ALT) ? 2 : LB_DEF;           // slots per block (B-D)
  static constexpr int NSLOT = L / 2 + 1;
  static constexpr int NTILE = (NSLOT + 3) / 4;
  static constexpr int NSB = NTILE * (4 / LB);                       // slot blocks per line set
};

template <typename R, int L, int ALT, class Src, typename Y>
int run_3d(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes, Skip skip, double* dpart,
           const gofd_cg::Level1& lv1, const gofd_cg::Finish& fin, const void* const* that_tab) {
  using C = Cfg3<R, L, ALT>;
  const int W = op->W, half = op->half;
  const long long z1s = (long long)C::NTILE * 4 * W * W;
  const long long z2s = (long long)C::NTILE * 4 * W * L;
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
  if (2 * (W - 1) > L) return gofd_fail(ctx, GOFD_E_ARG, "internal: window wider than half the period");
  if (!ctx->ws_Z) GOFD_TRY(dev_reserve(ctx, op->Z, sizeof(cplx<R>) * (z1s + z2s) * nrhs));
  cplx<R>* Z1 = ctx->ws_Z ? static_cast<cplx<R>*>(ctx->ws_Z) : op->Z.as<cplx<R>>();
  cplx<R>* Z2 = Z1 + z1s * nrhs;
  hipStream_t st = ctx->stream;
  const long long pairs = ((long long)W * W + 1) / 2;
  const unsigned nbA = (unsigned)((pairs + C::LINES - 1) / C::LINES);
  const dim3 gBD((unsigned)(C::NSB * W), nrhs), gC((unsigned)(C::NSB * L), nrhs);
  if (passes & 1)
    hipLaunchKernelGGL((k_p3A<R, L, C::E, C::LINES, Src>), dim3(nbA, nrhs), dim3(C::LINES * C::TPL), 0, st, src,
                       Z1, W, tw, z1s, skip);
  if (passes & 2) {
    hipLaunchKernelGGL((k_p3BD<R, L, C::E, C::LB, false>), gBD, dim3(C::LB * C::TPL), 0, st, Z1, Z2, W, C::NSB, tw,
                       z1s, z2s, skip);
    if (dpart)
      hipLaunchKernelGGL((k_p3C<R, L, C::E, C::LB, true>), gC, dim3(C::LB * C::TPL), 0, st, Z2, W, half, C::NSB,
                         That, tw, z2s, skip, dpart, lv1, that_tab);
    else
      hipLaunchKernelGGL((k_p3C<R, L, C::E, C::LB, false>), gC, dim3(C::LB * C::TPL), 0, st, Z2, W, half, C::NSB,
                         That, tw, z2s, skip, dpart, lv1, that_tab);
    hipLaunchKernelGGL((k_p3BD<R, L, C::E, C::LB, true>), gBD, dim3(C::LB * C::TPL), 0, st, Z1, Z2, W, C::NSB, tw,
                       z1s, z2s, skip);
  }
  if (passes & 4)
    hipLaunchKernelGGL((k_p3E<R, Y, L, C::E, C::LINES>), dim3(nbA + (fin.sc ? 1 : 0), nrhs),
                       dim3(C::LINES * C::TPL), 0, st, Z1, W, tw, z1s, y, (long long)W * W * W, skip, fin);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

// schedule of the 3D y/z/y passes in force for (L, precision): 0 or 1 (ALT)
int sched3_of(const gofd_ctx_s* ctx, int L, bool fp32) {
  auto it = ctx->sched3.find(std::make_pair(L, fp32));
  return it == ctx->sched3.end() ? 0 : it->second;
}

template <typename R, int L, class Src, typename Y>
int run_3d_s(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes, Skip skip,
             double* dpart, const gofd_cg::Level1& lv1, const gofd_cg::Finish& fin, const void* const* that_tab) {
  if (Cfg3<R, L>::HAS_ALT && sched3_of(op->ctx, L, sizeof(R) == 4) == 1)
    return run_3d<R, L, 1>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
  return run_3d<R, L, 0>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
}

template <typename R, class Src, typename Y>
int dispatch_3d(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes, Skip skip,
                double* dpart, const gofd_cg::Level1& lv1, const gofd_cg::Finish& fin, const void* const* that_tab) {
  switch (op->L) {
    case 8: return run_3d_s<R, 8>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 16: return run_3d_s<R, 16>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 32: return run_3d_s<R, 32>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 64: return run_3d_s<R, 64>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 128: return run_3d_s<R, 128>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 256: return run_3d_s<R, 256>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 512: return run_3d_s<R, 512>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    case 1024: return run_3d_s<R, 1024>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab);
    default: return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "3D FFT length " + std::to_string(op->L) + " not built");
  }
}

template <int L>
int p3c_blocks(const gofd_ctx_s* ctx, bool fp32) {
  const bool alt = sched3_of(ctx, L, fp32) == 1;
  if (fp32) return (alt ? Cfg3<float, L, 1>::NSB : Cfg3<float, L>::NSB) * L;
  return (alt ? Cfg3<double, L, 1>::NSB : Cfg3<double, L>::NSB) * L;
}

}  // namespace

long long conv3_workspace(const gofd_fdop_s* op) {
  const long long ntile = (op->L / 2 + 1 + 3) / 4;
  return ntile * 4 * (long long)op->W * (op->W + op->L);     // complex values per rhs (Z1 + Z2)
}

int conv3_passC_blocks(const gofd_fdop_s* op, bool fp32) {
  switch (op->L) {
    case 8: return p3c_blocks<8>(op->ctx, fp32);
    case 16: return p3c_blocks<16>(op->ctx, fp32);
    case 32: return p3c_blocks<32>(op->ctx, fp32);
    case 64: return p3c_blocks<64>(op->ctx, fp32);
    case 128: return p3c_blocks<128>(op->ctx, fp32);
    case 256: return p3c_blocks<256>(op->ctx, fp32);
    case 512: return p3c_blocks<512>(op->ctx, fp32);
    case 1024: return p3c_blocks<1024>(op->ctx, fp32);
    default: return 1;
  }
}

int conv3_run(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const double* v64, const float* v32, void* y, bool fp32,
              int passes, const int* skip_flag, int skip_stride, double* dpart, const gofd_cg::Level1& lv1,
              const gofd_cg::Finish& fin, const void* const* that_tab, const int* amap) {
  const Skip skip{skip_flag, skip_stride, amap};
  const long long nn = (long long)op->W * op->W * op->W;
  if (fp32) {
    if (v32) {
      SrcGrid<float> src{v32, nn};
      return dispatch_3d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes, skip, dpart, lv1, fin, that_tab);
    }
    SrcGrid<double> src{v64, nn};
    return dispatch_3d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes, skip, dpart, lv1, fin, that_tab);
  }
  SrcGrid<double> src{v64, nn};
  return dispatch_3d<double>(ctx, op, nrhs, src, static_cast<double*>(y), passes, skip, dpart, lv1, fin, that_tab);
}

// ---------------------------------------------------------------- schedule tuning (3D)

namespace {

template <typename R, int L, int ALT>
double time_yzy(gofd_ctx_s* ctx, gofd_fdop_s* op, double* dpart) {
  const long long nn = (long long)op->W * op->W * op->W;
  SrcGrid<double> src{nullptr, nn};
  const Skip skip{nullptr, 0};
  const gofd_cg::Level1 lv1;
  const gofd_cg::Finish fin;
  auto run = [&]() {
    return run_3d<R, L, ALT>(ctx, op, 1, src, static_cast<R*>(nullptr), 2, skip, dpart, lv1, fin, nullptr);
  };
  hipStream_t st = ctx->stream;
  for (int k = 0; k < 2; ++k)
    if (run() != GOFD_OK) return -1.0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  constexpr int reps = 10;
  (void)hipEventRecord(e0, st);
  for (int k = 0; k < reps; ++k) (void)run();
  (void)hipEventRecord(e1, st);
  float ms = -1.f;
  if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms < 0 ? -1.0 : ms / reps;
}

template <typename R, int L>
int tune3_L(gofd_ctx_s* ctx, gofd_fdop_s* op, double* times) {
  const bool fp32 = sizeof(R) == 4;
  const long long z = conv3_workspace(op);
  const long long nh = (long long)op->half * op->half * op->half;
  GOFD_TRY(dev_reserve(ctx, op->Z, sizeof(cplx<R>) * z));
  GOFD_TRY(dev_reserve(ctx, fp32 ? op->That32 : op->That64, sizeof(R) * nh));
  const long long nd = 3LL * std::max(Cfg3<R, L, 0>::NSB, Cfg3<R, L, 1>::NSB) * L;
  DevBuf dp;
  GOFD_TRY(dev_reserve(ctx, dp, sizeof(double) * nd));
  HIP_TRY(ctx, hipMemsetAsync(op->Z.p, 0, sizeof(cplx<R>) * z, ctx->stream));
  HIP_TRY(ctx, hipMemsetAsync((fp32 ? op->That32 : op->That64).p, 0, sizeof(R) * nh, ctx->stream));
  times[0] = time_yzy<R, L, 0>(ctx, op, dp.as<double>());
  if (times[0] < 0) return gofd_fail(ctx, GOFD_E_HIP, "timing the 3D passes failed");
  if (!Cfg3<R, L>::HAS_ALT) return 0;
  times[1] = time_yzy<R, L, 1>(ctx, op, dp.as<double>());
  if (times[1] < 0) return gofd_fail(ctx, GOFD_E_HIP, "timing the 3D passes failed");
  HIP_TRY(ctx, hipGetLastError());
  return times[1] < 0.95 * times[0] ? 1 : 0;   // the default unless the other is clearly faster
}

template <typename R>
int tune3(gofd_ctx_s* ctx, gofd_fdop_s* op, double* times) {
  switch (op->L) {
    case 8: return tune3_L<R, 8>(ctx, op, times);
    case 16: return tune3_L<R, 16>(ctx, op, times);
    case 32: return tune3_L<R, 32>(ctx, op, times);
    case 64: return tune3_L<R, 64>(ctx, op, times);
    case 128: return tune3_L<R, 128>(ctx, op, times);
    case 256: return tune3_L<R, 256>(ctx, op, times);
    case 512: return tune3_L<R, 512>(ctx, op, times);
    case 1024: return tune3_L<R, 1024>(ctx, op, times);
    default: return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "3D FFT length");
  }
}

}  // namespace

int conv3_tune(gofd_ctx_s* ctx, const gofd_grid* grid, bool fp32, double* times) {
  gofd_fdop_s op;
  GOFD_TRY(fdop_init_geometry(ctx, &op, 0.5, grid));
  if (!twiddles64(ctx, op.L) || !twiddles32(ctx, op.L)) return gofd_fail(ctx, GOFD_E_OOM, "twiddle table");
  // time with the default schedule installed, then record the choice
  ctx->sched3.erase(std::make_pair(op.L, fp32));
  const int best = fp32 ? tune3<float>(ctx, &op, times) : tune3<double>(ctx, &op, times);
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  if (best >= 0) ctx->sched3[std::make_pair(op.L, fp32)] = best;
  return best;
}

