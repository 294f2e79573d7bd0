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
#include <type_traits>

#include "bary.h"
#include "cg_items.h"
#include "cg_state.h"
#include "conv_common.h"
#include "fft.h"
#include "internal.h"

using gofd_fft::fft_regs;
using gofd_fft::padded_len;
using gofd_fft::pidx;

namespace {

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------- sources

// v = I u on the grid (eq. GoFD-1's interpolation): one thread per node, the
// weights from the record of the node's element; zero outside the mesh.  The
// optional per-vertex scale and mask multiply u first.  Kept apart from the
// row transform so that the dependent loads (element, record, vertex values)
// run with one node per thread.
#ifndef GOFD_GATHER_NPT
#define GOFD_GATHER_NPT 2
#endif
constexpr int GATHER_NPT = GOFD_GATHER_NPT;   // nodes per thread of the gather (build-time knob)

// Every load of the gathers is unconditional, from in-range indices: a node
// past the end reads the last node, a node outside the mesh reads the row of
// element 0 (compact row 0 in 3D) and weighs it by zero.  Per-lane branches
// around dependent loads would make each node of a thread wait for the one
// before it.

// 2D: interpolation rows of NPT nodes (column ci, row ri) from their element records
template <int NPT>
__device__ __forceinline__ void rows_2d_ij(const GridGeom& g, const ElemRec2* recs, const int* e, const int* ci,
                                           const int* ri, int (*vid)[4], double (*lam)[4]) {
  static_assert(sizeof(ElemRec2) == 64, "record layout");
  const int4* rq = reinterpret_cast<const int4*>(recs);
  const double2* rd = reinterpret_cast<const double2*>(recs);
  ElemRec2 rec[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const long long c = e[j] >= 0 ? e[j] : 0;
    const int4 v = gload(rq, 4 * c);
    const double2 x0 = gload(rd, 4 * c + 1), g0 = gload(rd, 4 * c + 2), g1 = gload(rd, 4 * c + 3);
    rec[j].v[0] = v.x, rec[j].v[1] = v.y, rec[j].v[2] = v.z, rec[j].v[3] = v.w;
    rec[j].x0[0] = x0.x, rec[j].x0[1] = x0.y;
    rec[j].g[0][0] = g0.x, rec[j].g[0][1] = g0.y, rec[j].g[1][0] = g1.x, rec[j].g[1][1] = g1.y;
  }
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int idx[2] = {ci[j], ri[j]};
    rec_weights<2>(g, rec[j], idx, vid[j], lam[j]);
    vid[j][3] = vid[j][0];
    lam[j][3] = 0.0;
    if (e[j] < 0) lam[j][0] = lam[j][1] = lam[j][2] = 0.0;
  }
}

// the same for nodes given by their linear numbers k
template <int NPT>
__device__ __forceinline__ void rows_2d(const GridGeom& g, const ElemRec2* recs, const int* e, const unsigned* k,
                                        int (*vid)[4], double (*lam)[4]) {
  int ci[NPT], ri[NPT];
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const unsigned W = (unsigned)g.W;
    ci[j] = (int)(k[j] % W);
    ri[j] = (int)(k[j] / W);
  }
  rows_2d_ij<NPT>(g, recs, e, ci, ri, vid, lam);
}

// 2D, FP32 pipeline: interpolation rows of NPT nodes k from the per-node
// single-precision rows (weights widened to double for the sum)
template <int NPT>
__device__ __forceinline__ void rows_2d_32(const int4* rv, const float2* rw, const long long* k, int (*vid)[4],
                                           double (*lam)[4]) {
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const int4 v = gload(rv, k[j]);
    const float2 w = gload(rw, k[j]);
    vid[j][0] = v.x, vid[j][1] = v.y, vid[j][2] = v.z, vid[j][3] = v.x;
    lam[j][0] = (double)__int_as_float(v.w), lam[j][1] = (double)w.x, lam[j][2] = (double)w.y, lam[j][3] = 0.0;
  }
}

// 3D: interpolation rows of NPT nodes from the compact per-node rows
template <int NPT>
__device__ __forceinline__ void rows_3d(const int4* ev, const double2* ew, const int* c, int (*vid)[4],
                                        double (*lam)[4]) {
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    const long long cc = c[j] >= 0 ? c[j] : 0;
    const int4 v = gload(ev, cc);
    const double2 w01 = gload(ew, 2 * cc), w23 = gload(ew, 2 * cc + 1);
    vid[j][0] = v.x, vid[j][1] = v.y, vid[j][2] = v.z, vid[j][3] = v.w;
    lam[j][0] = w01.x, lam[j][1] = w01.y, lam[j][2] = w23.x, lam[j][3] = w23.y;
    if (c[j] < 0) lam[j][0] = lam[j][1] = lam[j][2] = lam[j][3] = 0.0;
  }
}

// sum_r lam_r * (u * scale * mask)[vid_r] for NPT rows (scale and mask optional)
template <int D, int NPT>
__device__ __forceinline__ void row_values(const double* u, const double* scale, const double* mask,
                                           const int (*vid)[4], const double (*lam)[4], double* out) {
  const auto gu = gmem(u);
  double uv[NPT][D + 1];
#pragma unroll
  for (int j = 0; j < NPT; ++j)
#pragma unroll
    for (int r = 0; r <= D; ++r) uv[j][r] = gu[vid[j][r]];
  if (scale) {
    const auto gs = gmem(scale);
#pragma unroll
    for (int j = 0; j < NPT; ++j)
#pragma unroll
      for (int r = 0; r <= D; ++r) uv[j][r] *= gs[vid[j][r]];
  }
  if (mask) {
    const auto gm = gmem(mask);
#pragma unroll
    for (int j = 0; j < NPT; ++j)
#pragma unroll
      for (int r = 0; r <= D; ++r) uv[j][r] *= gm[vid[j][r]];
  }
#pragma unroll
  for (int j = 0; j < NPT; ++j) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r <= D; ++r) s += lam[j][r] * uv[j][r];
    out[j] = s;
  }
}

// 2D: the FP64 pipeline evaluates each node's weights from its element's
// record (element, record, vertex values: three dependent loads); the FP32
// pipeline reads the per-node single-precision rows (row, vertex values: two)
template <typename R, int D>
__global__ __launch_bounds__(256) void k_gather(GridGeom g, const ElemRec<D>* __restrict__ recs,
                                                const int* __restrict__ elem, const int4* __restrict__ rv,
                                                const float2* __restrict__ rw, const double* __restrict__ u,
                                                const double* __restrict__ scale, const double* __restrict__ mask,
                                                long long nv, long long n_nodes, R* __restrict__ out, Skip skip) {
  static_assert(D == 2, "3D gathers from compact rows");
  const long long k0 = (long long)xcd_remap(blockIdx.x, gridDim.x) * (256 * GATHER_NPT) + threadIdx.x;
  const int rhs = skip.item(blockIdx.y);
  int vid[GATHER_NPT][4];
  double lam[GATHER_NPT][4], val[GATHER_NPT];
  if constexpr (sizeof(R) == 4) {
    long long kc[GATHER_NPT];
#pragma unroll
    for (int j = 0; j < GATHER_NPT; ++j) {
      const long long k = k0 + j * 256;
      kc[j] = k < n_nodes ? k : n_nodes - 1;
    }
    rows_2d_32<GATHER_NPT>(rv, rw, kc, vid, lam);
    if (skip(rhs)) return;
  } else {
    int e[GATHER_NPT];
    unsigned kc[GATHER_NPT];
#pragma unroll
    for (int j = 0; j < GATHER_NPT; ++j) {
      const long long k = k0 + j * 256;
      kc[j] = (unsigned)(k < n_nodes ? k : n_nodes - 1);
      e[j] = gmem(elem)[kc[j]];
    }
    if (skip(rhs)) return;
    rows_2d<GATHER_NPT>(g, recs, e, kc, vid, lam);
  }
  row_values<2, GATHER_NPT>(u + rhs * nv, scale, mask, vid, lam, val);
#pragma unroll
  for (int j = 0; j < GATHER_NPT; ++j) {
    const long long k = k0 + j * 256;
    if (k < n_nodes) out[rhs * n_nodes + k] = (R)val[j];
  }
}

// The same from compact per-node rows (3D): row c = idx[k] of an inside node
// holds its four vertex ids and weights.
template <typename R>
__global__ __launch_bounds__(256) void k_gather_ell(const int* __restrict__ idx, const int4* __restrict__ ev,
                                                    const double2* __restrict__ ew, const double* __restrict__ u,
                                                    const double* __restrict__ scale,
                                                    const double* __restrict__ mask, long long nv, long long n_nodes,
                                                    R* __restrict__ out, Skip skip) {
  const long long k = (long long)xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const int rhs = skip.item(blockIdx.y);
  if (k >= n_nodes) return;
  const int c = idx[k];
  if (skip(rhs)) return;
  int vid[1][4];
  double lam[1][4], val[1];
  rows_3d<1>(ev, ew, &c, vid, lam);
  row_values<3, 1>(u + rhs * nv, scale, mask, vid, lam, val);
  out[rhs * n_nodes + k] = (R)val[0];
}

// Batched gather: item blockIdx.y of the batch (its mesh, its vector at
// ubase + off); with use_mask the interior mask multiplies u first.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_gather_items(const CgItem* __restrict__ items,
                                                      const double* __restrict__ ubase, int use_mask,
                                                      long long n_nodes, R* __restrict__ out, Skip skip) {
  const int it = skip.item(blockIdx.y);
  const CgItem& I = items[it];
  const long long k0 = (long long)xcd_remap(blockIdx.x, gridDim.x) * (256 * GATHER_NPT) + threadIdx.x;
  int vid[GATHER_NPT][4];
  double lam[GATHER_NPT][4], val[GATHER_NPT];
  if constexpr (D == 2 && sizeof(R) == 4) {
    // FP32 pipeline: per-node single-precision rows
    long long kc[GATHER_NPT];
#pragma unroll
    for (int j = 0; j < GATHER_NPT; ++j) {
      const long long k = k0 + j * 256;
      kc[j] = k < n_nodes ? k : n_nodes - 1;
    }
    rows_2d_32<GATHER_NPT>(I.row32_v, I.row32_w, kc, vid, lam);
    if (skip(it)) return;
  } else {
    const auto elem = gmem(D == 2 ? I.elem : I.ell_idx);
    int e[GATHER_NPT];
    unsigned kc[GATHER_NPT];
#pragma unroll
    for (int j = 0; j < GATHER_NPT; ++j) {
      const long long k = k0 + j * 256;
      kc[j] = (unsigned)(k < n_nodes ? k : n_nodes - 1);
      e[j] = elem[kc[j]];
    }
    if (skip(it)) return;
    if constexpr (D == 2)
      rows_2d<GATHER_NPT>(I.g, static_cast<const ElemRec2*>(I.recs), e, kc, vid, lam);
    else
      rows_3d<GATHER_NPT>(I.ell_v, I.ell_w, e, vid, lam);
  }
  row_values<D, GATHER_NPT>(ubase + I.off, nullptr, use_mask ? I.imask : nullptr, vid, lam, val);
#pragma unroll
  for (int j = 0; j < GATHER_NPT; ++j) {
    const long long k = k0 + j * 256;
    if (k < n_nodes) out[it * n_nodes + k] = (R)val[j];
  }
}

// ---------------------------------------------------------------- row-pair sources
// Input of the first row pass: for the row pair (row0, row0 + 1), thread t
// of the TPL threads of the pair gets element m of its line, the complex
// value (row0, col) + i (row0 + 1, col) at col = t + m TPL; columns past the
// window and rows past the grid give zero.  Loads read clamped in-range
// positions and are masked after.
template <int E, int TPL>
struct PairCols {
  static constexpr int M = E / 2 + 1;     // columns beyond L/2 are outside the window (W <= L/2 + 1)
  int r0c, r1c;
  bool has0, has1;
  __device__ __forceinline__ PairCols(int row0, int W) {
    has0 = row0 < W;
    has1 = row0 + 1 < W;
    r0c = has0 ? row0 : W - 1;
    r1c = has1 ? row0 + 1 : r0c;
  }
  __device__ __forceinline__ static int col(int t, int m) { return t + m * TPL; }
  __device__ __forceinline__ static int clamp(int c, int W) { return c < W ? c : W - 1; }
  template <typename R>
  __device__ __forceinline__ void put(cplx<R>* v, int t, int W, const double* a, const double* b) const {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      R x = 0, y = 0;
      if (m < M) {
        const bool in = col(t, m) < W;
        if (has0 && in) x = (R)a[m];
        if (has1 && in) y = (R)b[m];
      }
      v[m] = {x, y};
    }
  }
};

// a grid field (nrhs fields of W^2 values)
template <typename T>
struct SrcPairGrid {
  const T* f;
  long long n_nodes;
  template <typename R, int E, int TPL>
  __device__ __forceinline__ void load(int rhs, int row0, int W, int t, cplx<R>* v) const {
    const PairCols<E, TPL> pc(row0, W);
    constexpr int M = PairCols<E, TPL>::M;
    const T* fr = f + rhs * n_nodes;
    double a[M], b[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int cc = pc.clamp(pc.col(t, m), W);
      a[m] = (double)fr[(long long)pc.r0c * W + cc];
      b[m] = (double)fr[(long long)pc.r1c * W + cc];
    }
    pc.template put<R>(v, t, W, a, b);
  }
};

// the FP32 gather of batch item `it` (its mesh, its vector at ubase + off)
// straight from the per-node single-precision rows: row, then vertex values,
// for every node of the thread in flight together
struct SrcPairGatherRows {
  const CgItem* items;
  const double* ubase;
  int use_mask;
  template <typename R, int E, int TPL>
  __device__ __forceinline__ void load(int it, int row0, int W, int t, cplx<R>* v) const {
    const PairCols<E, TPL> pc(row0, W);
    constexpr int M = PairCols<E, TPL>::M;
    const CgItem& I = items[it];
    long long k[2 * M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int cc = pc.clamp(pc.col(t, m), W);
      k[m] = (long long)pc.r0c * W + cc;
      k[M + m] = (long long)pc.r1c * W + cc;
    }
    int vid[2 * M][4];
    double lam[2 * M][4], val[2 * M];
    rows_2d_32<2 * M>(I.row32_v, I.row32_w, k, vid, lam);
    row_values<2, 2 * M>(ubase + I.off, nullptr, use_mask ? I.imask : nullptr, vid, lam, val);
    pc.template put<R>(v, t, W, val, val + M);
  }
};

// The FP32 gather of batch item `it` through its row pair's slots: the line's
// threads stage the slot values of the row pair (one per vertex with entries
// in its two rows, at row-pair-major positions meta.z ..) in LDS while the
// node rows load, and each node then adds its three weighted values from
// there.  No load waits for another load's result but for the row pair's
// descriptor.
struct SrcPairSegRows {
  const CgItem* items;
  const float* us;
  long long ustride;
  template <typename R, int E, int TPL>
  __device__ __forceinline__ void load(int it, int row0, int W, int t, cplx<R>* v) const {
    const PairCols<E, TPL> pc(row0, W);
    constexpr int M = PairCols<E, TPL>::M;
    constexpr int LINES = TPL >= 64 ? 1 : 64 / TPL;     // row pairs per block of the row passes
    constexpr int SEGL = RP_SEGCAP / LINES;              // slots a row pair may have
    constexpr int NLD = SEGL / TPL;
    static_assert(NLD * TPL == SEGL, "slot staging");
    __shared__ float su[RP_SEGCAP];
    const CgItem& I = items[it];
    const int rp = min(row0 >> 1, ((W + 1) >> 1) - 1);
    const int4 meta = gload(reinterpret_cast<const int4*>(I.rp_meta), rp);   // z: first slot, w: slots
    int4 a[2 * M];
    float w2[2 * M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int cc = pc.clamp(pc.col(t, m), W);
      const long long k0 = (long long)pc.r0c * W + cc, k1 = (long long)pc.r1c * W + cc;
      a[m] = gload(I.seg_row, k0);
      a[M + m] = gload(I.seg_row, k1);
      w2[m] = gmem(I.seg_row_w2)[k0];
      w2[M + m] = gmem(I.seg_row_w2)[k1];
    }
    const float* ui = us + it * ustride + (meta.w > 0 ? meta.z : 0);
    float uv[NLD];
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int idx = t + j * TPL;
      uv[j] = gmem(ui)[idx < meta.w ? idx : 0];
    }
    float* sl = su + (threadIdx.x / TPL) * SEGL;
#pragma unroll
    for (int j = 0; j < NLD; ++j) sl[t + j * TPL] = (t + j * TPL < meta.w) ? uv[j] : 0.f;
    __syncthreads();
    double val[2 * M];
#pragma unroll
    for (int j = 0; j < 2 * M; ++j) {
      const int s0 = a[j].x & 0xffff, s1 = (int)((unsigned)a[j].x >> 16), s2 = a[j].y;
      float x = __int_as_float(a[j].z) * sl[s0];
      x = fmaf(__int_as_float(a[j].w), sl[s1], x);
      x = fmaf(w2[j], sl[s2], x);
      val[j] = (double)x;
    }
    pc.template put<R>(v, t, W, val, val + M);
  }
};

// ---------------------------------------------------------------- spectra layout
// Z holds, per rhs, the L/2 column slots of the W window rows after the row
// transform, in tiles of four slots: Z[slot/4][row][slot%4].  A block of the
// column pass reads one tile as a contiguous stretch, and a row pair of the
// row passes touches 2 x 4 consecutive entries per tile.  Slot c > 0 is
// spectrum column k0 = c; slot 0 carries the two real columns k0 = 0 and
// k0 = L/2 packed as one complex value (both are exactly real for real rows).
template <typename R>
__device__ __forceinline__ long long zidx(int slot, int row, int W) {
  return ((long long)(slot >> 2) * W + row) * 4 + (slot & 3);
}

// ---------------------------------------------------------------- pass A
// LINES row pairs per block, TPL = L/E threads per row pair.  Two real rows
// are packed as one complex line (a + i b); after the forward transform the
// half spectra are split off with the mirror entry L - k.
template <typename R, int L, int E, int LINES, class Src>
__global__ __launch_bounds__(LINES*(L / E)) void k_passA(Src src, cplx<R>* __restrict__ Z, int W,
                                                         const cplx<R>* __restrict__ tw, long long zs, Skip skip) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int H = L / 2;
  __shared__ cplx<R> sbuf[LINES * PL];
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* buf = sbuf + line * PL;
  const int row0 = (xcd_remap(blockIdx.x, gridDim.x) * LINES + line) * 2;   // row bands per XCD
  const int rhs = skip.item(blockIdx.y);
  const bool has0 = row0 < W;
  const bool has1 = row0 + 1 < W;
  cplx<R> v[E];
  src.template load<R, E, TPL>(rhs, row0, W, t, v);
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  // the finished-rhs test after the loads, so that its latency overlaps theirs
  if (skip(rhs)) return;
  fft_regs<R, L, E, false>(v, buf, tws, t);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) buf[pidx<E>(t + m * TPL)] = v[m];
  __syncthreads();
  if (!has0) return;
  cplx<R>* Zr = Z + rhs * zs;
#pragma unroll
  for (int q = 0; q < E / 2; ++q) {
    const int k = t + q * TPL;
    cplx<R> z0, z1;
    if (k == 0) {
      const cplx<R> dc = buf[pidx<E>(0)], nq = buf[pidx<E>(H)];
      z0 = {dc.x, nq.x};
      z1 = {dc.y, nq.y};
    } else {
      const cplx<R> zk = buf[pidx<E>(k)], zm = buf[pidx<E>(L - k)];
      z0 = {(zk.x + zm.x) * (R)0.5, (zk.y - zm.y) * (R)0.5};
      z1 = {(zk.y + zm.y) * (R)0.5, (zm.x - zk.x) * (R)0.5};
    }
    cplx<R>* dst = Zr + zidx<R>(k, row0, W);
    dst[0] = z0;
    if (has1) dst[4] = z1;
  }
}

// ---------------------------------------------------------------- pass B
// LB column slots per block (LB divides the tile width 4), TPL threads each.
// Forward FFT along the rows (W nonzero of L), multiply by the real spectrum,
// inverse FFT, keep the W window rows; the product happens in registers
// between the last forward and the first inverse stage.  For the packed slot
// 0, with C = FFT(a + i b) and m = L - k:
//   A_k = (C_k + conj C_m)/2,  i B_k = (C_k - conj C_m)/2, and the product
//   D = T0 A + i T1 B gives D_k = (T0+T1)/2 C_k + (T0-T1)/2 conj C_m;
// the inverse FFT of D is (T0 * a) + i (T1 * b) with both parts real.
//
// With dpart given, the block also leaves the partial sum of
//   (A v, v) = sum_k That_k |V_k|^2   (Parseval for the circulant embedding;
// the half spectrum counts the columns 0 < k0 < L/2 twice), which is the
// (K u, u) of CG when v = I u, and the sums of its slice of the level-1
// partials of gamma and (r, r): dpart[rhs][q][block], q = gamma, (r, r), delta.
template <typename R, int L, int E, int LB, bool DOT>
__global__ __launch_bounds__(LB*(L / E), (LB * (L / E) >= 256) ? 2 : 1) void k_passB(cplx<R>* __restrict__ Z, int W, int half,
                                                      const R* That, const cplx<R>* __restrict__ tw,
                                                      long long zs, Skip skip, double* __restrict__ dpart,
                                                      gofd_cg::Level1 lv1, const void* const* __restrict__ that_tab) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int H = L / 2;
  constexpr int NT = LB * TPL;
  __shared__ cplx<R> sbuf[LB * PL];
  __shared__ double shd[gofd_cg::block_sum_lds<NT, 3>()];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int c = threadIdx.x % LB, t = threadIdx.x / LB;
  cplx<R>* buf = sbuf + c * PL;
  const int slot = b * LB + c;
  const int rhs = skip.item(blockIdx.y);
  cplx<R>* Zc = Z + rhs * zs + zidx<R>(slot, 0, W);
  // rows i >= W are zero (W <= L/2 + 1: only elements m <= E/2 can hold rows
  // of the window); the loads read clamped rows and are masked after, so that
  // they are all in flight together
  cplx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int i = t + m * TPL;
    if (m <= E / 2) {
      v[m] = Zc[(long long)(i < W ? i : W - 1) * 4];
      if (i >= W) v[m] = cplx<R>{0, 0};
    } else {
      v[m] = cplx<R>{0, 0};
    }
  }
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  // multipliers of this slot, fetched before the transform; element k1 of the
  // line takes row min(k1, L - k1) of the stored (L/2+1)-row spectrum column
  // (for slot 0 this is column k0 = 0; column L/2 is read when it is used)
  R pm[E];
  if (that_tab) That = static_cast<const R*>(that_tab[rhs]);     // per-item spectrum (batched solves)
  {
    const R* Tc = That + (long long)slot * half;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k1 = t + m * TPL;
      pm[m] = Tc[(k1 <= H) ? k1 : L - k1];
    }
  }
  // this block's slice of the level-1 partials (usually one value per thread)
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
  double& dacc = red[2];
  fft_regs<R, L, E, false>(v, buf, tws, t);
  if (b == 0) {                     // block-uniform: this block holds slot 0
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) buf[pidx<E>(t + m * TPL)] = v[m];
    __syncthreads();
    if (c == 0) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int k1 = t + m * TPL;
        const R t0 = pm[m];                                                  // column k0 = 0
        const R t1 = That[(long long)H * half + ((k1 <= H) ? k1 : L - k1)];  // column k0 = L/2
        const R pp = (t0 + t1) * (R)0.5, qq = (t0 - t1) * (R)0.5;
        const cplx<R> ck = v[m], cm = buf[pidx<E>((L - k1) & (L - 1))];
        if constexpr (DOT) {
          // columns k0 = 0 and L/2: A = (C_k + conj C_m)/2, B = (C_k - conj C_m)/(2i)
          const double ax = (double)ck.x + cm.x, ay = (double)ck.y - cm.y;
          const double bx = (double)ck.y + cm.y, by = (double)ck.x - cm.x;
          dacc += 0.25 * ((double)t0 * (ax * ax + ay * ay) + (double)t1 * (bx * bx + by * by));
        }
        v[m] = {pp * ck.x + qq * cm.x, pp * ck.y - qq * cm.y};
      }
    }
  }
  if (slot != 0) {
    // terms That_k |V_k|^2 in the grid precision (products of grid values),
    // a thread's E terms summed in that precision, the threads' sums in double
    R dsum = 0;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      if constexpr (DOT) dsum += pm[m] * (v[m].x * v[m].x + v[m].y * v[m].y);
      v[m] = {v[m].x * pm[m], v[m].y * pm[m]};
    }
    dacc += 2.0 * (double)dsum;
  }
  if constexpr (DOT) {
    static_assert(NT % 64 == 0 || NT < 64, "block size");
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
#pragma unroll
  for (int m = 0; m <= E / 2; ++m) {
    const int i = t + m * TPL;
    if (i < W) Zc[(long long)i * 4] = v[m];
  }
}

// ---------------------------------------------------------------- pass C
// Row pairs: rebuild the Hermitian spectra of two real rows as one complex
// line (a + i b at k, conj(a) + i conj(b) at L - k), inverse FFT, write the
// W window values of both rows.
//
// With fin active, one extra block (the last) finishes the CG reductions of
// the iteration instead (the step's scalars are needed only by later
// kernels), concurrently with the transforms.
//
// With SCAT (2D CG iteration, row-pair form of I^T present for the item), the
// block does not write y: it sums, for each segment of its row pair (the
// entries of one vertex in these two rows), weight times y over the
// segment's entries and writes the sum to the segment's partial slot.  The
// entries, in the thread-interleaved layout of the transfer, are fetched at
// the start so that they arrive during the transform.
struct RowScatter {
  const CgItem* items;     // per-item row-pair arrays
  double* P;               // partial slots, item it at it * pstride
  long long pstride;
  int ent_ahead;           // entries read ahead per thread (covers most row pairs)
};
template <typename R, typename Y, int L, int E, int LINES, bool SCAT, int EPRE = 1>
__global__ __launch_bounds__(LINES*(L / E), (SCAT && LINES * (L / E) >= 256) ? (sizeof(R) == 4 ? 3 : 2) : 1) void k_passC(const cplx<R>* __restrict__ Z, int W,
                                                         const cplx<R>* __restrict__ tw, long long zs,
                                                         Y* __restrict__ y, long long n_nodes, Skip skip,
                                                         gofd_cg::Finish fin, RowScatter rs) {
  constexpr int TPL = L / E;
  constexpr int PL = padded_len<L, E>();
  constexpr int NT = LINES * TPL;
  constexpr int SEGL = RP_SEGCAP / LINES;                  // segment sums per row pair
  constexpr int QD = (SEGL + TPL - 1) / TPL;               // segments per thread in the write-out
  static_assert(2 * (L / 2 + 1) <= 2 * PL, "row pair fits the exchange buffer");
  __shared__ cplx<R> sbuf[LINES * PL];
  __shared__ double shf[gofd_cg::block_sum_lds<NT, 3>()];
  __shared__ R segs[SCAT ? RP_SEGCAP : 1];                // segment sums, grid precision
  const int line = threadIdx.x / TPL, t = threadIdx.x % TPL;
  cplx<R>* buf = sbuf + line * PL;
  const int nrb = gridDim.x - (fin.sc ? 1 : 0);                            // row-pair blocks
  const int row0 = (xcd_remap(min((int)blockIdx.x, nrb - 1), nrb) * LINES + line) * 2;   // row bands per XCD
  const int rhs = skip.item(blockIdx.y);
  const bool has0 = row0 < W;
  const bool has1 = row0 + 1 < W;
  const cplx<R>* Zr = Z + rhs * zs;
  if (fin.sc && blockIdx.x == gridDim.x - 1) {     // block-uniform: the finishing block
    fin.run<NT>(rhs, shf);
    return;
  }
  // rows past the window read a window row (loads in flight together) and
  // count as zero
  const int r0c = has0 ? row0 : W - 1, r1c = has1 ? row0 + 1 : r0c;
  cplx<R> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = t + m * TPL;
    const bool dcnq = (m == 0 || m == E / 2) && t == 0;      // k = 0 or k = L/2: packed slot 0
    const bool mirror = !dcnq && m >= E / 2;                  // k > L/2: conjugate of slot L - k
    const int sl = dcnq ? 0 : (mirror ? L - k : k);
    cplx<R> a = Zr[zidx<R>(sl, r0c, W)];
    cplx<R> bb = Zr[zidx<R>(sl, r1c, W)];
    if (!has0) a = cplx<R>{0, 0};
    if (!has1) bb = cplx<R>{0, 0};
    if (dcnq)
      v[m] = (m == 0) ? cplx<R>{a.x, bb.x} : cplx<R>{a.y, bb.y};
    else if (mirror)
      v[m] = {a.x + bb.y, bb.x - a.y};                        // conj(a) + i conj(b)
    else
      v[m] = {a.x - bb.y, a.y + bb.x};                        // a + i b
  }
  gofd_fft::Twiddles<R, L, E> tws;
  tws.load(tw, t);
  // row-pair I^T: this thread's entries and the row pair's segment slots
  int4 meta = make_int4(0, 0, 0, 0);
  int tseg = 0, tcnt = 0, mlast = 0;
  int code[SCAT ? EPRE : 1];
  R wt[SCAT ? EPRE : 1];
  int dst[SCAT ? QD : 1];
  const unsigned short* gcode = nullptr;
  const R* gw = nullptr;
  if constexpr (SCAT) {
    const CgItem& I = rs.items[rhs];
    const int rp = has0 ? row0 / 2 : 0;
    meta = gload(reinterpret_cast<const int4*>(I.rp_meta), rp);
    if (!has0) meta = make_int4(0, 0, 0, 0);
    if constexpr (LINES == 1) {                // one row pair per block: its descriptor is uniform
      meta.x = __builtin_amdgcn_readfirstlane(meta.x);
      meta.y = __builtin_amdgcn_readfirstlane(meta.y);
      meta.z = __builtin_amdgcn_readfirstlane(meta.z);
      meta.w = __builtin_amdgcn_readfirstlane(meta.w);
    }
    int tword = gmem(I.rp_tseg)[(long long)rp * TPL + t];
    if (!has0) tword = 0;
    tseg = tword & 0xffff;
    tcnt = tword >> 16;
    // entries m < EPRE of this thread, read ahead: a load past the thread's
    // own count (its padding, up to the row pair's count meta.y, and beyond)
    // re-reads its last entry, a line already fetched, and the value becomes
    // padding (node 0, weight 0), as the stored padding is.  The launch picks
    // EPRE from the count that covers most row pairs.
    mlast = tcnt > 0 ? tcnt - 1 : 0;
    gcode = I.rp_code + meta.x + t;
    if constexpr (sizeof(R) == 4)
      gw = reinterpret_cast<const R*>(I.rp_w32) + meta.x + t;
    else
      gw = reinterpret_cast<const R*>(I.rp_w64) + meta.x + t;
    // the second half only where the row pair's count needs it (a uniform
    // branch with one row pair per block)
#pragma unroll
    for (int m = 0; m < EPRE / 2; ++m) {
      const int mm = min(m, mlast);
      code[m] = gmem(gcode)[mm * TPL];
      wt[m] = gmem(gw)[mm * TPL];
    }
    if (LINES > 1 || meta.y > EPRE / 2) {
#pragma unroll
      for (int m = EPRE / 2; m < EPRE; ++m) {
        const int mm = min(m, mlast);
        code[m] = gmem(gcode)[mm * TPL];
        wt[m] = gmem(gw)[mm * TPL];
      }
    } else {
#pragma unroll
      for (int m = EPRE / 2; m < EPRE; ++m) {
        code[m] = 0;
        wt[m] = (R)0;
      }
    }
#pragma unroll
    for (int m = 0; m < EPRE; ++m)
      if (m >= tcnt) {
        code[m] = 0;
        wt[m] = (R)0;
      }
#pragma unroll
    for (int q = 0; q < QD; ++q) {
      const int i = t + q * TPL;
      dst[q] = gmem(I.rp_dest)[i < meta.w ? meta.z + i : 0];
    }
  }
  if (skip(rhs)) return;
  fft_regs<R, L, E, true>(v, buf, tws, t);
  if constexpr (SCAT) {
    // the row pair's values into the exchange buffer (after every thread has
    // left the transform), then the segment sums (every thread reaches the
    // barriers: a line without rows has no entries)
    R* yl = reinterpret_cast<R*>(buf);
    R* sg = segs + line * SEGL;
    __syncthreads();
#pragma unroll
    for (int m = 0; m <= E / 2; ++m) {
      const int col = t + m * TPL;
      if (col < W) {
        yl[col] = v[m].x;
        yl[W + col] = v[m].y;
      }
    }
    __syncthreads();
    // every node value first, then the sums in entry order: a segment's sum
    // is stored at its last entry (a predicated store, no branch around loads)
    R yv[EPRE];
#pragma unroll
    for (int m = 0; m < EPRE; ++m) yv[m] = yl[code[m] & RP_NODE];
    // (a segment's entries are summed in the grid precision, the segments of
    // a vertex in double by the vertex kernel)
    R acc = 0;
    int j = tseg;
#pragma unroll
    for (int m = 0; m < EPRE; ++m) {
      acc = fma(wt[m], yv[m], acc);
      const bool end = (code[m] & RP_END) != 0;
      if (end) sg[j] = acc;
      j += end ? 1 : 0;
      acc = end ? (R)0 : acc;
    }
    for (int m = EPRE; m < meta.y; ++m) {      // rows pairs with more entries per thread
      const int mm = min(m, mlast);
      const bool real = m < tcnt;
      int c = gmem(gcode)[(long long)mm * TPL];
      R wv = gmem(gw)[(long long)mm * TPL];
      if (!real) {
        c = 0;
        wv = (R)0;
      }
      acc = fma(wv, yl[c & RP_NODE], acc);
      if (c & RP_END) {
        sg[j++] = acc;
        acc = 0;
      }
    }
    __syncthreads();
    double* P = rs.P + rhs * rs.pstride;
#pragma unroll
    for (int q = 0; q < QD; ++q) {
      const int i = t + q * TPL;
      if (i < meta.w) P[dst[q]] = (double)sg[i];
    }
    return;
  }
  if (!has0) return;
  Y* yr = y + rhs * n_nodes + (long long)row0 * W;
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

// Values per thread of the row passes (C; A unless set apart) and of the
// default column-pass schedule (B): build-time knobs, powers of two in 4..16.
#ifndef GOFD_FFT_E_ROWS
#define GOFD_FFT_E_ROWS 8
#endif
#ifndef GOFD_FFT_E_PASSA
#define GOFD_FFT_E_PASSA GOFD_FFT_E_ROWS
#endif
#ifndef GOFD_FFT_E_COLS
#define GOFD_FFT_E_COLS 16
#endif
// most column slots per block of the default column-pass schedule (1, 2 or 4)
#ifndef GOFD_FFT_LB
#define GOFD_FFT_LB 2
#endif

template <typename R, int L>
struct Cfg {
  static constexpr int EA = (L >= GOFD_FFT_E_ROWS) ? GOFD_FFT_E_ROWS : L;
  static constexpr int TA = L / EA;                                         // threads per row pair
  static constexpr int LINES_A = (TA >= 64) ? 1 : 64 / TA;                  // row pairs per block
  static_assert(LINES_A * TA <= 1024 && LINES_A * padded_len<L, EA>() * (int)sizeof(cplx<R>) <= 150 * 1024,
                "row pass block");
  // the forward row pass (A)
  static constexpr int E1 = (L >= GOFD_FFT_E_PASSA) ? GOFD_FFT_E_PASSA : L;
  static constexpr int T1 = L / E1;
  static constexpr int LINES_1 = (T1 >= 64) ? 1 : 64 / T1;
  static_assert(LINES_1 * T1 <= 1024 && LINES_1 * padded_len<L, E1>() * (int)sizeof(cplx<R>) <= 150 * 1024,
                "row pass block");
};

// Schedules of the column pass (values per thread, column slots per block):
// schedule 0 is the built-in default; gofd_autotune times the others on the
// device and records the fastest per (L, precision) in the context.
struct ColSched {
  int e, lb;
};
constexpr ColSched kColSched[GOFD_N_COL_SCHED] = {{GOFD_FFT_E_COLS, GOFD_FFT_LB}, {16, 1}, {8, 2}, {16, 4}};

template <typename R, int L, int S>
struct ColCfg {
  static constexpr int E = (L >= kColSched[S].e) ? kColSched[S].e : L;
  static constexpr int T = L / E;                                           // threads per column slot
  static constexpr int LINE_BYTES = padded_len<L, E>() * (int)sizeof(cplx<R>);
  static constexpr int LB0 = kColSched[S].lb;
  static constexpr int LB_MEM = (LB0 >= 4 && 4 * LINE_BYTES <= 150 * 1024)
                                    ? 4
                                    : ((LB0 >= 2 && 2 * LINE_BYTES <= 150 * 1024) ? 2 : 1);
  static constexpr int LB = (LB_MEM * T <= 512) ? LB_MEM : ((2 * T <= 512) ? 2 : 1);     // slots per block
  static_assert(4 % LB == 0 && (L / 2) % 4 == 0, "tile layout");
};

template <typename R, int L, int S>
void launch_passB_s(gofd_ctx_s* ctx, hipStream_t st, int nrhs, cplx<R>* Z, int W, int half, const R* That,
                    const cplx<R>* tw, long long zs, Skip skip, double* dpart, const gofd_cg::Level1& lv1,
                    const void* const* that_tab) {
  using C = ColCfg<R, L, S>;
  if (dpart)
    GOFD_LAUNCH(ctx, (k_passB<R, L, C::E, C::LB, true>), dim3((L / 2) / C::LB, nrhs), dim3(C::LB * C::T), 0, st, Z,
                W, half, That, tw, zs, skip, dpart, lv1, that_tab);
  else
    GOFD_LAUNCH(ctx, (k_passB<R, L, C::E, C::LB, false>), dim3((L / 2) / C::LB, nrhs), dim3(C::LB * C::T), 0, st,
                Z, W, half, That, tw, zs, skip, dpart, lv1, that_tab);
}

template <typename R, int L>
int passB_blocks_L(int s) {
  switch (s) {
    case 1: return (L / 2) / ColCfg<R, L, 1>::LB;
    case 2: return (L / 2) / ColCfg<R, L, 2>::LB;
    case 3: return (L / 2) / ColCfg<R, L, 3>::LB;
    default: return (L / 2) / ColCfg<R, L, 0>::LB;
  }
}

// schedule in force for (L, precision) in this context
static int col_sched(const gofd_ctx_s* ctx, int L, bool fp32) {
  auto it = ctx->col_sched.find(std::make_pair(L, fp32));
  return it == ctx->col_sched.end() ? 0 : it->second;
}

// values per thread of the first row pass of the products (0: the default)
static int row_sched(const gofd_ctx_s* ctx, int L, bool fp32) {
  auto it = ctx->row_sched.find(std::make_pair(L, fp32));
  return it == ctx->row_sched.end() ? 0 : it->second;
}

template <typename R, int L, int EP, class Src>
void launch_passA(gofd_ctx_s* ctx, hipStream_t st, int nrhs, int pairs, const Src& src, cplx<R>* Z, int W,
                  const cplx<R>* tw, long long zs, Skip skip) {
  constexpr int TP = L / EP;
  constexpr int LP = (TP >= 64) ? 1 : 64 / TP;
  GOFD_LAUNCH(ctx, (k_passA<R, L, EP, LP, Src>), dim3((pairs + LP - 1) / LP, nrhs), dim3(LP * TP), 0, st, src, Z,
              W, tw, zs, skip);
}

template <typename R, int L, class Src, typename Y>
int run_2d(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes, Skip skip,
           double* dpart, const gofd_cg::Level1& lv1, const gofd_cg::Finish& fin, const void* const* that_tab,
           const RowScatter& rs) {
  const int W = op->W, half = op->half;
  const long long zs = (long long)W * (L / 2);
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
  if (!ctx->ws_Z) GOFD_TRY(dev_reserve(ctx, op->Z, sizeof(cplx<R>) * zs * nrhs));
  cplx<R>* Z = ctx->ws_Z ? static_cast<cplx<R>*>(ctx->ws_Z) : op->Z.as<cplx<R>>();
  using C = Cfg<R, L>;
  const int pairs = (W + 1) / 2;
  const int nbA = (pairs + C::LINES_A - 1) / C::LINES_A;
  hipStream_t st = ctx->stream;
  if (passes & 1) {
    // the gather through the slots does its FFT with 16 values per thread
    // when both row passes still hold one row pair per block (the slot
    // capacity of a row pair is the same then); the products from a grid
    // field take 8 by default, or 16 where the tuner found that faster
    constexpr bool SEG = std::is_same<Src, SrcPairSegRows>::value;
    constexpr bool BOTH = L / 16 >= 64 && C::TA >= 64 && C::E1 == 8;   // 8 and 16 both one row pair per block
    constexpr bool WIDE = SEG && BOTH;
    const bool wide = WIDE || (BOTH && !SEG && row_sched(ctx, L, sizeof(R) == 4) == 16);
    if (wide) {
      if constexpr (BOTH) launch_passA<R, L, 16, Src>(ctx, st, nrhs, pairs, src, Z, W, tw, zs, skip);
    } else if constexpr (!WIDE) {
      launch_passA<R, L, C::E1, Src>(ctx, st, nrhs, pairs, src, Z, W, tw, zs, skip);
    }
  }
  if (passes & 2) {
    switch (col_sched(ctx, L, sizeof(R) == 4)) {
      case 1: launch_passB_s<R, L, 1>(ctx, st, nrhs, Z, W, half, That, tw, zs, skip, dpart, lv1, that_tab); break;
      case 2: launch_passB_s<R, L, 2>(ctx, st, nrhs, Z, W, half, That, tw, zs, skip, dpart, lv1, that_tab); break;
      case 3: launch_passB_s<R, L, 3>(ctx, st, nrhs, Z, W, half, That, tw, zs, skip, dpart, lv1, that_tab); break;
      default: launch_passB_s<R, L, 0>(ctx, st, nrhs, Z, W, half, That, tw, zs, skip, dpart, lv1, that_tab);
    }
  }
  if ((passes & 4) && rs.items) {
    // entries read ahead per thread: 16, 24 or 32, as the transfer chose from
    // its row pairs' counts (more run in a loop)
    const dim3 gC(nbA + (fin.sc ? 1 : 0), nrhs), bC(C::LINES_A * C::TA);
    if (rs.ent_ahead <= 16)
      GOFD_LAUNCH(ctx, (k_passC<R, Y, L, C::EA, C::LINES_A, true, 16>), gC, bC, 0, st, Z, W, tw, zs, y,
                  (long long)W * W, skip, fin, rs);
    else if (rs.ent_ahead <= 24)
      GOFD_LAUNCH(ctx, (k_passC<R, Y, L, C::EA, C::LINES_A, true, 24>), gC, bC, 0, st, Z, W, tw, zs, y,
                  (long long)W * W, skip, fin, rs);
    else
      GOFD_LAUNCH(ctx, (k_passC<R, Y, L, C::EA, C::LINES_A, true, 32>), gC, bC, 0, st, Z, W, tw, zs, y,
                  (long long)W * W, skip, fin, rs);
  } else if (passes & 4)
    GOFD_LAUNCH(ctx, (k_passC<R, Y, L, C::EA, C::LINES_A, false>), dim3(nbA + (fin.sc ? 1 : 0), nrhs),
                dim3(C::LINES_A * C::TA), 0, st, Z, W, tw, zs, y, (long long)W * W, skip, fin, rs);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

template <typename R, class Src, typename Y>
int dispatch_2d(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const Src& src, Y* y, int passes, Skip skip,
                double* dpart = nullptr, const gofd_cg::Level1& lv1 = gofd_cg::Level1(),
                const gofd_cg::Finish& fin = gofd_cg::Finish(), const void* const* that_tab = nullptr,
                const RowScatter& rs = RowScatter{}) {
  switch (op->L) {
    case 8: return run_2d<R, 8>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 16: return run_2d<R, 16>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 32: return run_2d<R, 32>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 64: return run_2d<R, 64>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 128: return run_2d<R, 128>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 256: return run_2d<R, 256>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 512: return run_2d<R, 512>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 1024: return run_2d<R, 1024>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 2048: return run_2d<R, 2048>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
    case 4096: return run_2d<R, 4096>(ctx, op, nrhs, src, y, passes, skip, dpart, lv1, fin, that_tab, rs);
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
  long long zs = 1, nn = 1;
  for (int a = 0; a < op->d; ++a) {
    zs *= (a == 0 ? op->half : op->W);
    nn *= op->W;
  }
  if (op->d == 3) zs = conv3_workspace(op);
  GOFD_TRY(dev_reserve(ctx, op->G, sizeof(double) * nn * nrhs));
  return dev_reserve(ctx, op->Z, sizeof(cplx<double>) * zs * nrhs);
}

int conv_apply(gofd_ctx_s* ctx, gofd_fdop_s* op, int nrhs, const double* v, const GatherSpec* g, void* y,
               bool fp32, int passes) {
  const int d = op->d;
  if (d != 2 && d != 3) return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "dimension");
  long long nn = 1;
  for (int a = 0; a < d; ++a) nn *= op->W;
  const Skip skip{g ? g->skip : nullptr, g ? g->skip_stride : 0, g ? g->amap : nullptr};
  double* dpart = g ? g->dpart : nullptr;
  const gofd_cg::Level1 lv1 = g ? g->lv1 : gofd_cg::Level1();
  const gofd_cg::Finish fin = g ? g->fin : gofd_cg::Finish();
  const void* const* that_tab = g ? (fp32 ? g->that32_tab : g->that64_tab) : nullptr;
  if (v) {
    if (d == 3)
      return conv3_run(ctx, op, nrhs, v, nullptr, y, fp32, passes & 7, skip.flag, skip.stride, dpart, lv1, fin,
                       that_tab);
    SrcPairGrid<double> src{v, nn};
    return fp32 ? dispatch_2d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes, skip, dpart, lv1, fin,
                                     that_tab)
                : dispatch_2d<double>(ctx, op, nrhs, src, static_cast<double*>(y), passes, skip, dpart, lv1, fin,
                                      that_tab);
  }
  if (g->pregathered) passes &= ~8;
  hipStream_t st = ctx->stream;
  if (!ctx->ws_G) GOFD_TRY(dev_reserve(ctx, op->G, (fp32 ? sizeof(float) : sizeof(double)) * nn * nrhs));
  void* const Gp = ctx->ws_G ? ctx->ws_G : op->G.p;    // the gathered field I u
  const dim3 gg(grid1(nn, 256 * GATHER_NPT), nrhs);
  if (conv_gather_fused(op, fp32) && g->items && (passes & 8) && (passes & 1)) {
    // the FP32 gather of a batch runs inside the first row pass
    const RowScatter rs{g->rp_P ? g->items : nullptr, g->rp_P, g->rp_pstride, g->rp_ent_ahead};
#if GOFD_FFT_E_PASSA == GOFD_FFT_E_ROWS      // the slot capacity of a row pair follows the row passes' lines
    if (g->rp_us && d == 2) {
      SrcPairSegRows src{g->items, g->rp_us, g->rp_pstride};
      return dispatch_2d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes & 7, skip, dpart, lv1, fin,
                                that_tab, rs);
    }
#endif
    SrcPairGatherRows src{g->items, g->ubase, g->items_mask ? 1 : 0};
    return dispatch_2d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes & 7, skip, dpart, lv1, fin,
                              that_tab, rs);
  }
  if ((passes & 8) && g->items) {
    // batched: every item gathers from its own mesh
#define GOFD_GI(R, D) \
  GOFD_LAUNCH(ctx, (k_gather_items<R, D>), gg, dim3(256), 0, st, g->items, g->ubase, g->items_mask ? 1 : 0, nn, static_cast<R*>(Gp), skip)
    if (d == 2) {
      if (fp32) GOFD_GI(float, 2); else GOFD_GI(double, 2);
    } else {
      if (fp32) GOFD_GI(float, 3); else GOFD_GI(double, 3);
    }
#undef GOFD_GI
    HIP_TRY(ctx, hipGetLastError());
  } else if (passes & 8) {
    const gofd_transfer_s* tr = g->tr;
    GridGeom geom;
    geom.d = d;
    geom.W = tr->W;
    geom.h = tr->h;
    for (int a = 0; a < 3; ++a) geom.lo[a] = tr->lo[a];
    if (d == 2) {
      if (fp32)
        GOFD_LAUNCH(ctx, (k_gather<float, 2>), gg, dim3(256), 0, st, geom, tr->rec.as<ElemRec2>(),
                    tr->elem.as<int>(), tr->row32_v.as<int4>(), tr->row32_w.as<float2>(), g->u, g->col_scale, g->mask, (long long)tr->nv, nn, static_cast<float*>(Gp), skip);
      else
        GOFD_LAUNCH(ctx, (k_gather<double, 2>), gg, dim3(256), 0, st, geom, tr->rec.as<ElemRec2>(),
                    tr->elem.as<int>(), tr->row32_v.as<int4>(), tr->row32_w.as<float2>(), g->u, g->col_scale, g->mask, (long long)tr->nv, nn, static_cast<double*>(Gp), skip);
    } else {
      const dim3 ge(grid1(nn, 256), nrhs);
      if (fp32)
        GOFD_LAUNCH(ctx, (k_gather_ell<float>), ge, dim3(256), 0, st, tr->ell_idx.as<int>(), tr->ell_v.as<int4>(),
                    tr->ell_w.as<double2>(), g->u, g->col_scale, g->mask, (long long)tr->nv, nn, static_cast<float*>(Gp),
                    skip);
      else
        GOFD_LAUNCH(ctx, (k_gather_ell<double>), ge, dim3(256), 0, st, tr->ell_idx.as<int>(), tr->ell_v.as<int4>(),
                    tr->ell_w.as<double2>(), g->u, g->col_scale, g->mask, (long long)tr->nv, nn, static_cast<double*>(Gp),
                    skip);
    }
    HIP_TRY(ctx, hipGetLastError());
  }
  if (d == 3)
    return conv3_run(ctx, op, nrhs, fp32 ? nullptr : static_cast<double*>(Gp), fp32 ? static_cast<float*>(Gp) : nullptr, y, fp32,
                     passes & 7, skip.flag, skip.stride, dpart, lv1, fin, that_tab, skip.map);
  const RowScatter rs{g->rp_P ? g->items : nullptr, g->rp_P, g->rp_pstride, g->rp_ent_ahead};
  if (fp32) {
    SrcPairGrid<float> src{static_cast<float*>(Gp), nn};
    return dispatch_2d<float>(ctx, op, nrhs, src, static_cast<float*>(y), passes, skip, dpart, lv1, fin, that_tab,
                              rs);
  }
  SrcPairGrid<double> src{static_cast<double*>(Gp), nn};
  return dispatch_2d<double>(ctx, op, nrhs, src, static_cast<double*>(y), passes, skip, dpart, lv1, fin, that_tab,
                             rs);
}

template <typename R>
static int passB_blocks(int L, int s) {
  switch (L) {
    case 8: return passB_blocks_L<R, 8>(s);
    case 16: return passB_blocks_L<R, 16>(s);
    case 32: return passB_blocks_L<R, 32>(s);
    case 64: return passB_blocks_L<R, 64>(s);
    case 128: return passB_blocks_L<R, 128>(s);
    case 256: return passB_blocks_L<R, 256>(s);
    case 512: return passB_blocks_L<R, 512>(s);
    case 1024: return passB_blocks_L<R, 1024>(s);
    case 2048: return passB_blocks_L<R, 2048>(s);
    case 4096: return passB_blocks_L<R, 4096>(s);
    default: return 1;
  }
}

int conv_passB_blocks(const gofd_fdop_s* op, bool fp32) {
  if (op->d == 3) return conv3_passC_blocks(op, fp32);
  const int s = col_sched(op->ctx, op->L, fp32);
  return fp32 ? passB_blocks<float>(op->L, s) : passB_blocks<double>(op->L, s);
}

// ---------------------------------------------------------------- ABI

bool same_grid(const gofd_transfer_s* tr, const gofd_fdop_s* op) {
  return tr->d == op->d && tr->N == op->N && tr->R == op->R && tr->center[0] == op->center[0] &&
         tr->center[1] == op->center[1] && tr->center[2] == op->center[2];
}

// Column-pass schedule tuning (2D): time every schedule on a zero field of
// the grid's window (one field, the CG variant of the pass), keep the fastest.
template <typename R, int L>
static int tune_L(gofd_ctx_s* ctx, int W, double* times) {
  const int half = L / 2 + 1;
  const long long zs = (long long)W * (L / 2);
  const cplx<R>* tw = sizeof(R) == 8 ? reinterpret_cast<const cplx<R>*>(twiddles64(ctx, L))
                                     : reinterpret_cast<const cplx<R>*>(twiddles32(ctx, L));
  if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddle table");
  DevBuf Z, T, dp;
  GOFD_TRY(dev_reserve(ctx, Z, sizeof(cplx<R>) * zs));
  GOFD_TRY(dev_reserve(ctx, T, sizeof(R) * (long long)half * half));
  GOFD_TRY(dev_reserve(ctx, dp, sizeof(double) * 3 * (L / 2)));
  hipStream_t st = ctx->stream;
  HIP_TRY(ctx, hipMemsetAsync(Z.p, 0, sizeof(cplx<R>) * zs, st));
  HIP_TRY(ctx, hipMemsetAsync(T.p, 0, sizeof(R) * (long long)half * half, st));
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  const gofd_cg::Level1 lv1;
  const Skip skip{nullptr, 0};
  constexpr int reps = 20;
  int best = 0;
  for (int s = 0; s < GOFD_N_COL_SCHED; ++s) {
    auto run = [&]() {
      switch (s) {
        case 1: launch_passB_s<R, L, 1>(ctx, st, 1, Z.as<cplx<R>>(), W, half, T.as<R>(), tw, zs, skip, dp.as<double>(), lv1, nullptr); break;
        case 2: launch_passB_s<R, L, 2>(ctx, st, 1, Z.as<cplx<R>>(), W, half, T.as<R>(), tw, zs, skip, dp.as<double>(), lv1, nullptr); break;
        case 3: launch_passB_s<R, L, 3>(ctx, st, 1, Z.as<cplx<R>>(), W, half, T.as<R>(), tw, zs, skip, dp.as<double>(), lv1, nullptr); break;
        default: launch_passB_s<R, L, 0>(ctx, st, 1, Z.as<cplx<R>>(), W, half, T.as<R>(), tw, zs, skip, dp.as<double>(), lv1, nullptr);
      }
    };
    for (int k = 0; k < 3; ++k) run();
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < reps; ++k) run();
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return gofd_fail(ctx, GOFD_E_HIP, "timing the column pass failed");
    }
    times[s] = ms / reps;
  }
  // another schedule replaces the default only when clearly faster (5 %):
  // closer timings are within the noise of this measurement
  for (int s = 1; s < GOFD_N_COL_SCHED; ++s)
    if (times[s] < 0.95 * times[0] && times[s] < times[best]) best = s;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(ctx, hipGetLastError());
  return best;
}

// First row pass of the products (a grid-field source): 8 against 16 values
// per thread, where both hold one row pair per block (L >= 1024).  times[0]
// for 8, times[1] for 16; returns the values per thread to use (0: only one
// width exists for this length).
template <typename R, int L>
static int tune_rows_L(gofd_ctx_s* ctx, int W, double* times) {
  using C = Cfg<R, L>;
  constexpr bool BOTH = L / 16 >= 64 && C::TA >= 64 && C::E1 == 8;
  if constexpr (!BOTH) {
    return 0;
  } else {
    const long long zs = (long long)W * (L / 2), nn = (long long)W * W;
    const cplx<R>* tw = sizeof(R) == 8 ? reinterpret_cast<const cplx<R>*>(twiddles64(ctx, L))
                                       : reinterpret_cast<const cplx<R>*>(twiddles32(ctx, L));
    if (!tw) return gofd_fail(ctx, GOFD_E_OOM, "twiddle table");
    DevBuf Z, F;
    GOFD_TRY(dev_reserve(ctx, Z, sizeof(cplx<R>) * zs));
    GOFD_TRY(dev_reserve(ctx, F, sizeof(R) * nn));
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipMemsetAsync(F.p, 0, sizeof(R) * nn, st));
    const SrcPairGrid<R> src{F.as<R>(), nn};
    const Skip skip{nullptr, 0};
    const int pairs = (W + 1) / 2;
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    constexpr int reps = 20;
    for (int v = 0; v < 2; ++v) {
      auto run = [&]() {
        if (v == 0) launch_passA<R, L, 8>(ctx, st, 1, pairs, src, Z.as<cplx<R>>(), W, tw, zs, skip);
        else launch_passA<R, L, 16>(ctx, st, 1, pairs, src, Z.as<cplx<R>>(), W, tw, zs, skip);
      };
      for (int k = 0; k < 3; ++k) run();
      (void)hipEventRecord(e0, st);
      for (int k = 0; k < reps; ++k) run();
      (void)hipEventRecord(e1, st);
      float ms = 0.f;
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return gofd_fail(ctx, GOFD_E_HIP, "timing the row pass failed");
      }
      times[v] = ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(ctx, hipGetLastError());
    return times[1] < 0.95 * times[0] ? 16 : 8;   // 16 only when clearly faster than the default
  }
}

template <typename R>
static int tune_rows(gofd_ctx_s* ctx, int L, int W, double* times) {
  switch (L) {
    case 1024: return tune_rows_L<R, 1024>(ctx, W, times);
    case 2048: return tune_rows_L<R, 2048>(ctx, W, times);
    case 4096: return tune_rows_L<R, 4096>(ctx, W, times);
    default: return 0;
  }
}

template <typename R>
static int tune_2d(gofd_ctx_s* ctx, int L, int W, double* times) {
  switch (L) {
    case 8: return tune_L<R, 8>(ctx, W, times);
    case 16: return tune_L<R, 16>(ctx, W, times);
    case 32: return tune_L<R, 32>(ctx, W, times);
    case 64: return tune_L<R, 64>(ctx, W, times);
    case 128: return tune_L<R, 128>(ctx, W, times);
    case 256: return tune_L<R, 256>(ctx, W, times);
    case 512: return tune_L<R, 512>(ctx, W, times);
    case 1024: return tune_L<R, 1024>(ctx, W, times);
    case 2048: return tune_L<R, 2048>(ctx, W, times);
    case 4096: return tune_L<R, 4096>(ctx, W, times);
    default: return gofd_fail(ctx, GOFD_E_UNSUPPORTED, "FFT length");
  }
}

extern "C" int gofd_autotune(gofd_ctx ctx, const gofd_grid* grid, int flags, int* sched, double* times) {
  if (!ctx || !grid || grid->N < 1 || (grid->d != 2 && grid->d != 3)) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  const bool fp32 = flags & GOFD_FP32_GRID;
  const int L = conv_period(grid->N), W = 2 * grid->N + 1;
  double t[GOFD_N_TUNE_TIMES];
  for (double& x : t) x = HUGE_VAL;
  int out[2] = {0, 0};
  if (grid->d == 3) {
    const int best = conv3_tune(ctx, grid, fp32, t);
    if (best < 0) return best;
    out[0] = best;
  } else {
    const int best = fp32 ? tune_2d<float>(ctx, L, W, t) : tune_2d<double>(ctx, L, W, t);
    if (best < 0) return best;
    ctx->col_sched[std::make_pair(L, fp32)] = best;
    out[0] = best;
    ctx->row_sched.erase(std::make_pair(L, fp32));
    const int rows = fp32 ? tune_rows<float>(ctx, L, W, t + 4) : tune_rows<double>(ctx, L, W, t + 4);
    if (rows < 0) return rows;
    if (rows > 0) ctx->row_sched[std::make_pair(L, fp32)] = rows;
    out[1] = rows;
  }
  if (sched) {
    sched[0] = out[0];
    sched[1] = out[1];
  }
  if (times)
    for (int s = 0; s < GOFD_N_TUNE_TIMES; ++s) times[s] = t[s];
  return GOFD_OK;
}

extern "C" int gofd_set_schedule(gofd_ctx ctx, const gofd_grid* grid, int flags, int sched) {
  if (!ctx || !grid || grid->N < 1 || (grid->d != 2 && grid->d != 3)) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  const auto key = std::make_pair(conv_period(grid->N), (flags & GOFD_FP32_GRID) != 0);
  if (grid->d == 3) {
    if (sched != 0 && sched != 1) return gofd_fail(ctx, GOFD_E_ARG, "3D schedules are 0 and 1");
    ctx->sched3[key] = sched;
  } else if (flags & GOFD_SCHED_ROWS) {
    if (sched != 0 && sched != 8 && sched != 16) return gofd_fail(ctx, GOFD_E_ARG, "row pass: 0, 8 or 16 values");
    ctx->row_sched[key] = sched;
  } else {
    if (sched < 0 || sched >= GOFD_N_COL_SCHED) return gofd_fail(ctx, GOFD_E_ARG, "bad column schedule");
    ctx->col_sched[key] = sched;
  }
  return GOFD_OK;
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

int apply_Ah_impl(gofd_ctx_s* ctx, gofd_transfer_s* tr, gofd_fdop_s* op, int nrhs, const double* u, double* y,
                  int flags, void* ygrid) {
  if (!ctx || !tr || !op || !u || !y || nrhs < 1) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  if (!same_grid(tr, op)) return gofd_fail(ctx, GOFD_E_ARG, "transfer and operator use different grids");
  const bool fp32 = flags & GOFD_FP32_GRID;
  const bool sym = flags & GOFD_SYMMETRIC;
  const bool unscaled = flags & GOFD_UNSCALED;
  const bool interior = flags & GOFD_INTERIOR;
  if (sym && unscaled) return gofd_fail(ctx, GOFD_E_ARG, "SYMMETRIC and UNSCALED are exclusive");
  const long long n_nodes = tr->n_nodes;
  if (!ygrid) {
    GOFD_TRY(dev_reserve(ctx, op->Y, (fp32 ? sizeof(float) : sizeof(double)) * n_nodes * nrhs));
    ygrid = op->Y.p;
  }
  GatherSpec g;
  g.tr = tr;
  g.u = u;
  g.col_scale = sym ? tr->dsqrt.as<double>() : nullptr;
  g.mask = interior ? tr->imask.as<double>() : nullptr;
  GOFD_TRY(conv_apply(ctx, op, nrhs, nullptr, &g, ygrid, fp32));
  const double* scale = unscaled ? nullptr : (sym ? tr->dsqrt.as<double>() : tr->dscale.as<double>());
  GOFD_TRY(scatter_apply(ctx, tr, nrhs, ygrid, fp32, scale, interior ? tr->imask.as<double>() : nullptr, y));
  if (flags & GOFD_SCALE_H2S) {
    const double f = 1.0 / op->h2s;
    long long n = tr->nv * nrhs;
    hipLaunchKernelGGL(k_scale, dim3(grid1(n, 256)), dim3(256), 0, ctx->stream, y, n, f);
  }
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

extern "C" int gofd_apply_Ah(gofd_ctx ctx, gofd_transfer tr, gofd_fdop op, int nrhs, const double* u, double* y,
                             int flags) {
  return apply_Ah_impl(ctx, tr, op, nrhs, u, y, flags, nullptr);
}

// ---------------------------------------------------------------- operator from a table

static int next_pow2(long long x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

int conv_period(int N) { return std::max(8, next_pow2(4LL * N)); }

#ifndef GOFD_FUSE_GATHER
#define GOFD_FUSE_GATHER 1
#endif
bool conv_gather_fused(const gofd_fdop_s* op, bool fp32) { return GOFD_FUSE_GATHER && op->d == 2 && fp32; }

int conv_rowpass_threads(int L) {
  const int E = std::min(GOFD_FFT_E_ROWS, L);
  return L / E;
}

int conv_rowpass_lines(int L) {
  const int T = conv_rowpass_threads(L);
  return T >= 64 ? 1 : 64 / T;
}

int fdop_init_geometry(gofd_ctx_s* ctx, gofd_fdop_s* op, double s, const gofd_grid* grid) {
  if (!grid || (grid->d != 2 && grid->d != 3) || grid->N < 1 || !(grid->R > 0))
    return gofd_fail(ctx, GOFD_E_ARG, "bad grid");
  if (!(s > 0.0 && s < 1.0)) return gofd_fail(ctx, GOFD_E_ARG, "s must lie in (0, 1)");
  op->ctx = ctx;
  op->d = grid->d;
  op->N = grid->N;
  op->W = 2 * grid->N + 1;
  op->L = conv_period(grid->N);     // L >= 4N keeps the embedding exact (R7); 8 is the smallest built
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
  if (!ctx || !tr || !op || !u || !avg_ms || nrhs < 1 || reps < 1 || which < 0 || which > 4)
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
  GOFD_TRY(conv_apply(ctx, op, nrhs, nullptr, &g, op->Y.p, fp32, 15));
  auto launch = [&]() -> int {
    if (which == GOFD_K_SCATTER)
      return scatter_apply(ctx, tr, nrhs, op->Y.p, fp32, nullptr, tr->imask.as<double>(), z.as<double>());
    return conv_apply(ctx, op, nrhs, nullptr, &g, op->Y.p, fp32, which == GOFD_K_GATHER ? 8 : 1 << which);
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
