// Transfer matrix I_h^FD: point location, barycentric weights, the vertex-major
// (transposed) structure, column sums D_h, and the I^T scatter.
//
// Section 3.1 of the paper: (I_h^FD)_{k,j} = phi_j(x_k^FD) (eq. IhFD-1); a node
// outside the closed mesh has a zero row; D_{h,j} = sum_k (I_h^FD)_{k,j}.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <queue>
#include <thread>

#include "bary.h"
#include "internal.h"
#include "predicates.h"

namespace {

constexpr int NO_ELEM = 0x7fffffff;

GridGeom make_geom(const gofd_transfer_s* tr) {
  GridGeom g;
  g.d = tr->d;
  g.W = tr->W;
  g.h = tr->h;
  for (int a = 0; a < 3; ++a) g.lo[a] = tr->lo[a];
  return g;
}

// ---------------------------------------------------------------- K1: location
//
// One thread per element: the element's bounding box in grid-index space is
// enlarged by one node on each side (a conservative candidate set), and every
// candidate node is tested against the closed simplex with exact orientation
// signs.  elem_of_node[k] receives the smallest containing element id through
// an integer atomicMin, so the result does not depend on scheduling.
template <int D>
__global__ __launch_bounds__(256) void k_locate(GridGeom g, const double* __restrict__ X,
                                                const int* __restrict__ elems, long long ne,
                                                int* __restrict__ elem_of_node,
                                                unsigned long long* __restrict__ counters) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double V[D + 1][3];
  for (int r = 0; r <= D; ++r) {
    const int v = elems[e * (D + 1) + r];
    for (int a = 0; a < D; ++a) V[r][a] = X[(long long)v * D + a];
  }
  int exact_used = 0;
  int esign;
  if constexpr (D == 2)
    esign = gofd_exact::orient2_sign(V[0], V[1], V[2], &exact_used);
  else
    esign = gofd_exact::orient3_sign(V[0], V[1], V[2], V[3], &exact_used);
  if (esign == 0) {
    atomicOr((unsigned int*)&counters[1], 1u);   // degenerate element
    return;
  }
  if (esign == 2) {
    atomicOr((unsigned int*)&counters[2], 1u);   // expansion capacity
    return;
  }
  int ilo[3], ihi[3];
  for (int a = 0; a < D; ++a) {
    double mn = V[0][a], mx = V[0][a];
    for (int r = 1; r <= D; ++r) {
      mn = fmin(mn, V[r][a]);
      mx = fmax(mx, V[r][a]);
    }
    const double fl = floor((mn - g.lo[a]) / g.h) - 1.0;
    const double cl = ceil((mx - g.lo[a]) / g.h) + 1.0;
    ilo[a] = (int)fmax(0.0, fmin((double)(g.W - 1), fl));
    ihi[a] = (int)fmax(0.0, fmin((double)(g.W - 1), cl));
  }
  unsigned long long nexact = exact_used;
  const int nz = (D == 3) ? (ihi[2] - ilo[2] + 1) : 1;
  for (int iz = 0; iz < nz; ++iz) {
    for (int iy = ilo[1]; iy <= ihi[1]; ++iy) {
      for (int ix = ilo[0]; ix <= ihi[0]; ++ix) {
        double p[3];
        p[0] = node_coord(g, 0, ix);
        p[1] = node_coord(g, 1, iy);
        if constexpr (D == 3) p[2] = node_coord(g, 2, ilo[2] + iz);
        bool inside = true;
        for (int r = 0; r <= D && inside; ++r) {
          int ex = 0;
          int sg;
          if constexpr (D == 2) {
            const double* q[3] = {V[0], V[1], V[2]};
            q[r] = p;
            sg = gofd_exact::orient2_sign(q[0], q[1], q[2], &ex);
          } else {
            const double* q[4] = {V[0], V[1], V[2], V[3]};
            q[r] = p;
            sg = gofd_exact::orient3_sign(q[0], q[1], q[2], q[3], &ex);
          }
          nexact += ex;
          if (sg == 2) {
            atomicOr((unsigned int*)&counters[2], 1u);
            inside = false;
          } else if (sg * esign < 0) {
            inside = false;
          }
        }
        if (inside) {
          long long k = (long long)ix + (long long)g.W * iy;
          if constexpr (D == 3) k += (long long)g.W * g.W * (ilo[2] + iz);
          atomicMin(&elem_of_node[k], (int)e);
        }
      }
    }
  }
  if (nexact) atomicAdd(&counters[0], nexact);
}

__global__ void k_fill_i32(int* __restrict__ p, long long n, int v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_finish_location(int* __restrict__ elem_of_node, long long n,
                                  unsigned long long* __restrict__ counters) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  if (elem_of_node[k] == NO_ELEM)
    elem_of_node[k] = -1;
  else
    atomicAdd(&counters[3], 1ull);
}

// ---------------------------------------------------------------- K3: CSC
template <int D>
__global__ void k_count(const int* __restrict__ elem_of_node, const int* __restrict__ elems, long long n,
                        int* __restrict__ cnt) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int e = elem_of_node[k];
  if (e < 0) return;
  for (int r = 0; r <= D; ++r) atomicAdd(&cnt[elems[(long long)e * (D + 1) + r]], 1);
}

template <int D>
__global__ void k_make_records(const double* __restrict__ X, const int* __restrict__ elems, long long ne,
                               ElemRec<D>* __restrict__ recs) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  ElemRec<D> r;
  make_record<D>(X, elems, e, r);
  recs[e] = r;
}

template <int D>
__global__ void k_fill_csc(GridGeom g, const ElemRec<D>* __restrict__ recs,
                           const int* __restrict__ elem_of_node, long long n, int* __restrict__ cursor,
                           int* __restrict__ node_out, double* __restrict__ w_out) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int e = elem_of_node[k];
  if (e < 0) return;
  int vid[D + 1];
  double lam[D + 1];
  node_weights<D>(g, recs, e, k, vid, lam);
  for (int r = 0; r <= D; ++r) {
    const int pos = atomicAdd(&cursor[vid[r]], 1);
    node_out[pos] = (int)k;
    w_out[pos] = lam[r];
  }
}

// one 64-lane wavefront per vertex: rank each entry of the segment by node
// number (node numbers are distinct inside a segment) and scatter it to its
// sorted position.  Deterministic regardless of the fill order above.
__global__ __launch_bounds__(256) void k_sort_segments(const int* __restrict__ off, long long nv,
                                                       const int* __restrict__ node_in,
                                                       const double* __restrict__ w_in,
                                                       int* __restrict__ node_out, double* __restrict__ w_out) {
  const long long v = ((long long)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int lane = threadIdx.x & 63;
  if (v >= nv) return;
  const int b = off[v], e = off[v + 1];
  for (int i = b + lane; i < e; i += 64) {
    const int key = node_in[i];
    int rank = 0;
    for (int j = b; j < e; ++j) rank += (node_in[j] < key);
    node_out[b + rank] = key;
    w_out[b + rank] = w_in[i];
  }
}

// D_j = sum of the column's weights in ascending node order; scale factors
__global__ void k_colsum(const int* __restrict__ off, long long nv, const double* __restrict__ w,
                         const unsigned char* __restrict__ bmask, double* __restrict__ D,
                         double* __restrict__ dscale, double* __restrict__ dsqrt, double* __restrict__ imask,
                         float* __restrict__ w32, long long nnz) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double s = 0.0;
  for (int i = off[v]; i < off[v + 1]; ++i) {
    s += w[i];
    w32[i] = (float)w[i];
  }
  D[v] = s;
  dscale[v] = s > 0.0 ? 1.0 / s : 0.0;
  dsqrt[v] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  imask[v] = bmask[v] ? 0.0 : 1.0;
}

// single-precision interpolation row of every node (2D): vertex ids and the
// weights rounded to float exactly as the I^T entries are; nodes outside the
// mesh get vertex 0 with weight zero
__global__ void k_fill_rows32(GridGeom g, const ElemRec2* __restrict__ recs, const int* __restrict__ elem_of_node,
                              long long n, int4* __restrict__ rv, float2* __restrict__ rw) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int e = elem_of_node[k];
  if (e < 0) {
    rv[k] = make_int4(0, 0, 0, 0);
    rw[k] = make_float2(0.f, 0.f);
    return;
  }
  int vid[3];
  double lam[3];
  node_weights<2>(g, recs, e, k, vid, lam);
  rv[k] = make_int4(vid[0], vid[1], vid[2], __float_as_int((float)lam[0]));
  rw[k] = make_float2((float)lam[1], (float)lam[2]);
}

template <int D>
__global__ void k_export_ell(GridGeom g, const ElemRec<D>* __restrict__ recs,
                             const int* __restrict__ elem_of_node, long long n, int* __restrict__ verts,
                             double* __restrict__ wts) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int e = elem_of_node[k];
  if (e < 0) {
    for (int r = 0; r <= D; ++r) {
      if (verts) verts[k * (D + 1) + r] = -1;
      if (wts) wts[k * (D + 1) + r] = 0.0;
    }
    return;
  }
  int vid[D + 1];
  double lam[D + 1];
  node_weights<D>(g, recs, e, k, vid, lam);
  for (int r = 0; r <= D; ++r) {
    if (verts) verts[k * (D + 1) + r] = vid[r];
    if (wts) wts[k * (D + 1) + r] = lam[r];
  }
}

__global__ void k_inside_flag(const int* __restrict__ elem, long long n, int* __restrict__ flag) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) flag[k] = elem[k] >= 0 ? 1 : 0;
}

// Interpolation rows of the inside nodes, compacted: idx holds the exclusive
// prefix of the inside flags on entry and the row (or -1) on exit.
template <int D>
__global__ void k_fill_ell(GridGeom g, const ElemRec<D>* __restrict__ recs, const int* __restrict__ elem_of_node,
                           long long n, int* __restrict__ idx, int* __restrict__ ev, double* __restrict__ ew) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int e = elem_of_node[k];
  if (e < 0) {
    idx[k] = -1;
    return;
  }
  const long long c = idx[k];
  int vid[D + 1];
  double lam[D + 1];
  node_weights<D>(g, recs, e, k, vid, lam);
  for (int r = 0; r <= D; ++r) {
    ev[c * (D + 1) + r] = vid[r];
    ew[c * (D + 1) + r] = lam[r];
  }
}

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- host helpers

// Dirichlet vertices: vertices of facets owned by exactly one element.
static void boundary_mask(int d, int64_t nv, const std::vector<int32_t>& el, std::vector<uint8_t>& mask) {
  const int64_t ne = (int64_t)el.size() / (d + 1);
  std::vector<std::pair<uint64_t, uint64_t>> keys;
  keys.reserve(ne * (d + 1));
  for (int64_t e = 0; e < ne; ++e) {
    for (int r = 0; r <= d; ++r) {
      int32_t f[3];
      int c = 0;
      for (int q = 0; q <= d; ++q)
        if (q != r) f[c++] = el[e * (d + 1) + q];
      std::sort(f, f + d);
      uint64_t k0 = (uint64_t)(uint32_t)f[0] << 32 | (uint32_t)f[1];
      uint64_t k1 = (d == 3) ? (uint64_t)(uint32_t)f[2] : 0;
      keys.push_back({k0, k1});
    }
  }
  std::sort(keys.begin(), keys.end());
  mask.assign(nv, 0);
  for (size_t i = 0; i < keys.size();) {
    size_t j = i + 1;
    while (j < keys.size() && keys[j] == keys[i]) ++j;
    if (j - i == 1) {
      mask[(uint32_t)(keys[i].first >> 32)] = 1;
      mask[(uint32_t)(keys[i].first & 0xffffffffu)] = 1;
      if (d == 3) mask[(uint32_t)keys[i].second] = 1;
    }
    i = j;
  }
}

static double min_height(int d, const std::vector<double>& X, const std::vector<int32_t>& el) {
  const int64_t ne = (int64_t)el.size() / (d + 1);
  double best = INFINITY;
  for (int64_t e = 0; e < ne; ++e) {
    double P[4][3];
    for (int r = 0; r <= d; ++r)
      for (int a = 0; a < d; ++a) P[r][a] = X[(int64_t)el[e * (d + 1) + r] * d + a];
    if (d == 2) {
      const double area2 = std::fabs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]));
      for (int j = 0; j < 3; ++j) {
        const int a = (j + 1) % 3, b = (j + 2) % 3;
        const double len = std::hypot(P[b][0] - P[a][0], P[b][1] - P[a][1]);
        best = std::min(best, area2 / len);
      }
    } else {
      double u[3], v[3], w[3];
      for (int a = 0; a < 3; ++a) {
        u[a] = P[1][a] - P[0][a];
        v[a] = P[2][a] - P[0][a];
        w[a] = P[3][a] - P[0][a];
      }
      const double vol6 = std::fabs(u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
                                    u[2] * (v[0] * w[1] - v[1] * w[0]));
      for (int j = 0; j < 4; ++j) {
        int o[3], c = 0;
        for (int q = 0; q < 4; ++q)
          if (q != j) o[c++] = q;
        double s[3], t[3];
        for (int a = 0; a < 3; ++a) {
          s[a] = P[o[1]][a] - P[o[0]][a];
          t[a] = P[o[2]][a] - P[o[0]][a];
        }
        const double cx = s[1] * t[2] - s[2] * t[1], cy = s[2] * t[0] - s[0] * t[2], cz = s[0] * t[1] - s[1] * t[0];
        const double area2 = std::sqrt(cx * cx + cy * cy + cz * cz);
        best = std::min(best, vol6 / area2);
      }
    }
  }
  return best;
}

// ---------------------------------------------------------------- ABI

// ---------------------------------------------------------------- row-pair form of I^T (2D)
//
// The CG iteration forms (I^T y)_j = sum_k lambda_j(k) y_k inside the last
// row pass, which holds two rows of y at a time: for each row pair the
// entries (j, k) of the rows' nodes are grouped by vertex into segments, each
// segment's sum goes to one partial slot of its vertex (slots of a vertex are
// contiguous, in row-pair order), and a vertex kernel adds its partials.
// The sums run in a fixed order, so results are reproducible.
//
// Layout for the row pass (T threads per row pair, as it is launched): the
// segments of a row pair, in vertex order, are split into T contiguous runs
// of about equal entry count; thread t's entries are stored at
// base + m T + t (m = 0..ENT-1, padded with zero weights), each with its
// local node (row offset times W plus column) and a flag on the last entry
// of each segment.  Leaves rp_ok false (nothing built) when a row pair has
// more segments than a block can hold.
static int build_rowpairs(gofd_ctx_s* ctx, gofd_transfer_s* tr, const std::vector<int32_t>& offh) {
  hipStream_t st = ctx->stream;
  tr->rp_ok = false;
  tr->seg_rows_ok = false;
  if (tr->d != 2 || tr->nnz == 0) return GOFD_OK;
  const int64_t nv = tr->nv, nnz = tr->nnz;
  const int W = tr->W;
  const int L = conv_period(tr->N);
  const int T = conv_rowpass_threads(L);
  const int lines = conv_rowpass_lines(L);
  const int pairs = (W + 1) / 2;
  std::vector<int32_t> node(nnz);
  std::vector<double> wv(nnz);
  HIP_TRY(ctx, hipMemcpyAsync(node.data(), tr->csc_node.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(wv.data(), tr->csc_w.p, sizeof(double) * nnz, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  // segments: runs of a vertex's entries (sorted by node) within one row
  // pair; numbered vertex-major, which makes a segment's number its slot
  std::vector<int32_t> seg_rp, seg_a, seg_b;
  std::vector<int32_t> pv(nv + 1, 0);
  for (int64_t v = 0; v < nv; ++v) {
    int32_t i = offh[v];
    while (i < offh[v + 1]) {
      const int rp = (node[i] / W) / 2;
      int32_t j = i + 1;
      while (j < offh[v + 1] && (node[j] / W) / 2 == rp) ++j;
      seg_rp.push_back(rp);
      seg_a.push_back(i);
      seg_b.push_back(j);
      i = j;
    }
    pv[v + 1] = (int32_t)seg_rp.size();
  }
  const int64_t nseg = (int64_t)seg_rp.size();
  // segments of each row pair, in vertex order
  std::vector<int32_t> rp_cnt(pairs + 1, 0);
  for (int64_t q = 0; q < nseg; ++q) ++rp_cnt[seg_rp[q] + 1];
  for (int r = 0; r < pairs; ++r) {
    if (rp_cnt[r + 1] > RP_SEGCAP / lines) return GOFD_OK;     // too many for a block: keep the CSC form
    rp_cnt[r + 1] += rp_cnt[r];
  }
  std::vector<int32_t> dest(nseg), fill(rp_cnt.begin(), rp_cnt.end() - 1);
  for (int64_t q = 0; q < nseg; ++q) dest[fill[seg_rp[q]]++] = (int32_t)q;
  // per row pair: a balanced contiguous split over the T threads
  if (2 * (int64_t)W > RP_NODE + 1) return GOFD_OK;        // local node numbers must fit the 15-bit code
  // per row pair: segments over the T threads by longest-first onto the
  // least-loaded thread (ties: the lower thread), then laid out thread by
  // thread, each thread's in vertex order.  Row pairs are independent: the
  // plans and then the entries are made by host threads over row pairs.
  std::vector<int32_t> meta(4 * (size_t)pairs), tseg((size_t)pairs * T), tcnt((size_t)pairs * T), ent(pairs),
      plan(nseg);
  auto len = [&](int32_t p) { return seg_b[dest[p]] - seg_a[dest[p]]; };
  const int nthr = std::max(1, std::min<int>(16, (int)std::thread::hardware_concurrency()));
  auto parallel_rows = [&](auto&& body) {
    std::vector<std::thread> pool;
    for (int h = 0; h < nthr; ++h)
      pool.emplace_back([&, h]() {
        for (int r = h; r < pairs; r += nthr) body(r);
      });
    for (auto& th : pool) th.join();
  };
  parallel_rows([&](int r) {
    const int32_t s0 = rp_cnt[r], s1 = rp_cnt[r + 1];
    std::vector<int32_t> order(s1 - s0), load(T, 0);
    std::vector<std::vector<int32_t>> owned(T);
    for (int32_t p = s0; p < s1; ++p) order[p - s0] = p;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return len(x) > len(y); });
    std::priority_queue<std::pair<int32_t, int>, std::vector<std::pair<int32_t, int>>,
                        std::greater<std::pair<int32_t, int>>> heap;
    for (int c = 0; c < T; ++c) heap.push({0, c});
    for (int32_t p : order) {
      const int k = heap.top().second;
      heap.pop();
      load[k] += len(p);
      owned[k].push_back(p);
      heap.push({load[k], k});
    }
    int32_t pos = s0, e = 0;
    for (int k = 0; k < T; ++k) {
      std::sort(owned[k].begin(), owned[k].end());
      tseg[(size_t)r * T + k] = pos - s0;
      tcnt[(size_t)r * T + k] = load[k];
      for (int32_t p : owned[k]) plan[pos++] = dest[p];     // segment (= slot) at each position
      e = std::max(e, load[k]);
    }
    ent[r] = e;
  });
  int64_t ebase = 0;
  for (int r = 0; r < pairs; ++r) {
    meta[4 * (size_t)r + 0] = (int32_t)ebase;
    meta[4 * (size_t)r + 1] = ent[r];
    meta[4 * (size_t)r + 2] = rp_cnt[r];
    meta[4 * (size_t)r + 3] = rp_cnt[r + 1] - rp_cnt[r];
    ebase += (int64_t)ent[r] * T;
    if (ebase >= ((int64_t)1 << 30)) return GOFD_OK;
  }
  // entries (padding: node 0, weight 0; RP_EPRE * T more read ahead past the last row pair)
  const int64_t total = ebase + (int64_t)RP_EPRE * T;
  std::vector<uint16_t> code(total, 0);
  std::vector<float> w32(total, 0.f);
  std::vector<double> w64(total, 0.0);
  // per node: the local segments (position within the row pair) and weights
  // of its entries, for the FP32 gather through the slots
  const int64_t n_nodes = (int64_t)W * W;
  std::vector<int32_t> srow(4 * (size_t)n_nodes, 0);
  std::vector<float> srow_w2(n_nodes, 0.f);
  std::vector<uint8_t> scnt(n_nodes, 0);
  std::atomic<bool> srow_ok{true};
  parallel_rows([&](int r) {
    const int64_t base = meta[4 * (size_t)r];
    const int32_t s0 = rp_cnt[r], s1 = rp_cnt[r + 1];
    for (int k = 0; k < T; ++k) {
      const int32_t p0 = s0 + tseg[(size_t)r * T + k];
      const int32_t p1 = (k + 1 < T) ? s0 + tseg[(size_t)r * T + k + 1] : s1;
      int64_t m = 0;
      for (int32_t p = p0; p < p1; ++p) {
        const int32_t q = plan[p];
        for (int32_t i = seg_a[q]; i < seg_b[q]; ++i, ++m) {
          const int32_t row = node[i] / W, col = node[i] % W;
          const int64_t at = base + m * T + k;
          code[at] = (uint16_t)(((row - 2 * r) * W + col) | (i + 1 == seg_b[q] ? RP_END : 0));
          w64[at] = wv[i];
          w32[at] = (float)wv[i];
          // the nodes of rows 2r, 2r+1 belong to this row pair only
          const int64_t n = node[i];
          const int c = scnt[n]++;
          const int32_t loc = p - s0;
          if (c == 0) {
            srow[4 * n] = loc;
            srow[4 * n + 2] = (int32_t)__builtin_bit_cast(uint32_t, (float)wv[i]);
          } else if (c == 1) {
            srow[4 * n] |= loc << 16;
            srow[4 * n + 3] = (int32_t)__builtin_bit_cast(uint32_t, (float)wv[i]);
          } else if (c == 2) {
            srow[4 * n + 1] = loc;
            srow_w2[n] = (float)wv[i];
          } else {
            srow_ok = false;
          }
        }
      }
    }
  });
  dest.swap(plan);                                  // the slot of each segment, row pair by row pair in thread order
  std::vector<int32_t> pos(std::max<int64_t>(nseg, 1), 0);
  for (int64_t p = 0; p < nseg; ++p) pos[dest[p]] = (int32_t)p;
  GOFD_TRY(dev_reserve(ctx, tr->rp_meta, sizeof(int32_t) * meta.size()));
  // on the device each thread's word also carries its entry count (bits 16..31), so that its loads stop at
  // its last entry: first segment < RP_SEGCAP fits the low 16 bits
  for (size_t i = 0; i < tseg.size(); ++i) {
    if (tcnt[i] > 0xffff) return GOFD_OK;
    tseg[i] |= tcnt[i] << 16;
  }
  GOFD_TRY(dev_reserve(ctx, tr->rp_tseg, sizeof(int32_t) * tseg.size()));
  GOFD_TRY(dev_reserve(ctx, tr->rp_code, sizeof(uint16_t) * total));
  GOFD_TRY(dev_reserve(ctx, tr->rp_w32, sizeof(float) * total));
  GOFD_TRY(dev_reserve(ctx, tr->rp_w64, sizeof(double) * total));
  GOFD_TRY(dev_reserve(ctx, tr->rp_dest, sizeof(int32_t) * std::max<int64_t>(nseg, 1)));
  GOFD_TRY(dev_reserve(ctx, tr->pv_off, sizeof(int32_t) * (nv + 1)));
  HIP_TRY(ctx, hipMemcpyAsync(tr->rp_meta.p, meta.data(), sizeof(int32_t) * meta.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->rp_tseg.p, tseg.data(), sizeof(int32_t) * tseg.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->rp_code.p, code.data(), sizeof(uint16_t) * total, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->rp_w32.p, w32.data(), sizeof(float) * total, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->rp_w64.p, w64.data(), sizeof(double) * total, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->rp_dest.p, dest.data(), sizeof(int32_t) * nseg, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->pv_off.p, pv.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, st));
  tr->seg_rows_ok = srow_ok;
  if (srow_ok) {
    GOFD_TRY(dev_reserve(ctx, tr->rp_pos, sizeof(int32_t) * pos.size()));
    GOFD_TRY(dev_reserve(ctx, tr->seg_row, sizeof(int32_t) * srow.size()));
    GOFD_TRY(dev_reserve(ctx, tr->seg_row_w2, sizeof(float) * srow_w2.size()));
    HIP_TRY(ctx, hipMemcpyAsync(tr->rp_pos.p, pos.data(), sizeof(int32_t) * pos.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(tr->seg_row.p, srow.data(), sizeof(int32_t) * srow.size(), hipMemcpyHostToDevice,
                                st));
    HIP_TRY(ctx, hipMemcpyAsync(tr->seg_row_w2.p, srow_w2.data(), sizeof(float) * srow_w2.size(),
                                hipMemcpyHostToDevice, st));
  }
  HIP_TRY(ctx, hipStreamSynchronize(st));      // the host arrays go out of scope
  tr->n_slots = nseg;
  // entries the last row pass reads ahead per thread: the largest of 16, 24,
  // 32 not above the median count of the row pairs (the rest of a row pair's
  // entries run in a loop).  On the L-shape (25-29 entries per thread) 24
  // took 11.7 us against 12.3 for 28 and 13.1 for 32: loads read ahead past a
  // thread's count cost more than the few loop iterations
  {
    std::vector<int> e(ent.begin(), ent.end());
    std::sort(e.begin(), e.end());
    const int med = e.empty() ? 0 : e[e.size() / 2];
    tr->rp_ent_ahead = med >= 32 ? 32 : (med >= 24 ? 24 : 16);
  }
  tr->info.rp_slots = nseg;
  tr->info.rp_entries = ebase;
  tr->info.rp_seg_rows = srow_ok ? 1 : 0;
  tr->rp_ok = true;
  return GOFD_OK;
}

// device time of the build's stages: events recorded at each kernel's start and end
struct BuildTimer {
  hipEvent_t ev[8][2] = {};
  bool ok = true;
  BuildTimer() {
    for (auto& p : ev)
      for (auto& e : p) ok = ok && hipEventCreate(&e) == hipSuccess;
  }
  ~BuildTimer() {
    for (auto& p : ev)
      for (auto& e : p)
        if (e) (void)hipEventDestroy(e);
  }
  void write(double* us) const {     // after the stream has been synchronised
    for (int k = 0; k < 8; ++k) {
      float ms = 0.0f;
      us[k] = ok && hipEventElapsedTime(&ms, ev[k][0], ev[k][1]) == hipSuccess ? ms * 1e3 : 0.0;
    }
  }
};

#define TR_LAUNCH(TM, K, KERNEL, GRID, BLOCK, STREAM, ...)                                              \
  do {                                                                                                  \
    if ((TM).ok)                                                                                        \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, (TM).ev[K][0], (TM).ev[K][1], 0, __VA_ARGS__); \
    else                                                                                                \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                                  \
  } while (0)

extern "C" int gofd_build_transfer(gofd_ctx ctx, int d, int64_t nv, const double* X_dev, int64_t ne,
                                   const int32_t* elems_dev, const gofd_grid* grid, gofd_transfer* out,
                                   gofd_transfer_info* info) {
  if (!ctx || !out || !grid || !X_dev || !elems_dev) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  if (d != 2 && d != 3) return gofd_fail(ctx, GOFD_E_ARG, "d must be 2 or 3");
  if (grid->d != d || grid->N < 1 || !(grid->R > 0)) return gofd_fail(ctx, GOFD_E_ARG, "bad grid");
  if (nv < d + 1 || ne < 1) return gofd_fail(ctx, GOFD_E_ARG, "empty mesh");
  const int W = 2 * grid->N + 1;
  int64_t n_nodes = 1;
  for (int a = 0; a < d; ++a) n_nodes *= W;
  if (n_nodes >= (int64_t)1 << 31) return gofd_fail(ctx, GOFD_E_ARG, "grid too large for 32-bit node numbers");
  if (n_nodes < nv)
    return gofd_fail(ctx, GOFD_E_RANK, "(2N+1)^d < N_v: I_h^FD cannot have full column rank");
  auto* tr = new (std::nothrow) gofd_transfer_s();
  if (!tr) return GOFD_E_OOM;
  std::unique_ptr<gofd_transfer_s> guard(tr);
  tr->ctx = ctx;
  tr->d = d;
  tr->N = grid->N;
  tr->W = W;
  tr->R = grid->R;
  tr->h = grid->R / (double)grid->N;
  for (int a = 0; a < 3; ++a) {
    tr->center[a] = a < d ? grid->center[a] : 0.0;
    tr->lo[a] = tr->center[a] - grid->R;
  }
  tr->nv = nv;
  tr->ne = ne;
  tr->n_nodes = n_nodes;
  hipStream_t st = ctx->stream;

  // host copies for topology (boundary facets) and heights
  tr->elems_host.resize(ne * (d + 1));
  tr->X_host.resize(nv * d);
  HIP_TRY(ctx, hipMemcpyAsync(tr->elems_host.data(), elems_dev, sizeof(int32_t) * ne * (d + 1),
                              hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->X_host.data(), X_dev, sizeof(double) * nv * d, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  for (int64_t i = 0; i < ne * (d + 1); ++i)
    if (tr->elems_host[i] < 0 || tr->elems_host[i] >= nv)
      return gofd_fail(ctx, GOFD_E_ARG, "element vertex id out of range");
  for (int64_t i = 0; i < nv * d; ++i)
    if (!std::isfinite(tr->X_host[i])) return gofd_fail(ctx, GOFD_E_ARG, "non-finite vertex coordinate");

  GOFD_TRY(dev_reserve(ctx, tr->X, sizeof(double) * nv * d));
  GOFD_TRY(dev_reserve(ctx, tr->elems, sizeof(int32_t) * ne * (d + 1)));
  GOFD_TRY(dev_reserve(ctx, tr->elem, sizeof(int32_t) * n_nodes));
  HIP_TRY(ctx, hipMemcpyAsync(tr->X.p, X_dev, sizeof(double) * nv * d, hipMemcpyDeviceToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(tr->elems.p, elems_dev, sizeof(int32_t) * ne * (d + 1), hipMemcpyDeviceToDevice, st));

  GridGeom g = make_geom(tr);
  BuildTimer tm;
  GOFD_TRY(dev_reserve(ctx, tr->rec, (d == 2 ? sizeof(ElemRec2) : sizeof(ElemRec3)) * ne));
  if (d == 2)
    TR_LAUNCH(tm, GOFD_TR_K_RECORDS, k_make_records<2>, dim3(grid1(ne, 256)), dim3(256), st, tr->X.as<double>(),
              tr->elems.as<int>(), (long long)ne, tr->rec.as<ElemRec2>());
  else
    TR_LAUNCH(tm, GOFD_TR_K_RECORDS, k_make_records<3>, dim3(grid1(ne, 256)), dim3(256), st, tr->X.as<double>(),
              tr->elems.as<int>(), (long long)ne, tr->rec.as<ElemRec3>());
  unsigned long long* counters = ctx->scratch.as<unsigned long long>();
  HIP_TRY(ctx, hipMemsetAsync(counters, 0, 8 * sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_fill_i32, dim3(grid1(n_nodes, 256)), dim3(256), 0, st, tr->elem.as<int>(), n_nodes, NO_ELEM);
  if (d == 2)
    TR_LAUNCH(tm, GOFD_TR_K_LOCATE, k_locate<2>, dim3(grid1(ne, 256)), dim3(256), st, g, tr->X.as<double>(),
              tr->elems.as<int>(), (long long)ne, tr->elem.as<int>(), counters);
  else
    TR_LAUNCH(tm, GOFD_TR_K_LOCATE, k_locate<3>, dim3(grid1(ne, 256)), dim3(256), st, g, tr->X.as<double>(),
              tr->elems.as<int>(), (long long)ne, tr->elem.as<int>(), counters);
  hipLaunchKernelGGL(k_finish_location, dim3(grid1(n_nodes, 256)), dim3(256), 0, st, tr->elem.as<int>(),
                     n_nodes, counters);
  HIP_TRY(ctx, hipGetLastError());
  unsigned long long hc[4];
  HIP_TRY(ctx, hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (hc[1]) return gofd_fail(ctx, GOFD_E_DEGENERATE, "mesh has an element of zero volume");
  if (hc[2]) return gofd_fail(ctx, GOFD_E_NUMERIC, "exact orientation exceeded its expansion capacity");
  const int64_t n_inside = (int64_t)hc[3];
  const int64_t nnz = n_inside * (d + 1);
  tr->nnz = nnz;

  // boundary (host topology)
  boundary_mask(d, nv, tr->elems_host, tr->bmask_host);
  GOFD_TRY(dev_reserve(ctx, tr->bmask, nv));
  HIP_TRY(ctx, hipMemcpyAsync(tr->bmask.p, tr->bmask_host.data(), nv, hipMemcpyHostToDevice, st));

  // CSC: counts, offsets, fill, per-segment sort, column sums
  DevBuf cnt, cursor, node_tmp, w_tmp;
  GOFD_TRY(dev_reserve(ctx, cnt, sizeof(int32_t) * (nv + 1)));
  GOFD_TRY(dev_reserve(ctx, cursor, sizeof(int32_t) * (nv + 1)));
  GOFD_TRY(dev_reserve(ctx, tr->csc_off, sizeof(int32_t) * (nv + 1)));
  GOFD_TRY(dev_reserve(ctx, tr->csc_node, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
  GOFD_TRY(dev_reserve(ctx, tr->csc_w, sizeof(double) * std::max<int64_t>(nnz, 1)));
  GOFD_TRY(dev_reserve(ctx, tr->csc_w32, sizeof(float) * std::max<int64_t>(nnz, 1)));
  GOFD_TRY(dev_reserve(ctx, node_tmp, sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
  GOFD_TRY(dev_reserve(ctx, w_tmp, sizeof(double) * std::max<int64_t>(nnz, 1)));
  if (nnz == 0) {
    // one zero entry (node 0, weight 0): kernels read entry 0 in place of a
    // missing one and weight it by zero
    HIP_TRY(ctx, hipMemsetAsync(tr->csc_node.p, 0, sizeof(int32_t), st));
    HIP_TRY(ctx, hipMemsetAsync(tr->csc_w.p, 0, sizeof(double), st));
    HIP_TRY(ctx, hipMemsetAsync(tr->csc_w32.p, 0, sizeof(float), st));
  }
  HIP_TRY(ctx, hipMemsetAsync(cnt.p, 0, sizeof(int32_t) * (nv + 1), st));
  if (d == 2)
    TR_LAUNCH(tm, GOFD_TR_K_COUNT, k_count<2>, dim3(grid1(n_nodes, 256)), dim3(256), st, tr->elem.as<int>(),
              tr->elems.as<int>(), n_nodes, cnt.as<int>());
  else
    TR_LAUNCH(tm, GOFD_TR_K_COUNT, k_count<3>, dim3(grid1(n_nodes, 256)), dim3(256), st, tr->elem.as<int>(),
              tr->elems.as<int>(), n_nodes, cnt.as<int>());
  GOFD_TRY(scan_prepare(ctx, nv));
  if (tm.ok) HIP_TRY(ctx, hipEventRecord(tm.ev[GOFD_TR_K_SCAN][0], st));
  GOFD_TRY(scan_exclusive_i32(ctx, cnt.as<int32_t>(), tr->csc_off.as<int32_t>(), nv));
  if (tm.ok) HIP_TRY(ctx, hipEventRecord(tm.ev[GOFD_TR_K_SCAN][1], st));
  HIP_TRY(ctx, hipMemcpyAsync(cursor.p, tr->csc_off.p, sizeof(int32_t) * (nv + 1), hipMemcpyDeviceToDevice, st));
  if (d == 2)
    TR_LAUNCH(tm, GOFD_TR_K_FILL, k_fill_csc<2>, dim3(grid1(n_nodes, 256)), dim3(256), st, g,
              tr->rec.as<ElemRec2>(), tr->elem.as<int>(), n_nodes, cursor.as<int>(), node_tmp.as<int>(),
              w_tmp.as<double>());
  else
    TR_LAUNCH(tm, GOFD_TR_K_FILL, k_fill_csc<3>, dim3(grid1(n_nodes, 256)), dim3(256), st, g,
              tr->rec.as<ElemRec3>(), tr->elem.as<int>(), n_nodes, cursor.as<int>(), node_tmp.as<int>(),
              w_tmp.as<double>());
  TR_LAUNCH(tm, GOFD_TR_K_SORT, k_sort_segments, dim3(grid1(nv * 64, 256)), dim3(256), st, tr->csc_off.as<int>(),
            (long long)nv, node_tmp.as<int>(), w_tmp.as<double>(), tr->csc_node.as<int>(), tr->csc_w.as<double>());
  if (d == 3) {
    // compact interpolation rows for the gather: in 3D the nodes of an element
    // lie in different planes, so per-node rows stream better than records
    GOFD_TRY(dev_reserve(ctx, tr->ell_idx, sizeof(int32_t) * (n_nodes + 1)));
    GOFD_TRY(dev_reserve(ctx, tr->ell_v, sizeof(int32_t) * 4 * std::max<int64_t>(n_inside, 1)));
    GOFD_TRY(dev_reserve(ctx, tr->ell_w, sizeof(double) * 4 * std::max<int64_t>(n_inside, 1)));
    if (n_inside == 0) {
      // one zero row (vertex 0, weights 0), read in place of a missing one
      HIP_TRY(ctx, hipMemsetAsync(tr->ell_v.p, 0, sizeof(int32_t) * 4, st));
      HIP_TRY(ctx, hipMemsetAsync(tr->ell_w.p, 0, sizeof(double) * 4, st));
    }
    DevBuf flag;
    GOFD_TRY(dev_reserve(ctx, flag, sizeof(int32_t) * (n_nodes + 1)));
    hipLaunchKernelGGL(k_inside_flag, dim3(grid1(n_nodes, 256)), dim3(256), 0, st, tr->elem.as<int>(),
                       (long long)n_nodes, flag.as<int>());
    GOFD_TRY(scan_exclusive_i32(ctx, flag.as<int32_t>(), tr->ell_idx.as<int32_t>(), n_nodes));
    TR_LAUNCH(tm, GOFD_TR_K_ROWS, k_fill_ell<3>, dim3(grid1(n_nodes, 256)), dim3(256), st, g,
              tr->rec.as<ElemRec3>(), tr->elem.as<int>(), (long long)n_nodes, tr->ell_idx.as<int>(),
              tr->ell_v.as<int>(), tr->ell_w.as<double>());
    HIP_TRY(ctx, hipStreamSynchronize(st));
  }
  if (d == 2) {
    GOFD_TRY(dev_reserve(ctx, tr->row32_v, sizeof(int4) * n_nodes));
    GOFD_TRY(dev_reserve(ctx, tr->row32_w, sizeof(float2) * n_nodes));
    TR_LAUNCH(tm, GOFD_TR_K_ROWS, k_fill_rows32, dim3(grid1(n_nodes, 256)), dim3(256), st, g,
              tr->rec.as<ElemRec2>(), tr->elem.as<int>(), (long long)n_nodes, tr->row32_v.as<int4>(),
              tr->row32_w.as<float2>());
  }
  GOFD_TRY(dev_reserve(ctx, tr->D, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, tr->dscale, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, tr->dsqrt, sizeof(double) * nv));
  GOFD_TRY(dev_reserve(ctx, tr->imask, sizeof(double) * nv));
  TR_LAUNCH(tm, GOFD_TR_K_COLSUM, k_colsum, dim3(grid1(nv, 256)), dim3(256), st, tr->csc_off.as<int>(),
            (long long)nv, tr->csc_w.as<double>(), tr->bmask.as<unsigned char>(), tr->D.as<double>(),
            tr->dscale.as<double>(), tr->dsqrt.as<double>(), tr->imask.as<double>(), tr->csc_w32.as<float>(),
            (long long)nnz);
  HIP_TRY(ctx, hipGetLastError());

  // statistics and checks on the host
  std::vector<double> Dh(nv);
  std::vector<int32_t> offh(nv + 1);
  HIP_TRY(ctx, hipMemcpyAsync(Dh.data(), tr->D.p, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipMemcpyAsync(offh.data(), tr->csc_off.p, sizeof(int32_t) * (nv + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  gofd_transfer_info inf{};
  inf.n_nodes = n_nodes;
  inf.n_inside = n_inside;
  inf.nnz = nnz;
  inf.exact_tests = (int64_t)hc[0];
  double dmin = INFINITY;
  int64_t nb = 0, maxc = 0;
  for (int64_t j = 0; j < nv; ++j) {
    maxc = std::max<int64_t>(maxc, offh[j + 1] - offh[j]);
    if (tr->bmask_host[j]) {
      ++nb;
    } else {
      dmin = std::min(dmin, Dh[j]);
    }
  }
  inf.n_boundary = nb;
  inf.n_interior = nv - nb;
  inf.dmin_interior = dmin;
  inf.max_col_count = maxc;
  inf.a_h = min_height(d, tr->X_host, tr->elems_host);
  inf.h_bound = inf.a_h / ((d + 1) * std::sqrt((double)d));
  tm.write(inf.kernel_us);     // the stream was synchronised above
  tr->info = inf;
  if (info) *info = inf;
  if (inf.n_interior > 0 && !(dmin > 0.0))
    return gofd_fail(ctx, GOFD_E_ZERO_COLSUM, "an interior vertex has zero column sum D_j (grid too coarse)");
  GOFD_TRY(build_rowpairs(ctx, tr, offh));
  if (info) *info = tr->info;
  *out = guard.release();
  return GOFD_OK;
}

extern "C" int gofd_transfer_free(gofd_transfer tr) {
  if (!tr) return GOFD_E_ARG;
  (void)hipDeviceSynchronize();   // the creating context may already be gone
  delete tr;
  return GOFD_OK;
}

extern "C" int gofd_transfer_export(gofd_ctx ctx, gofd_transfer tr, int part, void* dst) {
  if (!ctx || !tr || !dst) return gofd_fail(ctx, GOFD_E_ARG, "null argument");
  hipStream_t st = ctx->stream;
  const int d = tr->d;
  GridGeom g = make_geom(tr);
  switch (part) {
    case GOFD_TR_ELEM:
      HIP_TRY(ctx, hipMemcpyAsync(dst, tr->elem.p, sizeof(int32_t) * tr->n_nodes, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD_TR_ELL_VERTS:
    case GOFD_TR_ELL_WEIGHTS: {
      int* vv = part == GOFD_TR_ELL_VERTS ? static_cast<int*>(dst) : nullptr;
      double* ww = part == GOFD_TR_ELL_WEIGHTS ? static_cast<double*>(dst) : nullptr;
      if (d == 2)
        hipLaunchKernelGGL(k_export_ell<2>, dim3(grid1(tr->n_nodes, 256)), dim3(256), 0, st, g,
                           tr->rec.as<ElemRec2>(), tr->elem.as<int>(), (long long)tr->n_nodes, vv, ww);
      else
        hipLaunchKernelGGL(k_export_ell<3>, dim3(grid1(tr->n_nodes, 256)), dim3(256), 0, st, g,
                           tr->rec.as<ElemRec3>(), tr->elem.as<int>(), (long long)tr->n_nodes, vv, ww);
      break;
    }
    case GOFD_TR_CSC_OFFSETS:
      HIP_TRY(ctx, hipMemcpyAsync(dst, tr->csc_off.p, sizeof(int32_t) * (tr->nv + 1), hipMemcpyDeviceToDevice, st));
      break;
    case GOFD_TR_CSC_NODES:
      HIP_TRY(ctx, hipMemcpyAsync(dst, tr->csc_node.p, sizeof(int32_t) * tr->nnz, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD_TR_CSC_WEIGHTS:
      HIP_TRY(ctx, hipMemcpyAsync(dst, tr->csc_w.p, sizeof(double) * tr->nnz, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD_TR_D:
      HIP_TRY(ctx, hipMemcpyAsync(dst, tr->D.p, sizeof(double) * tr->nv, hipMemcpyDeviceToDevice, st));
      break;
    case GOFD_TR_BOUNDARY:
      HIP_TRY(ctx, hipMemcpyAsync(dst, tr->bmask.p, tr->nv, hipMemcpyDeviceToDevice, st));
      break;
    default:
      return gofd_fail(ctx, GOFD_E_ARG, "unknown transfer part");
  }
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

// ---------------------------------------------------------------- K8: I^T scatter
//
// z_j = scale_j * mask_j * sum_{k in column j} w_kj y_k.  A group of G lanes
// owns one vertex; lanes stride through the column (ascending node order) and
// the partial sums are combined with cross-lane shuffles, always in the same
// order, so the result is deterministic.
template <typename Y, typename WT, int G>
__global__ __launch_bounds__(256) void k_scatter(const int* __restrict__ off, const int* __restrict__ node,
                                                 const WT* __restrict__ w, const Y* __restrict__ y,
                                                 long long nv, long long n_nodes, int nrhs,
                                                 const double* __restrict__ scale, const double* __restrict__ mask,
                                                 double* __restrict__ z) {
  const long long gid = (long long)xcd_remap(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const long long v = gid / G;
  const int lane = threadIdx.x % G;
  const int rhs = blockIdx.y;
  if (v >= nv) return;
  const int b = off[v], e = off[v + 1];
  const Y* yr = y + (long long)rhs * n_nodes;
  double acc = 0.0;
  for (int i = b + lane; i < e; i += G) acc += (double)w[i] * (double)yr[node[i]];
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, G);
  if (lane == 0) {
    double r = acc;
    if (scale) r *= scale[v];
    if (mask) r *= mask[v];
    z[(long long)rhs * nv + v] = r;
  }
}

int scatter_apply(gofd_ctx_s* ctx, const gofd_transfer_s* tr, int nrhs, const void* y, bool fp32,
                  const double* scale, const double* mask, double* z) {
  constexpr int G = 16;
  dim3 grid(grid1(tr->nv * G, 256), nrhs);
  if (fp32)
    hipLaunchKernelGGL((k_scatter<float, float, G>), grid, dim3(256), 0, ctx->stream, tr->csc_off.as<int>(),
                       tr->csc_node.as<int>(), tr->csc_w32.as<float>(), static_cast<const float*>(y),
                       (long long)tr->nv, (long long)tr->n_nodes, nrhs, scale, mask, z);
  else
    hipLaunchKernelGGL((k_scatter<double, double, G>), grid, dim3(256), 0, ctx->stream, tr->csc_off.as<int>(),
                       tr->csc_node.as<int>(), tr->csc_w.as<double>(), static_cast<const double*>(y),
                       (long long)tr->nv, (long long)tr->n_nodes, nrhs, scale, mask, z);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}
