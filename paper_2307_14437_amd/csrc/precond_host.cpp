// Host construction of the sparse preconditioner of Section 3.3:
//   A_FD^(p): the entries of A_FD on the 5/9/27-point pattern,
//   A_h^(p) = I^T A_FD^(p) I restricted to the interior vertices (eq. Ah-4),
//   incomplete Cholesky with level-1 fill.
// The factor is assembled over all N_v vertices in the mesh's numbering, with
// identity rows for Dirichlet vertices (their unknowns are fixed at zero).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <queue>
#include <vector>

#include "precond_host.h"

namespace {

struct Pattern {
  std::vector<int> off[3];   // offsets per axis
  int n = 0;
};

Pattern stencil(int d, int npts) {
  Pattern p;
  auto add = [&](int a, int b, int c) {
    p.off[0].push_back(a);
    p.off[1].push_back(b);
    p.off[2].push_back(c);
    ++p.n;
  };
  if (d == 2 && npts == 5) {
    add(0, 0, 0); add(1, 0, 0); add(-1, 0, 0); add(0, 1, 0); add(0, -1, 0);
  } else if (d == 2 && npts == 9) {
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a) add(a, b, 0);
  } else if (d == 3 && npts == 27) {
    for (int c = -1; c <= 1; ++c)
      for (int b = -1; b <= 1; ++b)
        for (int a = -1; a <= 1; ++a) add(a, b, c);
  }
  return p;
}

}  // namespace

// A = I_J^T A^(p) I_J as CSR over all vertices (Dirichlet rows/cols dropped).
// T holds the stencil values by |offset| in the octant layout with row length
// Wt (axis 0 fastest): the table of A_FD (Wt = W), or a 2^d table.
bool assemble_pattern_matrix(const HostTransfer& t, const double* T, int64_t Wt, int npts, HostCsr& A) {
  const int d = t.d, W = t.W;
  Pattern pat = stencil(d, npts);
  if (pat.n == 0) return false;
  const int64_t nv = t.nv;
  const int d1 = d + 1;
  A.n = nv;
  A.rowptr.assign(nv + 1, 0);
  A.col.clear();
  A.val.clear();
  std::vector<double> acc(nv, 0.0);
  std::vector<int32_t> touched;
  std::vector<char> mark(nv, 0);
  for (int64_t j = 0; j < nv; ++j) {
    touched.clear();
    if (!t.bnd[j]) {
      for (int32_t e = t.csc_off[j]; e < t.csc_off[j + 1]; ++e) {
        const int64_t k = t.csc_node[e];
        const double lkj = t.csc_w[e];
        int64_t ik[3] = {k % W, (k / W) % W, d == 3 ? k / ((int64_t)W * W) : 0};
        for (int q = 0; q < pat.n; ++q) {
          int64_t jk[3];
          bool ok = true;
          for (int a = 0; a < d; ++a) {
            jk[a] = ik[a] + pat.off[a][q];
            ok = ok && jk[a] >= 0 && jk[a] < W;
          }
          if (!ok) continue;
          const int64_t k2 = jk[0] + (int64_t)W * jk[1] + (d == 3 ? (int64_t)W * W * jk[2] : 0);
          const int32_t e2 = t.elem[k2];
          if (e2 < 0) continue;
          // T at |offset| (octant layout, axis 0 fastest)
          int64_t ti = std::abs(pat.off[0][q]) + Wt * std::abs(pat.off[1][q]);
          if (d == 3) ti += Wt * Wt * std::abs(pat.off[2][q]);
          const double tv = T[ti];
          for (int r = 0; r < d1; ++r) {
            const int32_t j2 = t.elems[(int64_t)e2 * d1 + r];
            if (t.bnd[j2]) continue;
            const double w2 = t.node_w[k2 * d1 + r];
            if (!mark[j2]) {
              mark[j2] = 1;
              touched.push_back(j2);
            }
            acc[j2] += lkj * tv * w2;
          }
        }
      }
    }
    if (t.bnd[j]) {
      touched.push_back((int32_t)j);   // identity row
      acc[j] = 1.0;
      mark[j] = 1;
    }
    std::sort(touched.begin(), touched.end());
    for (int32_t c : touched) {
      A.col.push_back(c);
      A.val.push_back(acc[c]);
      acc[c] = 0.0;
      mark[c] = 0;
    }
    A.rowptr[j + 1] = (int64_t)A.col.size();
  }
  return true;
}

// Lower-triangular level-of-fill <= level pattern (rows sorted, diagonal last).
void ic_symbolic(const HostCsr& A, int level, std::vector<int64_t>& Lptr, std::vector<int32_t>& Lcol) {
  const int64_t n = A.n;
  // upper parts of finished rows: columns > i with their levels
  std::vector<std::vector<std::pair<int32_t, int8_t>>> upper(n);
  Lptr.assign(n + 1, 0);
  Lcol.clear();
  std::vector<int8_t> lev(n, 127);
  std::vector<int32_t> cols;
  std::vector<int32_t> heap;
  for (int64_t i = 0; i < n; ++i) {
    cols.clear();
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
      const int32_t c = A.col[e];
      lev[c] = 0;
      cols.push_back(c);
    }
    if (lev[i] != 0) {
      lev[i] = 0;
      cols.push_back((int32_t)i);
    }
    // process k < i in increasing order, including fill discovered on the way
    heap.clear();
    for (int32_t c : cols)
      if (c < i) heap.push_back(c);
    std::make_heap(heap.begin(), heap.end(), std::greater<int32_t>());
    while (!heap.empty()) {
      std::pop_heap(heap.begin(), heap.end(), std::greater<int32_t>());
      const int32_t k = heap.back();
      heap.pop_back();
      const int lik = lev[k];
      if (lik > level) continue;
      for (auto& pr : upper[k]) {
        const int32_t j = pr.first;
        const int nl = lik + pr.second + 1;
        if (nl <= level && nl < lev[j]) {
          const bool fresh = lev[j] == 127;
          lev[j] = (int8_t)nl;
          if (fresh) {
            cols.push_back(j);
            if (j < i) {
              heap.push_back(j);
              std::push_heap(heap.begin(), heap.end(), std::greater<int32_t>());
            }
          }
        }
      }
    }
    std::sort(cols.begin(), cols.end());
    std::vector<std::pair<int32_t, int8_t>> up;
    for (int32_t c : cols) {
      if (lev[c] <= level) {
        if (c <= i) Lcol.push_back(c);
        if (c > i) up.push_back({c, lev[c]});
      }
      lev[c] = 127;
    }
    upper[i].swap(up);
    Lptr[i + 1] = (int64_t)Lcol.size();
  }
}

// Numeric IC on the pattern; false on a non-positive pivot.
bool ic_numeric(const HostCsr& A, double shift, const std::vector<int64_t>& Lptr, const std::vector<int32_t>& Lcol,
                std::vector<double>& Lval) {
  const int64_t n = A.n;
  Lval.assign(Lcol.size(), 0.0);
  std::vector<double> work(n, 0.0);   // row i of L under construction, by column
  std::vector<int64_t> diag_pos(n);
  for (int64_t i = 0; i < n; ++i) {
    // scatter a_i (lower part) into work on the pattern
    for (int64_t e = Lptr[i]; e < Lptr[i + 1]; ++e) work[Lcol[e]] = 0.0;
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
      const int32_t c = A.col[e];
      if (c <= i) work[c] = A.val[e] + (c == i ? shift * A.val[e] : 0.0);
    }
    // columns j < i in increasing order
    double diag_acc = 0.0;
    for (int64_t e = Lptr[i]; e < Lptr[i + 1]; ++e) {
      const int32_t j = Lcol[e];
      if (j == i) break;
      // L_ij = (a_ij - sum_{k<j} L_ik L_jk) / L_jj, using row j of L
      double s = work[j];
      for (int64_t f = Lptr[j]; f < Lptr[j + 1]; ++f) {
        const int32_t k = Lcol[f];
        if (k >= j) break;
        s -= work[k] * Lval[f];   // work[k] = L_ik for k < j (zero off the pattern)
      }
      const double lij = s / Lval[diag_pos[j]];
      work[j] = lij;
      Lval[e] = lij;
      diag_acc += lij * lij;
    }
    const int64_t de = Lptr[i + 1] - 1;
    const double piv = work[i] - diag_acc;
    if (!(piv > 0.0) || !std::isfinite(piv)) return false;
    Lval[de] = std::sqrt(piv);
    diag_pos[i] = de;
    for (int64_t e = Lptr[i]; e < Lptr[i + 1]; ++e) work[Lcol[e]] = 0.0;
  }
  return true;
}

int greedy_colouring(const HostCsr& A, std::vector<int32_t>& colour) {
  const int64_t n = A.n;
  colour.assign(n, -1);
  std::vector<int64_t> stamp(1, -1);    // stamp[c] == i: colour c is taken by a neighbour of i
  int ncol = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
      const int32_t c = colour[A.col[e]];
      if (c >= 0) stamp[c] = i;
    }
    int32_t c = 0;
    while (c < (int32_t)stamp.size() && stamp[c] == i) ++c;
    if (c == (int32_t)stamp.size()) stamp.push_back(-1);
    colour[i] = c;
    ncol = std::max(ncol, (int)c + 1);
  }
  return ncol;
}

int smallest_last_colouring(const HostCsr& A, std::vector<int32_t>& colour) {
  const int64_t n = A.n;
  std::vector<int32_t> deg(n, 0);
  for (int64_t v = 0; v < n; ++v)
    for (int64_t e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) deg[v] += A.col[e] != v;
  // least degree first, then the smallest index; entries made stale by a later decrease are skipped
  std::priority_queue<std::pair<int32_t, int32_t>, std::vector<std::pair<int32_t, int32_t>>, std::greater<>> heap;
  for (int64_t v = 0; v < n; ++v) heap.push({deg[v], (int32_t)v});
  std::vector<char> removed(n, 0);
  std::vector<int32_t> order;
  order.reserve(n);
  while (!heap.empty()) {
    const auto [d, v] = heap.top();
    heap.pop();
    if (removed[v] || d != deg[v]) continue;
    removed[v] = 1;
    order.push_back(v);
    for (int64_t e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) {
      const int32_t j = A.col[e];
      if (j != v && !removed[j]) heap.push({--deg[j], j});
    }
  }
  colour.assign(n, -1);
  std::vector<int64_t> stamp(1, -1);
  int ncol = 0;
  for (auto it = order.rbegin(); it != order.rend(); ++it) {
    const int32_t v = *it;
    for (int64_t e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) {
      const int32_t c = colour[A.col[e]];
      if (c >= 0) stamp[c] = v;
    }
    int32_t c = 0;
    while (c < (int32_t)stamp.size() && stamp[c] == v) ++c;
    if (c == (int32_t)stamp.size()) stamp.push_back(-1);
    colour[v] = c;
    ncol = std::max(ncol, (int)c + 1);
  }
  return ncol;
}

void permute_symmetric(const HostCsr& A, const std::vector<int32_t>& perm, HostCsr& B) {
  const int64_t n = A.n;
  std::vector<int32_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
  B.n = n;
  B.rowptr.assign(n + 1, 0);
  B.col.clear();
  B.val.clear();
  std::vector<std::pair<int32_t, double>> row;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t v = perm[i];
    row.clear();
    for (int64_t e = A.rowptr[v]; e < A.rowptr[v + 1]; ++e) row.push_back({inv[A.col[e]], A.val[e]});
    std::sort(row.begin(), row.end());
    for (auto& pr : row) {
      B.col.push_back(pr.first);
      B.val.push_back(pr.second);
    }
    B.rowptr[i + 1] = (int64_t)B.col.size();
  }
}

int grow_blocks(const HostCsr& A, int size, std::vector<int32_t>& blk) {
  const int64_t n = A.n;
  blk.assign(n, -1);
  std::vector<int32_t> queue;
  int nb = 0;
  for (int64_t v = 0; v < n; ++v) {
    if (blk[v] >= 0) continue;
    blk[v] = nb;
    queue.assign(1, (int32_t)v);
    size_t head = 0;
    int count = 1;
    while (head < queue.size() && count < size) {
      const int32_t u = queue[head++];
      for (int64_t e = A.rowptr[u]; e < A.rowptr[u + 1] && count < size; ++e) {
        const int32_t j = A.col[e];
        if (blk[j] < 0) {
          blk[j] = nb;
          queue.push_back(j);
          ++count;
        }
      }
    }
    ++nb;
  }
  return nb;
}

void block_graph(const HostCsr& A, const std::vector<int32_t>& blk, int nb, HostCsr& G) {
  std::vector<std::vector<int32_t>> adj(nb);
  for (int64_t i = 0; i < A.n; ++i)
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e)
      if (blk[A.col[e]] != blk[i]) adj[blk[i]].push_back(blk[A.col[e]]);
  G.n = nb;
  G.rowptr.assign(nb + 1, 0);
  G.col.clear();
  G.val.clear();
  for (int b = 0; b < nb; ++b) {
    auto& a = adj[b];
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    G.col.insert(G.col.end(), a.begin(), a.end());
    G.rowptr[b + 1] = (int64_t)G.col.size();
  }
  G.val.assign(G.col.size(), 1.0);
}

void drop_same_colour(const std::vector<int32_t>& colour, std::vector<int64_t>& Lptr, std::vector<int32_t>& Lcol,
                      const std::vector<int32_t>* group) {
  const int64_t n = (int64_t)Lptr.size() - 1;
  std::vector<int64_t> ptr(n + 1, 0);
  std::vector<int32_t> col;
  col.reserve(Lcol.size());
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = Lptr[i]; e < Lptr[i + 1]; ++e) {
      const int32_t j = Lcol[e];
      if (j == i || colour[j] != colour[i] || (group && (*group)[j] == (*group)[i])) col.push_back(j);
    }
    ptr[i + 1] = (int64_t)col.size();
  }
  Lptr.swap(ptr);
  Lcol.swap(col);
}

