// Grid-node coordinates and barycentric weights on the device.
//
// Both the gather (I u, inside the first FFT pass) and the construction of the
// transposed structure (I^T) evaluate the weights with these functions, so the
// two sides of the symmetric product I^T A I use bit-identical values.
// Floating-point contraction is switched off here: node coordinates must be
// rounded exactly like the interface describes, and the weights must not
// depend on how the surrounding kernel is optimised.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

struct GridGeom {
  int d;
  int W;
  double lo[3];   // c_a - R
  double h;       // R / N
};

// coordinate of node index i along axis a: lo_a + i*h, two separate roundings
__device__ __forceinline__ double node_coord(const GridGeom& g, int a, int i) {
#pragma clang fp contract(off)
  const double t = (double)i * g.h;
  return g.lo[a] + t;
}

// barycentric weights of point p in the simplex with vertex coordinates V
// (V[r*d + a]); lambda_r = orient(V with vertex r replaced by p) / orient(V)
__device__ __forceinline__ void bary2(const double* V, const double* p, double* lam) {
#pragma clang fp contract(off)
  const double ax = V[0], ay = V[1], bx = V[2], by = V[3], cx = V[4], cy = V[5];
  const double det = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
  const double l0 = (bx - p[0]) * (cy - p[1]) - (by - p[1]) * (cx - p[0]);
  const double l1 = (p[0] - ax) * (cy - ay) - (p[1] - ay) * (cx - ax);
  const double l2 = (bx - ax) * (p[1] - ay) - (by - ay) * (p[0] - ax);
  const double inv = 1.0 / det;
  lam[0] = l0 * inv;
  lam[1] = l1 * inv;
  lam[2] = l2 * inv;
}

__device__ __forceinline__ double det3(double a0, double a1, double a2, double b0, double b1, double b2,
                                       double c0, double c1, double c2) {
#pragma clang fp contract(off)
  return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

__device__ __forceinline__ void bary3(const double* V, const double* p, double* lam) {
#pragma clang fp contract(off)
  // orient3(q0,q1,q2,q3) = det[q1-q0, q2-q0, q3-q0]
  double Q[4][3];
  for (int r = 0; r < 4; ++r)
    for (int a = 0; a < 3; ++a) Q[r][a] = V[r * 3 + a];
  const double det = det3(Q[1][0] - Q[0][0], Q[1][1] - Q[0][1], Q[1][2] - Q[0][2],
                          Q[2][0] - Q[0][0], Q[2][1] - Q[0][1], Q[2][2] - Q[0][2],
                          Q[3][0] - Q[0][0], Q[3][1] - Q[0][1], Q[3][2] - Q[0][2]);
  const double inv = 1.0 / det;
  for (int r = 0; r < 4; ++r) {
    double S[4][3];
    for (int q = 0; q < 4; ++q)
      for (int a = 0; a < 3; ++a) S[q][a] = (q == r) ? p[a] : Q[q][a];
    const double dr = det3(S[1][0] - S[0][0], S[1][1] - S[0][1], S[1][2] - S[0][2],
                           S[2][0] - S[0][0], S[2][1] - S[0][1], S[2][2] - S[0][2],
                           S[3][0] - S[0][0], S[3][1] - S[0][1], S[3][2] - S[0][2]);
    lam[r] = dr * inv;
  }
}

// Per-element record of the affine barycentric map, built once per transfer:
// lambda_r(x) = g_r . (x - x_0) for r >= 1, lambda_0 = 1 - sum_{r>=1} lambda_r.
// Every kernel that needs the weight of a node evaluates it from the record of
// its element with the same function, so the two sides of I^T A I use
// bit-identical weights.
struct ElemRec2 {
  int v[4];        // vertex ids (v[3] unused)
  double x0[2];    // vertex 0
  double g[2][2];  // gradients of lambda_1, lambda_2
};
struct ElemRec3 {
  int v[4];
  double x0[3];
  double g[3][3];
  double pad;
};
template <int D>
using ElemRec = typename std::conditional<D == 2, ElemRec2, ElemRec3>::type;

template <int D>
__device__ __forceinline__ void make_record(const double* __restrict__ X, const int* __restrict__ elems, long long e,
                                            ElemRec<D>& rec) {
#pragma clang fp contract(off)
  double P[D + 1][D];
  for (int r = 0; r <= D; ++r) {
    rec.v[r] = elems[e * (D + 1) + r];
    for (int a = 0; a < D; ++a) P[r][a] = X[(long long)rec.v[r] * D + a];
  }
  for (int a = 0; a < D; ++a) rec.x0[a] = P[0][a];
  if constexpr (D == 2) {
    rec.v[3] = -1;
    const double ax = P[1][0] - P[0][0], ay = P[1][1] - P[0][1];
    const double bx = P[2][0] - P[0][0], by = P[2][1] - P[0][1];
    const double inv = 1.0 / (ax * by - ay * bx);
    rec.g[0][0] = by * inv;
    rec.g[0][1] = -bx * inv;
    rec.g[1][0] = -ay * inv;
    rec.g[1][1] = ax * inv;
  } else {
    // columns of M are the edge vectors x_r - x_0; rows of M^{-1} are the gradients
    double M[3][3];
    for (int r = 0; r < 3; ++r)
      for (int a = 0; a < 3; ++a) M[a][r] = P[r + 1][a] - P[0][a];
    const double c00 = M[1][1] * M[2][2] - M[1][2] * M[2][1];
    const double c01 = M[1][2] * M[2][0] - M[1][0] * M[2][2];
    const double c02 = M[1][0] * M[2][1] - M[1][1] * M[2][0];
    const double det = M[0][0] * c00 + M[0][1] * c01 + M[0][2] * c02;
    const double inv = 1.0 / det;
    rec.g[0][0] = c00 * inv;
    rec.g[1][0] = c01 * inv;
    rec.g[2][0] = c02 * inv;
    rec.g[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * inv;
    rec.g[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * inv;
    rec.g[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * inv;
    rec.g[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * inv;
    rec.g[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * inv;
    rec.g[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * inv;
    rec.pad = 0.0;
  }
}

// weights of the grid node with axis indices idx[0..D-1] from its element's record
template <int D>
__device__ __forceinline__ void rec_weights(const GridGeom& g, const ElemRec<D>& rec, const int* idx, int* vid,
                                            double* lam) {
#pragma clang fp contract(off)
  double dx[3];
  for (int a = 0; a < D; ++a) dx[a] = node_coord(g, a, idx[a]) - rec.x0[a];
  double s = 0.0;
  for (int r = 1; r <= D; ++r) {
    double l = 0.0;
    for (int a = 0; a < D; ++a) l += rec.g[r - 1][a] * dx[a];
    lam[r] = l;
    s += l;
  }
  lam[0] = 1.0 - s;
  for (int r = 0; r <= D; ++r) vid[r] = rec.v[r];
}

// weights of grid node k (linear number) from its element's record
template <int D>
__device__ __forceinline__ void node_weights(const GridGeom& g, const ElemRec<D>* __restrict__ recs, int e,
                                             long long k, int* vid, double* lam) {
  const ElemRec<D> rec = recs[e];
  int idx[3];
  long long rem = k;
  for (int a = 0; a < D; ++a) {
    idx[a] = (int)(rem % g.W);
    rem /= g.W;
  }
  rec_weights<D>(g, rec, idx, vid, lam);
}

// inverse of the (D+1)x(D+1) matrix E = [[x_0 .. x_D]; [1 .. 1]] by Gauss-Jordan
template <int D>
__device__ void inverse_E(const double* V, double* Ei) {
  constexpr int n = D + 1;
  double A[n][2 * n];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) A[i][j] = 0.0;
  for (int r = 0; r < n; ++r) {        // column r = vertex r
    for (int a = 0; a < D; ++a) A[a][r] = V[r * D + a];
    A[D][r] = 1.0;
  }
  for (int i = 0; i < n; ++i) A[i][n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int i = c + 1; i < n; ++i)
      if (fabs(A[i][c]) > fabs(A[piv][c])) piv = i;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) {
        const double t = A[c][j];
        A[c][j] = A[piv][j];
        A[piv][j] = t;
      }
    const double inv = 1.0 / A[c][c];
    for (int j = 0; j < 2 * n; ++j) A[c][j] *= inv;
    for (int i = 0; i < n; ++i) {
      if (i == c) continue;
      const double f = A[i][c];
      for (int j = 0; j < 2 * n; ++j) A[i][j] -= f * A[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ei[i * n + j] = A[i][n + j];
}
