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

// weights of grid node k (linear number) in element e; writes d+1 vertex ids
// and weights
template <int D>
__device__ __forceinline__ void node_weights(const GridGeom& g, const double* __restrict__ X,
                                             const int* __restrict__ elems, int e, long long k,
                                             int* vid, double* lam) {
  double p[3];
  long long rem = k;
  for (int a = 0; a < D; ++a) {
    const int i = (int)(rem % g.W);
    rem /= g.W;
    p[a] = node_coord(g, a, i);
  }
  double V[(D + 1) * D];
  for (int r = 0; r <= D; ++r) {
    vid[r] = elems[(long long)e * (D + 1) + r];
    for (int a = 0; a < D; ++a) V[r * D + a] = X[(long long)vid[r] * D + a];
  }
  if constexpr (D == 2)
    bary2(V, p, lam);
  else
    bary3(V, p, lam);
}
