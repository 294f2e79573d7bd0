// Exact orientation signs on the device.
//
// orient(q_0..q_d) = det[q_1 - q_0, ..., q_d - q_0].  A double-precision
// evaluation decides whenever its magnitude clears a generous rounding bound;
// otherwise the determinant is expanded into exact products of the raw
// coordinates and summed exactly with floating-point expansions (Shewchuk,
// "Adaptive precision floating-point arithmetic and fast robust geometric
// predicates", 1997: Two-Sum, Two-Product via FMA, Grow-Expansion with zero
// elimination).  The sign of a nonoverlapping expansion is the sign of its
// largest component.  Contraction into fused multiply-adds is switched off in
// every function: a product fused into the following sum is no longer the
// rounded product that Two-Product's error term refers to.
#pragma once

#include <hip/hip_runtime.h>

namespace gofd_exact {

// x + y == a + b exactly, x = fl(a + b)
__device__ __forceinline__ void two_sum(double a, double b, double& x, double& y) {
#pragma clang fp contract(off)
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}

// x + y == a * b exactly, x = fl(a * b)
__device__ __forceinline__ void two_prod(double a, double b, double& x, double& y) {
#pragma clang fp contract(off)
  x = a * b;
  y = __builtin_fma(a, b, -x);
}

// Add b to the nonoverlapping expansion e[0..len) (increasing magnitude), in
// place, dropping zero components.  Returns the new length, or -1 on overflow.
template <int CAP>
__device__ __forceinline__ int grow(double* e, int len, double b) {
#pragma clang fp contract(off)
  double q = b;
  int out = 0;
  for (int i = 0; i < len; ++i) {
    double qn, h;
    two_sum(q, e[i], qn, h);
    q = qn;
    if (h != 0.0) e[out++] = h;
  }
  if (q != 0.0 || out == 0) {
    if (out >= CAP) return -1;
    e[out++] = q;
  }
  return out;
}

template <int CAP>
__device__ __forceinline__ int expansion_sign(const double* e, int len) {
#pragma clang fp contract(off)
  for (int i = len - 1; i >= 0; --i) {
    if (e[i] > 0.0) return 1;
    if (e[i] < 0.0) return -1;
  }
  return 0;
}

// exact sign of det[b - a, c - a] in 2D; returns 2 on capacity overflow
__device__ __noinline__ int orient2_exact(const double* a, const double* b, const double* c) {
#pragma clang fp contract(off)
  constexpr int CAP = 40;
  double e[CAP];
  int len = 0;
  double u0, u1, v0, v1, p0, p1, q0, q1;
  two_sum(b[0], -a[0], u0, u1);   // b_x - a_x = u0 + u1
  two_sum(c[1], -a[1], v0, v1);   // c_y - a_y
  two_sum(b[1], -a[1], p0, p1);   // b_y - a_y
  two_sum(c[0], -a[0], q0, q1);   // c_x - a_x
  const double us[2] = {u0, u1}, vs[2] = {v0, v1}, ps[2] = {p0, p1}, qs[2] = {q0, q1};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double x, y;
      two_prod(us[i], vs[j], x, y);
      len = grow<CAP>(e, len, x);
      if (len < 0) return 2;
      len = grow<CAP>(e, len, y);
      if (len < 0) return 2;
      two_prod(ps[i], qs[j], x, y);
      len = grow<CAP>(e, len, -x);
      if (len < 0) return 2;
      len = grow<CAP>(e, len, -y);
      if (len < 0) return 2;
    }
  return expansion_sign<CAP>(e, len);
}

// exact sign of det[b - a, c - a, d - a] in 3D; returns 2 on overflow
__device__ __noinline__ int orient3_exact(const double* a, const double* b, const double* c,
                                          const double* d) {
#pragma clang fp contract(off)
  constexpr int CAP = 96;
  double e[CAP];
  int len = 0;
  double M[3][3][2];   // rows: b-a, c-a, d-a; each entry a 2-term expansion
  const double* rows[3] = {b, c, d};
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) two_sum(rows[r][k], -a[k], M[r][k][0], M[r][k][1]);
  // det = sum over permutations (k0,k1,k2) of sign * M[0][k0] M[1][k1] M[2][k2]
  const int perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {2, 1, 0}, {1, 0, 2}};
  for (int pi = 0; pi < 6; ++pi) {
    const double sg = pi < 3 ? 1.0 : -1.0;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k) {
          double x, y;
          two_prod(M[0][perm[pi][0]][i], M[1][perm[pi][1]][j], x, y);
          const double w = M[2][perm[pi][2]][k];
          double t[4];
          two_prod(x, w, t[0], t[1]);
          two_prod(y, w, t[2], t[3]);
          for (int q = 0; q < 4; ++q) {
            len = grow<CAP>(e, len, sg * t[q]);
            if (len < 0) return 2;
          }
        }
  }
  return expansion_sign<CAP>(e, len);
}

// filtered sign of orient in 2D; *exact_used set when the exact path ran
__device__ __forceinline__ int orient2_sign(const double* a, const double* b, const double* c,
                                            int* exact_used) {
#pragma clang fp contract(off)
  const double ux = b[0] - a[0], uy = b[1] - a[1];
  const double vx = c[0] - a[0], vy = c[1] - a[1];
  const double t1 = ux * vy, t2 = uy * vx;
  const double det = t1 - t2;
  double sc = fmax(fmax(fabs(a[0]), fabs(a[1])), fmax(fmax(fabs(b[0]), fabs(b[1])), fmax(fabs(c[0]), fabs(c[1]))));
  const double bound = 1e-13 * (fabs(t1) + fabs(t2) + sc * sc);
  if (det > bound) return 1;
  if (det < -bound) return -1;
  *exact_used = 1;
  return orient2_exact(a, b, c);
}

__device__ __forceinline__ int orient3_sign(const double* a, const double* b, const double* c,
                                            const double* d, int* exact_used) {
#pragma clang fp contract(off)
  const double e00 = b[0] - a[0], e01 = b[1] - a[1], e02 = b[2] - a[2];
  const double e10 = c[0] - a[0], e11 = c[1] - a[1], e12 = c[2] - a[2];
  const double e20 = d[0] - a[0], e21 = d[1] - a[1], e22 = d[2] - a[2];
  const double m0 = e11 * e22 - e12 * e21;
  const double m1 = e10 * e22 - e12 * e20;
  const double m2 = e10 * e21 - e11 * e20;
  const double det = e00 * m0 - e01 * m1 + e02 * m2;
  const double pm0 = fabs(e11 * e22) + fabs(e12 * e21);
  const double pm1 = fabs(e10 * e22) + fabs(e12 * e20);
  const double pm2 = fabs(e10 * e21) + fabs(e11 * e20);
  double sc = 0.0;
  for (int k = 0; k < 3; ++k)
    sc = fmax(sc, fmax(fmax(fabs(a[k]), fabs(b[k])), fmax(fabs(c[k]), fabs(d[k]))));
  const double bound = 1e-13 * (fabs(e00) * pm0 + fabs(e01) * pm1 + fabs(e02) * pm2 + sc * sc * sc);
  if (det > bound) return 1;
  if (det < -bound) return -1;
  *exact_used = 1;
  return orient3_exact(a, b, c, d);
}

}  // namespace gofd_exact
