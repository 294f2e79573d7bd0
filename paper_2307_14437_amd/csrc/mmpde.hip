// Mesh adaptation by the MMPDE moving mesh method (Section 4, Algorithm
// amGoFD), 2D, on the device.
//
//  - Hessian recovery: at every vertex the least-squares quadratic through
//    u_h at the vertices of its two-ring (monomials 1, dx, dy, dx^2/2, dx dy,
//    dy^2/2 in coordinates relative to the vertex, scaled by the patch
//    radius), solved through its 6 x 6 normal equations; H_K = mean of the
//    vertex Hessians of K.
//  - Metric of eq. MK-1 with |H| = sqrt(H^2) (closed-form 2 x 2 eigen
//    decomposition) at every vertex, alpha_h the root of sum_K |K| det(I +
//    |H_K|/alpha)^{1/3} = 2 |Omega| found by bisection in log(alpha) inside
//    one workgroup.  During a move the metric is the piecewise-linear
//    interpolant of the vertex metrics on the mesh the move started from,
//    and M_K its value at the current centroid of K, located by a walk
//    (across the edge opposite the most negative barycentric coordinate,
//    from where the centroid was at the last accepted step; beyond a
//    boundary edge the value is extrapolated).
//  - Energy of eq. I-h and its gradient by the chain rule: with E = [x1 - x0,
//    x2 - x0], V = det E, A = M^{-1}, B = E_ref^T E_ref (equilateral
//    reference triangle of unit area), C = E^{-T} B E^{-1}, t = tr(A C),
//    q = sqrt(det M): dV/dE = V E^{-T}, dt/dE = -2 E^{-T} B E^{-1} A E^{-T},
//    dq/dM = q A / 2, dt/dM = -A C A; the metric's variation adds
//    1/3 sum_c dG/dm_c grad m_c at each vertex of K.
//  - Moving mesh equations x-1: dx_i/dt = -sqrt(det M(x_i))/tau dI_h/dx_i,
//    M(x_i) the vertex metric of the starting mesh, boundary vertices
//    sliding on the unit circle or fixed.  The system is stiff, so it is
//    integrated by linearly implicit (Rosenbrock-Euler) steps
//        P (tau/h Q^{-1} + J) P dx = -P dI_h/dx,  Q = diag(sqrt(det M(x_i))),
//    P the projection onto the allowed motions, J the Hessian of I_h with
//    the current M_K held fixed, from element Hessians taken by central
//    differences of the element gradient (step 1e-5 times the longest edge,
//    symmetrised), solved by conjugate
//    gradients with the 2 x 2 vertex blocks as preconditioner; a trial step
//    is halved until the solve succeeds (the matrix is positive definite on
//    the Krylov space), no element inverts and I_h decreases, and the next
//    trial step is twice the accepted one (the same after a halving); the move ends at t_end, at rest
//    (small projected gradient), or once no step of at least 1e-6 times the
//    longest accepted one (and 1e-14) decreases I_h.
// Vertex sums over elements run in a fixed order (vertex -> element lists
// sorted by element), and every reduction over blocks in a fixed order, so
// every result is reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <memory>
#include <set>
#include <vector>

#include "internal.h"

struct gofd_mmpde_s {
  int64_t nv = 0, ne = 0;
  int boundary = GOFD_MMPDE_BOUNDARY_CIRCLE;
  DevBuf elems;       // int32[ne*3]
  DevBuf ring_off;    // int32[nv+1]: two-ring of every vertex (sorted, the vertex included)
  DevBuf ring;        // int32[...]
  DevBuf ve_off;      // int32[nv+1]: elements around every vertex (sorted)
  DevBuf ve;          // int32[...]: element * 3 + corner
  DevBuf bnd;         // uint8[nv]: vertex on an edge owned by one element
  DevBuf nbr;         // int32[ne*3]: element across the edge opposite each corner, -1 on the boundary
  DevBuf iwork;       // int32[2*ne]: centroid locations (accepted, trial)
  DevBuf work;        // scratch: vertex Hessians, element data, gradients, trial positions, partials
  size_t work_bytes = 0;
  double* hst = nullptr;       // page-locked copies of a step solve's state, one slot per chunk in flight
  hipEvent_t ev[2] = {};       // recorded after each chunk's copy
  ~gofd_mmpde_s() {
    if (hst) (void)hipHostFree(hst);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

constexpr int MB = 256;          // threads per block
constexpr int MNB = 256;         // blocks of the reductions (fixed: sums in a fixed order)

inline unsigned grid1(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// reference triangle: equilateral, unit area, side a with a^2 = 4/sqrt(3); B = E_ref^T E_ref
struct RefTri {
  double b11, b12, b22, det;
};
__host__ __device__ inline RefTri ref_tri() {
  const double a2 = 4.0 / sqrt(3.0);
  return RefTri{a2, 0.5 * a2, a2, 2.0};   // E_ref = a [[1, 1/2], [0, sqrt(3)/2]]: det = a^2 sqrt(3)/2 = 2
}

// symmetric 2 x 2 [[a, b], [b, c]]: |H| and its eigenvalues' magnitudes
__device__ inline void abs_sym2(double a, double b, double c, double* o, double* lam) {
  const double m = 0.5 * (a + c), r = sqrt(0.25 * (a - c) * (a - c) + b * b);
  const double l1 = m + r, l2 = m - r;
  lam[0] = fabs(l1);
  lam[1] = fabs(l2);
  if (r == 0.0) {                 // a multiple of the identity
    o[0] = fabs(l1);
    o[1] = 0.0;
    o[2] = fabs(l1);
    return;
  }
  // projector onto the eigenvector of l1: P1 = (H - l2 I) / (l1 - l2)
  const double p11 = (a - l2) / (l1 - l2), p12 = b / (l1 - l2), p22 = (c - l2) / (l1 - l2);
  // |H| = |l1| P1 + |l2| (I - P1)
  o[0] = lam[0] * p11 + lam[1] * (1.0 - p11);
  o[1] = (lam[0] - lam[1]) * p12;
  o[2] = lam[0] * p22 + lam[1] * (1.0 - p22);
}

// least-squares quadratic at vertex i over its two-ring: Hv[i] = (h11, h12, h22)
__global__ __launch_bounds__(MB) void k_vertex_hessian(const double* __restrict__ X, const int* __restrict__ roff,
                                                       const int* __restrict__ ring, const double* __restrict__ u,
                                                       long long nv, double* __restrict__ Hv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const double xi = X[2 * i], yi = X[2 * i + 1];
  double rho = 0.0;
  for (int q = roff[i]; q < roff[i + 1]; ++q) {
    const int j = ring[q];
    rho = fmax(rho, fmax(fabs(X[2 * j] - xi), fabs(X[2 * j + 1] - yi)));
  }
  if (rho == 0.0) rho = 1.0;
  double N[6][7] = {};
  for (int q = roff[i]; q < roff[i + 1]; ++q) {
    const int j = ring[q];
    const double dx = (X[2 * j] - xi) / rho, dy = (X[2 * j + 1] - yi) / rho;
    const double phi[6] = {1.0, dx, dy, 0.5 * dx * dx, dx * dy, 0.5 * dy * dy};
    const double uj = u[j];
    for (int a = 0; a < 6; ++a) {
      for (int b = 0; b < 6; ++b) N[a][b] += phi[a] * phi[b];
      N[a][6] += phi[a] * uj;
    }
  }
  // Gauss elimination with partial pivoting on the normal equations; a two-ring on which the
  // quadratics are not unisolvent (a vanishing pivot) gives a zero Hessian
  const double scale = (N[0][0] + N[1][1] + N[2][2] + N[3][3] + N[4][4] + N[5][5]) / 6.0;
  for (int c = 0; c < 6; ++c) {
    int piv = c;
    for (int r = c + 1; r < 6; ++r)
      if (fabs(N[r][c]) > fabs(N[piv][c])) piv = r;
    if (piv != c)
      for (int k = 0; k < 7; ++k) {
        const double t = N[c][k];
        N[c][k] = N[piv][k];
        N[piv][k] = t;
      }
    if (!(fabs(N[c][c]) > 1e-13 * scale)) {
      Hv[3 * i] = Hv[3 * i + 1] = Hv[3 * i + 2] = 0.0;
      return;
    }
    for (int r = c + 1; r < 6; ++r) {
      const double f = N[r][c] / N[c][c];
      for (int k = c; k < 7; ++k) N[r][k] -= f * N[c][k];
    }
  }
  double cf[6];
  for (int r = 5; r >= 0; --r) {
    double s = N[r][6];
    for (int k = r + 1; k < 6; ++k) s -= N[r][k] * cf[k];
    cf[r] = s / N[r][r];
  }
  const double r2 = rho * rho;
  Hv[3 * i] = cf[3] / r2;
  Hv[3 * i + 1] = cf[4] / r2;
  Hv[3 * i + 2] = cf[5] / r2;
}

// per element: |H_K| (3 values), its eigenvalue magnitudes (2) and area
__global__ void k_element_absH(const double* __restrict__ X, const int* __restrict__ el, const double* __restrict__ Hv,
                               long long ne, double* __restrict__ aH, double* __restrict__ lam,
                               double* __restrict__ area) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  const int v0 = el[3 * k], v1 = el[3 * k + 1], v2 = el[3 * k + 2];
  double h[3];
  for (int a = 0; a < 3; ++a) h[a] = (Hv[3 * v0 + a] + Hv[3 * v1 + a] + Hv[3 * v2 + a]) / 3.0;
  double o[3], l[2];
  abs_sym2(h[0], h[1], h[2], o, l);
  for (int a = 0; a < 3; ++a) aH[3 * k + a] = o[a];
  lam[2 * k] = l[0];
  lam[2 * k + 1] = l[1];
  const double e1x = X[2 * v1] - X[2 * v0], e1y = X[2 * v1 + 1] - X[2 * v0 + 1];
  const double e2x = X[2 * v2] - X[2 * v0], e2y = X[2 * v2 + 1] - X[2 * v0 + 1];
  area[k] = 0.5 * (e1x * e2y - e1y * e2x);
}

// sum over elements of area * ((1 + l1/alpha)(1 + l2/alpha))^{1/3}, by one block in a fixed order
__device__ double alpha_sum(const double* lam, const double* area, long long ne, double alpha, double* sh) {
  double v[1] = {0.0};
  for (long long k = threadIdx.x; k < ne; k += 1024)
    v[0] += area[k] * cbrt((1.0 + lam[2 * k] / alpha) * (1.0 + lam[2 * k + 1] / alpha));
  gofd_cg::block_sum_n<1024, 1>(v, sh);
  return v[0];
}

// alpha_h by bisection in log(alpha), the same search as the oracle's; +inf when every |H_K| vanishes
__global__ __launch_bounds__(1024) void k_alpha(const double* __restrict__ lam, const double* __restrict__ area,
                                                long long ne, double* __restrict__ out) {
  __shared__ double sh[1024 / 64];
  double v[2] = {0.0, 0.0};
  for (long long k = threadIdx.x; k < ne; k += 1024) {
    v[0] += area[k];
    v[1] = fmax(v[1], fmax(lam[2 * k], lam[2 * k + 1]));
  }
  double s[1] = {v[0]};
  gofd_cg::block_sum_n<1024, 1>(s, sh);
  const double omega = s[0];
  if (!(omega > 0.0)) {            // an inverted or empty mesh: no metric
    if (threadIdx.x == 0) out[0] = NAN;
    return;
  }
  // max over the block (every lane ends with the same value)
  double mx = v[1];
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __shared__ double shm[1024 / 64];
  if ((threadIdx.x & 63) == 0) shm[threadIdx.x / 64] = mx;
  __syncthreads();
  mx = 0.0;
  for (int w = 0; w < 1024 / 64; ++w) mx = fmax(mx, shm[w]);
  __syncthreads();
  if (!(mx > 0.0)) {
    if (threadIdx.x == 0) out[0] = HUGE_VAL;
    return;
  }
  auto f = [&](double a) { return alpha_sum(lam, area, ne, a, sh) - 2.0 * omega; };
  double hi = 1.0;
  while (f(hi) > 0) hi *= 2.0;
  double lo = hi / 2.0;
  while (f(lo) <= 0) lo /= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = sqrt(lo * hi);
    if (f(mid) > 0) lo = mid;
    else hi = mid;
    if (hi / lo - 1.0 < 1e-15) break;
  }
  if (threadIdx.x == 0) out[0] = sqrt(lo * hi);
}

// vertex metric M_i = det(B)^{-1/6} B, B = I + |H_i| / alpha (the identity for alpha = inf); (m11, m12, m22)
__global__ void k_vertex_metric(const double* __restrict__ Hv, const double* __restrict__ alpha, long long nv,
                                double* __restrict__ M) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  const double al = alpha[0];
  if (!isfinite(al)) {
    M[3 * i] = 1.0;
    M[3 * i + 1] = 0.0;
    M[3 * i + 2] = 1.0;
    return;
  }
  double o[3], l[2];
  abs_sym2(Hv[3 * i], Hv[3 * i + 1], Hv[3 * i + 2], o, l);
  const double b11 = 1.0 + o[0] / al, b12 = o[1] / al, b22 = 1.0 + o[2] / al;
  const double s = pow(b11 * b22 - b12 * b12, -1.0 / 6.0);
  M[3 * i] = s * b11;
  M[3 * i + 1] = s * b12;
  M[3 * i + 2] = s * b22;
}

// ---------------------------------------------------------------- the metric field

// gradient of each component of the linear interpolant on background element k: GM[6k + 2c + (x, y)]
__global__ void k_field_grad(const double* __restrict__ Xb, const int* __restrict__ el, const double* __restrict__ Mv,
                             long long ne, double* __restrict__ GM) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  const int v0 = el[3 * k], v1 = el[3 * k + 1], v2 = el[3 * k + 2];
  const double t11 = Xb[2 * v1] - Xb[2 * v0], t12 = Xb[2 * v2] - Xb[2 * v0];
  const double t21 = Xb[2 * v1 + 1] - Xb[2 * v0 + 1], t22 = Xb[2 * v2 + 1] - Xb[2 * v0 + 1];
  const double det = t11 * t22 - t12 * t21;
  for (int c = 0; c < 3; ++c) {
    // grad^T T = (f1 - f0, f2 - f0)
    const double d1 = Mv[3 * v1 + c] - Mv[3 * v0 + c], d2 = Mv[3 * v2 + c] - Mv[3 * v0 + c];
    GM[6 * k + 2 * c] = (d1 * t22 - d2 * t21) / det;
    GM[6 * k + 2 * c + 1] = (d2 * t11 - d1 * t12) / det;
  }
}

__global__ void k_iota(int* __restrict__ a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = (int)i;
}

// barycentric coordinates of (x, y) in background element k
__device__ inline void bary(const double* Xb, const int* el, int k, double x, double y, double* lam) {
  const int v0 = el[3 * k], v1 = el[3 * k + 1], v2 = el[3 * k + 2];
  const double t11 = Xb[2 * v1] - Xb[2 * v0], t12 = Xb[2 * v2] - Xb[2 * v0];
  const double t21 = Xb[2 * v1 + 1] - Xb[2 * v0 + 1], t22 = Xb[2 * v2 + 1] - Xb[2 * v0 + 1];
  const double bx = x - Xb[2 * v0], by = y - Xb[2 * v0 + 1];
  const double det = t11 * t22 - t12 * t21;
  lam[1] = (t22 * bx - t12 * by) / det;
  lam[2] = (t11 * by - t21 * bx) / det;
  lam[0] = 1.0 - lam[1] - lam[2];
}

constexpr int WALK_MAX = 4096;   // moves of one walk at most (then the value is taken where it stopped)

// M_K and the component gradients at the centroid of every element of X, walking from loc_in
__global__ void k_field_eval(const double* __restrict__ X, const int* __restrict__ el, const double* __restrict__ Xb,
                             const int* __restrict__ nbr, const double* __restrict__ Mv,
                             const double* __restrict__ GMb, const int* __restrict__ loc_in, long long ne,
                             int* __restrict__ loc_out, double* __restrict__ MK, double* __restrict__ GK) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  const int v0 = el[3 * k], v1 = el[3 * k + 1], v2 = el[3 * k + 2];
  const double cx = (X[2 * v0] + X[2 * v1] + X[2 * v2]) / 3.0;
  const double cy = (X[2 * v0 + 1] + X[2 * v1 + 1] + X[2 * v2 + 1]) / 3.0;
  int kb = loc_in[k];
  double lam[3];
  for (int mv = 0; mv < WALK_MAX; ++mv) {
    bary(Xb, el, kb, cx, cy, lam);
    int a = 0;
    if (lam[1] < lam[a]) a = 1;
    if (lam[2] < lam[a]) a = 2;
    if (lam[a] >= 0.0) break;
    const int nb = nbr[3 * kb + a];
    if (nb < 0) break;
    kb = nb;
  }
  loc_out[k] = kb;
  const int w0 = el[3 * kb], w1 = el[3 * kb + 1], w2 = el[3 * kb + 2];
  for (int c = 0; c < 3; ++c) MK[3 * k + c] = lam[0] * Mv[3 * w0 + c] + lam[1] * Mv[3 * w1 + c] + lam[2] * Mv[3 * w2 + c];
  for (int c = 0; c < 6; ++c) GK[6 * k + c] = GMb[6 * kb + c];
}

__global__ void k_sqrtdet(const double* __restrict__ Mv, long long nv, double* __restrict__ qv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  qv[i] = sqrt(Mv[3 * i] * Mv[3 * i + 2] - Mv[3 * i + 1] * Mv[3 * i + 1]);
}

// energy term of one element and its gradient with respect to the six coordinates of its vertices,
// P = (x0, y0, x1, y1, x2, y2), metric (m11, m12, m22); g in the order of P
__device__ inline double elem_energy_grad(const double* P, double m11, double m12, double m22, double* g) {
  const RefTri R = ref_tri();
  const double e11 = P[2] - P[0], e21 = P[3] - P[1];   // column 1: x1 - x0
  const double e12 = P[4] - P[0], e22 = P[5] - P[1];   // column 2: x2 - x0
  const double V = e11 * e22 - e12 * e21;
  // E^{-1}
  const double i11 = e22 / V, i12 = -e12 / V, i21 = -e21 / V, i22 = e11 / V;
  const double dm = m11 * m22 - m12 * m12;
  const double q = sqrt(dm);
  const double a11 = m22 / dm, a12 = -m12 / dm, a22 = m11 / dm;          // A = M^{-1}
  // X1 = E^{-1} A E^{-T}
  const double t11 = i11 * a11 + i12 * a12, t12 = i11 * a12 + i12 * a22;
  const double t21 = i21 * a11 + i22 * a12, t22 = i21 * a12 + i22 * a22;
  const double x11 = t11 * i11 + t12 * i12, x12 = t11 * i21 + t12 * i22;
  const double x21 = t21 * i11 + t22 * i12, x22 = t21 * i21 + t22 * i22;
  const double t = x11 * R.b11 + x12 * R.b12 + x21 * R.b12 + x22 * R.b22;   // tr(X1 B)
  const double p = 1.5;
  const double tp = pow(t, p);
  // dV = V E^{-T}; dt = -2 E^{-T} B X1
  const double dV11 = V * i11, dV12 = V * i21, dV21 = V * i12, dV22 = V * i22;
  // Y = B X1
  const double y11 = R.b11 * x11 + R.b12 * x21, y12 = R.b11 * x12 + R.b12 * x22;
  const double y21 = R.b12 * x11 + R.b22 * x21, y22 = R.b12 * x12 + R.b22 * x22;
  const double dt11 = -2.0 * (i11 * y11 + i21 * y21), dt12 = -2.0 * (i11 * y12 + i21 * y22);
  const double dt21 = -2.0 * (i12 * y11 + i22 * y21), dt22 = -2.0 * (i12 * y12 + i22 * y22);
  const double fac = 0.5 * q;
  const double c1 = fac / 3.0 * tp, c2 = fac / 3.0 * V * p * pow(t, p - 1.0);
  const double d2p = pow(2.0, p);
  const double c3 = d2p / 3.0 * fac * pow(q / R.det, -p) * (1.0 - p) * pow(V, -p);
  const double g11 = (c1 + c3) * dV11 + c2 * dt11, g12 = (c1 + c3) * dV12 + c2 * dt12;
  const double g21 = (c1 + c3) * dV21 + c2 * dt21, g22 = (c1 + c3) * dV22 + c2 * dt22;
  // column j of dG/dE -> vertex j (1, 2); vertex 0 takes minus their sum
  g[2] = g11;
  g[3] = g21;
  g[4] = g12;
  g[5] = g22;
  g[0] = -(g11 + g12);
  g[1] = -(g21 + g22);
  const double area = 0.5 * V;
  return q * area * tp / 3.0 + d2p / 3.0 * q * area * pow(q * V / R.det, -p);
}

__device__ inline void load_elem(const double* X, const int* el, long long k, double* P) {
  for (int a = 0; a < 3; ++a) {
    const int v = el[3 * k + a];
    P[2 * a] = X[2 * v];
    P[2 * a + 1] = X[2 * v + 1];
  }
}

// dG/dm_c for the components (m11, m12, m22) of the element's metric (m12 for both off-diagonal entries)
__device__ inline void elem_metric_deriv(const double* P, double m11, double m12, double m22, double* dm) {
  const RefTri R = ref_tri();
  const double e11 = P[2] - P[0], e21 = P[3] - P[1];
  const double e12 = P[4] - P[0], e22 = P[5] - P[1];
  const double V = e11 * e22 - e12 * e21;
  const double i11 = e22 / V, i12 = -e12 / V, i21 = -e21 / V, i22 = e11 / V;
  // C = E^{-T} B E^{-1}: first BE = B E^{-1}, then E^{-T} BE
  const double f11 = R.b11 * i11 + R.b12 * i21, f12 = R.b11 * i12 + R.b12 * i22;
  const double f21 = R.b12 * i11 + R.b22 * i21, f22 = R.b12 * i12 + R.b22 * i22;
  const double c11 = i11 * f11 + i21 * f21, c12 = i11 * f12 + i21 * f22, c22 = i12 * f12 + i22 * f22;
  const double dmt = m11 * m22 - m12 * m12;
  const double q = sqrt(dmt);
  const double a11 = m22 / dmt, a12 = -m12 / dmt, a22 = m11 / dmt;
  const double t = a11 * c11 + 2.0 * a12 * c12 + a22 * c22;      // tr(A C), both symmetric
  const double p = 1.5;
  const double area = 0.5 * V;
  const double dG_dq = area * pow(t, p) / 3.0 + pow(2.0, p) / 3.0 * area * (1.0 - p) * pow(q, -p) * pow(V / R.det, -p);
  const double dG_dt = q * area * p * pow(t, p - 1.0) / 3.0;
  // A C A
  const double u11 = a11 * c11 + a12 * c12, u12 = a11 * c12 + a12 * c22;
  const double u21 = a12 * c11 + a22 * c12, u22 = a12 * c12 + a22 * c22;
  const double w11 = u11 * a11 + u12 * a12, w12 = u11 * a12 + u12 * a22, w22 = u21 * a12 + u22 * a22;
  dm[0] = dG_dq * 0.5 * q * a11 - dG_dt * w11;
  dm[1] = dG_dq * q * a12 - dG_dt * 2.0 * w12;
  dm[2] = dG_dq * 0.5 * q * a22 - dG_dt * w22;
}

// element gradients with the metric M_K at the centroid; with GK, the metric's variation (grad m_c of the
// background element holding the centroid) adds 1/3 sum_c dG/dm_c grad m_c at each vertex
__global__ void k_elem_grad(const double* __restrict__ X, const int* __restrict__ el, const double* __restrict__ M,
                            const double* __restrict__ GK, long long ne, double* __restrict__ G) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  double P[6], g[6];
  load_elem(X, el, k, P);
  (void)elem_energy_grad(P, M[3 * k], M[3 * k + 1], M[3 * k + 2], g);
  if (GK) {
    double dm[3];
    elem_metric_deriv(P, M[3 * k], M[3 * k + 1], M[3 * k + 2], dm);
    double ex = 0.0, ey = 0.0;
    for (int c = 0; c < 3; ++c) {
      ex += dm[c] * GK[6 * k + 2 * c];
      ey += dm[c] * GK[6 * k + 2 * c + 1];
    }
    ex /= 3.0;
    ey /= 3.0;
    for (int a = 0; a < 3; ++a) {
      g[2 * a] += ex;
      g[2 * a + 1] += ey;
    }
  }
  for (int a = 0; a < 6; ++a) G[6 * k + a] = g[a];
}

// element Hessians (6 x 6, row-major, symmetrised) by central differences of the element gradient with
// the step 1e-5 times the element's longest edge
__global__ __launch_bounds__(MB) void k_elem_hess_fd(const double* __restrict__ X, const int* __restrict__ el,
                                                     const double* __restrict__ M, long long ne,
                                                     double* __restrict__ Hk) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  double P[6];
  load_elem(X, el, k, P);
  double L = 0.0;
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3;
    const double dx = P[2 * a] - P[2 * b], dy = P[2 * a + 1] - P[2 * b + 1];
    L = fmax(L, sqrt(dx * dx + dy * dy));
  }
  const double eps = 1e-5 * L;
  const double m11 = M[3 * k], m12 = M[3 * k + 1], m22 = M[3 * k + 2];
  double H[36];
  for (int c = 0; c < 6; ++c) {
    double Q[6], gp[6], gm[6];
    for (int a = 0; a < 6; ++a) Q[a] = P[a];
    Q[c] = P[c] + eps;
    (void)elem_energy_grad(Q, m11, m12, m22, gp);
    Q[c] = P[c] - eps;
    (void)elem_energy_grad(Q, m11, m12, m22, gm);
    for (int r = 0; r < 6; ++r) H[6 * r + c] = (gp[r] - gm[r]) / (2.0 * eps);
  }
  for (int r = 0; r < 6; ++r)
    for (int c = 0; c < 6; ++c) Hk[36 * k + 6 * r + c] = 0.5 * (H[6 * r + c] + H[6 * c + r]);
}

// partials of (energy, inverted) over elements: a non-positive area counts as an inverted element
__global__ __launch_bounds__(MB) void k_energy_check(const double* __restrict__ X, const int* __restrict__ el,
                                                     const double* __restrict__ M, long long ne,
                                                     double* __restrict__ part) {
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 1>()];
  __shared__ int bad_sh;
  if (threadIdx.x == 0) bad_sh = 0;
  __syncthreads();
  double e[1] = {0.0};
  int bad = 0;
  for (long long k = (long long)blockIdx.x * MB + threadIdx.x; k < ne; k += (long long)gridDim.x * MB) {
    double P[6], g[6];
    load_elem(X, el, k, P);
    const double V = (P[2] - P[0]) * (P[5] - P[1]) - (P[4] - P[0]) * (P[3] - P[1]);
    if (!(V > 0.0)) {
      bad = 1;
      continue;
    }
    e[0] += elem_energy_grad(P, M[3 * k], M[3 * k + 1], M[3 * k + 2], g);
  }
  if (bad) atomicOr(&bad_sh, 1);
  gofd_cg::block_sum_n<MB, 1>(e, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = e[0];
    part[gridDim.x + blockIdx.x] = bad_sh ? 1.0 : 0.0;
  }
}

// out = (sum of part[0..nb), max of part[nb..2 nb)) by one block in a fixed order
__global__ __launch_bounds__(MB) void k_finish2(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 1>()];
  __shared__ double shb[MB];
  double e[1] = {0.0};
  double bad = 0.0;
  for (int b = threadIdx.x; b < nb; b += MB) {
    e[0] += part[b];
    bad = fmax(bad, part[nb + b]);
  }
  gofd_cg::block_sum_n<MB, 1>(e, sh);
  shb[threadIdx.x] = bad;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int t = 0; t < MB; ++t) b = fmax(b, shb[t]);
    out[0] = e[0];
    out[1] = b;
  }
}

// sum over the elements around vertex i of their 6-vectors' entries at corner i
__device__ inline void gather2(const int* voff, const int* ve, const double* Z, long long i, double& gx, double& gy) {
  gx = 0.0;
  gy = 0.0;
  for (int q = voff[i]; q < voff[i + 1]; ++q) {
    const int kc = ve[q];
    gx += Z[2 * kc];
    gy += Z[2 * kc + 1];
  }
}

// projection onto the allowed motions of vertex i (mode < 0: none)
__device__ inline void project(int mode, uint8_t b, double x, double y, double& vx, double& vy) {
  if (mode < 0 || !b) return;
  if (mode == GOFD_MMPDE_BOUNDARY_CIRCLE) {
    const double r = sqrt(x * x + y * y);
    const double tx = -y / r, ty = x / r;
    const double s = tx * vx + ty * vy;
    vx = s * tx;
    vy = s * ty;
  } else {
    vx = vy = 0.0;
  }
}

// partial block sums of NQ values per thread, stored as part[q * gridDim.x + block]
template <int NQ>
__device__ inline void store_partials(double* v, double* sh, double* part) {
  gofd_cg::block_sum_n<MB, NQ>(v, sh);
  if (threadIdx.x == 0)
    for (int q = 0; q < NQ; ++q) part[q * gridDim.x + blockIdx.x] = v[q];
}

// sum of the nb partials part[0..nb) (nb <= MB), the same bits in every block
__device__ inline double sum_partials(const double* part, int nb, double* sh) {
  double v[1] = {threadIdx.x < nb ? part[threadIdx.x] : 0.0};
  gofd_cg::block_sum_n<MB, 1>(v, sh);
  return v[0];
}

// (projected) gradient at the vertices; partial sums of its squared norm when part is given
__global__ __launch_bounds__(MB) void k_grad_vert(const int* __restrict__ voff, const int* __restrict__ ve,
                                                  const double* __restrict__ G, const uint8_t* __restrict__ bnd,
                                                  const double* __restrict__ X, long long nv, int mode,
                                                  double* __restrict__ out, double* __restrict__ part) {
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 2>()];
  double v[2] = {0.0, 0.0};      // squared norm, and a zero for the max slot of k_finish2
  for (long long i = (long long)blockIdx.x * MB + threadIdx.x; i < nv; i += (long long)gridDim.x * MB) {
    double gx, gy;
    gather2(voff, ve, G, i, gx, gy);
    project(mode, bnd[i], X[2 * i], X[2 * i + 1], gx, gy);
    out[2 * i] = gx;
    out[2 * i + 1] = gy;
    v[0] += gx * gx + gy * gy;
  }
  if (part) store_partials<2>(v, sh, part);
}

// diagonal 2 x 2 blocks of J at the vertices: (j11, j12, j22)
__global__ void k_hess_diag(const int* __restrict__ voff, const int* __restrict__ ve, const double* __restrict__ Hk,
                            long long nv, double* __restrict__ Jd) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int q = voff[i]; q < voff[i + 1]; ++q) {
    const int k = ve[q] / 3, cn = ve[q] % 3;
    const double* H = Hk + 36 * (long long)k;
    a += H[6 * (2 * cn) + 2 * cn];
    b += H[6 * (2 * cn) + 2 * cn + 1];
    c += H[6 * (2 * cn + 1) + 2 * cn + 1];
  }
  Jd[3 * i] = a;
  Jd[3 * i + 1] = b;
  Jd[3 * i + 2] = c;
}

// ---------------------------------------------------------------- conjugate gradients on the step system
// state: st[0] 0 running / 1 converged / 2 failed, st[1] tol^2 (r0, r0), st[2] iterations

// true when the solve has ended; read once per block (block 0 of the kernel may set the flag while other
// blocks run), so that a block either runs or leaves as a whole
__device__ inline bool stopped(const double* st) {
  __shared__ int flag;
  if (threadIdx.x == 0) flag = st[0] != 0.0;
  __syncthreads();
  const bool r = flag != 0;
  __syncthreads();
  return r;
}

struct StepSys {
  const uint8_t* bnd;
  const double* X;
  const double* Jd;
  const double* qv;
  double tau, h;
  int mode;
  long long nv;
};

// z = B_i^{-1} r on the allowed motions, B_i = Jd_i + tau / (h q_i) I; false if B_i is not positive there
__device__ inline bool precond(const StepSys& S, long long i, double rx, double ry, double& zx, double& zy) {
  const double c = S.tau / (S.h * S.qv[i]);
  const double b11 = S.Jd[3 * i] + c, b12 = S.Jd[3 * i + 1], b22 = S.Jd[3 * i + 2] + c;
  if (S.mode >= 0 && S.bnd[i]) {
    if (S.mode != GOFD_MMPDE_BOUNDARY_CIRCLE) {
      zx = zy = 0.0;
      return true;
    }
    const double x = S.X[2 * i], y = S.X[2 * i + 1];
    const double r = sqrt(x * x + y * y);
    const double tx = -y / r, ty = x / r;
    const double sb = tx * (b11 * tx + b12 * ty) + ty * (b12 * tx + b22 * ty);
    if (!(sb > 0.0)) return false;
    const double s = (tx * rx + ty * ry) / sb;
    zx = s * tx;
    zy = s * ty;
    return true;
  }
  const double det = b11 * b22 - b12 * b12;
  if (!(b11 > 0.0 && det > 0.0)) return false;
  zx = (b22 * rx - b12 * ry) / det;
  zy = (b11 * ry - b12 * rx) / det;
  return true;
}

// dx = 0, r = -P g, z = B^{-1} r, p = 0 (the first direction is z: see k_cg_elem); partials of (r, z),
// (r, r) and failure
__global__ __launch_bounds__(MB) void k_cg_init(StepSys S, const double* __restrict__ pg, double* __restrict__ dx,
                                                double* __restrict__ r, double* __restrict__ z,
                                                double* __restrict__ p, double* __restrict__ part) {
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 3>()];
  double v[3] = {0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * MB + threadIdx.x; i < S.nv; i += (long long)gridDim.x * MB) {
    const double rx = -pg[2 * i], ry = -pg[2 * i + 1];
    double zx = 0.0, zy = 0.0;
    if (!precond(S, i, rx, ry, zx, zy)) v[2] += 1.0;
    dx[2 * i] = dx[2 * i + 1] = 0.0;
    r[2 * i] = rx;
    r[2 * i + 1] = ry;
    z[2 * i] = zx;
    z[2 * i + 1] = zy;
    p[2 * i] = p[2 * i + 1] = 0.0;
    v[0] += rx * zx + ry * zy;
    v[1] += rx * rx + ry * ry;
  }
  store_partials<3>(v, sh, part);
}

// state from the initial partials; the partial slots of the iterations: pr[0] = (r, z) and (r, r) of the
// first iterate, pr[1] = the same (r, z), read as the previous one (so that the first beta is 1 and the first
// direction z + 1 * 0 = z)
__global__ __launch_bounds__(MB) void k_cg_start(const double* __restrict__ part, int nb, double tol,
                                                 double* __restrict__ st, double* __restrict__ pr0,
                                                 double* __restrict__ pr1) {
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 1>()];
  const double rr = sum_partials(part + nb, nb, sh);
  const double bad = sum_partials(part + 2 * nb, nb, sh);
  for (int b = threadIdx.x; b < 2 * nb; b += MB) pr0[b] = part[b];
  for (int b = threadIdx.x; b < nb; b += MB) pr1[b] = part[b];
  if (threadIdx.x == 0) {
    st[0] = bad > 0.0 ? 2.0 : (rr == 0.0 ? 1.0 : 0.0);
    st[1] = tol * tol * rr;
    st[2] = 0.0;
  }
}

// the new direction at one coordinate (the same code in both kernels that form it, so the same bits)
__device__ __forceinline__ double new_dir(double z, double beta, double p) { return z + beta * p; }

// beta = (r, z)_cur / (r, z)_prev from the partials, and the convergence test (r, r)_cur <= tol^2 (r0, r0)
__device__ inline bool cg_beta(const double* pcur, const double* pprev, int nb, const double* st, double* sh,
                               double& beta) {
  const double rz = sum_partials(pcur, nb, sh);
  const double rzp = sum_partials(pprev, nb, sh);
  const double rr = sum_partials(pcur + nb, nb, sh);
  beta = rz / rzp;
  return rr <= st[1];
}

// converged: flag set by block 0, every block leaves; else Z_K = H_K p_K, p = z + beta p_prev formed on the fly
__global__ __launch_bounds__(MB) void k_cg_elem(const int* __restrict__ el, const double* __restrict__ Hk,
                                                const double* __restrict__ z, const double* __restrict__ p,
                                                long long ne, const double* __restrict__ pcur,
                                                const double* __restrict__ pprev, int nb, double* __restrict__ st,
                                                double* __restrict__ Z) {
  if (stopped(st)) return;
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 1>()];
  double beta;
  const bool conv = cg_beta(pcur, pprev, nb, st, sh, beta);
  if (conv) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = 1.0;
    return;
  }
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  double zk[6], pk[6];
  load_elem(z, el, k, zk);
  load_elem(p, el, k, pk);
  for (int c = 0; c < 6; ++c) pk[c] = new_dir(zk[c], beta, pk[c]);
  const double* H = Hk + 36 * k;
  for (int r = 0; r < 6; ++r) {
    double s = 0.0;
    for (int c = 0; c < 6; ++c) s += H[6 * r + c] * pk[c];
    Z[6 * k + r] = s;
  }
}

// p = z + beta p_prev (stored); w = P (J p + tau / (h q) p); partials of (p, w)
__global__ __launch_bounds__(MB) void k_cg_vert(StepSys S, const int* __restrict__ voff, const int* __restrict__ ve,
                                                const double* __restrict__ Z, const double* __restrict__ z,
                                                double* __restrict__ p, const double* __restrict__ pcur,
                                                const double* __restrict__ pprev, int nb, double* __restrict__ st,
                                                double* __restrict__ w, double* __restrict__ part) {
  if (stopped(st)) return;
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 1>()];
  double beta;
  (void)cg_beta(pcur, pprev, nb, st, sh, beta);
  double v[1] = {0.0};
  for (long long i = (long long)blockIdx.x * MB + threadIdx.x; i < S.nv; i += (long long)gridDim.x * MB) {
    const double px = new_dir(z[2 * i], beta, p[2 * i]), py = new_dir(z[2 * i + 1], beta, p[2 * i + 1]);
    p[2 * i] = px;
    p[2 * i + 1] = py;
    double wx, wy;
    gather2(voff, ve, Z, i, wx, wy);
    const double c = S.tau / (S.h * S.qv[i]);
    wx += c * px;
    wy += c * py;
    project(S.mode, S.bnd[i], S.X[2 * i], S.X[2 * i + 1], wx, wy);
    w[2 * i] = wx;
    w[2 * i + 1] = wy;
    v[0] += px * wx + py * wy;
  }
  store_partials<1>(v, sh, part);
}

// alpha = (r, z) / (p, w); dx += alpha p, r -= alpha w, z = B^{-1} r; partials of the new (r, z) and (r, r);
// counts the iteration
__global__ __launch_bounds__(MB) void k_cg_update(StepSys S, const double* __restrict__ part_pw,
                                                  const double* __restrict__ part_rz, int nb, double* __restrict__ st,
                                                  double* __restrict__ dx, double* __restrict__ r,
                                                  double* __restrict__ z, const double* __restrict__ p,
                                                  const double* __restrict__ w, double* __restrict__ part_out) {
  if (stopped(st)) return;
  __shared__ double sh[gofd_cg::block_sum_lds<MB, 2>()];
  const double pw = sum_partials(part_pw, nb, sh);
  const double rz = sum_partials(part_rz, nb, sh);
  if (!(pw > 0.0) || !isfinite(rz)) {      // not positive definite on the Krylov space
    if (blockIdx.x == 0 && threadIdx.x == 0) st[0] = 2.0;
    return;
  }
  const double alpha = rz / pw;
  double v[2] = {0.0, 0.0};
  for (long long i = (long long)blockIdx.x * MB + threadIdx.x; i < S.nv; i += (long long)gridDim.x * MB) {
    dx[2 * i] += alpha * p[2 * i];
    dx[2 * i + 1] += alpha * p[2 * i + 1];
    const double rx = r[2 * i] - alpha * w[2 * i], ry = r[2 * i + 1] - alpha * w[2 * i + 1];
    r[2 * i] = rx;
    r[2 * i + 1] = ry;
    double zx = 0.0, zy = 0.0;
    (void)precond(S, i, rx, ry, zx, zy);    // positive: checked by k_cg_init for the same matrix
    z[2 * i] = zx;
    z[2 * i + 1] = zy;
    v[0] += rx * zx + ry * zy;
    v[1] += rx * rx + ry * ry;
  }
  store_partials<2>(v, sh, part_out);
  if (blockIdx.x == 0 && threadIdx.x == 0) st[2] += 1.0;
}

// Y = X + dx; boundary vertices put back on the unit circle
__global__ void k_place(const double* __restrict__ X, const double* __restrict__ dx, const uint8_t* __restrict__ bnd,
                        long long nv, int mode, double* __restrict__ Y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double x = X[2 * i] + dx[2 * i], y = X[2 * i + 1] + dx[2 * i + 1];
  if (bnd[i] && mode == GOFD_MMPDE_BOUNDARY_CIRCLE) {
    const double r = sqrt(x * x + y * y);
    x /= r;
    y /= r;
  }
  Y[2 * i] = x;
  Y[2 * i + 1] = y;
}

// kernel timing of a move: the first launches of each kernel record HIP events at their start and end
struct KTimer {
  static constexpr int SAMPLES = 32;
  bool on = false;
  hipEvent_t ev[GOFD_MMPDE_N_KERNELS][SAMPLES][2] = {};
  int used[GOFD_MMPDE_N_KERNELS] = {};
  long long launches[GOFD_MMPDE_N_KERNELS] = {};
  ~KTimer() {
    for (auto& k : ev)
      for (auto& smp : k)
        for (auto& e : smp)
          if (e) (void)hipEventDestroy(e);
  }
  // events for the next launch of kernel k, or false
  bool next(int k, hipEvent_t* a, hipEvent_t* b) {
    ++launches[k];
    if (!on || used[k] >= SAMPLES) return false;
    hipEvent_t* p = ev[k][used[k]];
    if (!p[0] && (hipEventCreate(&p[0]) != hipSuccess || hipEventCreate(&p[1]) != hipSuccess)) return false;
    *a = p[0];
    *b = p[1];
    ++used[k];
    return true;
  }
  void write(gofd_mmpde_kernel_stats* out) const {
    for (int k = 0; k < GOFD_MMPDE_N_KERNELS; ++k) {
      double sum = 0.0;
      int n = 0;
      for (int i = 0; i < used[k]; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[k][i][0], ev[k][i][1]) == hipSuccess) {
          sum += ms;
          ++n;
        }
      }
      out->avg_us[k] = n ? sum * 1e3 / n : 0.0;
      out->launches[k] = launches[k];
    }
  }
};

// launch, timed by the move's KTimer when it has events left for this kernel
#define MM_LAUNCH(T, K, KERNEL, GRID, BLOCK, STREAM, ...)                                          \
  do {                                                                                             \
    hipEvent_t ea_, eb_;                                                                           \
    if ((T) && (T)->next((K), &ea_, &eb_))                                                          \
      hipExtLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, ea_, eb_, 0, __VA_ARGS__);             \
    else                                                                                           \
      hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                             \
  } while (0)

// scratch (doubles): Hv 3nv | aH 3ne | lam 2ne | area ne | alpha 1 | G 6ne | Hk 36ne | Jd 3nv | qv nv |
// pg, dx, r, z, p, w, Y, Xb 2nv each | GMb 6ne | MK 2 x 3ne | GK 2 x 6ne | part 8 MNB | st 4 | out 2;
// ints: loc 2 x ne
struct Scratch {
  double *Hv, *aH, *lam, *area, *alpha, *G, *Hk, *Jd, *qv, *pg, *dx, *r, *z, *p, *w, *Y, *Xb, *GMb, *MK[2], *GK[2],
      *part, *st, *out;
  int* loc[2];
};
int scratch(gofd_ctx_s* ctx, gofd_mmpde_s* m, Scratch& s) {
  const long long nv = m->nv, ne = m->ne;
  const long long n = 3 * nv + 3 * ne + 2 * ne + ne + 1 + 6 * ne + 36 * ne + 3 * nv + nv + 16 * nv + 6 * ne +
                      6 * ne + 12 * ne + 8 * MNB + 4 + 2;
  GOFD_TRY(dev_reserve(ctx, m->work, sizeof(double) * n));
  GOFD_TRY(dev_reserve(ctx, m->iwork, sizeof(int) * 2 * ne));
  double* q = m->work.as<double>();
  auto take = [&](long long k) {
    double* r = q;
    q += k;
    return r;
  };
  s.Hv = take(3 * nv);
  s.aH = take(3 * ne);
  s.lam = take(2 * ne);
  s.area = take(ne);
  s.alpha = take(1);
  s.G = take(6 * ne);
  s.Hk = take(36 * ne);
  s.Jd = take(3 * nv);
  s.qv = take(nv);
  s.pg = take(2 * nv);
  s.dx = take(2 * nv);
  s.r = take(2 * nv);
  s.z = take(2 * nv);
  s.p = take(2 * nv);
  s.w = take(2 * nv);
  s.Y = take(2 * nv);
  s.Xb = take(2 * nv);
  s.GMb = take(6 * ne);
  s.MK[0] = take(3 * ne);
  s.MK[1] = take(3 * ne);
  s.GK[0] = take(6 * ne);
  s.GK[1] = take(6 * ne);
  s.part = take(8 * MNB);
  s.st = take(4);
  s.out = take(2);
  s.loc[0] = m->iwork.as<int>();
  s.loc[1] = s.loc[0] + ne;
  return GOFD_OK;
}

// blocks of the vertex reductions: a function of N_v only, so that the sums keep their order
inline int vertex_blocks(long long nv) { return (int)std::min<long long>(MNB, grid1(nv, MB)); }

int energy_check(gofd_ctx_s* ctx, gofd_mmpde_s* m, const double* X, const double* M, Scratch& s, double* host2,
                 KTimer* T = nullptr) {
  hipStream_t st = ctx->stream;
  MM_LAUNCH(T, GOFD_MMPDE_K_ENERGY, k_energy_check, dim3(MNB), dim3(MB), st, X, m->elems.as<int>(), M,
            (long long)m->ne, s.part);
  hipLaunchKernelGGL(k_finish2, dim3(1), dim3(MB), 0, st, s.part, MNB, s.out);
  HIP_TRY(ctx, hipMemcpyAsync(host2, s.out, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  return GOFD_OK;
}

// projected gradient at X into s.pg; returns its norm
int projected_gradient(gofd_ctx_s* ctx, gofd_mmpde_s* m, const double* X, const double* M, const double* GK,
                       Scratch& s, double* norm) {
  hipStream_t st = ctx->stream;
  const long long nv = m->nv, ne = m->ne;
  const int nb = vertex_blocks(nv);
  hipLaunchKernelGGL(k_elem_grad, dim3(grid1(ne, MB)), dim3(MB), 0, st, X, m->elems.as<int>(), M, GK, ne, s.G);
  hipLaunchKernelGGL(k_grad_vert, dim3(nb), dim3(MB), 0, st, m->ve_off.as<int>(), m->ve.as<int>(), s.G,
                     m->bnd.as<uint8_t>(), X, nv, m->boundary, s.pg, s.part);
  hipLaunchKernelGGL(k_finish2, dim3(1), dim3(MB), 0, st, s.part, nb, s.out);
  double o[2];
  HIP_TRY(ctx, hipMemcpyAsync(o, s.out, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  *norm = sqrt(o[0]);
  return GOFD_OK;
}

// conjugate gradients on the step system of length h (Hk, Jd, qv, pg ready); *ok = converged, *its added.
// Iterations go out in chunks of 8; each chunk ends with a copy of the state to a page-locked slot and an
// event, and the host reads a chunk's state while the next one runs (kernels of a chunk issued past the end
// return at once).
int step_solve(gofd_ctx_s* ctx, gofd_mmpde_s* m, const double* X, Scratch& s, double tau, double h, double tol,
               int max_cg, bool* ok, long long* its, KTimer* T) {
  hipStream_t st = ctx->stream;
  const long long nv = m->nv, ne = m->ne;
  const int nb = vertex_blocks(nv);
  StepSys S{m->bnd.as<uint8_t>(), X, s.Jd, s.qv, tau, h, m->boundary, nv};
  if (!m->hst) {
    HIP_TRY(ctx, hipHostMalloc((void**)&m->hst, 8 * sizeof(double), hipHostMallocDefault));
    for (auto& e : m->ev) HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  // partial slots: pr[j] = (r, z) then (r, r) of an iterate, ping-pong; (p, w); the initial three
  double* pr[2] = {s.part, s.part + 2 * MNB};
  double* ppw = s.part + 4 * MNB;
  double* pinit = s.part + 5 * MNB;
  hipLaunchKernelGGL(k_cg_init, dim3(nb), dim3(MB), 0, st, S, s.pg, s.dx, s.r, s.z, s.p, pinit);
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(MB), 0, st, pinit, nb, tol, s.st, pr[0], pr[1]);
  const int CH = 8;
  int it = 0, chunk = 0;
  double last[3] = {0.0, 0.0, 0.0};
  bool done = false;
  while (!done && it < max_cg) {
    for (int q = 0; q < CH && it < max_cg; ++q, ++it) {
      const int cur = it & 1;
      MM_LAUNCH(T, GOFD_MMPDE_K_CG_ELEM, k_cg_elem, dim3(grid1(ne, MB)), dim3(MB), st, m->elems.as<int>(), s.Hk,
                s.z, s.p, ne, pr[cur], pr[cur ^ 1], nb, s.st, s.G);
      MM_LAUNCH(T, GOFD_MMPDE_K_CG_VERT, k_cg_vert, dim3(nb), dim3(MB), st, S, m->ve_off.as<int>(),
                m->ve.as<int>(), s.G, s.z, s.p, pr[cur], pr[cur ^ 1], nb, s.st, s.w, ppw);
      MM_LAUNCH(T, GOFD_MMPDE_K_CG_UPDATE, k_cg_update, dim3(nb), dim3(MB), st, S, ppw, pr[cur], nb, s.st, s.dx,
                s.r, s.z, s.p, s.w, pr[cur ^ 1]);
    }
    double* slot = m->hst + 4 * (chunk & 1);
    HIP_TRY(ctx, hipMemcpyAsync(slot, s.st, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipEventRecord(m->ev[chunk & 1], st));
    if (chunk > 0) {          // the previous chunk's state, while this one runs
      HIP_TRY(ctx, hipEventSynchronize(m->ev[(chunk - 1) & 1]));
      const double* prev = m->hst + 4 * ((chunk - 1) & 1);
      if (prev[0] != 0.0) done = true;
    }
    ++chunk;
  }
  // the last chunk's state is final (nothing changes the state once it has ended)
  HIP_TRY(ctx, hipEventSynchronize(m->ev[(chunk - 1) & 1]));
  for (int k = 0; k < 3; ++k) last[k] = m->hst[4 * ((chunk - 1) & 1) + k];
  HIP_TRY(ctx, hipGetLastError());
  *ok = last[0] == 1.0;
  *its += (long long)last[2];
  return GOFD_OK;
}

// the metric field of (Xb, Mv): component gradients per background element
void field_setup(gofd_ctx_s* ctx, gofd_mmpde_s* m, const double* Xb, const double* Mv, Scratch& s) {
  hipLaunchKernelGGL(k_field_grad, dim3(grid1(m->ne, MB)), dim3(MB), 0, ctx->stream, Xb, m->elems.as<int>(), Mv,
                     (long long)m->ne, s.GMb);
}

// M_K, GK at the centroids of X into slot j, walking from loc_in
void field_eval(gofd_ctx_s* ctx, gofd_mmpde_s* m, const double* X, const double* Xb, const double* Mv,
                const int* loc_in, Scratch& s, int j, KTimer* T = nullptr) {
  MM_LAUNCH(T, GOFD_MMPDE_K_FIELD, k_field_eval, dim3(grid1(m->ne, MB)), dim3(MB), ctx->stream, X,
            m->elems.as<int>(), Xb, m->nbr.as<int>(), Mv, s.GMb, loc_in, (long long)m->ne, s.loc[j], s.MK[j],
            s.GK[j]);
}

}  // namespace

extern "C" int gofd_mmpde_create(gofd_ctx ctx, int64_t nv, int64_t ne, const int32_t* elems_dev, int boundary,
                                 gofd_mmpde* out) {
  if (!ctx || !elems_dev || !out || nv < 3 || ne < 1 ||
      (boundary != GOFD_MMPDE_BOUNDARY_CIRCLE && boundary != GOFD_MMPDE_BOUNDARY_FIXED))
    return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  auto m = std::unique_ptr<gofd_mmpde_s>(new (std::nothrow) gofd_mmpde_s());
  if (!m) return gofd_fail(ctx, GOFD_E_OOM, "mmpde handle");
  m->nv = nv;
  m->ne = ne;
  m->boundary = boundary;
  std::vector<int32_t> el(3 * ne);
  HIP_TRY(ctx, hipMemcpyAsync(el.data(), elems_dev, sizeof(int32_t) * 3 * ne, hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int32_t v : el)
    if (v < 0 || v >= nv) return gofd_fail(ctx, GOFD_E_ARG, "element vertex out of range");
  // neighbours, two-rings, vertex -> element corners, boundary edges
  std::vector<std::set<int32_t>> nb(nv);
  std::vector<std::vector<int32_t>> vel(nv);
  std::vector<std::pair<int32_t, int32_t>> edges;
  for (int64_t k = 0; k < ne; ++k)
    for (int a = 0; a < 3; ++a) {
      const int32_t v = el[3 * k + a];
      for (int b = 0; b < 3; ++b) nb[v].insert(el[3 * k + b]);
      vel[v].push_back((int32_t)(3 * k + a));
      const int32_t w = el[3 * k + (a + 1) % 3];
      edges.push_back({std::min(v, w), std::max(v, w)});
    }
  std::sort(edges.begin(), edges.end());
  // element neighbours across the edge opposite each corner
  std::vector<std::pair<std::pair<int32_t, int32_t>, int64_t>> half;   // (edge, 3 k + corner)
  half.reserve(3 * ne);
  for (int64_t k = 0; k < ne; ++k)
    for (int a = 0; a < 3; ++a) {
      const int32_t p = el[3 * k + (a + 1) % 3], q = el[3 * k + (a + 2) % 3];
      half.push_back({{std::min(p, q), std::max(p, q)}, 3 * k + a});
    }
  std::sort(half.begin(), half.end());
  std::vector<int32_t> nbr(3 * ne, -1);
  for (size_t e = 0; e + 1 < half.size(); ++e)
    if (half[e].first == half[e + 1].first) {
      nbr[half[e].second] = (int32_t)(half[e + 1].second / 3);
      nbr[half[e + 1].second] = (int32_t)(half[e].second / 3);
    }
  std::vector<uint8_t> bnd(nv, 0);
  for (size_t e = 0; e < edges.size();) {
    size_t f = e;
    while (f < edges.size() && edges[f] == edges[e]) ++f;
    if (f - e == 1) bnd[edges[e].first] = bnd[edges[e].second] = 1;
    e = f;
  }
  for (int64_t i = 0; i < nv; ++i)
    if (vel[i].empty()) return gofd_fail(ctx, GOFD_E_ARG, "a vertex belongs to no element");
  std::vector<int32_t> roff(nv + 1, 0), ring, voff(nv + 1, 0), ve;
  for (int64_t i = 0; i < nv; ++i) {
    std::set<int32_t> r2(nb[i].begin(), nb[i].end());
    r2.insert((int32_t)i);
    for (int32_t j : nb[i]) r2.insert(nb[j].begin(), nb[j].end());
    ring.insert(ring.end(), r2.begin(), r2.end());
    roff[i + 1] = (int32_t)ring.size();
    ve.insert(ve.end(), vel[i].begin(), vel[i].end());     // element order (k ascending by construction)
    voff[i + 1] = (int32_t)ve.size();
  }
  hipStream_t st = ctx->stream;
  GOFD_TRY(dev_reserve(ctx, m->elems, sizeof(int32_t) * 3 * ne));
  GOFD_TRY(dev_reserve(ctx, m->ring_off, sizeof(int32_t) * (nv + 1)));
  GOFD_TRY(dev_reserve(ctx, m->ring, sizeof(int32_t) * ring.size()));
  GOFD_TRY(dev_reserve(ctx, m->ve_off, sizeof(int32_t) * (nv + 1)));
  GOFD_TRY(dev_reserve(ctx, m->ve, sizeof(int32_t) * ve.size()));
  GOFD_TRY(dev_reserve(ctx, m->bnd, nv));
  GOFD_TRY(dev_reserve(ctx, m->nbr, sizeof(int32_t) * 3 * ne));
  HIP_TRY(ctx, hipMemcpyAsync(m->elems.p, el.data(), sizeof(int32_t) * 3 * ne, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(m->ring_off.p, roff.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(m->ring.p, ring.data(), sizeof(int32_t) * ring.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(m->ve_off.p, voff.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(m->ve.p, ve.data(), sizeof(int32_t) * ve.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(m->bnd.p, bnd.data(), nv, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipMemcpyAsync(m->nbr.p, nbr.data(), sizeof(int32_t) * 3 * ne, hipMemcpyHostToDevice, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  *out = m.release();
  return GOFD_OK;
}

extern "C" int gofd_mmpde_free(gofd_mmpde m) {
  delete m;
  return GOFD_OK;
}

extern "C" int gofd_mmpde_metric(gofd_ctx ctx, gofd_mmpde m, const double* X_dev, const double* u_dev,
                                 double* Mv_dev, double* hess_dev, double* alpha_host) {
  if (!ctx || !m || !X_dev || !u_dev || !Mv_dev) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  Scratch s;
  GOFD_TRY(scratch(ctx, m, s));
  hipStream_t st = ctx->stream;
  const long long nv = m->nv, ne = m->ne;
  hipLaunchKernelGGL(k_vertex_hessian, dim3(grid1(nv, MB)), dim3(MB), 0, st, X_dev, m->ring_off.as<int>(),
                     m->ring.as<int>(), u_dev, nv, hess_dev ? hess_dev : s.Hv);
  hipLaunchKernelGGL(k_element_absH, dim3(grid1(ne, MB)), dim3(MB), 0, st, X_dev, m->elems.as<int>(),
                     hess_dev ? hess_dev : s.Hv, ne, s.aH, s.lam, s.area);
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(1024), 0, st, s.lam, s.area, ne, s.alpha);
  hipLaunchKernelGGL(k_vertex_metric, dim3(grid1(nv, MB)), dim3(MB), 0, st, hess_dev ? hess_dev : s.Hv, s.alpha, nv,
                     Mv_dev);
  HIP_TRY(ctx, hipGetLastError());
  double a = 0.0;
  HIP_TRY(ctx, hipMemcpyAsync(&a, s.alpha, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(ctx, hipStreamSynchronize(st));
  if (std::isnan(a)) return gofd_fail(ctx, GOFD_E_DEGENERATE, "the mesh has no positive area");
  if (alpha_host) *alpha_host = a;
  return GOFD_OK;
}

extern "C" int gofd_mmpde_energy(gofd_ctx ctx, gofd_mmpde m, const double* Xb_dev, const double* Mv_dev,
                                 const double* X_dev, double* grad_dev, double* MK_dev, double* energy_host) {
  if (!ctx || !m || !Xb_dev || !Mv_dev || !X_dev) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  Scratch s;
  GOFD_TRY(scratch(ctx, m, s));
  hipStream_t st = ctx->stream;
  const long long nv = m->nv, ne = m->ne;
  field_setup(ctx, m, Xb_dev, Mv_dev, s);
  hipLaunchKernelGGL(k_iota, dim3(grid1(ne, MB)), dim3(MB), 0, st, s.loc[1], ne);
  field_eval(ctx, m, X_dev, Xb_dev, Mv_dev, s.loc[1], s, 0);
  if (grad_dev) {
    hipLaunchKernelGGL(k_elem_grad, dim3(grid1(ne, MB)), dim3(MB), 0, st, X_dev, m->elems.as<int>(), s.MK[0],
                       s.GK[0], ne, s.G);
    hipLaunchKernelGGL(k_grad_vert, dim3(vertex_blocks(nv)), dim3(MB), 0, st, m->ve_off.as<int>(), m->ve.as<int>(),
                       s.G, m->bnd.as<uint8_t>(), X_dev, nv, -1, grad_dev, nullptr);
  }
  if (MK_dev)
    HIP_TRY(ctx, hipMemcpyAsync(MK_dev, s.MK[0], sizeof(double) * 3 * ne, hipMemcpyDeviceToDevice, st));
  double h2[2];
  GOFD_TRY(energy_check(ctx, m, X_dev, s.MK[0], s, h2));
  if (energy_host) *energy_host = h2[1] > 0 ? HUGE_VAL : h2[0];
  return GOFD_OK;
}

extern "C" int gofd_mmpde_element_hessians(gofd_ctx ctx, gofd_mmpde m, const double* X_dev, const double* MK_dev,
                                           double* hess_dev) {
  if (!ctx || !m || !X_dev || !MK_dev || !hess_dev) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  hipLaunchKernelGGL(k_elem_hess_fd, dim3(grid1(m->ne, MB)), dim3(MB), 0, ctx->stream, X_dev, m->elems.as<int>(),
                     MK_dev, (long long)m->ne, hess_dev);
  HIP_TRY(ctx, hipGetLastError());
  return GOFD_OK;
}

extern "C" int gofd_mmpde_move(gofd_ctx ctx, gofd_mmpde m, double* X_dev, const double* Mv_dev,
                               const gofd_mmpde_opts* opts, gofd_mmpde_info* info) {
  if (!ctx || !m || !X_dev || !Mv_dev) return gofd_fail(ctx, GOFD_E_ARG, "bad argument");
  gofd_mmpde_opts o{};
  if (opts) o = *opts;
  const double tau = o.tau > 0 ? o.tau : 1e-2;
  const double t_end = o.t_end > 0 ? o.t_end : 1.0;
  const double dt0 = o.dt0 > 0 ? o.dt0 : 1e-3;
  const int max_steps = o.max_steps > 0 ? o.max_steps : 400;
  const double gtol = o.gtol > 0 ? o.gtol : 1e-6;
  const double cg_tol = o.cg_tol > 0 ? o.cg_tol : 1e-10;
  const int max_cg = o.max_cg > 0 ? o.max_cg : 20000;
  const bool fixed = o.fixed_dt > 0;
  Scratch s;
  GOFD_TRY(scratch(ctx, m, s));
  hipStream_t st = ctx->stream;
  const long long nv = m->nv, ne = m->ne;
  const int* el = m->elems.as<int>();
  std::unique_ptr<KTimer> timer;
  if (o.stats) {
    timer.reset(new (std::nothrow) KTimer());
    if (!timer) return gofd_fail(ctx, GOFD_E_OOM, "kernel timer");
    timer->on = true;
  }
  KTimer* T = timer.get();
  // the metric field lives on the mesh the move starts from
  HIP_TRY(ctx, hipMemcpyAsync(s.Xb, X_dev, sizeof(double) * 2 * nv, hipMemcpyDeviceToDevice, st));
  field_setup(ctx, m, s.Xb, Mv_dev, s);
  hipLaunchKernelGGL(k_sqrtdet, dim3(grid1(nv, MB)), dim3(MB), 0, st, Mv_dev, nv, s.qv);
  hipLaunchKernelGGL(k_iota, dim3(grid1(ne, MB)), dim3(MB), 0, st, s.loc[1], ne);
  int acc = 0;   // slot of the accepted mesh's field values
  field_eval(ctx, m, X_dev, s.Xb, Mv_dev, s.loc[1], s, acc);
  double e0[2];
  GOFD_TRY(energy_check(ctx, m, X_dev, s.MK[acc], s, e0));
  if (e0[1] > 0) return gofd_fail(ctx, GOFD_E_DEGENERATE, "the mesh given has an inverted element");
  const double I_start = e0[0];
  double I0 = I_start, t = 0.0, dt = fixed ? o.fixed_dt : dt0, g0 = -1.0, gn = 0.0, h_max = 0.0;
  int steps = 0, rejected = 0;
  long long cg_its = 0;
  bool stalled = false;
  while (steps < max_steps && (fixed || t < t_end)) {
    GOFD_TRY(projected_gradient(ctx, m, X_dev, s.MK[acc], s.GK[acc], s, &gn));
    if (g0 < 0) g0 = gn;
    if (!fixed && gn <= gtol * g0) break;
    MM_LAUNCH(T, GOFD_MMPDE_K_HESS, k_elem_hess_fd, dim3(grid1(ne, MB)), dim3(MB), st, X_dev, el, s.MK[acc], ne,
              s.Hk);
    hipLaunchKernelGGL(k_hess_diag, dim3(grid1(nv, MB)), dim3(MB), 0, st, m->ve_off.as<int>(), m->ve.as<int>(), s.Hk,
                       nv, s.Jd);
    double h = fixed ? dt : std::min(dt, t_end - t);
    double e1[2] = {I0, 0.0};
    bool halved = false;
    for (;;) {
      bool ok = false;
      GOFD_TRY(step_solve(ctx, m, X_dev, s, tau, h, cg_tol, max_cg, &ok, &cg_its, T));
      if (fixed && !ok) return gofd_fail(ctx, GOFD_E_BREAKDOWN, "step system not positive definite");
      if (ok) {
        hipLaunchKernelGGL(k_place, dim3(grid1(nv, MB)), dim3(MB), 0, st, X_dev, s.dx, m->bnd.as<uint8_t>(), nv,
                           m->boundary, s.Y);
        field_eval(ctx, m, s.Y, s.Xb, Mv_dev, s.loc[acc], s, acc ^ 1, T);
        GOFD_TRY(energy_check(ctx, m, s.Y, s.MK[acc ^ 1], s, e1, T));
        if (fixed || (e1[1] == 0.0 && e1[0] < I0)) break;
      }
      h *= 0.5;
      ++rejected;
      halved = true;
      if (h < 1e-14 || h < 1e-6 * h_max) {
        stalled = true;
        break;
      }
    }
    if (stalled) break;
    HIP_TRY(ctx, hipMemcpyAsync(X_dev, s.Y, sizeof(double) * 2 * nv, hipMemcpyDeviceToDevice, st));
    acc ^= 1;
    I0 = e1[1] > 0 ? HUGE_VAL : e1[0];
    t += h;
    ++steps;
    h_max = std::max(h_max, h);
    if (!fixed) dt = halved ? h : 2.0 * h;     // after a halving the step is kept, else doubled
  }
  GOFD_TRY(projected_gradient(ctx, m, X_dev, s.MK[acc], s.GK[acc], s, &gn));
  if (g0 < 0) g0 = gn;
  if (T) {
    HIP_TRY(ctx, hipStreamSynchronize(st));
    T->write(o.stats);
  }
  if (info) {
    info->steps = steps;
    info->rejected = rejected;
    info->t = t;
    info->energy_start = I_start;
    info->energy_end = I0;
    info->cg_iterations = cg_its;
    info->grad_start = g0;
    info->grad_end = gn;
  }
  return GOFD_OK;
}
