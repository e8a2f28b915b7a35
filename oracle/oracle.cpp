// CPU FP64 oracle of the unified ABD-IPC time step (Taccel, arXiv 2504.12908).
//
// TEST INFRASTRUCTURE ONLY: the slow, plain reference the GPU library is checked against.
// It shares no code with the GPU library and must never be called from the product path.
//
// What it computes, and where each part comes from:
//  * Incremental potential of one backward-Euler step (Sec. 3.2 Eq. 1, App. A.2):
//      E(z) = sum_i 1/2 m_i |x_i - xhat_i|^2 + sum_b 1/2 (y_b - yhat_b)^T My_b (y_b - yhat_b)
//           + h^2 [ sum_e V_e Psi(F_e) + sum_b kappa_s V_b |A_b - R(A_b)|_F^2
//                   + kappa sum_k m_k b(d_k) ]
//           + sum_{prescribed b} augmented-Lagrangian term (Sec. 3.4 Eq. 6, App. A.5),
//    with xhat = x^n + h v^n + h^2 g (external force folded into the inertia term).
//  * Neo-Hookean density Psi = mu/2 (tr F^T F - 3) - mu ln J + lambda/2 (ln J)^2 from
//    (E, nu) (Sec. 3.1, App. A.1), lumped mass rho V_e / 4 per tet vertex.
//  * Log barrier b(d) = -(d - dhat)^2 ln(d/dhat) for 0 < d < dhat (App. A.3 Eq. A6) on
//    point-triangle and edge-edge pairs of the surface meshes (App. A.3), unsquared
//    Euclidean distance, near-parallel edge-edge pairs multiplied by the standard IPC
//    mollifier.  Lagged friction mu lambda f0(|u|) (App. A.3) when a scene sets mu > 0.
//  * Affine bodies (Sec. 3.3, App. A.4): y = [p; c1; c2; c3] with x = p + sum_j xbar_j c_j,
//    xbar in the centre-of-mass frame, reduced mass My = J^T M J from exact volume
//    integrals, an as-rigid-as-possible stiffness kappa_s V |A - R(A)|^2.
//  * Minimisation by Newton's method: exact element derivatives by second-order forward-mode
//    jets; far from the minimiser each FEM and barrier Hessian is replaced by its nearest
//    positive semidefinite matrix (Jacobi eigen-decomposition, eigenvalues clamped at zero),
//    and once the last step of the loop was a full one of at most 1e-2 dhat the exact
//    Hessians are used (the projected ones again if that system is not positive definite);
//    a direct (skyline Cholesky) solve, additive continuous collision detection to bound the
//    step, backtracking line search, convergence when the largest vertex displacement of the
//    Newton direction is below tol * h * L.
//  * Kinematic constraints: soft Dirichlet vertices are hard; prescribed affine bodies use
//    the method of multipliers and are snapped onto their target once close enough and the
//    snap is collision-free.
//
// Contact candidates are enumerated by brute force over all admissible pairs.
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <unordered_map>
#include <vector>

#include "jet.h"

namespace oracle {

using std::array;
using std::vector;
typedef array<double, 3> V3;
static const double kInf = std::numeric_limits<double>::infinity();

static inline V3 ld3(const double* p) { return {p[0], p[1], p[2]}; }
static inline V3 operator-(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
static inline V3 operator+(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
static inline V3 operator*(double s, const V3& a) { return {s * a[0], s * a[1], s * a[2]}; }
static inline double dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline V3 cross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
static inline double norm(const V3& a) { return std::sqrt(dot(a, a)); }

// ============================================================ symmetric eigen-solver
// Cyclic Jacobi rotations until the off-diagonal mass is below 1e-15 of the total.
static void sym_eigen(int n, const double* Ain, double* w, double* Vout) {
  vector<double> A(Ain, Ain + n * n), V(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
  if (Vout) std::memcpy(Vout, V.data(), sizeof(double) * n * n);
}

// Frobenius-nearest positive semi-definite matrix: eigenvalues clamped at zero.
static void psd_project(int n, const double* A, double* out) {
  vector<double> w(n), V(n * n);
  sym_eigen(n, A, w.data(), V.data());
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k)
        if (w[k] > 0.0) acc += V[i * n + k] * w[k] * V[j * n + k];
      out[i * n + j] = acc;
    }
}

// ============================================================ 3x3 helpers (any scalar)
template <class T>
static T det3(const T* F) {
  return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}
static void inv3(const double* A, double* out) {
  const double d = det3(A);
  out[0] = (A[4] * A[8] - A[5] * A[7]) / d;
  out[1] = (A[2] * A[7] - A[1] * A[8]) / d;
  out[2] = (A[1] * A[5] - A[2] * A[4]) / d;
  out[3] = (A[5] * A[6] - A[3] * A[8]) / d;
  out[4] = (A[0] * A[8] - A[2] * A[6]) / d;
  out[5] = (A[2] * A[3] - A[0] * A[5]) / d;
  out[6] = (A[3] * A[7] - A[4] * A[6]) / d;
  out[7] = (A[1] * A[6] - A[0] * A[7]) / d;
  out[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

// ============================================================ neo-Hookean (Sec. 3.1)
template <class T>
static T nh_psi(const T* F, double mu, double lam) {
  using std::log;
  T I1 = F[0] * F[0];
  for (int k = 1; k < 9; ++k) I1 = I1 + F[k] * F[k];
  T lnJ = log(det3(F));
  return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

// Edge matrix D[3*i+k] = X_{k+1,i} - X_{0,i} of a tet given as 4 stacked points.
static void edge_matrix(const double* x12, double* D) {
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) D[3 * i + k] = x12[3 * (k + 1) + i] - x12[i];
}

// Energy V*Psi(F) of one tet with gradient and Hessian (raw and PSD-projected in F space).
static void nh_tet_eval(const double* rest, const double* x, double mu, double lam, double* e,
                        double* g, double* H, double* Hp) {
  double Dm[9], Ds[9], Dminv[9], F[9];
  edge_matrix(rest, Dm);
  edge_matrix(x, Ds);
  inv3(Dm, Dminv);
  const double vol = det3(Dm) / 6.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Ds[3 * i + k] * Dminv[3 * k + j];
      F[3 * i + j] = acc;
    }
  if (g) std::memset(g, 0, sizeof(double) * 12);
  if (H) std::memset(H, 0, sizeof(double) * 144);
  if (Hp) std::memset(Hp, 0, sizeof(double) * 144);
  if (!(det3(F) > 0.0)) {
    *e = kInf;
    return;
  }
  Jet<9> Fj[9];
  for (int k = 0; k < 9; ++k) Fj[k] = Jet<9>::variable(F[k], k);
  const Jet<9> psi = nh_psi(Fj, mu, lam);
  *e = vol * psi.v;
  // B[k][m] = d vec(F)_k / d x_m, k = 3i+j, m = 3a+c.
  double B[9][12];
  std::memset(B, 0, sizeof(B));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double colsum = 0.0;
      for (int a = 1; a <= 3; ++a) {
        B[3 * i + j][3 * a + i] = Dminv[3 * (a - 1) + j];
        colsum += Dminv[3 * (a - 1) + j];
      }
      B[3 * i + j][i] = -colsum;
    }
  if (g)
    for (int m = 0; m < 12; ++m) {
      double acc = 0.0;
      for (int k = 0; k < 9; ++k) acc += B[k][m] * psi.g[k];
      g[m] = vol * acc;
    }
  double HF[81], HFp[81];
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) HF[9 * a + b] = psi.h[a][b];
  psd_project(9, HF, HFp);
  for (int pass = 0; pass < 2; ++pass) {
    double* out = pass == 0 ? H : Hp;
    const double* M = pass == 0 ? HF : HFp;
    if (!out) continue;
    for (int m = 0; m < 12; ++m)
      for (int n = 0; n < 12; ++n) {
        double acc = 0.0;
        for (int a = 0; a < 9; ++a) {
          if (B[a][m] == 0.0) continue;
          for (int b = 0; b < 9; ++b) acc += B[a][m] * M[9 * a + b] * B[b][n];
        }
        out[12 * m + n] = vol * acc;
      }
  }
}

static double nh_tet_energy(const double* rest, const double* x, double mu, double lam) {
  double Dm[9], Ds[9], Dminv[9], F[9];
  edge_matrix(rest, Dm);
  edge_matrix(x, Ds);
  inv3(Dm, Dminv);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += Ds[3 * i + k] * Dminv[3 * k + j];
      F[3 * i + j] = acc;
    }
  if (!(det3(F) > 0.0)) return kInf;
  return det3(Dm) / 6.0 * nh_psi(F, mu, lam);
}

// ============================================================ distances (App. A.3)
// Squared distance formulas per closest-feature type, any scalar type.
template <class T>
static T sq_pp(const T* a, const T* b) {
  T d0 = a[0] - b[0], d1 = a[1] - b[1], d2 = a[2] - b[2];
  return d0 * d0 + d1 * d1 + d2 * d2;
}
template <class T>
static void tcross(const T* a, const T* b, T* out) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}
template <class T>
static void tsub(const T* a, const T* b, T* out) {
  for (int i = 0; i < 3; ++i) out[i] = a[i] - b[i];
}
template <class T>
static T tdot(const T* a, const T* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
// Point p to the line through a, b: |(a-p) x (b-p)|^2 / |b-a|^2.
template <class T>
static T sq_pe(const T* p, const T* a, const T* b) {
  T u[3], v[3], c[3], e[3];
  tsub(a, p, u);
  tsub(b, p, v);
  tcross(u, v, c);
  tsub(b, a, e);
  return tdot(c, c) / tdot(e, e);
}
// Point p to the plane through t0, t1, t2.
template <class T>
static T sq_plane(const T* p, const T* t0, const T* t1, const T* t2) {
  T e1[3], e2[3], n[3], r[3];
  tsub(t1, t0, e1);
  tsub(t2, t0, e2);
  tcross(e1, e2, n);
  tsub(p, t0, r);
  T q = tdot(r, n);
  return q * q / tdot(n, n);
}
// Line a0a1 to line b0b1.
template <class T>
static T sq_ll(const T* a0, const T* a1, const T* b0, const T* b1) {
  T u[3], v[3], n[3], r[3];
  tsub(a1, a0, u);
  tsub(b1, b0, v);
  tcross(u, v, n);
  tsub(b0, a0, r);
  T q = tdot(r, n);
  return q * q / tdot(n, n);
}

// Point-triangle types: 0..2 point-vertex t0,t1,t2; 3..5 point-edge t0t1,t1t2,t2t0; 6 plane.
// Edge-edge types: 0 a0b0, 1 a0b1, 2 a1b0, 3 a1b1; 4 a0-edge b, 5 a1-edge b, 6 b0-edge a,
// 7 b1-edge a; 8 line-line.
template <class T>
static T typed_sqdist(int kind, int type, const T* x) {
  const T* P[4] = {x, x + 3, x + 6, x + 9};
  if (kind == 0) {
    switch (type) {
      case 0: return sq_pp(P[0], P[1]);
      case 1: return sq_pp(P[0], P[2]);
      case 2: return sq_pp(P[0], P[3]);
      case 3: return sq_pe(P[0], P[1], P[2]);
      case 4: return sq_pe(P[0], P[2], P[3]);
      case 5: return sq_pe(P[0], P[3], P[1]);
      default: return sq_plane(P[0], P[1], P[2], P[3]);
    }
  }
  switch (type) {
    case 0: return sq_pp(P[0], P[2]);
    case 1: return sq_pp(P[0], P[3]);
    case 2: return sq_pp(P[1], P[2]);
    case 3: return sq_pp(P[1], P[3]);
    case 4: return sq_pe(P[0], P[2], P[3]);
    case 5: return sq_pe(P[1], P[2], P[3]);
    case 6: return sq_pe(P[2], P[0], P[1]);
    case 7: return sq_pe(P[3], P[0], P[1]);
    default: return sq_ll(P[0], P[1], P[2], P[3]);
  }
}

// Projection parameter of p onto segment ab (unclamped).
static double seg_param(const double* p, const double* a, const double* b) {
  double e[3], r[3];
  tsub(b, a, e);
  tsub(p, a, r);
  return tdot(r, e) / tdot(e, e);
}

// True distance = minimum over the features whose closest point lies on the primitive.
// Candidates are visited from the highest-dimensional feature down and only a strictly
// smaller value replaces the current one, so ties resolve to the interior feature.
static int closest_type(int kind, const double* x, double* s_out) {
  double best = kInf;
  int type = -1;
  const double* P[4] = {x, x + 3, x + 6, x + 9};
  if (kind == 0) {
    double e1[3], e2[3], r[3];
    tsub(P[2], P[1], e1);
    tsub(P[3], P[1], e2);
    tsub(P[0], P[1], r);
    const double a11 = tdot(e1, e1), a12 = tdot(e1, e2), a22 = tdot(e2, e2);
    const double b1 = tdot(r, e1), b2 = tdot(r, e2);
    const double det = a11 * a22 - a12 * a12;
    if (det > 0.0) {
      const double l1 = (b1 * a22 - b2 * a12) / det, l2 = (a11 * b2 - a12 * b1) / det;
      const double l0 = 1.0 - l1 - l2;
      if (l0 >= 0.0 && l1 >= 0.0 && l2 >= 0.0) {
        best = typed_sqdist(0, 6, x);
        type = 6;
      }
    }
    const int ea[3] = {1, 2, 3}, eb[3] = {2, 3, 1};
    for (int k = 0; k < 3; ++k) {
      const double u = seg_param(P[0], P[ea[k]], P[eb[k]]);
      if (u >= 0.0 && u <= 1.0) {
        const double s = typed_sqdist(0, 3 + k, x);
        if (s < best) { best = s; type = 3 + k; }
      }
    }
    for (int k = 0; k < 3; ++k) {
      const double s = typed_sqdist(0, k, x);
      if (s < best) { best = s; type = k; }
    }
  } else {
    double u[3], v[3], w[3], n[3];
    tsub(P[1], P[0], u);
    tsub(P[3], P[2], v);
    tsub(P[0], P[2], w);
    tcross(u, v, n);
    const double A = tdot(u, u), B = tdot(u, v), C = tdot(v, v), D = tdot(u, w), E = tdot(v, w);
    if (tdot(n, n) > 1e-20 * A * C) {
      const double den = A * C - B * B;
      const double sa = (B * E - C * D) / den, sb = (A * E - B * D) / den;
      if (sa >= 0.0 && sa <= 1.0 && sb >= 0.0 && sb <= 1.0) {
        best = typed_sqdist(1, 8, x);
        type = 8;
      }
    }
    const int pt[4] = {0, 1, 2, 3};
    const int sa_[4] = {2, 2, 0, 0}, sb_[4] = {3, 3, 1, 1};
    for (int k = 0; k < 4; ++k) {
      const double t = seg_param(P[pt[k]], P[sa_[k]], P[sb_[k]]);
      if (t >= 0.0 && t <= 1.0) {
        const double s = typed_sqdist(1, 4 + k, x);
        if (s < best) { best = s; type = 4 + k; }
      }
    }
    for (int k = 0; k < 4; ++k) {
      const double s = typed_sqdist(1, k, x);
      if (s < best) { best = s; type = k; }
    }
  }
  *s_out = best;
  return type;
}

static double pair_sqdist(int kind, const double* x) {
  double s;
  closest_type(kind, x, &s);
  return s;
}

// ============================================================ barrier (App. A.3 Eq. A6)
template <class T>
static T barrier_of_d(const T& d, double dhat) {
  using std::log;
  return -((d - dhat) * (d - dhat)) * log(d / dhat);
}

template <class T>
static T edge_cross_sq(const T* x) {
  T u[3], v[3], n[3];
  tsub(x + 3, x, u);
  tsub(x + 9, x + 6, v);
  tcross(u, v, n);
  return tdot(n, n);
}

// Mollifier of near-parallel edge pairs: 2c/eps - c^2/eps^2 below eps, 1 above.
template <class T>
static T mollifier(const T& c, double eps) {
  if (value_of(c) < eps) return (2.0 / eps) * c - (c * c) * (1.0 / (eps * eps));
  return T(1.0);
}

static double pair_energy(int kind, const double* x, double meps, double dhat, double kappa) {
  const double s = pair_sqdist(kind, x);
  if (!(s > 0.0)) return kInf;
  const double d = std::sqrt(s);
  if (d >= dhat) return 0.0;
  double e = kappa * barrier_of_d(d, dhat);
  if (kind == 1) e *= mollifier(edge_cross_sq(x), meps);
  return e;
}

static int pair_eval(int kind, const double* x, double meps, double dhat, double kappa,
                     double* e, double* g, double* H, double* Hp) {
  double s;
  const int type = closest_type(kind, x, &s);
  if (g) std::memset(g, 0, sizeof(double) * 12);
  if (H) std::memset(H, 0, sizeof(double) * 144);
  if (Hp) std::memset(Hp, 0, sizeof(double) * 144);
  if (!(s > 0.0)) { *e = kInf; return type; }
  if (std::sqrt(s) >= dhat) { *e = 0.0; return type; }
  Jet<12> X[12];
  for (int k = 0; k < 12; ++k) X[k] = Jet<12>::variable(x[k], k);
  Jet<12> S = typed_sqdist(kind, type, X);
  Jet<12> E = kappa * barrier_of_d(sqrt(S), dhat);
  if (kind == 1) E = E * mollifier(edge_cross_sq(X), meps);
  *e = E.v;
  if (g) for (int k = 0; k < 12; ++k) g[k] = E.g[k];
  double Hraw[144];
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) Hraw[12 * a + b] = E.h[a][b];
  if (H) std::memcpy(H, Hraw, sizeof(Hraw));
  if (Hp) psd_project(12, Hraw, Hp);
  return type;
}

// ============================================================ friction (App. A.3)
// A friction pair with the data lagged at the start of the step: four world vertex ids, the
// weights of the closest-point difference c = sum_v gam_v X_v, its value c0 at the start of
// the step, the unit normal c0/|c0| and mu * lambda.
struct FPair {
  int w[4];
  double gam[4];
  V3 c0, n;
  double mul;
};
// Weights gam of the closest-point difference c = sum_v gam_v x_v of the closest features of
// a pair of the given distance type (the same types closest_type returns): c is the vector
// from the closest point of the second primitive to that of the first, |c| the distance.
static void closest_weights(int kind, int type, const double* x, double* gam) {
  const double* P[4] = {x, x + 3, x + 6, x + 9};
  for (int v = 0; v < 4; ++v) gam[v] = 0.0;
  if (kind == 0) {
    gam[0] = 1.0;
    if (type <= 2) {
      gam[1 + type] = -1.0;
    } else if (type <= 5) {
      const int ea[3] = {1, 2, 3}, eb[3] = {2, 3, 1};
      const int k = type - 3;
      const double u = seg_param(P[0], P[ea[k]], P[eb[k]]);
      gam[ea[k]] = -(1.0 - u);
      gam[eb[k]] = -u;
    } else {
      // barycentric coordinates of the projection of p onto the triangle's plane
      double e1[3], e2[3], r[3];
      tsub(P[2], P[1], e1);
      tsub(P[3], P[1], e2);
      tsub(P[0], P[1], r);
      const double a11 = tdot(e1, e1), a12 = tdot(e1, e2), a22 = tdot(e2, e2);
      const double b1 = tdot(r, e1), b2 = tdot(r, e2);
      const double det = a11 * a22 - a12 * a12;
      const double l1 = (b1 * a22 - b2 * a12) / det, l2 = (a11 * b2 - a12 * b1) / det;
      gam[1] = -(1.0 - l1 - l2);
      gam[2] = -l1;
      gam[3] = -l2;
    }
    return;
  }
  if (type <= 3) {
    const int a = type < 2 ? 0 : 1, b = (type & 1) ? 3 : 2;
    gam[a] = 1.0;
    gam[b] = -1.0;
  } else if (type <= 5) {  // a0 or a1 against edge b
    const double t = seg_param(P[type - 4], P[2], P[3]);
    gam[type - 4] = 1.0;
    gam[2] = -(1.0 - t);
    gam[3] = -t;
  } else if (type <= 7) {  // b0 or b1 against edge a
    const double t = seg_param(P[type - 4], P[0], P[1]);
    gam[0] = 1.0 - t;
    gam[1] = t;
    gam[type - 4] = -1.0;
  } else {  // closest points of the two lines
    double u[3], v[3], w[3];
    tsub(P[1], P[0], u);
    tsub(P[3], P[2], v);
    tsub(P[0], P[2], w);
    const double A = tdot(u, u), B = tdot(u, v), C = tdot(v, v), D = tdot(u, w), E = tdot(v, w);
    const double den = A * C - B * B;
    const double sa = (B * E - C * D) / den, sb = (A * E - B * D) / den;
    gam[0] = 1.0 - sa;
    gam[1] = sa;
    gam[2] = -(1.0 - sb);
    gam[3] = -sb;
  }
}

// Lagged data of one pair at the start-of-step configuration xn: weights, c0, normal and
// mu * lambda, lambda = -kappa m d b/dd the magnitude of the pair's normal force (the
// mollifier value m of an edge-edge pair held fixed).  Returns false for a pair not closer
// than dhat (or at zero distance).
static bool friction_lag(int kind, const double* xn, double meps, double dhat, double kappa,
                         double mu, FPair& f) {
  double s;
  const int type = closest_type(kind, xn, &s);
  if (!(s > 0.0) || !(s < dhat * dhat)) return false;
  closest_weights(kind, type, xn, f.gam);
  f.c0 = {0, 0, 0};
  for (int v = 0; v < 4; ++v) f.c0 = f.c0 + f.gam[v] * ld3(xn + 3 * v);
  f.n = (1.0 / norm(f.c0)) * f.c0;
  Jet<1> d = Jet<1>::variable(std::sqrt(s), 0);
  const double db = barrier_of_d(d, dhat).g[0];
  const double m = kind == 1 ? mollifier(edge_cross_sq(xn), meps) : 1.0;
  f.mul = mu * (-kappa * m * db);
  return true;
}

// f0 of the friction mollifier with eh = eps_v h, as a function of s = |u|^2: the closed form
// -|u|^3/(3 eh^2) + |u|^2/eh + eh/3 below eh and |u| above.  At s = 0 exactly the cubic term,
// whose first and second derivatives vanish there, is dropped (its jet would divide by 0).
template <class T>
static T friction_f0(const T& s, double eh) {
  using std::sqrt;
  if (value_of(s) == 0.0) return s * (1.0 / eh) + eh / 3.0;
  const T y = sqrt(s);
  if (value_of(y) < eh) return -(s * y) * (1.0 / (3.0 * eh * eh)) + s * (1.0 / eh) + eh / 3.0;
  return y;
}

// Friction energy mu lambda f0(|u|) of a lagged pair at the configuration x (12 values), with
// u the tangential part of c(x) - c0; gradient and Hessian by jets when g is given.
static double friction_eval(const FPair& f, const double* x, double eh, double* g, double* H) {
  if (!g) {
    V3 dl = {0, 0, 0};
    for (int v = 0; v < 4; ++v) dl = dl + f.gam[v] * ld3(x + 3 * v);
    dl = dl - f.c0;
    const V3 u = dl - dot(f.n, dl) * f.n;
    return f.mul * friction_f0(dot(u, u), eh);
  }
  Jet<12> X[12];
  for (int k = 0; k < 12; ++k) X[k] = Jet<12>::variable(x[k], k);
  Jet<12> dl[3];
  for (int c = 0; c < 3; ++c) {
    dl[c] = Jet<12>(-f.c0[c]);
    for (int v = 0; v < 4; ++v) dl[c] = dl[c] + f.gam[v] * X[3 * v + c];
  }
  const Jet<12> nd = f.n[0] * dl[0] + f.n[1] * dl[1] + f.n[2] * dl[2];
  Jet<12> ss(0.0);
  for (int c = 0; c < 3; ++c) {
    const Jet<12> uc = dl[c] - f.n[c] * nd;
    ss = ss + uc * uc;
  }
  const Jet<12> E = f.mul * friction_f0(ss, eh);
  for (int k = 0; k < 12; ++k) g[k] = E.g[k];
  for (int a = 0; a < 12; ++a)
    for (int b = 0; b < 12; ++b) H[12 * a + b] = E.h[a][b];
  return E.v;
}

// ============================================================ additive CCD
// Conservative advancement: with the common mean displacement removed, the distance can
// shrink at most at rate l_p (sum of the largest displacement on each side).  Advance by
// a fraction of the current distance over l_p until the remaining motion is covered (return
// 1) or the distance would fall below gap_ratio * d(0) (return the last safe time).
static double accd(int kind, const double* x, const double* p, double gap_ratio, int max_iter) {
  double q[12];
  for (int c = 0; c < 3; ++c) {
    const double mean = 0.25 * (p[c] + p[3 + c] + p[6 + c] + p[9 + c]);
    for (int v = 0; v < 4; ++v) q[3 * v + c] = p[3 * v + c] - mean;
  }
  double len[4];
  for (int v = 0; v < 4; ++v) len[v] = std::sqrt(tdot(q + 3 * v, q + 3 * v));
  const double lp = kind == 0 ? len[0] + std::max(len[1], std::max(len[2], len[3]))
                              : std::max(len[0], len[1]) + std::max(len[2], len[3]);
  if (lp == 0.0) return 1.0;
  const double d0 = std::sqrt(pair_sqdist(kind, x));
  if (!(d0 > 0.0)) return 0.0;
  const double gap = gap_ratio * d0;
  double t = 0.0;
  double step = (1.0 - gap_ratio) * d0 / lp;
  double xt[12];
  for (int it = 0; it < max_iter; ++it) {
    const double tn = t + step;
    for (int k = 0; k < 12; ++k) xt[k] = x[k] + tn * q[k];
    const double d = std::sqrt(pair_sqdist(kind, xt));
    if (it > 0 && d < gap) return t;
    t = tn;
    if (t > 1.0) return 1.0;
    step = 0.9 * d / lp;
  }
  return t;
}

// ============================================================ affine-body pieces (Sec. 3.3)
// Volume integrals of 1, x and x x^T by a signed tetrahedral fan from the vertex centroid.
static void abd_mass(int nv, const double* verts, int nf, const int* tris, double rho,
                     double* out) {
  V3 o = {0, 0, 0};
  for (int i = 0; i < nv; ++i) o = o + ld3(verts + 3 * i);
  o = (1.0 / nv) * o;
  double vol = 0.0, m1[3] = {0, 0, 0}, m2[9] = {0};
  for (int f = 0; f < nf; ++f) {
    const V3 a = ld3(verts + 3 * tris[3 * f]), b = ld3(verts + 3 * tris[3 * f + 1]),
             c = ld3(verts + 3 * tris[3 * f + 2]);
    const double v = dot(a - o, cross(b - o, c - o)) / 6.0;
    const V3 pts[4] = {o, a, b, c};
    const V3 s = o + a + b + c;
    vol += v;
    for (int i = 0; i < 3; ++i) m1[i] += v * s[i] / 4.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = s[i] * s[j];
        for (int k = 0; k < 4; ++k) acc += pts[k][i] * pts[k][j];
        m2[3 * i + j] += v * acc / 20.0;
      }
  }
  const double com[3] = {m1[0] / vol, m1[1] / vol, m1[2] / vol};
  out[0] = rho * vol;
  out[1] = vol;
  for (int i = 0; i < 3; ++i) out[2 + i] = com[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) out[5 + 3 * i + j] = rho * (m2[3 * i + j] - vol * com[i] * com[j]);
}

// |A - R(A)|_F^2 with R the polar rotation, R found by the Newton iteration
// X <- (X + X^{-T}) / 2 carried out in jet arithmetic.  A is given row-major.
template <class T>
static T arap_energy_t(const T* A) {
  T X[9];
  for (int k = 0; k < 9; ++k) X[k] = A[k];
  for (int it = 0; it < 40; ++it) {
    const T d = det3(X);
    T C[9];  // cofactor matrix = det * X^{-T}
    C[0] = X[4] * X[8] - X[5] * X[7];
    C[1] = X[5] * X[6] - X[3] * X[8];
    C[2] = X[3] * X[7] - X[4] * X[6];
    C[3] = X[2] * X[7] - X[1] * X[8];
    C[4] = X[0] * X[8] - X[2] * X[6];
    C[5] = X[1] * X[6] - X[0] * X[7];
    C[6] = X[1] * X[5] - X[2] * X[4];
    C[7] = X[2] * X[3] - X[0] * X[5];
    C[8] = X[0] * X[4] - X[1] * X[3];
    const T invd = 1.0 / d;
    T Y[9];
    for (int k = 0; k < 9; ++k) Y[k] = 0.5 * (X[k] + C[k] * invd);
    for (int k = 0; k < 9; ++k) X[k] = Y[k];
  }
  T acc = (A[0] - X[0]) * (A[0] - X[0]);
  for (int k = 1; k < 9; ++k) acc = acc + (A[k] - X[k]) * (A[k] - X[k]);
  return acc;
}

static double arap_eval(const double* A, double* g, double* H, double* Hp) {
  Jet<9> Aj[9];
  for (int k = 0; k < 9; ++k) Aj[k] = Jet<9>::variable(A[k], k);
  const Jet<9> e = arap_energy_t(Aj);
  if (g) for (int k = 0; k < 9; ++k) g[k] = e.g[k];
  double Hr[81];
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) Hr[9 * a + b] = e.h[a][b];
  if (H) std::memcpy(H, Hr, sizeof(Hr));
  if (Hp) psd_project(9, Hr, Hp);
  return e.v;
}
static double arap_energy(const double* A) { return arap_energy_t(A); }

// ============================================================ skyline Cholesky
// Symmetric positive-definite solve on the envelope of a reverse Cuthill-McKee ordering.
struct BlockMatrix {
  int n_nodes = 0;
  std::unordered_map<uint64_t, int> index;
  vector<array<double, 9>> blocks;
  vector<std::pair<int, int>> keys;
  array<double, 9>& at(int i, int j) {
    const uint64_t k = (uint64_t)(uint32_t)i << 32 | (uint32_t)j;
    auto it = index.find(k);
    if (it != index.end()) return blocks[it->second];
    index.emplace(k, (int)blocks.size());
    array<double, 9> z;
    z.fill(0.0);
    blocks.push_back(z);
    keys.emplace_back(i, j);
    return blocks.back();
  }
};

static bool skyline_solve(const BlockMatrix& M, const vector<double>& rhs, vector<double>& sol) {
  const int nn = M.n_nodes;
  vector<vector<int>> adj(nn);
  for (const auto& k : M.keys)
    if (k.first != k.second) adj[k.first].push_back(k.second);
  // Reverse Cuthill-McKee over every connected component.
  vector<int> order, deg(nn);
  for (int i = 0; i < nn; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
    deg[i] = (int)adj[i].size();
  }
  vector<char> seen(nn, 0);
  for (;;) {
    int start = -1;
    for (int i = 0; i < nn; ++i)
      if (!seen[i] && (start < 0 || deg[i] < deg[start])) start = i;
    if (start < 0) break;
    size_t head = order.size();
    order.push_back(start);
    seen[start] = 1;
    while (head < order.size()) {
      const int u = order[head++];
      vector<int> nb;
      for (int w : adj[u])
        if (!seen[w]) { nb.push_back(w); seen[w] = 1; }
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  vector<int> pos(nn);
  for (int i = 0; i < nn; ++i) pos[order[i]] = i;
  const int n = 3 * nn;
  vector<int> first(n);
  for (int r = 0; r < n; ++r) first[r] = r;
  for (const auto& k : M.keys) {
    const int pi = pos[k.first], pj = pos[k.second];
    if (pj > pi) continue;
    for (int a = 0; a < 3; ++a) {
      const int r = 3 * pi + a;
      first[r] = std::min(first[r], 3 * pj);
    }
  }
  vector<size_t> start(n + 1, 0);
  for (int r = 0; r < n; ++r) start[r + 1] = start[r] + (size_t)(r - first[r] + 1);
  vector<double> L(start[n], 0.0);
  auto ref = [&](int r, int c) -> double& { return L[start[r] + (size_t)(c - first[r])]; };
  for (size_t b = 0; b < M.keys.size(); ++b) {
    const int pi = pos[M.keys[b].first], pj = pos[M.keys[b].second];
    if (pj > pi) continue;
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        const int r = 3 * pi + a, col = 3 * pj + c;
        if (col <= r) ref(r, col) += M.blocks[b][3 * a + c];
      }
  }
  for (int i = 0; i < n; ++i) {
    for (int j = first[i]; j <= i; ++j) {
      double acc = ref(i, j);
      const int k0 = std::max(first[i], first[j]);
      for (int k = k0; k < j; ++k) acc -= ref(i, k) * ref(j, k);
      if (j < i) {
        ref(i, j) = acc / ref(j, j);
      } else {
        if (!(acc > 0.0)) return false;
        ref(i, i) = std::sqrt(acc);
      }
    }
  }
  vector<double> yv(n);
  for (int node = 0; node < nn; ++node)
    for (int a = 0; a < 3; ++a) yv[3 * pos[node] + a] = rhs[3 * node + a];
  for (int i = 0; i < n; ++i) {
    double acc = yv[i];
    for (int k = first[i]; k < i; ++k) acc -= ref(i, k) * yv[k];
    yv[i] = acc / ref(i, i);
  }
  for (int i = n - 1; i >= 0; --i) {
    yv[i] /= ref(i, i);
    const double v = yv[i];
    for (int k = first[i]; k < i; ++k) yv[k] -= ref(i, k) * v;
  }
  sol.assign(n, 0.0);
  for (int node = 0; node < nn; ++node)
    for (int a = 0; a < 3; ++a) sol[3 * node + a] = yv[3 * pos[node] + a];
  return true;
}

// ============================================================ scene
struct Body {
  int nv = 0, off = 0;  // off: first world vertex id
  vector<V3> xbar;      // creation-pose vertices relative to the centre of mass
  double rho = 0, m = 0, vol = 0, Q[9] = {0};
  V3 com0 = {0, 0, 0};
  bool prescribed = false;
  double My[144] = {0};
  double y[12] = {0}, yd[12] = {0};
  double yn[12] = {0}, yhat[12] = {0}, ystar[12] = {0}, lambda[12] = {0};
  double kappaA = 0, r0 = 0, rprev = 0;
  bool snapped = false;
};

struct Pair {
  int kind, i, j;
};

struct Scene {
  // parameters
  double h, dhat, kappa, kappa_s, tol, grav[3], mu, lam, rho;
  double fmu = 0.0, epsv = 0.0;  // friction coefficient and velocity threshold
  int max_newton, max_al;
  // soft body
  int nv = 0;
  vector<V3> X, x, v, xn, xhat;
  vector<uint8_t> dir;
  vector<array<int, 4>> tets;
  vector<array<double, 12>> rest;
  vector<double> mass;
  vector<int> moving;  // vertex ids flagged 2, increasing
  vector<Body> bodies;
  // contact topology over world vertex ids
  int nw = 0;
  vector<int> owner;  // -1 soft, else body index
  vector<char> fixed;
  vector<int> cverts;
  vector<array<int, 3>> ctris;
  vector<array<int, 2>> cedges;
  vector<double> edge_len2;  // rest squared length per contact edge
  double L = 0;
  // friction pairs of the current step (lagged at its start)
  vector<FPair> fric;
  // diagnostics
  vector<double> ls_log;
  vector<double> it_log;  // per Newton iteration of the last step, kItLog values each
  int al_round = 0;
};
constexpr int kItLog = 8;

static void world_positions(const Scene& S, vector<V3>& P) {
  P.resize(S.nw);
  for (int i = 0; i < S.nv; ++i) P[i] = S.x[i];
  for (const Body& b : S.bodies)
    for (int k = 0; k < b.nv; ++k) {
      V3 p = {b.y[0], b.y[1], b.y[2]};
      for (int j = 0; j < 3; ++j) p = p + b.xbar[k][j] * V3{b.y[3 + 3 * j], b.y[4 + 3 * j], b.y[5 + 3 * j]};
      P[b.off + k] = p;
    }
}

static void body_vertex(const Body& b, const double* y, int k, double* out) {
  for (int c = 0; c < 3; ++c) {
    double acc = y[c];
    for (int j = 0; j < 3; ++j) acc += b.xbar[k][j] * y[3 + 3 * j + c];
    out[c] = acc;
  }
}

static void pair_verts(const Scene& S, const Pair& pr, int* w) {
  if (pr.kind == 0) {
    w[0] = S.cverts[pr.i];
    for (int k = 0; k < 3; ++k) w[1 + k] = S.ctris[pr.j][k];
  } else {
    w[0] = S.cedges[pr.i][0];
    w[1] = S.cedges[pr.i][1];
    w[2] = S.cedges[pr.j][0];
    w[3] = S.cedges[pr.j][1];
  }
}

static double pair_meps(const Scene& S, const Pair& pr) {
  return pr.kind == 1 ? 1e-3 * S.edge_len2[pr.i] * S.edge_len2[pr.j] : 0.0;
}

static void gather12(const vector<V3>& P, const int* w, double* x12) {
  for (int v = 0; v < 4; ++v)
    for (int c = 0; c < 3; ++c) x12[3 * v + c] = P[w[v]][c];
}

// Axis-aligned box overlap with the activation distance folded in (same expression for
// every pair so a hash-based broad phase can reproduce the set bit for bit).
static bool boxes_close(const double* lo_a, const double* hi_a, const double* lo_b,
                        const double* hi_b, double dhat) {
  for (int c = 0; c < 3; ++c)
    if (!(lo_a[c] - dhat <= hi_b[c] && lo_b[c] - dhat <= hi_a[c])) return false;
  return true;
}

static void prim_box(const vector<V3>& P0, const vector<V3>* P1, const int* w, int n,
                     double* lo, double* hi) {
  for (int c = 0; c < 3; ++c) {
    lo[c] = kInf;
    hi[c] = -kInf;
  }
  for (int k = 0; k < n; ++k)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], P0[w[k]][c]);
      hi[c] = std::max(hi[c], P0[w[k]][c]);
      if (P1) {
        lo[c] = std::min(lo[c], (*P1)[w[k]][c]);
        hi[c] = std::max(hi[c], (*P1)[w[k]][c]);
      }
    }
}

// Admissible pairs (no shared vertex, not inside one affine body, not entirely on
// permanently fixed vertices) whose boxes pass the predicate, by brute force.
static void brute_candidates(const Scene& S, const vector<V3>& P0, const vector<V3>* P1,
                             vector<Pair>& out) {
  out.clear();
  const int nvq = (int)S.cverts.size(), nt = (int)S.ctris.size(), ne = (int)S.cedges.size();
  vector<array<double, 6>> vb(nvq), tb(nt), eb(ne);
  for (int i = 0; i < nvq; ++i) prim_box(P0, P1, &S.cverts[i], 1, vb[i].data(), vb[i].data() + 3);
  for (int i = 0; i < nt; ++i) prim_box(P0, P1, S.ctris[i].data(), 3, tb[i].data(), tb[i].data() + 3);
  for (int i = 0; i < ne; ++i) prim_box(P0, P1, S.cedges[i].data(), 2, eb[i].data(), eb[i].data() + 3);
  for (int i = 0; i < nvq; ++i) {
    const int v = S.cverts[i];
    for (int j = 0; j < nt; ++j) {
      const auto& t = S.ctris[j];
      if (v == t[0] || v == t[1] || v == t[2]) continue;
      const int ob = S.owner[v];
      if (ob >= 0 && ob == S.owner[t[0]] && ob == S.owner[t[1]] && ob == S.owner[t[2]]) continue;
      if (S.fixed[v] && S.fixed[t[0]] && S.fixed[t[1]] && S.fixed[t[2]]) continue;
      if (!boxes_close(vb[i].data(), vb[i].data() + 3, tb[j].data(), tb[j].data() + 3, S.dhat)) continue;
      out.push_back({0, i, j});
    }
  }
  for (int i = 0; i < ne; ++i) {
    const auto& a = S.cedges[i];
    for (int j = i + 1; j < ne; ++j) {
      const auto& b = S.cedges[j];
      if (a[0] == b[0] || a[0] == b[1] || a[1] == b[0] || a[1] == b[1]) continue;
      const int ob = S.owner[a[0]];
      if (ob >= 0 && ob == S.owner[a[1]] && ob == S.owner[b[0]] && ob == S.owner[b[1]]) continue;
      if (S.fixed[a[0]] && S.fixed[a[1]] && S.fixed[b[0]] && S.fixed[b[1]]) continue;
      if (!boxes_close(eb[i].data(), eb[i].data() + 3, eb[j].data(), eb[j].data() + 3, S.dhat)) continue;
      out.push_back({1, i, j});
    }
  }
}

// ---------------------------------------------------------------- unknowns
// Nodes of the linear system: free soft vertices (3 dof each) and, per unsnapped affine
// body, 4 pseudo-nodes p, c1, c2, c3 (3 dof each).
struct Dofs {
  vector<int> soft_node;  // per soft vertex: node or -1
  vector<int> body_node;  // per body: first node or -1
  int n_nodes = 0;
};

static Dofs make_dofs(const Scene& S) {
  Dofs D;
  D.soft_node.assign(S.nv, -1);
  for (int i = 0; i < S.nv; ++i)
    if (S.dir[i] == 0) D.soft_node[i] = D.n_nodes++;
  D.body_node.assign(S.bodies.size(), -1);
  for (size_t b = 0; b < S.bodies.size(); ++b)
    if (!S.bodies[b].snapped) {
      D.body_node[b] = D.n_nodes;
      D.n_nodes += 4;
    }
  return D;
}

// Node entries (node, weight) through which a world vertex moves.
static int vertex_nodes(const Scene& S, const Dofs& D, int w, int* node, double* wt) {
  if (S.owner[w] < 0) {
    if (D.soft_node[w] < 0) return 0;
    node[0] = D.soft_node[w];
    wt[0] = 1.0;
    return 1;
  }
  const int b = S.owner[w];
  if (D.body_node[b] < 0) return 0;
  const Body& B = S.bodies[b];
  const int k = w - B.off;
  node[0] = D.body_node[b];
  wt[0] = 1.0;
  for (int j = 0; j < 3; ++j) {
    node[1 + j] = D.body_node[b] + 1 + j;
    wt[1 + j] = B.xbar[k][j];
  }
  return 4;
}

// ---------------------------------------------------------------- energy
// Terms of the incremental potential, selectable for tests (all of them in the solve).
enum : unsigned {
  kTermInertia = 1,      // soft lumped inertia and body inertia
  kTermElastic = 2,      // neo-Hookean elasticity, h^2 V Psi
  kTermBodyStiff = 4,    // affine-body orthogonality (ARAP) term
  kTermConstraint = 8,   // augmented-Lagrangian kinematic constraint
  kTermContact = 16,     // barrier of the active pairs
  kTermFriction = 32,    // lagged friction potential
  kTermAll = 63
};

static double total_energy(const Scene& S, const vector<Pair>& pairs, unsigned terms = kTermAll) {
  double E = 0.0;
  for (int i = 0; i < S.nv; ++i)
    if ((terms & kTermInertia) && S.dir[i] == 0) {
      const V3 d = S.x[i] - S.xhat[i];
      E += 0.5 * S.mass[i] * dot(d, d);
    }
  const double h2 = S.h * S.h;
  double Eel = 0.0;
  for (size_t e = 0; e < S.tets.size() && (terms & kTermElastic); ++e) {
    double x12[12];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) x12[3 * a + c] = S.x[S.tets[e][a]][c];
    const double te = nh_tet_energy(S.rest[e].data(), x12, S.mu, S.lam);
    if (std::isinf(te)) return kInf;
    Eel += te;
  }
  E += h2 * Eel;
  for (const Body& b : S.bodies) {
    if (b.snapped) continue;
    double dy[12];
    for (int k = 0; k < 12; ++k) dy[k] = b.y[k] - b.yhat[k];
    double q = 0.0;
    for (int a = 0; a < 12; ++a)
      for (int c = 0; c < 12; ++c) q += dy[a] * b.My[12 * a + c] * dy[c];
    if (terms & kTermInertia) E += 0.5 * q;
    double A[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[3 * i + j] = b.y[3 + 3 * j + i];
    if (terms & kTermBodyStiff) E += h2 * S.kappa_s * b.vol * arap_energy(A);
    if (b.prescribed && (terms & kTermConstraint)) {
      double c[12];
      for (int k = 0; k < 12; ++k) c[k] = b.y[k] - b.ystar[k];
      double cc = 0.0, lc = 0.0;
      for (int a = 0; a < 12; ++a)
        for (int k = 0; k < 12; ++k) {
          cc += c[a] * b.My[12 * a + k] * c[k];
          lc += b.lambda[a] * b.My[12 * a + k] * c[k];
        }
      E += 0.5 * b.kappaA * cc - lc;
    }
  }
  vector<V3> P;
  world_positions(S, P);
  double Eb = 0.0;
  for (const Pair& pr : pairs) {
    if (!(terms & kTermContact)) break;
    int w[4];
    pair_verts(S, pr, w);
    double x12[12];
    gather12(P, w, x12);
    const double pe = pair_energy(pr.kind, x12, pair_meps(S, pr), S.dhat, S.kappa);
    if (std::isinf(pe)) return kInf;
    Eb += pe;
  }
  for (const FPair& f : S.fric) {
    if (!(terms & kTermFriction)) break;
    double x12[12];
    gather12(P, f.w, x12);
    Eb += friction_eval(f, x12, S.epsv * S.h, nullptr, nullptr);
  }
  E += h2 * Eb;
  return E;
}

// ---------------------------------------------------------------- gradient and Hessian
// exact: the FEM and barrier Hessians enter unprojected (Newton's method proper); otherwise
// each is replaced by its nearest positive semidefinite matrix (projected Newton).
static void assemble(const Scene& S, const Dofs& D, const vector<Pair>& active,
                     vector<double>& G, BlockMatrix& H, unsigned terms = kTermAll,
                     bool exact = false) {
  const double h2 = S.h * S.h;
  G.assign(3 * D.n_nodes, 0.0);
  H = BlockMatrix();
  H.n_nodes = D.n_nodes;
  for (int i = 0; i < S.nv; ++i) {
    const int n = D.soft_node[i];
    if (n < 0 || !(terms & kTermInertia)) continue;
    for (int c = 0; c < 3; ++c) G[3 * n + c] += S.mass[i] * (S.x[i][c] - S.xhat[i][c]);
    auto& blk = H.at(n, n);
    for (int c = 0; c < 3; ++c) blk[4 * c] += S.mass[i];
  }
  for (size_t e = 0; e < S.tets.size() && (terms & kTermElastic); ++e) {
    double x12[12], en, g[12], Hp[144];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) x12[3 * a + c] = S.x[S.tets[e][a]][c];
    if (exact) nh_tet_eval(S.rest[e].data(), x12, S.mu, S.lam, &en, g, Hp, nullptr);
    else nh_tet_eval(S.rest[e].data(), x12, S.mu, S.lam, &en, g, nullptr, Hp);
    for (int a = 0; a < 4; ++a) {
      const int na = D.soft_node[S.tets[e][a]];
      if (na < 0) continue;
      for (int c = 0; c < 3; ++c) G[3 * na + c] += h2 * g[3 * a + c];
      for (int b = 0; b < 4; ++b) {
        const int nb = D.soft_node[S.tets[e][b]];
        if (nb < 0) continue;
        auto& blk = H.at(na, nb);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) blk[3 * r + c] += h2 * Hp[12 * (3 * a + r) + 3 * b + c];
      }
    }
  }
  for (size_t bi = 0; bi < S.bodies.size(); ++bi) {
    const Body& b = S.bodies[bi];
    const int n0 = D.body_node[bi];
    if (n0 < 0) continue;
    double g[12] = {0}, Hb[144] = {0};
    if (terms & kTermInertia) {
      for (int k = 0; k < 144; ++k) Hb[k] = b.My[k];
      for (int a = 0; a < 12; ++a)
        for (int c = 0; c < 12; ++c) g[a] += b.My[12 * a + c] * (b.y[c] - b.yhat[c]);
    }
    double A[9], ga[9], Hap[81];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[3 * i + j] = b.y[3 + 3 * j + i];
    arap_eval(A, ga, nullptr, Hap);
    const double ks = (terms & kTermBodyStiff) ? h2 * S.kappa_s * b.vol : 0.0;
    // A row-major index 3i+j  <->  y index 3 + 3j + i.
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        g[3 + 3 * j + i] += ks * ga[3 * i + j];
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l)
            Hb[12 * (3 + 3 * j + i) + 3 + 3 * l + k] += ks * Hap[9 * (3 * i + j) + 3 * k + l];
      }
    if (b.prescribed && (terms & kTermConstraint)) {
      for (int a = 0; a < 12; ++a)
        for (int c = 0; c < 12; ++c) {
          g[a] += b.My[12 * a + c] * (b.kappaA * (b.y[c] - b.ystar[c]) - b.lambda[c]);
          Hb[12 * a + c] += b.kappaA * b.My[12 * a + c];
        }
    }
    for (int u = 0; u < 4; ++u) {
      for (int c = 0; c < 3; ++c) G[3 * (n0 + u) + c] += g[3 * u + c];
      for (int w = 0; w < 4; ++w) {
        auto& blk = H.at(n0 + u, n0 + w);
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) blk[3 * r + c] += Hb[12 * (3 * u + r) + 3 * w + c];
      }
    }
  }
  vector<V3> P;
  world_positions(S, P);
  const size_t npair = active.size();
  for (size_t k = 0; k < npair + S.fric.size(); ++k) {
    if (k < npair && !(terms & kTermContact)) continue;
    if (k >= npair && !(terms & kTermFriction)) continue;
    int w[4];
    double x12[12], e, g[12], Hp[144];
    if (k < npair) {
      const Pair& pr = active[k];
      pair_verts(S, pr, w);
      gather12(P, w, x12);
      if (exact) pair_eval(pr.kind, x12, pair_meps(S, pr), S.dhat, S.kappa, &e, g, Hp, nullptr);
      else pair_eval(pr.kind, x12, pair_meps(S, pr), S.dhat, S.kappa, &e, g, nullptr, Hp);
    } else {
      // friction: the exact Hessian, positive semidefinite by construction (the lagged normal
      // and weights make u linear in x, and f0 is convex in |u| with f1 >= 0)
      const FPair& f = S.fric[k - npair];
      for (int v = 0; v < 4; ++v) w[v] = f.w[v];
      gather12(P, w, x12);
      friction_eval(f, x12, S.epsv * S.h, g, Hp);
    }
    int nodes[4][4];
    double wts[4][4];
    int cnt[4];
    for (int a = 0; a < 4; ++a) cnt[a] = vertex_nodes(S, D, w[a], nodes[a], wts[a]);
    for (int a = 0; a < 4; ++a)
      for (int ia = 0; ia < cnt[a]; ++ia) {
        const int na = nodes[a][ia];
        const double wa = wts[a][ia];
        for (int c = 0; c < 3; ++c) G[3 * na + c] += h2 * wa * g[3 * a + c];
        for (int b = 0; b < 4; ++b)
          for (int ib = 0; ib < cnt[b]; ++ib) {
            auto& blk = H.at(na, nodes[b][ib]);
            const double s = h2 * wa * wts[b][ib];
            for (int r = 0; r < 3; ++r)
              for (int c = 0; c < 3; ++c) blk[3 * r + c] += s * Hp[12 * (3 * a + r) + 3 * b + c];
          }
      }
  }
}

// World-space displacement of every vertex for a node-space direction p.
static void world_displacement(const Scene& S, const Dofs& D, const vector<double>& p,
                               vector<V3>& out) {
  out.assign(S.nw, V3{0, 0, 0});
  for (int i = 0; i < S.nv; ++i) {
    const int n = D.soft_node[i];
    if (n >= 0) out[i] = {p[3 * n], p[3 * n + 1], p[3 * n + 2]};
  }
  for (size_t bi = 0; bi < S.bodies.size(); ++bi) {
    const int n0 = D.body_node[bi];
    if (n0 < 0) continue;
    const Body& b = S.bodies[bi];
    for (int k = 0; k < b.nv; ++k) body_vertex(b, &p[3 * n0], k, out[b.off + k].data());
  }
}

static void apply_step(Scene& S, const Dofs& D, const vector<double>& p, double alpha) {
  for (int i = 0; i < S.nv; ++i) {
    const int n = D.soft_node[i];
    if (n >= 0)
      for (int c = 0; c < 3; ++c) S.x[i][c] += alpha * p[3 * n + c];
  }
  for (size_t bi = 0; bi < S.bodies.size(); ++bi) {
    const int n0 = D.body_node[bi];
    if (n0 < 0) continue;
    for (int k = 0; k < 12; ++k) S.bodies[bi].y[k] += alpha * p[3 * n0 + k];
  }
}

static double min_ccd(const Scene& S, const vector<V3>& P0, const vector<V3>& disp,
                      const vector<Pair>& pairs) {
  double alpha = 1.0;
  for (const Pair& pr : pairs) {
    int w[4];
    pair_verts(S, pr, w);
    double x12[12], p12[12];
    gather12(P0, w, x12);
    gather12(disp, w, p12);
    alpha = std::min(alpha, accd(pr.kind, x12, p12, 0.1, 100000));
  }
  return alpha;
}

enum { kOk = 0, kNotConverged = 3, kLineSearchFailed = 4, kALFailed = 5, kNaN = 6, kInfeasible = 7 };

// One Newton loop on the current constraint set.  Returns a status and counts iterations.
static double body_residual(const Body& b);

static int newton_loop(Scene& S, int* iters) {
  const Dofs D = make_dofs(S);
  vector<Pair> cand, active, swept;
  vector<V3> P, disp, P1;
  vector<double> G, p;
  BlockMatrix H;
  const double stop = S.tol * S.h * S.L;
  double prev_alpha = 0.0, prev_pmax = 0.0;
  for (int it = 0; it < S.max_newton; ++it) {
    ++*iters;
    world_positions(S, P);
    brute_candidates(S, P, nullptr, cand);
    active.clear();
    for (const Pair& pr : cand) {
      int w[4];
      pair_verts(S, pr, w);
      double x12[12];
      gather12(P, w, x12);
      if (pair_sqdist(pr.kind, x12) < S.dhat * S.dhat) active.push_back(pr);
    }
    // Close to the minimiser (the last step was a full one and small against dhat) the
    // Hessian is taken exactly, so that the iteration converges quadratically; when that
    // system is not positive definite, the projected one is solved instead.
    const bool exact = it > 0 && prev_alpha == 1.0 && prev_pmax <= 1e-2 * S.dhat;
    assemble(S, D, active, G, H, kTermAll, exact);
    for (double gv : G)
      if (!std::isfinite(gv)) return kNaN;
    vector<double> rhs(G.size());
    for (size_t k = 0; k < G.size(); ++k) rhs[k] = -G[k];
    if (D.n_nodes == 0) return kOk;
    bool solved = skyline_solve(H, rhs, p);
    if (!solved && exact) {
      assemble(S, D, active, G, H);
      solved = skyline_solve(H, rhs, p);
    }
    if (!solved) return kNaN;
    world_displacement(S, D, p, disp);
    double pmax = 0.0;
    for (const V3& d : disp)
      for (int c = 0; c < 3; ++c) pmax = std::max(pmax, std::fabs(d[c]));
    const bool last = pmax <= stop;
    P1.resize(S.nw);
    for (int k = 0; k < S.nw; ++k) P1[k] = P[k] + disp[k];
    brute_candidates(S, P, &P1, swept);
    const double amax = min_ccd(S, P, disp, swept);
    double alpha = amax;
    if (!last) {
      const double E0 = total_energy(S, swept);
      const vector<V3> x_keep = S.x;
      vector<array<double, 12>> y_keep(S.bodies.size());
      for (size_t b = 0; b < S.bodies.size(); ++b) std::memcpy(y_keep[b].data(), S.bodies[b].y, sizeof(double) * 12);
      for (;;) {
        apply_step(S, D, p, alpha);
        const double E1 = total_energy(S, swept);
        S.x = x_keep;
        for (size_t b = 0; b < S.bodies.size(); ++b) std::memcpy(S.bodies[b].y, y_keep[b].data(), sizeof(double) * 12);
        if (E1 <= E0) {
          S.ls_log.push_back(E0);
          S.ls_log.push_back(E1);
          break;
        }
        alpha *= 0.5;
        if (alpha < 1e-12) return kLineSearchFailed;
      }
    }
    apply_step(S, D, p, alpha);
    prev_alpha = alpha;
    prev_pmax = pmax;
    {
      double kap = 0.0, res = 0.0;
      for (const Body& b : S.bodies)
        if (b.prescribed && !b.snapped) {
          kap = std::max(kap, b.kappaA);
          res = std::max(res, body_residual(b));
        }
      const double row[kItLog] = {(double)S.al_round, (double)it, pmax, amax, alpha,
                                  (double)active.size(), kap, res};
      S.it_log.insert(S.it_log.end(), row, row + kItLog);
    }
    if (last) return kOk;
  }
  return kNotConverged;
}

static double body_residual(const Body& b) {
  double r = 0.0;
  for (int k = 0; k < b.nv; ++k) {
    double a[3], c[3];
    body_vertex(b, b.y, k, a);
    body_vertex(b, b.ystar, k, c);
    r = std::max(r, std::sqrt((a[0] - c[0]) * (a[0] - c[0]) + (a[1] - c[1]) * (a[1] - c[1]) +
                              (a[2] - c[2]) * (a[2] - c[2])));
  }
  return r;
}

// Can body bi move from y to y* with every other vertex frozen, collision-free?
static bool snap_feasible(const Scene& S, int bi) {
  const Body& b = S.bodies[bi];
  vector<V3> P, disp(S.nw, V3{0, 0, 0}), P1;
  world_positions(S, P);
  for (int k = 0; k < b.nv; ++k) {
    double a[3], c[3];
    body_vertex(b, b.y, k, a);
    body_vertex(b, b.ystar, k, c);
    disp[b.off + k] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  }
  P1.resize(S.nw);
  for (int k = 0; k < S.nw; ++k) P1[k] = P[k] + disp[k];
  vector<Pair> swept;
  brute_candidates(S, P, &P1, swept);
  return min_ccd(S, P, disp, swept) >= 1.0;
}

static void to_public(const Body& b, const double* y, double* q) {
  // x = A X0 + t with t = p - A com0.
  double A[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[3 * i + j] = y[3 + 3 * j + i];
  for (int i = 0; i < 3; ++i) {
    double acc = y[i];
    for (int j = 0; j < 3; ++j) acc -= A[3 * i + j] * b.com0[j];
    q[i] = acc;
  }
  for (int k = 0; k < 9; ++k) q[3 + k] = A[k];
}
static void from_public(const Body& b, const double* q, double* y) {
  const double* A = q + 3;
  for (int i = 0; i < 3; ++i) {
    double acc = q[i];
    for (int j = 0; j < 3; ++j) acc += A[3 * i + j] * b.com0[j];
    y[i] = acc;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) y[3 + 3 * j + i] = A[3 * i + j];
}
static void to_public_rate(const Body& b, const double* yd, double* qd) {
  double Ad[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ad[3 * i + j] = yd[3 + 3 * j + i];
  for (int i = 0; i < 3; ++i) {
    double acc = yd[i];
    for (int j = 0; j < 3; ++j) acc -= Ad[3 * i + j] * b.com0[j];
    qd[i] = acc;
  }
  for (int k = 0; k < 9; ++k) qd[3 + k] = Ad[k];
}
static void from_public_rate(const Body& b, const double* qd, double* yd) { from_public(b, qd, yd); }

// Brute-force minimum distance over every admissible pair, number of pairs closer than
// dhat and the minimum det(F) over all tets, at the current state.
static void diagnostics(const Scene& S, double* dmin_out, double* jmin_out, int* nact_out) {
  vector<V3> P;
  world_positions(S, P);
  vector<Pair> all;
  // Every admissible pair: an infinite activation distance makes the box test pass.
  Scene T = S;
  T.dhat = kInf;
  brute_candidates(T, P, nullptr, all);
  double dmin = kInf;
  int nact = 0;
  for (const Pair& pr : all) {
    int w[4];
    pair_verts(S, pr, w);
    double x12[12];
    gather12(P, w, x12);
    const double d = std::sqrt(pair_sqdist(pr.kind, x12));
    dmin = std::min(dmin, d);
    if (d < S.dhat) ++nact;
  }
  double jmin = kInf;
  for (size_t e = 0; e < S.tets.size(); ++e) {
    double x12[12], Dm[9], Ds[9], Dminv[9];
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) x12[3 * a + c] = S.x[S.tets[e][a]][c];
    edge_matrix(S.rest[e].data(), Dm);
    edge_matrix(x12, Ds);
    inv3(Dm, Dminv);
    jmin = std::min(jmin, det3(Ds) * det3(Dminv));
  }
  *nact_out = nact;
  *dmin_out = dmin;
  *jmin_out = jmin;
}

// First half of a time step: prediction (Sec. 3.2 Eq. 1), kinematic targets, the friction
// lag and the jump of moving Dirichlet vertices.  Returns kOk or kInfeasible.
static int step_begin(Scene& S, const double* body_targets, const double* dir_targets) {
  S.ls_log.clear();
  S.xn = S.x;
  const double h = S.h;
  S.xhat.assign(S.nv, V3{0, 0, 0});
  for (int i = 0; i < S.nv; ++i)
    for (int c = 0; c < 3; ++c) S.xhat[i][c] = S.x[i][c] + h * S.v[i][c] + h * h * S.grav[c];
  for (size_t bi = 0; bi < S.bodies.size(); ++bi) {
    Body& b = S.bodies[bi];
    std::memcpy(b.yn, b.y, sizeof(b.y));
    for (int k = 0; k < 12; ++k) b.yhat[k] = b.y[k] + h * b.yd[k];
    if (!b.prescribed)
      for (int c = 0; c < 3; ++c) b.yhat[c] += h * h * S.grav[c];
    b.snapped = false;
    if (b.prescribed) {
      from_public(b, body_targets + 12 * bi, b.ystar);
      std::memset(b.lambda, 0, sizeof(b.lambda));
      b.kappaA = 1e6;
      b.r0 = body_residual(b);
      b.rprev = b.r0;
      // A body that starts the step on its target (a held indenter) satisfies its constraint
      // already: its DOFs are fixed from the start, as a Dirichlet DOF is.  The relative snap
      // test below could never pass for it (its start-of-step residual is zero).
      if (b.r0 == 0.0) b.snapped = true;
    }
  }
  // Friction pairs and their lagged data at the start-of-step configuration.
  S.fric.clear();
  if (S.fmu > 0.0) {
    vector<V3> P;
    world_positions(S, P);
    vector<Pair> cand;
    brute_candidates(S, P, nullptr, cand);
    for (const Pair& pr : cand) {
      FPair f;
      pair_verts(S, pr, f.w);
      double x12[12];
      gather12(P, f.w, x12);
      if (friction_lag(pr.kind, x12, pair_meps(S, pr), S.dhat, S.kappa, S.fmu, f)) S.fric.push_back(f);
    }
  }
  // Moving Dirichlet vertices jump to their targets; the move must be collision-free.
  if (!S.moving.empty()) {
    vector<V3> P, disp(S.nw, V3{0, 0, 0}), P1;
    world_positions(S, P);
    for (size_t k = 0; k < S.moving.size(); ++k) {
      const int v = S.moving[k];
      for (int c = 0; c < 3; ++c) disp[v][c] = dir_targets[3 * k + c] - S.x[v][c];
    }
    P1.resize(S.nw);
    for (int k = 0; k < S.nw; ++k) P1[k] = P[k] + disp[k];
    vector<Pair> swept;
    brute_candidates(S, P, &P1, swept);
    const double a = min_ccd(S, P, disp, swept);
    bool ok = a >= 1.0;
    vector<V3> keep = S.x;
    for (size_t k = 0; k < S.moving.size(); ++k)
      for (int c = 0; c < 3; ++c) S.x[S.moving[k]][c] = dir_targets[3 * k + c];
    if (ok) {
      for (size_t e = 0; e < S.tets.size() && ok; ++e) {
        double x12[12];
        for (int a2 = 0; a2 < 4; ++a2)
          for (int c = 0; c < 3; ++c) x12[3 * a2 + c] = S.x[S.tets[e][a2]][c];
        ok = std::isfinite(nh_tet_energy(S.rest[e].data(), x12, S.mu, S.lam));
      }
    }
    if (!ok) {
      S.x = keep;
      return kInfeasible;
    }
  }
  return kOk;
}

// Second half: Newton loops with the augmented-Lagrangian rounds and snaps (Sec. 3.4), then
// the velocity update (App. A.2 Eq. A2), or a roll-back to the start of the step.
static int step_finish(Scene& S, orc_stats* st) {
  const double h = S.h;
  int iters = 0, rounds = 0, status = kOk;
  S.it_log.clear();
  for (;;) {
    ++rounds;
    S.al_round = rounds;
    status = newton_loop(S, &iters);
    if (status != kOk) break;
    bool pending = false;
    for (size_t bi = 0; bi < S.bodies.size(); ++bi) {
      Body& b = S.bodies[bi];
      if (!b.prescribed || b.snapped) continue;
      const double r = body_residual(b);
      if (r <= 1e-3 * b.r0 && snap_feasible(S, (int)bi)) {
        std::memcpy(b.y, b.ystar, sizeof(b.y));
        b.snapped = true;
        pending = true;  // the others must re-equilibrate with the body fixed
        continue;
      }
      for (int k = 0; k < 12; ++k) b.lambda[k] -= b.kappaA * (b.y[k] - b.ystar[k]);
      if (r > 0.5 * b.rprev) b.kappaA *= 2.0;
      b.rprev = r;
      pending = true;
    }
    if (!pending) break;
    if (rounds >= S.max_al) { status = kALFailed; break; }
  }
  if (st) {
    st->status = status;
    st->newton_iters = iters;
    st->al_rounds = rounds;
  }
  if (status != kOk) {
    S.x = S.xn;
    for (Body& b : S.bodies) std::memcpy(b.y, b.yn, sizeof(b.y));
    return status;
  }
  for (int i = 0; i < S.nv; ++i)
    for (int c = 0; c < 3; ++c) S.v[i][c] = (S.x[i][c] - S.xn[i][c]) / h;
  for (Body& b : S.bodies)
    for (int k = 0; k < 12; ++k) b.yd[k] = (b.y[k] - b.yn[k]) / h;
  return kOk;
}

static int step(Scene& S, const double* body_targets, const double* dir_targets, orc_stats* st) {
  const int rc = step_begin(S, body_targets, dir_targets);
  if (rc != kOk) {
    if (st) st->status = rc;
    return rc;
  }
  return step_finish(S, st);
}

// The Newton system at the current state over the current unknowns: active pairs of the
// current positions, energy, gradient and projected Hessian of the selected terms.
static int current_system(const Scene& S, unsigned terms, double* energy, vector<double>& G,
                          BlockMatrix& H, Dofs& D) {
  D = make_dofs(S);
  vector<V3> P;
  world_positions(S, P);
  vector<Pair> cand, active;
  brute_candidates(S, P, nullptr, cand);
  for (const Pair& pr : cand) {
    int w[4];
    pair_verts(S, pr, w);
    double x12[12];
    gather12(P, w, x12);
    if (pair_sqdist(pr.kind, x12) < S.dhat * S.dhat) active.push_back(pr);
  }
  assemble(S, D, active, G, H, terms);
  if (energy) *energy = total_energy(S, active, terms);
  return D.n_nodes;
}

static Scene* create(const orc_desc* d, std::string& err) {
  Scene* S = new Scene();
  S->h = d->h;
  S->dhat = d->dhat;
  S->kappa = d->kappa;
  S->kappa_s = d->kappa_s;
  S->tol = d->newton_tol;
  for (int c = 0; c < 3; ++c) S->grav[c] = d->gravity[c];
  S->max_newton = d->max_newton > 0 ? d->max_newton : 100;
  S->max_al = d->max_al > 0 ? d->max_al : 30;
  S->fmu = d->friction;
  S->epsv = d->eps_v;
  if (S->fmu < 0.0 || (S->fmu > 0.0 && !(S->epsv > 0.0))) {
    err = "friction needs mu >= 0 and, when mu > 0, eps_v > 0";
    delete S;
    return nullptr;
  }
  S->mu = d->youngs / (2.0 * (1.0 + d->poisson));
  S->lam = d->youngs * d->poisson / ((1.0 + d->poisson) * (1.0 - 2.0 * d->poisson));
  S->rho = d->density;
  S->nv = d->nv;
  S->X.resize(S->nv);
  for (int i = 0; i < S->nv; ++i) S->X[i] = ld3(d->verts + 3 * i);
  S->x = S->X;
  S->v.assign(S->nv, V3{0, 0, 0});
  S->dir.assign(S->nv, 0);
  if (d->dirichlet)
    for (int i = 0; i < S->nv; ++i) S->dir[i] = d->dirichlet[i];
  for (int i = 0; i < S->nv; ++i)
    if (S->dir[i] == 2) S->moving.push_back(i);
  S->mass.assign(S->nv, 0.0);
  for (int e = 0; e < d->nt; ++e) {
    array<int, 4> t;
    for (int a = 0; a < 4; ++a) {
      t[a] = d->tets[4 * e + a];
      if (t[a] < 0 || t[a] >= S->nv) { err = "tet index out of range"; delete S; return nullptr; }
    }
    array<double, 12> r;
    for (int a = 0; a < 4; ++a)
      for (int c = 0; c < 3; ++c) r[3 * a + c] = S->X[t[a]][c];
    double Dm[9];
    edge_matrix(r.data(), Dm);
    const double vol = det3(Dm) / 6.0;
    if (!(vol > 0.0)) { err = "inverted or degenerate tet"; delete S; return nullptr; }
    for (int a = 0; a < 4; ++a) S->mass[t[a]] += S->rho * vol / 4.0;
    S->tets.push_back(t);
    S->rest.push_back(r);
  }
  // Boundary faces: faces used by exactly one tet.
  std::unordered_map<uint64_t, std::pair<int, array<int, 3>>> faces;
  auto fkey = [](int a, int b, int c) {
    int s[3] = {a, b, c};
    std::sort(s, s + 3);
    return (uint64_t)s[0] << 42 | (uint64_t)s[1] << 21 | (uint64_t)s[2];
  };
  for (const auto& t : S->tets) {
    const int f[4][3] = {{t[1], t[2], t[3]}, {t[0], t[3], t[2]}, {t[0], t[1], t[3]}, {t[0], t[2], t[1]}};
    for (int k = 0; k < 4; ++k) {
      auto& ent = faces[fkey(f[k][0], f[k][1], f[k][2])];
      ent.first += 1;
      ent.second = {f[k][0], f[k][1], f[k][2]};
    }
  }
  vector<array<int, 3>> soft_tris;
  for (const auto& kv : faces)
    if (kv.second.first == 1) soft_tris.push_back(kv.second.second);
  std::sort(soft_tris.begin(), soft_tris.end());
  int nw = S->nv;
  int voff = 0, foff = 0;
  for (int b = 0; b < d->nb; ++b) {
    Body B;
    B.nv = d->body_nv[b];
    B.off = nw;
    B.rho = d->body_density[b];
    B.prescribed = d->body_prescribed[b] != 0;
    double mp[14];
    abd_mass(B.nv, d->body_verts + 3 * voff, d->body_nf[b], d->body_tris + 3 * foff, B.rho, mp);
    B.m = mp[0];
    B.vol = mp[1];
    B.com0 = {mp[2], mp[3], mp[4]};
    for (int k = 0; k < 9; ++k) B.Q[k] = mp[5 + k];
    if (!(B.vol > 0.0)) { err = "affine body with non-positive volume"; delete S; return nullptr; }
    for (int k = 0; k < B.nv; ++k) B.xbar.push_back(ld3(d->body_verts + 3 * (voff + k)) - B.com0);
    for (int c = 0; c < 3; ++c) B.My[12 * c + c] = B.m;
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int c = 0; c < 3; ++c) B.My[12 * (3 + 3 * j + c) + 3 + 3 * k + c] = B.Q[3 * j + k];
    for (int c = 0; c < 3; ++c) B.y[c] = B.com0[c];
    for (int j = 0; j < 3; ++j) B.y[3 + 3 * j + j] = 1.0;
    for (int f = 0; f < d->body_nf[b]; ++f) {
      array<int, 3> t;
      for (int k = 0; k < 3; ++k) {
        const int li = d->body_tris[3 * (foff + f) + k];
        if (li < 0 || li >= B.nv) { err = "body triangle index out of range"; delete S; return nullptr; }
        t[k] = nw + li;
      }
      soft_tris.push_back(t);
    }
    nw += B.nv;
    voff += B.nv;
    foff += d->body_nf[b];
    S->bodies.push_back(B);
  }
  S->nw = nw;
  S->owner.assign(nw, -1);
  S->fixed.assign(nw, 0);
  for (int i = 0; i < S->nv; ++i) S->fixed[i] = S->dir[i] == 1;
  for (size_t b = 0; b < S->bodies.size(); ++b)
    for (int k = 0; k < S->bodies[b].nv; ++k) S->owner[S->bodies[b].off + k] = (int)b;
  S->ctris = soft_tris;
  vector<char> on_surf(nw, 0);
  std::unordered_map<uint64_t, int> emap;
  for (const auto& t : S->ctris)
    for (int k = 0; k < 3; ++k) {
      on_surf[t[k]] = 1;
      int a = t[k], b = t[(k + 1) % 3];
      if (a > b) std::swap(a, b);
      const uint64_t key = (uint64_t)a << 32 | (uint32_t)b;
      if (emap.emplace(key, (int)S->cedges.size()).second) S->cedges.push_back({a, b});
    }
  for (int w = 0; w < nw; ++w)
    if (on_surf[w]) S->cverts.push_back(w);
  // Rest positions of every world vertex for edge rest lengths and the scene scale.
  vector<V3> R(nw);
  for (int i = 0; i < S->nv; ++i) R[i] = S->X[i];
  for (const Body& B : S->bodies)
    for (int k = 0; k < B.nv; ++k) R[B.off + k] = B.xbar[k] + B.com0;
  for (const auto& e : S->cedges) {
    const V3 dv = R[e[1]] - R[e[0]];
    S->edge_len2.push_back(dot(dv, dv));
  }
  V3 lo = {kInf, kInf, kInf}, hi = {-kInf, -kInf, -kInf};
  for (const V3& p : R)
    for (int c = 0; c < 3; ++c) {
      lo[c] = std::min(lo[c], p[c]);
      hi[c] = std::max(hi[c], p[c]);
    }
  S->L = norm(hi - lo);
  return S;
}

}  // namespace oracle

using namespace oracle;

extern "C" {

void* orc_create(const orc_desc* d, char* err, int32_t errlen) {
  std::string msg;
  Scene* S = create(d, msg);
  if (!S && err && errlen > 0) std::snprintf(err, errlen, "%s", msg.c_str());
  return S;
}
void orc_destroy(void* s) { delete static_cast<Scene*>(s); }
int32_t orc_step(void* s, const double* body_targets, const double* dir_targets, orc_stats* st) {
  if (st) std::memset(st, 0, sizeof(*st));
  return step(*static_cast<Scene*>(s), body_targets, dir_targets, st);
}
int32_t orc_step_begin(void* s, const double* body_targets, const double* dir_targets) {
  return step_begin(*static_cast<Scene*>(s), body_targets, dir_targets);
}
int32_t orc_step_finish(void* s, orc_stats* st) {
  if (st) std::memset(st, 0, sizeof(*st));
  return step_finish(*static_cast<Scene*>(s), st);
}
int32_t orc_system(const void* s, uint32_t terms, double* energy, double* G, int32_t g_cap,
                   int32_t* brow, int32_t* bcol, double* bval, int32_t blk_cap, int32_t* n_blocks,
                   int32_t* node_of) {
  const Scene& S = *static_cast<const Scene*>(s);
  vector<double> Gv;
  BlockMatrix H;
  Dofs D;
  const int nn = current_system(S, terms, energy, Gv, H, D);
  for (int k = 0; k < (int)Gv.size() && k < g_cap; ++k) G[k] = Gv[k];
  const int nb = (int)H.keys.size();
  for (int b = 0; b < nb && b < blk_cap; ++b) {
    brow[b] = H.keys[b].first;
    bcol[b] = H.keys[b].second;
    for (int k = 0; k < 9; ++k) bval[9 * b + k] = H.blocks[b][k];
  }
  *n_blocks = nb;
  if (node_of) {
    for (int i = 0; i < S.nv; ++i) node_of[i] = D.soft_node[i];
    for (size_t b = 0; b < S.bodies.size(); ++b) node_of[S.nv + b] = D.body_node[b];
  }
  return nn;
}
int32_t orc_newton_direction(const void* s, double* p, int32_t cap) {
  const Scene& S = *static_cast<const Scene*>(s);
  vector<double> Gv, sol;
  BlockMatrix H;
  Dofs D;
  const int nn = current_system(S, kTermAll, nullptr, Gv, H, D);
  vector<double> rhs(Gv.size());
  for (size_t k = 0; k < Gv.size(); ++k) rhs[k] = -Gv[k];
  if (nn == 0) return 0;
  if (!skyline_solve(H, rhs, sol)) return -1;
  for (int k = 0; k < (int)sol.size() && k < cap; ++k) p[k] = sol[k];
  return nn;
}
int32_t orc_num_world_verts(const void* s) { return static_cast<const Scene*>(s)->nw; }
double orc_scene_scale(const void* s) { return static_cast<const Scene*>(s)->L; }
void orc_diagnostics(const void* s, double* min_distance, double* min_volume_ratio,
                     int32_t* n_active) {
  int n = 0;
  diagnostics(*static_cast<const Scene*>(s), min_distance, min_volume_ratio, &n);
  *n_active = n;
}
void orc_get_state(const void* s, double* x, double* v, double* q, double* qd) {
  const Scene& S = *static_cast<const Scene*>(s);
  for (int i = 0; i < S.nv; ++i)
    for (int c = 0; c < 3; ++c) {
      if (x) x[3 * i + c] = S.x[i][c];
      if (v) v[3 * i + c] = S.v[i][c];
    }
  for (size_t b = 0; b < S.bodies.size(); ++b) {
    if (q) to_public(S.bodies[b], S.bodies[b].y, q + 12 * b);
    if (qd) to_public_rate(S.bodies[b], S.bodies[b].yd, qd + 12 * b);
  }
}
void orc_set_state(void* s, const double* x, const double* v, const double* q, const double* qd) {
  Scene& S = *static_cast<Scene*>(s);
  for (int i = 0; i < S.nv; ++i)
    for (int c = 0; c < 3; ++c) {
      if (x) S.x[i][c] = x[3 * i + c];
      if (v) S.v[i][c] = v[3 * i + c];
    }
  for (size_t b = 0; b < S.bodies.size(); ++b) {
    if (q) from_public(S.bodies[b], q + 12 * b, S.bodies[b].y);
    if (qd) from_public_rate(S.bodies[b], qd + 12 * b, S.bodies[b].yd);
  }
}
void orc_world_positions(const void* s, double* out) {
  const Scene& S = *static_cast<const Scene*>(s);
  vector<V3> P;
  world_positions(S, P);
  for (int w = 0; w < S.nw; ++w)
    for (int c = 0; c < 3; ++c) out[3 * w + c] = P[w][c];
}
int32_t orc_newton_log(const void* s, double* out, int32_t cap) {
  const Scene& S = *static_cast<const Scene*>(s);
  const int n = (int)S.it_log.size();
  for (int k = 0; k < n && k < cap; ++k) out[k] = S.it_log[k];
  return n;
}

int32_t orc_ls_log(const void* s, double* out, int32_t cap) {
  const Scene& S = *static_cast<const Scene*>(s);
  const int n = (int)S.ls_log.size();
  for (int k = 0; k < n && k < cap; ++k) out[k] = S.ls_log[k];
  return n;
}
int32_t orc_candidates(const void* s, const double* P0, const double* P1, int32_t* out, int32_t cap) {
  const Scene& S = *static_cast<const Scene*>(s);
  vector<V3> A(S.nw), B;
  for (int w = 0; w < S.nw; ++w) A[w] = ld3(P0 + 3 * w);
  if (P1) {
    B.resize(S.nw);
    for (int w = 0; w < S.nw; ++w) B[w] = ld3(P1 + 3 * w);
  }
  vector<Pair> c;
  brute_candidates(S, A, P1 ? &B : nullptr, c);
  int n = 0;
  for (const Pair& pr : c) {
    int w[4];
    pair_verts(S, pr, w);
    int rec[5];
    rec[0] = pr.kind;
    if (pr.kind == 0) {
      rec[1] = w[0];
      int t[3] = {w[1], w[2], w[3]};
      std::sort(t, t + 3);
      rec[2] = t[0]; rec[3] = t[1]; rec[4] = t[2];
    } else {
      int a0 = std::min(w[0], w[1]), a1 = std::max(w[0], w[1]);
      int b0 = std::min(w[2], w[3]), b1 = std::max(w[2], w[3]);
      if (std::make_pair(b0, b1) < std::make_pair(a0, a1)) { std::swap(a0, b0); std::swap(a1, b1); }
      rec[1] = a0; rec[2] = a1; rec[3] = b0; rec[4] = b1;
    }
    if (n < cap)
      for (int k = 0; k < 5; ++k) out[5 * n + k] = rec[k];
    ++n;
  }
  return n;
}
void orc_nh_tet(const double rest[12], const double x[12], double mu, double lam, double* e,
                double g[12], double H[144], double Hp[144]) {
  nh_tet_eval(rest, x, mu, lam, e, g, H, Hp);
}
int32_t orc_pair_barrier(int32_t kind, const double x[12], double meps, double dhat, double kappa,
                         double* e, double g[12], double H[144], double Hp[144]) {
  return pair_eval(kind, x, meps, dhat, kappa, e, g, H, Hp);
}
double orc_pair_sqdist(int32_t kind, const double x[12], int32_t* dtype) {
  double s;
  const int t = closest_type(kind, x, &s);
  if (dtype) *dtype = t;
  return s;
}
double orc_accd(int32_t kind, const double x[12], const double p[12], double gap_ratio, int32_t max_iter) {
  return accd(kind, x, p, gap_ratio, max_iter);
}
double orc_barrier(double d, double dhat, double* d1, double* d2) {
  const Jet<1> D = Jet<1>::variable(d, 0);
  const Jet<1> b = barrier_of_d(D, dhat);
  if (d1) *d1 = b.g[0];
  if (d2) *d2 = b.h[0][0];
  return b.v;
}
void orc_abd_mass(int32_t nv, const double* verts, int32_t nf, const int32_t* tris, double rho, double out[14]) {
  abd_mass(nv, verts, nf, tris, rho, out);
}
double orc_arap(const double A[9], double g[9], double H[81], double Hp[81]) {
  return arap_eval(A, g, H, Hp);
}
void orc_psd_project(int32_t n, const double* A, double* out) { psd_project(n, A, out); }
double orc_pair_friction(int32_t kind, const double xn[12], const double x[12], double meps,
                         double dhat, double kappa, double mu, double eps_v_h, double* e,
                         double g[12], double H[144]) {
  FPair f;
  for (int v = 0; v < 4; ++v) f.w[v] = v;
  if (!friction_lag(kind, xn, meps, dhat, kappa, mu, f)) {
    *e = 0.0;
    std::memset(g, 0, sizeof(double) * 12);
    std::memset(H, 0, sizeof(double) * 144);
    return 0.0;
  }
  *e = friction_eval(f, x, eps_v_h, g, H);
  return mu > 0.0 ? f.mul / mu : 0.0;
}

}  // extern "C"
