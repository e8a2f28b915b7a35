// Neo-Hookean tetrahedra and the affine-body ARAP term (Taccel Sec. 3.1 and Sec. 3.3).
//
// Neo-Hookean density from (E, nu):  Psi(F) = mu/2 (tr F^T F - 3) - mu ln J + lambda/2 (ln J)^2,
// first Piola-Kirchhoff stress P = mu (F - F^{-T}) + lambda ln J F^{-T}.  Psi = +inf for J <= 0.
// The projected Hessian comes from the analytic eigensystem of an isotropic energy in
// singular values (3 scaling, 3 twist, 3 flip modes), with negative eigenvalues clamped at
// zero and each mode pulled back to vertex space as a rank-one 12x12 term.
#pragma once
#include "dmath.h"

namespace tc {

// F = D_s D_m^{-1} with D_s = [x1-x0, x2-x0, x3-x0].
TC_HD void deformation_gradient(const double* x12, const double* Dminv, double* F) {
  double Ds[9];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) Ds[3 * i + k] = x12[3 * (k + 1) + i] - x12[i];
  matmul3(Ds, Dminv, F);
}

TC_HD double nh_density(const double* F, double mu, double lam) {
  const double J = det3(F);
  if (!(J > 0.0)) return INFINITY;
  double I1 = 0.0;
  for (int k = 0; k < 9; ++k) I1 += F[k] * F[k];
  const double lnJ = log(J);
  return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
}

TC_HD void nh_stress(const double* F, double mu, double lam, double* P) {
  double C[9];
  cofactor3(F, C);
  const double J = det3(F);
  const double lnJ = log(J);
  const double invJ = 1.0 / J;
  for (int k = 0; k < 9; ++k) P[k] = mu * F[k] + (lam * lnJ - mu) * C[k] * invJ;
}

// The same stress in single precision from the displacement gradient G = F - I, in forms
// without the cancellations of F - F^{-T} and ln J near the rest state:
//   F - F^{-T} = F^{-T} (G + G^T + G^T G),  J - 1 = tr G + (tr^2 G - tr G^2)/2 + det G,
//   ln J = log1p(J - 1),  P = mu (F - F^{-T}) + lambda ln J F^{-T}.
TC_HD void nh_stress_disp(const float* G, float mu, float lam, float* P) {
  float F[9], C[9];
  for (int k = 0; k < 9; ++k) F[k] = G[k] + ((k % 4 == 0) ? 1.0f : 0.0f);
  cofactor3(F, C);
  const float trG = G[0] + G[4] + G[8];
  float trG2 = 0.0f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) trG2 += G[3 * i + j] * G[3 * j + i];
  const float Jm1 = trG + 0.5f * (trG * trG - trG2) + det3(G);
  const float J = 1.0f + Jm1;
  const float lnJ = log1pf(Jm1);
  // E2 = G + G^T + G^T G (= F^T F - I); F^{-T} = C / J
  float E2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      E2[3 * i + j] = G[3 * i + j] + G[3 * j + i] +
                      (G[i] * G[j] + G[3 + i] * G[3 + j] + G[6 + i] * G[6 + j]);
  const float invJ = 1.0f / J;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      // (F^{-T} E2)_{ij} = sum_k C_ik E2_kj / J
      const float fe = (C[3 * i] * E2[j] + C[3 * i + 1] * E2[3 + j] + C[3 * i + 2] * E2[6 + j]) * invJ;
      P[3 * i + j] = mu * fe + lam * lnJ * C[3 * i + j] * invJ;
    }
}

// Vertex-space pull-back of an F-space matrix M: w = vol * B^T vec(M), i.e. the columns of
// M D_m^{-T} for vertices 1..3 and minus their sum for vertex 0.
template <class R>
TC_HD void pullback(const R* M, const R* Dminv, R scale, R* w12) {
  for (int i = 0; i < 3; ++i) {
    R s = R(0);
    for (int a = 0; a < 3; ++a) {
      const R v = scale * (M[3 * i] * Dminv[3 * a] + M[3 * i + 1] * Dminv[3 * a + 1] +
                           M[3 * i + 2] * Dminv[3 * a + 2]);
      w12[3 * (a + 1) + i] = v;
      s += v;
    }
    w12[i] = -s;
  }
}

// Eigen-structure of an isotropic energy at F: SVD and the 9 mode eigenvalues.
template <class R>
struct ModesT {
  R U[9], V[9], E[9];  // E: eigenvectors of the 3x3 sigma-Hessian (columns)
  R lam[9];            // 0..2 scaling, then (twist, flip) for pairs (0,1),(0,2),(1,2)
};
using Modes = ModesT<double>;

template <class R>
TC_HD void nh_modes(const R* F, R mu, R lam, ModesT<R>& m) {
  R s[3];
  svd3(F, m.U, s, m.V);
  const R lnJ = log(det3(F));
  R hs[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      hs[3 * i + j] = i == j ? mu + (mu + lam * (R(1) - lnJ)) / (s[i] * s[i]) : lam / (s[i] * s[j]);
  R A[9], w[3];
  for (int k = 0; k < 9; ++k) A[k] = hs[k];
  sym_eig3(A, w, m.E);
  for (int k = 0; k < 3; ++k) m.lam[k] = w[k];
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int p = 0; p < 3; ++p) {
    const R inv = R(1) / (s[pa[p]] * s[pb[p]]);
    m.lam[3 + 2 * p] = mu + (lam * lnJ - mu) * inv;      // twist
    m.lam[4 + 2 * p] = mu + (mu - lam * lnJ) * inv;      // flip
  }
}

// ARAP term |A - R(A)|_F^2 = sum (s_i - 1)^2 with R = U V^T.
TC_HD void arap_modes(const double* A, Modes& m, double* e, double* grad /*9, row-major*/) {
  double s[3];
  svd3(A, m.U, s, m.V);
  *e = (s[0] - 1.0) * (s[0] - 1.0) + (s[1] - 1.0) * (s[1] - 1.0) + (s[2] - 1.0) * (s[2] - 1.0);
  double R[9];
  matmul3_bt(m.U, m.V, R);
  for (int k = 0; k < 9; ++k) grad[k] = 2.0 * (A[k] - R[k]);
  for (int k = 0; k < 9; ++k) m.E[k] = (k % 4 == 0) ? 1.0 : 0.0;
  m.lam[0] = m.lam[1] = m.lam[2] = 2.0;
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int p = 0; p < 3; ++p) {
    m.lam[3 + 2 * p] = 2.0 - 4.0 / (s[pa[p]] + s[pb[p]]);
    m.lam[4 + 2 * p] = 2.0;
  }
}

// F-space matrix Q_k of mode k (row-major).
template <class R>
TC_HD void mode_matrix(const ModesT<R>& m, int k, R* Q) {
  if (k < 3) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Q[3 * i + j] = m.U[3 * i] * m.E[k] * m.V[3 * j] + m.U[3 * i + 1] * m.E[3 + k] * m.V[3 * j + 1] +
                       m.U[3 * i + 2] * m.E[6 + k] * m.V[3 * j + 2];
    return;
  }
  const int p = (k - 3) >> 1;
  const R sb = ((k - 3) & 1) ? R(1) : R(-1);
  const int a = p == 2 ? 1 : 0, b = p == 0 ? 1 : 2;
  const R r = R(0.70710678118654752440);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Q[3 * i + j] = r * (m.U[3 * i + a] * m.V[3 * j + b] + sb * m.U[3 * i + b] * m.V[3 * j + a]);
}

}  // namespace tc
