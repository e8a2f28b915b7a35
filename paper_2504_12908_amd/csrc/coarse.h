// Coarse level of the two-level PCG preconditioner (host side, formed once per scene).
//
// The Newton systems of a soft pad are dominated by the elastic stiffness, whose smooth,
// long-range modes block-Jacobi PCG resolves only slowly.  An additive coarse correction
// M^{-1} = D^{-1} + P A_c^{-1} P^T removes most of them:
//   * aggregates are runs of consecutive 64-node blocks of a scene (one block each while the
//     scene has at most max_agg blocks with soft nodes); with the soft vertices stored along
//     a Morton curve every block is a compact patch of the pad;
//   * the coarse space holds the 6 rigid modes u = t + w x d of each aggregate, d being the
//     rest offset of a free soft node from its aggregate's centroid, scaled by the RMS
//     radius;
//   * A_c = P^T K P with K the rest-state Newton matrix of the soft body: lumped mass plus h^2
//     times the neo-Hookean Hessian at F = I (linear elasticity: dP = mu (dF + dF^T) +
//     lambda tr(dF) I).  Contact and affine-body terms stay with the block-Jacobi part.  Any
//     symmetric positive semi-definite A_c keeps the preconditioner SPD, so the rest-state
//     operator serves every Newton iteration of every step.
// Plain C++ (no device code), so it can be checked on the host.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace tc {

// Inverse of the principal submatrix of a symmetric positive semi-definite m x m matrix
// (row-major, overwritten) over the indices whose Cholesky pivot is not negligible (relative
// 1e-10 of the diagonal); the other rows and columns come out zero.
inline void spd_pinv(int m, std::vector<double>& A) {
  std::vector<double> L((size_t)m * m, 0.0);
  std::vector<char> keep(m, 0);
  for (int j = 0; j < m; ++j) {
    const double* Lj = &L[(size_t)j * m];
    double d = A[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= Lj[k] * Lj[k];
    if (!(A[(size_t)j * m + j] > 0.0) || !(d > 1e-10 * A[(size_t)j * m + j])) {
      for (int k = 0; k < j; ++k) L[(size_t)j * m + k] = 0.0;
      continue;
    }
    keep[j] = 1;
    const double ljj = std::sqrt(d);
    L[(size_t)j * m + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      const double* Li = &L[(size_t)i * m];
      double v = A[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) v -= Li[k] * Lj[k];
      L[(size_t)i * m + j] = v / ljj;
    }
  }
  // X = L^{-1} on the kept indices (forward substitution, column by column)
  std::vector<double> X((size_t)m * m, 0.0);
  for (int c = 0; c < m; ++c) {
    if (!keep[c]) continue;
    X[(size_t)c * m + c] = 1.0 / L[(size_t)c * m + c];
    for (int i = c + 1; i < m; ++i) {
      if (!keep[i]) continue;
      double v = 0.0;
      for (int k = c; k < i; ++k) v -= L[(size_t)i * m + k] * X[(size_t)k * m + c];
      X[(size_t)i * m + c] = v / L[(size_t)i * m + i];
    }
  }
  // A^{-1} = X^T X
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
      for (int k = i; k < m; ++k) v += X[(size_t)k * m + i] * X[(size_t)k * m + j];
      A[(size_t)i * m + j] = A[(size_t)j * m + i] = v;
    }
}

// One scene's inputs (global node / tet numbering of the batch).
struct CoarseScene {
  int node0 = 0, nv = 0;           // soft nodes node0 .. node0 + nv - 1
  const int* nfree = nullptr;      // [nodes]
  const double* X = nullptr;       // [nodes][3] rest positions
  const double* mass = nullptr;    // [nodes] lumped mass
  int tet0 = 0, tet1 = 0;
  const int* tv = nullptr;         // [tets][4] node ids
  const double* Dminv = nullptr;   // [tets][9] inverse rest edge matrix, row-major
  const double* vol = nullptr;     // [tets]
  double h = 0, mu = 0, lam = 0;
  const int* tn_b0 = nullptr;      // [blocks] first node of each 64-node block
  int bfirst = 0, bend = 0;        // the scene's blocks
  int block = 64;
  int max_agg = 128;
};

// Appends the scene's aggregates (block ranges), sets blk_agg for its blocks and the scaled
// offsets d of its free soft nodes, appends A_c^{-1} (m x m, row-major) and returns m.
inline int build_coarse(const CoarseScene& cs, std::vector<int>& blk_agg, std::vector<int>& agg_b0,
                        std::vector<int>& agg_b1, std::vector<double>& d_out,
                        std::vector<double>& ainv_out) {
  int nsb = 0;
  while (cs.bfirst + nsb < cs.bend && cs.tn_b0[cs.bfirst + nsb] < cs.node0 + cs.nv) ++nsb;
  if (nsb == 0) return 0;
  const int grp = (nsb + cs.max_agg - 1) / cs.max_agg;
  const int na = (nsb + grp - 1) / grp;
  const int a0 = (int)agg_b0.size(), m = 6 * na;
  std::vector<int> agg_of_block(nsb);
  for (int a = 0; a < na; ++a) {
    const int b0 = cs.bfirst + a * grp, b1 = std::min(cs.bfirst + (a + 1) * grp, cs.bfirst + nsb);
    agg_b0.push_back(b0);
    agg_b1.push_back(b1);
    for (int b = b0; b < b1; ++b) {
      blk_agg[b] = a0 + a;
      agg_of_block[b - cs.bfirst] = a;
    }
  }
  auto soft_free = [&](int n) { return n >= cs.node0 && n < cs.node0 + cs.nv && cs.nfree[n]; };
  auto agg_of = [&](int n) { return agg_of_block[(n - cs.node0) / cs.block]; };
  // centroids and RMS radii of the free soft nodes of each aggregate
  std::vector<double> cen(3 * (size_t)na, 0.0), rad(na, 0.0);
  std::vector<int> cnt(na, 0);
  for (int n = cs.node0; n < cs.node0 + cs.nv; ++n) {
    if (!soft_free(n)) continue;
    const int a = agg_of(n);
    for (int c = 0; c < 3; ++c) cen[3 * a + c] += cs.X[3 * (size_t)n + c];
    ++cnt[a];
  }
  for (int a = 0; a < na; ++a)
    for (int c = 0; c < 3; ++c) cen[3 * a + c] = cnt[a] ? cen[3 * a + c] / cnt[a] : 0.0;
  for (int n = cs.node0; n < cs.node0 + cs.nv; ++n) {
    if (!soft_free(n)) continue;
    const int a = agg_of(n);
    for (int c = 0; c < 3; ++c) {
      const double dd = cs.X[3 * (size_t)n + c] - cen[3 * a + c];
      rad[a] += dd * dd;
    }
  }
  for (int a = 0; a < na; ++a) rad[a] = (cnt[a] && rad[a] > 0.0) ? std::sqrt(rad[a] / cnt[a]) : 1.0;
  for (int n = cs.node0; n < cs.node0 + cs.nv; ++n) {
    if (!soft_free(n)) continue;
    const int a = agg_of(n);
    for (int c = 0; c < 3; ++c) d_out[3 * (size_t)n + c] = (cs.X[3 * (size_t)n + c] - cen[3 * a + c]) / rad[a];
  }
  // displacement of node n under coarse mode k: t = e_k (k < 3), w = e_{k-3} (k >= 3)
  auto mode = [&](int n, int k, double* u) {
    const double* d = &d_out[3 * (size_t)n];
    u[0] = u[1] = u[2] = 0.0;
    if (k < 3) {
      u[k] = 1.0;
      return;
    }
    const int a = k - 3;  // e_a x d
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    u[b] = -d[c];
    u[c] = d[b];
  };
  std::vector<double> Ac((size_t)m * m, 0.0);
  for (int n = cs.node0; n < cs.node0 + cs.nv; ++n) {
    if (!soft_free(n)) continue;
    const int a = agg_of(n);
    double U[6][3];
    for (int k = 0; k < 6; ++k) mode(n, k, U[k]);
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j)
        Ac[(size_t)(6 * a + i) * m + 6 * a + j] +=
            cs.mass[n] * (U[i][0] * U[j][0] + U[i][1] * U[j][1] + U[i][2] * U[j][2]);
  }
  const double h2 = cs.h * cs.h;
  for (int t = cs.tet0; t < cs.tet1; ++t) {
    const int* tvn = cs.tv + 4 * (size_t)t;
    const double* Di = cs.Dminv + 9 * (size_t)t;
    // gradients of the linear shape functions: F = sum_v x_v (x) gN_v
    double gN[4][3];
    for (int j = 0; j < 3; ++j) {
      gN[0][j] = -(Di[j] + Di[3 + j] + Di[6 + j]);
      for (int v = 1; v < 4; ++v) gN[v][j] = Di[3 * (v - 1) + j];
    }
    int aggs[4], nat = 0;
    for (int v = 0; v < 4; ++v) {
      if (!soft_free(tvn[v])) continue;
      const int a = agg_of(tvn[v]);
      bool seen = false;
      for (int q = 0; q < nat; ++q) seen = seen || aggs[q] == a;
      if (!seen) aggs[nat++] = a;
    }
    if (nat == 0) continue;
    const int L = 6 * nat;
    double dF[24][9];
    for (int q = 0; q < nat; ++q)
      for (int k = 0; k < 6; ++k) {
        double* F = dF[6 * q + k];
        for (int e = 0; e < 9; ++e) F[e] = 0.0;
        for (int v = 0; v < 4; ++v) {
          if (!soft_free(tvn[v]) || agg_of(tvn[v]) != aggs[q]) continue;
          double u[3];
          mode(tvn[v], k, u);
          for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) F[3 * i + j] += u[i] * gN[v][j];
        }
      }
    const double w = h2 * cs.vol[t];
    for (int p = 0; p < L; ++p)
      for (int q = 0; q < L; ++q) {
        const double* A = dF[p];
        const double* B = dF[q];
        double ff = 0.0, ft = 0.0;
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            ff += A[3 * i + j] * B[3 * i + j];
            ft += A[3 * i + j] * B[3 * j + i];
          }
        const double tr = (A[0] + A[4] + A[8]) * (B[0] + B[4] + B[8]);
        const int gp = 6 * aggs[p / 6] + p % 6, gq = 6 * aggs[q / 6] + q % 6;
        Ac[(size_t)gp * m + gq] += w * (cs.mu * (ff + ft) + cs.lam * tr);
      }
  }
  spd_pinv(m, Ac);
  ainv_out.insert(ainv_out.end(), Ac.begin(), Ac.end());
  return m;
}

}  // namespace tc
