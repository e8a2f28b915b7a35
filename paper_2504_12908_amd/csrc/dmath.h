// Small dense linear algebra for the per-element work of the IPC time step.
// Everything is __host__ __device__ so it can be compiled into GPU kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define TC_HD __host__ __device__ __forceinline__

namespace tc {

struct d3 {
  double x, y, z;
};
TC_HD d3 mk(double x, double y, double z) { return d3{x, y, z}; }
TC_HD d3 ld(const double* p) { return d3{p[0], p[1], p[2]}; }
TC_HD void st(double* p, const d3& a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
TC_HD d3 operator+(const d3& a, const d3& b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }
TC_HD d3 operator-(const d3& a, const d3& b) { return d3{a.x - b.x, a.y - b.y, a.z - b.z}; }
TC_HD d3 operator*(double s, const d3& a) { return d3{s * a.x, s * a.y, s * a.z}; }
TC_HD double dot(const d3& a, const d3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
TC_HD d3 cross(const d3& a, const d3& b) {
  return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
TC_HD double at(const d3& a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// 3x3 matrices are row-major double[9].
TC_HD double det3(const double* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
// Cofactor matrix (= det(A) * A^{-T}).
TC_HD void cofactor3(const double* A, double* C) {
  C[0] = A[4] * A[8] - A[5] * A[7];
  C[1] = A[5] * A[6] - A[3] * A[8];
  C[2] = A[3] * A[7] - A[4] * A[6];
  C[3] = A[2] * A[7] - A[1] * A[8];
  C[4] = A[0] * A[8] - A[2] * A[6];
  C[5] = A[1] * A[6] - A[0] * A[7];
  C[6] = A[1] * A[5] - A[2] * A[4];
  C[7] = A[2] * A[3] - A[0] * A[5];
  C[8] = A[0] * A[4] - A[1] * A[3];
}
TC_HD void matmul3(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
// C = A * B^T
TC_HD void matmul3_bt(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations.  A is row-major and is
// destroyed; on return w holds the eigenvalues and V (row-major) the eigenvectors as
// columns.
TC_HD void sym_eig3(double* A, double* w, double* V) {
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 10; ++sweep) {
    const double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    const double dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = A[3 * p + q];
      if (apq == 0.0) continue;
      const double theta = (A[3 * q + q] - A[3 * p + p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int k = 0; k < 3; ++k) {
        const double akp = A[3 * k + p], akq = A[3 * k + q];
        A[3 * k + p] = c * akp - s * akq;
        A[3 * k + q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        const double apk = A[3 * p + k], aqk = A[3 * q + k];
        A[3 * p + k] = c * apk - s * aqk;
        A[3 * q + k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[3 * k + p], vkq = V[3 * k + q];
        V[3 * k + p] = c * vkp - s * vkq;
        V[3 * k + q] = s * vkp + c * vkq;
      }
    }
  }
  w[0] = A[0];
  w[1] = A[4];
  w[2] = A[8];
}

// Rotation-variant SVD F = U diag(s) V^T with det U = det V = +1 (s[2] carries the sign
// of det F), singular values in decreasing order of magnitude.  V from the eigenvectors of
// F^T F; U by Gram-Schmidt on the columns of F V.
TC_HD void svd3(const double* F, double* U, double* s, double* V) {
  double A[9], w[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      A[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
  sym_eig3(A, w, V);
  // sort eigenpairs by decreasing eigenvalue
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2 - a; ++b)
      if (w[b] < w[b + 1]) {
        const double tw = w[b]; w[b] = w[b + 1]; w[b + 1] = tw;
        for (int k = 0; k < 3; ++k) {
          const double tv = V[3 * k + b]; V[3 * k + b] = V[3 * k + b + 1]; V[3 * k + b + 1] = tv;
        }
      }
  if (det3(V) < 0.0)
    for (int k = 0; k < 3; ++k) V[3 * k + 2] = -V[3 * k + 2];
  double B[9];
  matmul3(F, V, B);
  d3 b0 = mk(B[0], B[3], B[6]), b1 = mk(B[1], B[4], B[7]), b2 = mk(B[2], B[5], B[8]);
  double n0 = sqrt(dot(b0, b0));
  d3 u0 = n0 > 0.0 ? (1.0 / n0) * b0 : mk(1, 0, 0);
  d3 r1 = b1 - dot(u0, b1) * u0;
  double n1 = sqrt(dot(r1, r1));
  d3 u1;
  if (n1 > 1e-300) {
    u1 = (1.0 / n1) * r1;
  } else {  // any unit vector orthogonal to u0
    d3 t = fabs(u0.x) < 0.9 ? mk(1, 0, 0) : mk(0, 1, 0);
    t = t - dot(u0, t) * u0;
    u1 = (1.0 / sqrt(dot(t, t))) * t;
  }
  d3 u2 = cross(u0, u1);
  s[0] = n0;
  s[1] = dot(u1, b1);
  s[2] = dot(u2, b2);
  U[0] = u0.x; U[3] = u0.y; U[6] = u0.z;
  U[1] = u1.x; U[4] = u1.y; U[7] = u1.z;
  U[2] = u2.x; U[5] = u2.y; U[8] = u2.z;
}

// Projected Hessian of an isotropic energy psi(sigma) in F space, as 9 rank-one modes
// lambda_k vec(Q_k) vec(Q_k)^T (Q_k orthonormal in the Frobenius product): 3 scaling modes
// from the 3x3 Hessian in sigma, and per pair (i,j) a twist (antisymmetric) mode with
// eigenvalue (psi_i + psi_j)/(s_i + s_j) and a flip (symmetric) mode with
// (psi_i - psi_j)/(s_i - s_j); the latter two are passed in already simplified so that no
// division by s_i - s_j occurs.  Writes the 9 eigenvalues and the 9 matrices Q (row-major).
TC_HD void isotropic_modes(const double* U, const double* V, const double* hs /*3x3*/,
                           const double* twist /*[3] for pairs (0,1),(0,2),(1,2)*/,
                           const double* flip, double* lam, double* Q /*[9][9]*/) {
  double A[9], w[3], E[9];
  for (int k = 0; k < 9; ++k) A[k] = hs[k];
  sym_eig3(A, w, E);
  for (int m = 0; m < 3; ++m) {
    lam[m] = w[m];
    // U diag(e_m) V^T
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += U[3 * i + k] * E[3 * k + m] * V[3 * j + k];
        Q[9 * m + 3 * i + j] = acc;
      }
  }
  const double r = 0.70710678118654752440;
  const int pi_[3] = {0, 0, 1}, pj_[3] = {1, 2, 2};
  for (int p = 0; p < 3; ++p) {
    const int a = pi_[p], b = pj_[p];
    for (int sgn = 0; sgn < 2; ++sgn) {
      const int m = 3 + 2 * p + sgn;
      lam[m] = sgn == 0 ? twist[p] : flip[p];
      const double sb = sgn == 0 ? -1.0 : 1.0;
      // U (e_a e_b^T + sb e_b e_a^T) V^T / sqrt(2)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          Q[9 * m + 3 * i + j] = r * (U[3 * i + a] * V[3 * j + b] + sb * U[3 * i + b] * V[3 * j + a]);
    }
  }
}

// In-place PSD projection of a symmetric n x n matrix stored with element (i,j) at
// A[(i*n+j)*stride], using cyclic Jacobi; V is scratch of the same layout.  Eigenvalues
// are clamped at zero and the matrix is rebuilt.
template <int n>
TC_HD void psd_project_strided(double* A, double* V, int stride) {
#define AE(i, j) A[((i) * n + (j)) * stride]
#define VE(i, j) V[((i) * n + (j)) * stride]
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) VE(i, j) = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double a = AE(i, j);
        tot += a * a;
        if (i != j) off += a * a;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = AE(p, q);
        if (apq == 0.0) continue;
        const double theta = (AE(q, q) - AE(p, p)) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = AE(k, p), akq = AE(k, q);
          AE(k, p) = c * akp - s * akq;
          AE(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = AE(p, k), aqk = AE(q, k);
          AE(p, k) = c * apk - s * aqk;
          AE(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = VE(k, p), vkq = VE(k, q);
          VE(k, p) = c * vkp - s * vkq;
          VE(k, q) = s * vkp + c * vkq;
        }
      }
  }
  double w[n];
  for (int k = 0; k < n; ++k) w[k] = AE(k, k) > 0.0 ? AE(k, k) : 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      double acc = 0.0;
      for (int k = 0; k < n; ++k) acc += VE(i, k) * w[k] * VE(j, k);
      AE(i, j) = acc;
      AE(j, i) = acc;
    }
#undef AE
#undef VE
}

// Inverse of a symmetric positive-definite n x n matrix (row-major) by Gauss-Jordan with
// partial pivoting; returns false if a pivot vanishes.
template <int n>
TC_HD bool spd_inverse(const double* A, double* out) {
  double M[n * n];
  for (int k = 0; k < n * n; ++k) M[k] = A[k];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = i == j ? 1.0 : 0.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(M[r * n + c]) > fabs(M[piv * n + c])) piv = r;
    if (!(fabs(M[piv * n + c]) > 0.0)) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        double t = M[c * n + k]; M[c * n + k] = M[piv * n + k]; M[piv * n + k] = t;
        t = out[c * n + k]; out[c * n + k] = out[piv * n + k]; out[piv * n + k] = t;
      }
    const double inv = 1.0 / M[c * n + c];
    for (int k = 0; k < n; ++k) {
      M[c * n + k] *= inv;
      out[c * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        M[r * n + k] -= f * M[c * n + k];
        out[r * n + k] -= f * out[c * n + k];
      }
    }
  }
  return true;
}

}  // namespace tc
