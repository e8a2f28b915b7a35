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
// Scalar traits of the templated 3x3 routines: the Jacobi stopping ratio (off-diagonal over
// diagonal mass, about the square of the unit roundoff) and a tiny positive norm.
template <class R> struct Tiny;
template <> struct Tiny<double> {
  static constexpr double jacobi = 1e-34, norm = 1e-300;
};
template <> struct Tiny<float> {
  static constexpr float jacobi = 1e-14f, norm = 1e-30f;
};

template <class R>
TC_HD R det3(const R* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
         A[2] * (A[3] * A[7] - A[4] * A[6]);
}
// Cofactor matrix (= det(A) * A^{-T}).
template <class R>
TC_HD void cofactor3(const R* A, R* C) {
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
template <class R>
TC_HD void matmul3(const R* A, const R* B, R* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
// C = A * B^T
template <class R>
TC_HD void matmul3_bt(const R* A, const R* B, R* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations.  A is row-major and is
// destroyed; on return w holds the eigenvalues and V (row-major) the eigenvectors as
// columns.
template <class R>
TC_HD void sym_eig3(R* A, R* w, R* V) {
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? R(1) : R(0);
  for (int sweep = 0; sweep < 10; ++sweep) {
    const R off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    const R dia = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
    if (off <= Tiny<R>::jacobi * dia || off == R(0)) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const R apq = A[3 * p + q];
      if (apq == R(0)) continue;
      const R theta = (A[3 * q + q] - A[3 * p + p]) / (R(2) * apq);
      const R t = (theta >= R(0) ? R(1) : R(-1)) / (fabs(theta) + sqrt(theta * theta + R(1)));
      const R c = R(1) / sqrt(t * t + R(1)), s = t * c;
      for (int k = 0; k < 3; ++k) {
        const R akp = A[3 * k + p], akq = A[3 * k + q];
        A[3 * k + p] = c * akp - s * akq;
        A[3 * k + q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        const R apk = A[3 * p + k], aqk = A[3 * q + k];
        A[3 * p + k] = c * apk - s * aqk;
        A[3 * q + k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        const R vkp = V[3 * k + p], vkq = V[3 * k + q];
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
template <class R>
TC_HD void svd3(const R* F, R* U, R* s, R* V) {
  R A[9], w[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      A[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
  sym_eig3(A, w, V);
  // sort eigenpairs by decreasing eigenvalue
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2 - a; ++b)
      if (w[b] < w[b + 1]) {
        const R tw = w[b]; w[b] = w[b + 1]; w[b + 1] = tw;
        for (int k = 0; k < 3; ++k) {
          const R tv = V[3 * k + b]; V[3 * k + b] = V[3 * k + b + 1]; V[3 * k + b + 1] = tv;
        }
      }
  if (det3(V) < R(0))
    for (int k = 0; k < 3; ++k) V[3 * k + 2] = -V[3 * k + 2];
  R B[9];
  matmul3(F, V, B);
  // columns b_j of F V; u0 = b0 / |b0|, u1 from b1 orthogonalised against u0, u2 = u0 x u1
  const R b0[3] = {B[0], B[3], B[6]}, b1[3] = {B[1], B[4], B[7]}, b2[3] = {B[2], B[5], B[8]};
  const R n0 = sqrt(b0[0] * b0[0] + b0[1] * b0[1] + b0[2] * b0[2]);
  R u0[3];
  if (n0 > R(0)) {
    for (int k = 0; k < 3; ++k) u0[k] = b0[k] / n0;
  } else {
    u0[0] = R(1); u0[1] = R(0); u0[2] = R(0);
  }
  const R d01 = u0[0] * b1[0] + u0[1] * b1[1] + u0[2] * b1[2];
  R r1[3];
  for (int k = 0; k < 3; ++k) r1[k] = b1[k] - d01 * u0[k];
  const R n1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
  R u1[3];
  if (n1 > Tiny<R>::norm) {
    for (int k = 0; k < 3; ++k) u1[k] = r1[k] / n1;
  } else {  // any unit vector orthogonal to u0
    R t[3] = {R(0), R(0), R(0)};
    t[fabs(u0[0]) < R(0.9) ? 0 : 1] = R(1);
    const R d = u0[0] * t[0] + u0[1] * t[1] + u0[2] * t[2];
    for (int k = 0; k < 3; ++k) t[k] -= d * u0[k];
    const R nt = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    for (int k = 0; k < 3; ++k) u1[k] = t[k] / nt;
  }
  const R u2[3] = {u0[1] * u1[2] - u0[2] * u1[1], u0[2] * u1[0] - u0[0] * u1[2],
                   u0[0] * u1[1] - u0[1] * u1[0]};
  s[0] = n0;
  s[1] = u1[0] * b1[0] + u1[1] * b1[1] + u1[2] * b1[2];
  s[2] = u2[0] * b2[0] + u2[1] * b2[1] + u2[2] * b2[2];
  for (int k = 0; k < 3; ++k) {
    U[3 * k] = u0[k];
    U[3 * k + 1] = u1[k];
    U[3 * k + 2] = u2[k];
  }
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
