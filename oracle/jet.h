// Second-order forward-mode numbers ("jets") for the CPU oracle.
//
// TEST INFRASTRUCTURE ONLY: this oracle checks the GPU library; nothing in the product
// path may include, link or call it.
//
// A Jet<N> carries a value, its gradient and its full Hessian with respect to N seed
// variables.  Every energy of the method (neo-Hookean density, barrier of a contact pair,
// ARAP term of an affine body) is written once as a template over the scalar type and
// evaluated in Jet arithmetic, which yields exact first and second derivatives without any
// hand-derived formula.  This keeps the oracle independent of the closed forms used by
// the GPU kernels.
#pragma once
#include <cmath>
#include <cstring>

namespace oracle {

template <int N>
struct Jet {
  double v;
  double g[N];
  double h[N][N];

  Jet() : v(0.0) {
    std::memset(g, 0, sizeof(g));
    std::memset(h, 0, sizeof(h));
  }
  Jet(double c) : v(c) {  // NOLINT: implicit constant promotion is intended
    std::memset(g, 0, sizeof(g));
    std::memset(h, 0, sizeof(h));
  }
  static Jet variable(double value, int i) {
    Jet r(value);
    r.g[i] = 1.0;
    return r;
  }
};

template <int N>
inline Jet<N> operator+(const Jet<N>& a, const Jet<N>& b) {
  Jet<N> r;
  r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] + b.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] + b.h[i][j];
  return r;
}
template <int N>
inline Jet<N> operator-(const Jet<N>& a, const Jet<N>& b) {
  Jet<N> r;
  r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.g[i] - b.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = a.h[i][j] - b.h[i][j];
  return r;
}
template <int N>
inline Jet<N> operator-(const Jet<N>& a) {
  Jet<N> r;
  r.v = -a.v;
  for (int i = 0; i < N; ++i) r.g[i] = -a.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = -a.h[i][j];
  return r;
}
template <int N>
inline Jet<N> operator*(const Jet<N>& a, const Jet<N>& b) {
  Jet<N> r;
  r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      r.h[i][j] = a.v * b.h[i][j] + b.v * a.h[i][j] + a.g[i] * b.g[j] + b.g[i] * a.g[j];
  return r;
}
template <int N>
inline Jet<N> operator*(double c, const Jet<N>& a) {
  Jet<N> r;
  r.v = c * a.v;
  for (int i = 0; i < N; ++i) r.g[i] = c * a.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = c * a.h[i][j];
  return r;
}
template <int N>
inline Jet<N> operator*(const Jet<N>& a, double c) { return c * a; }
template <int N>
inline Jet<N> operator+(const Jet<N>& a, double c) { Jet<N> r = a; r.v += c; return r; }
template <int N>
inline Jet<N> operator+(double c, const Jet<N>& a) { return a + c; }
template <int N>
inline Jet<N> operator-(const Jet<N>& a, double c) { Jet<N> r = a; r.v -= c; return r; }
template <int N>
inline Jet<N> operator-(double c, const Jet<N>& a) { return (-a) + c; }

// Chain rule for a scalar function f with value f0, first derivative f1, second f2 at a.v.
template <int N>
inline Jet<N> chain(const Jet<N>& a, double f0, double f1, double f2) {
  Jet<N> r;
  r.v = f0;
  for (int i = 0; i < N; ++i) r.g[i] = f1 * a.g[i];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) r.h[i][j] = f1 * a.h[i][j] + f2 * a.g[i] * a.g[j];
  return r;
}
template <int N>
inline Jet<N> inv(const Jet<N>& a) {
  const double x = a.v;
  return chain(a, 1.0 / x, -1.0 / (x * x), 2.0 / (x * x * x));
}
template <int N>
inline Jet<N> operator/(const Jet<N>& a, const Jet<N>& b) { return a * inv(b); }
template <int N>
inline Jet<N> operator/(double c, const Jet<N>& a) { return c * inv(a); }
template <int N>
inline Jet<N> operator/(const Jet<N>& a, double c) { return (1.0 / c) * a; }
template <int N>
inline Jet<N> log(const Jet<N>& a) {
  const double x = a.v;
  return chain(a, std::log(x), 1.0 / x, -1.0 / (x * x));
}
template <int N>
inline Jet<N> sqrt(const Jet<N>& a) {
  const double s = std::sqrt(a.v);
  return chain(a, s, 0.5 / s, -0.25 / (s * a.v));
}

// Plain-double overloads so the same templates evaluate with T = double.
inline double value_of(double x) { return x; }
template <int N>
inline double value_of(const Jet<N>& x) { return x.v; }

}  // namespace oracle
