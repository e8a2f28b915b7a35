// Point-triangle / edge-edge distances, the IPC log barrier and additive CCD
// (Taccel App. A.3; contact pairs from the surface meshes of soft and affine bodies).
//
// Local vertex order of a pair: point-triangle (PT) = [p, t0, t1, t2]; edge-edge (EE) =
// [a0, a1, b0, b1].  The squared distance s is evaluated with the closed form of the
// closest-feature type; its first and second derivatives are assembled from a few
// "reduced" variables (differences of vertex positions):
//   vertex-vertex  s = |r|^2                         r = x_i - x_j
//   vertex-edge    s = |r x e|^2 / |e|^2             r = p - a, e = b - a
//   vertex-plane / line-line
//                  s = (r . (e1 x e2))^2 / |e1 x e2|^2
// The barrier b(d) = -(d - dhat)^2 ln(d / dhat) on 0 < d < dhat acts on d = sqrt(s); an
// edge-edge pair is multiplied by the mollifier m(c) = 2c/eps - c^2/eps^2 (c < eps) of
// c = |(a1 - a0) x (b1 - b0)|^2, eps = 1e-3 |a1 - a0|^2_rest |b1 - b0|^2_rest, which removes
// the discontinuity of the edge-edge distance at parallel edges.
#pragma once
#include "dmath.h"

namespace tc {

enum { KIND_PT = 0, KIND_EE = 1 };

// Reduced-variable description of a distance type: nred differences, each a signed
// combination of the 4 local vertices (coefficients -1, 0, +1).
struct DistForm {
  int nred;
  signed char C[3][4];
};

TC_HD DistForm dist_form(int kind, int type) {
  DistForm f;
  for (int j = 0; j < 3; ++j)
    for (int v = 0; v < 4; ++v) f.C[j][v] = 0;
  auto diff = [&](int j, int plus, int minus) { f.C[j][plus] += 1; f.C[j][minus] -= 1; };
  if (kind == KIND_PT) {
    if (type < 3) { f.nred = 1; diff(0, 0, type + 1); }
    else if (type < 6) {
      const int a = type - 2, b = type == 5 ? 1 : type - 1;  // edges (1,2), (2,3), (3,1)
      f.nred = 2; diff(0, 0, a); diff(1, b, a);
    } else { f.nred = 3; diff(0, 0, 1); diff(1, 2, 1); diff(2, 3, 1); }
  } else {
    if (type < 4) { f.nred = 1; diff(0, type < 2 ? 0 : 1, (type & 1) ? 3 : 2); }
    else if (type < 6) { f.nred = 2; diff(0, type - 4, 2); diff(1, 3, 2); }
    else if (type < 8) { f.nred = 2; diff(0, type - 4, 0); diff(1, 1, 0); }
    else { f.nred = 3; diff(0, 2, 0); diff(1, 1, 0); diff(2, 3, 2); }
  }
  return f;
}

TC_HD d3 reduced(const DistForm& f, int j, const double* x12) {
  d3 r = mk(0, 0, 0);
  for (int v = 0; v < 4; ++v)
    if (f.C[j][v]) r = r + (double)f.C[j][v] * ld(x12 + 3 * v);
  return r;
}

// Closest-feature classification.
//  PT: 0..2 point-vertex t0,t1,t2; 3..5 point-edge t0t1, t1t2, t2t0; 6 point-plane.
//  EE: 0 a0b0, 1 a0b1, 2 a1b0, 3 a1b1; 4 a0-edge b, 5 a1-edge b, 6 b0-edge a, 7 b1-edge a;
//      8 line-line.
TC_HD int classify_pt(const double* x12) {
  const d3 p = ld(x12), t0 = ld(x12 + 3), t1 = ld(x12 + 6), t2 = ld(x12 + 9);
  const d3 e1 = t1 - t0, e2 = t2 - t0, r = p - t0;
  const double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
  const double b1 = dot(r, e1), b2 = dot(r, e2);
  const double det = a11 * a22 - a12 * a12;
  if (det > 0.0) {
    const double l1 = (a22 * b1 - a12 * b2) / det, l2 = (a11 * b2 - a12 * b1) / det;
    if (l1 >= 0.0 && l2 >= 0.0 && l1 + l2 <= 1.0) return 6;
  }
  const d3 T[3] = {t0, t1, t2};
  double best = INFINITY;
  int type = 0;
  for (int k = 0; k < 3; ++k) {
    const d3 a = T[k], b = T[(k + 1) % 3];
    const d3 e = b - a;
    double u = dot(p - a, e) / dot(e, e);
    u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
    const d3 q = a + u * e;
    const double s = dot(p - q, p - q);
    if (s < best) {
      best = s;
      type = u == 0.0 ? k : (u == 1.0 ? (k + 1) % 3 : 3 + k);
    }
  }
  return type;
}

TC_HD int classify_ee(const double* x12) {
  const d3 a0 = ld(x12), a1 = ld(x12 + 3), b0 = ld(x12 + 6), b1 = ld(x12 + 9);
  const d3 d1 = a1 - a0, d2 = b1 - b0, r = a0 - b0;
  const double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  const double c = dot(d1, r), b = dot(d1, d2);
  const double den = a * e - b * b;
  const d3 n = cross(d1, d2);
  double s = 0.0;
  if (dot(n, n) > 1e-20 * a * e) {
    s = (b * f - c * e) / den;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  }
  double t = (b * s + f) / e;
  if (t < 0.0) {
    t = 0.0;
    s = -c / a;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  } else if (t > 1.0) {
    t = 1.0;
    s = (b - c) / a;
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  }
  const bool s_in = s > 0.0 && s < 1.0, t_in = t > 0.0 && t < 1.0;
  if (s_in && t_in) return 8;
  if (!s_in && t_in) return s == 0.0 ? 4 : 5;
  if (s_in && !t_in) return t == 0.0 ? 6 : 7;
  return (s == 0.0 ? 0 : 2) + (t == 0.0 ? 0 : 1);
}

TC_HD int classify(int kind, const double* x12) {
  return kind == KIND_PT ? classify_pt(x12) : classify_ee(x12);
}

// Squared distance for a known type.
TC_HD double typed_sqdist(const DistForm& f, const double* x12) {
  const d3 r = reduced(f, 0, x12);
  if (f.nred == 1) return dot(r, r);
  const d3 e1 = reduced(f, 1, x12);
  if (f.nred == 2) {
    const d3 c = cross(r, e1);
    return dot(c, c) / dot(e1, e1);
  }
  const d3 e2 = reduced(f, 2, x12);
  const d3 n = cross(e1, e2);
  const double q = dot(r, n);
  return q * q / dot(n, n);
}

TC_HD double pair_sqdist(int kind, const double* x12, int* type_out) {
  const int type = classify(kind, x12);
  if (type_out) *type_out = type;
  return typed_sqdist(dist_form(kind, type), x12);
}

// |u x v|^2 with derivatives in (u, v): gradient g[6], Hessian blocks H[2][2][9].
TC_HD double cross_sq(const d3& u, const d3& v, double* g, double* H) {
  const double uu = dot(u, u), vv = dot(v, v), uv = dot(u, v);
  const d3 gu = 2.0 * (vv * u - uv * v), gv = 2.0 * (uu * v - uv * u);
  st(g, gu);
  st(g + 3, gv);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double dij = i == j ? 1.0 : 0.0;
      H[0 * 9 + 3 * i + j] = 2.0 * (vv * dij - at(v, i) * at(v, j));
      H[3 * 9 + 3 * i + j] = 2.0 * (uu * dij - at(u, i) * at(u, j));
      H[1 * 9 + 3 * i + j] = 4.0 * at(u, i) * at(v, j) - 2.0 * uv * dij - 2.0 * at(v, i) * at(u, j);
      H[2 * 9 + 3 * j + i] = H[1 * 9 + 3 * i + j];
    }
  return uu * vv - uv * uv;
}

// Derivatives of s for the form f in reduced space: g[3*nred], H[nred][nred][9] (blocks
// stored at H[(j*nred+k)*9]).
TC_HD double sqdist_reduced(const DistForm& f, const double* x12, double* g, double* H) {
  const d3 r = reduced(f, 0, x12);
  if (f.nred == 1) {
    st(g, 2.0 * r);
    for (int k = 0; k < 9; ++k) H[k] = (k % 4 == 0) ? 2.0 : 0.0;
    return dot(r, r);
  }
  const d3 e = reduced(f, 1, x12);
  if (f.nred == 2) {
    double gA[6], HA[36];
    const double A = cross_sq(r, e, gA, HA);
    const double B = dot(e, e);
    const double iB = 1.0 / B;
    const double gB[6] = {0, 0, 0, 2 * e.x, 2 * e.y, 2 * e.z};
    for (int k = 0; k < 6; ++k) g[k] = gA[k] * iB - A * gB[k] * iB * iB;
    for (int bj = 0; bj < 2; ++bj)
      for (int bk = 0; bk < 2; ++bk)
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            const int a = 3 * bj + i, c = 3 * bk + j;
            double v = HA[(2 * bj + bk) * 9 + 3 * i + j] * iB;
            v -= (gA[a] * gB[c] + gB[a] * gA[c]) * iB * iB;
            if (bj == 1 && bk == 1 && i == j) v -= A * 2.0 * iB * iB;
            v += 2.0 * A * gB[a] * gB[c] * iB * iB * iB;
            H[(2 * bj + bk) * 9 + 3 * i + j] = v;
          }
    return A * iB;
  }
  const d3 e2 = reduced(f, 2, x12);
  const d3 n = cross(e, e2);
  const double q = dot(r, n);
  double gq[9];
  st(gq, n);
  st(gq + 3, cross(e2, r));
  st(gq + 6, cross(r, e));
  double gN6[6], HN[36];
  const double N = cross_sq(e, e2, gN6, HN);
  const double gN[9] = {0, 0, 0, gN6[0], gN6[1], gN6[2], gN6[3], gN6[4], gN6[5]};
  const double iN = 1.0 / N;
  for (int k = 0; k < 9; ++k) g[k] = 2.0 * q * gq[k] * iN - q * q * gN[k] * iN * iN;
  // Hessian of q: (r,e1) = -[e2]x, (r,e2) = [e1]x, (e1,e2) = -[r]x (+ transposes).
  auto skew = [](const d3& v, int i, int j) -> double {
    // ([v]x)_ij
    if (i == j) return 0.0;
    const int k = 3 - i - j;
    const double s = ((j - i + 3) % 3 == 1) ? -1.0 : 1.0;
    return s * at(v, k);
  };
  for (int bj = 0; bj < 3; ++bj)
    for (int bk = 0; bk < 3; ++bk)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double hq = 0.0;
          if (bj == 0 && bk == 1) hq = -skew(e2, i, j);
          else if (bj == 1 && bk == 0) hq = -skew(e2, j, i);
          else if (bj == 0 && bk == 2) hq = skew(e, i, j);
          else if (bj == 2 && bk == 0) hq = skew(e, j, i);
          else if (bj == 1 && bk == 2) hq = -skew(r, i, j);
          else if (bj == 2 && bk == 1) hq = -skew(r, j, i);
          double hN = 0.0;
          if (bj > 0 && bk > 0) hN = HN[(2 * (bj - 1) + (bk - 1)) * 9 + 3 * i + j];
          const int a = 3 * bj + i, c = 3 * bk + j;
          double v = 2.0 * gq[a] * gq[c] * iN + 2.0 * q * hq * iN;
          v -= 2.0 * q * (gq[a] * gN[c] + gN[a] * gq[c]) * iN * iN;
          v -= q * q * hN * iN * iN;
          v += 2.0 * q * q * gN[a] * gN[c] * iN * iN * iN;
          H[(3 * bj + bk) * 9 + 3 * i + j] = v;
        }
  return q * q * iN;
}

// Barrier b(d) and its first two derivatives in d.
TC_HD void barrier_d(double d, double dhat, double* b, double* b1, double* b2) {
  const double t = d - dhat;
  const double L = log(d / dhat);
  *b = -t * t * L;
  *b1 = -2.0 * t * L - t * t / d;
  *b2 = -2.0 * L - 4.0 * t / d + t * t / (d * d);
}

// Entry (i, j) of the Hessian of |u x v|^2 in (u, v); bu, bv pick the blocks (0: u, 1: v).
TC_HD double cross_sq_hess(const d3& u, const d3& v, int bu, int bv, int i, int j) {
  const double dij = i == j ? 1.0 : 0.0;
  if (bu == 0 && bv == 0) return 2.0 * (dot(v, v) * dij - at(v, i) * at(v, j));
  if (bu == 1 && bv == 1) return 2.0 * (dot(u, u) * dij - at(u, i) * at(u, j));
  if (bu == 1) {  // (v, u) block is the transpose of the (u, v) block
    const int t = i; i = j; j = t;
  }
  return 4.0 * at(u, i) * at(v, j) - 2.0 * dot(u, v) * dij - 2.0 * at(v, i) * at(u, j);
}

// ([v]x)_ij, the cross-product matrix of v.
TC_HD double skew_entry(const d3& v, int i, int j) {
  if (i == j) return 0.0;
  const int k = 3 - i - j;
  const double sg = ((j - i + 3) % 3 == 1) ? -1.0 : 1.0;
  return sg * at(v, k);
}

// Everything one pair's barrier derivatives need besides per-entry arithmetic: the distance
// type, the reduced vectors and their first derivatives, and the chain-rule coefficients.
// Every lane of a wavefront evaluates it (it is a few hundred flops), then each lane forms
// its own Hessian entries with barrier_hess_entry.
struct BarrierCore {
  int kind, type, regime;  // regime 0: 0 < d < dhat; 1: s <= 0 (e = +inf); 2: d >= dhat (0)
  DistForm f;
  double e;         // kappa m b(d)
  double cs;        // kappa m b'(d) / (2d)           (multiplies Hess s)
  double cr;        // kappa m (b'' - b'/d) / (4s)    (multiplies grad s grad s^T)
  double cc;        // kappa m' b                     (multiplies Hess c)
  double cx;        // kappa m' b'(d) / (2d)          (grad s grad c^T + grad c grad s^T)
  double cm;        // kappa m'' b                    (grad c grad c^T)
  d3 r, e1, e2;     // reduced vectors
  d3 u, v;          // edge vectors (EE mollifier)
  double iB, A2, gA[6];         // nred 2: s = A2 iB, A2 = |r x e1|^2, B = |e1|^2
  double q, iN, gq[9], gN[9];   // nred 3: s = q^2 iN, q = r.(e1 x e2), N = |e1 x e2|^2
  double gs[12], gc12[12];      // grad s, grad c in the 12 local coordinates
};

TC_HD void barrier_core(int kind, const double* x12, double meps, double dhat, double kappa,
                        BarrierCore& B) {
  B.kind = kind;
  B.type = classify(kind, x12);
  const DistForm& f = B.f = dist_form(kind, B.type);
  B.r = reduced(f, 0, x12);
  B.e1 = f.nred > 1 ? reduced(f, 1, x12) : mk(0, 0, 0);
  B.e2 = f.nred > 2 ? reduced(f, 2, x12) : mk(0, 0, 0);
  double gr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double s;
  if (f.nred == 1) {
    st(gr, 2.0 * B.r);
    s = dot(B.r, B.r);
  } else if (f.nred == 2) {
    double HA[36];
    B.A2 = cross_sq(B.r, B.e1, B.gA, HA);
    B.iB = 1.0 / dot(B.e1, B.e1);
    const double gB[6] = {0, 0, 0, 2 * B.e1.x, 2 * B.e1.y, 2 * B.e1.z};
    for (int k = 0; k < 6; ++k) gr[k] = B.gA[k] * B.iB - B.A2 * gB[k] * B.iB * B.iB;
    s = B.A2 * B.iB;
  } else {
    const d3 n = cross(B.e1, B.e2);
    B.q = dot(B.r, n);
    st(B.gq, n);
    st(B.gq + 3, cross(B.e2, B.r));
    st(B.gq + 6, cross(B.r, B.e1));
    double gN6[6], HN[36];
    const double N = cross_sq(B.e1, B.e2, gN6, HN);
    B.gN[0] = B.gN[1] = B.gN[2] = 0.0;
    for (int k = 0; k < 6; ++k) B.gN[3 + k] = gN6[k];
    B.iN = 1.0 / N;
    for (int k = 0; k < 9; ++k) gr[k] = 2.0 * B.q * B.gq[k] * B.iN - B.q * B.q * B.gN[k] * B.iN * B.iN;
    s = B.q * B.q * B.iN;
  }
  for (int k = 0; k < 12; ++k) B.gs[k] = B.gc12[k] = 0.0;
  B.e = B.cs = B.cr = B.cc = B.cx = B.cm = 0.0;
  if (!(s > 0.0)) { B.regime = 1; B.e = INFINITY; return; }
  const double d = sqrt(s);
  if (d >= dhat) { B.regime = 2; return; }
  B.regime = 0;
  double b, b1, b2;
  barrier_d(d, dhat, &b, &b1, &b2);
  const double Bs = b1 / (2.0 * d), Bss = (b2 - b1 / d) / (4.0 * s);
  double m = 1.0, m1 = 0.0, m2 = 0.0;
  if (kind == KIND_EE) {
    B.u = ld(x12 + 3) - ld(x12);
    B.v = ld(x12 + 9) - ld(x12 + 6);
    double gc[6], Hc[36];
    const double c = cross_sq(B.u, B.v, gc, Hc);
    if (c < meps) {
      m = 2.0 * c / meps - c * c / (meps * meps);
      m1 = 2.0 / meps - 2.0 * c / (meps * meps);
      m2 = -2.0 / (meps * meps);
    }
    for (int i = 0; i < 3; ++i) {
      B.gc12[i] = -gc[i];
      B.gc12[3 + i] = gc[i];
      B.gc12[6 + i] = -gc[3 + i];
      B.gc12[9 + i] = gc[3 + i];
    }
  }
  for (int j = 0; j < f.nred; ++j)
    for (int v = 0; v < 4; ++v)
      if (f.C[j][v])
        for (int i = 0; i < 3; ++i) B.gs[3 * v + i] += f.C[j][v] * gr[3 * j + i];
  B.e = kappa * m * b;
  B.cs = kappa * m * Bs;
  B.cr = kappa * m * Bss;
  B.cc = kappa * m1 * b;
  B.cx = kappa * m1 * Bs;
  B.cm = kappa * m2 * b;
}

// Entry (a, c) of block (j, k) of the Hessian of s in reduced space.
TC_HD double sqdist_reduced_hess(const BarrierCore& B, int j, int k, int a, int c) {
  const int nred = B.f.nred;
  if (nred == 1) return a == c ? 2.0 : 0.0;
  if (nred == 2) {
    const int ia = 3 * j + a, ic = 3 * k + c;
    const double gBa = j == 1 ? 2.0 * at(B.e1, a) : 0.0, gBc = k == 1 ? 2.0 * at(B.e1, c) : 0.0;
    double v = cross_sq_hess(B.r, B.e1, j, k, a, c) * B.iB;
    v -= (B.gA[ia] * gBc + gBa * B.gA[ic]) * B.iB * B.iB;
    if (j == 1 && k == 1 && a == c) v -= B.A2 * 2.0 * B.iB * B.iB;
    v += 2.0 * B.A2 * gBa * gBc * B.iB * B.iB * B.iB;
    return v;
  }
  // Hessian of q: (r,e1) = -[e2]x, (r,e2) = [e1]x, (e1,e2) = -[r]x (and transposes)
  double hq = 0.0;
  if (j == 0 && k == 1) hq = -skew_entry(B.e2, a, c);
  else if (j == 1 && k == 0) hq = -skew_entry(B.e2, c, a);
  else if (j == 0 && k == 2) hq = skew_entry(B.e1, a, c);
  else if (j == 2 && k == 0) hq = skew_entry(B.e1, c, a);
  else if (j == 1 && k == 2) hq = -skew_entry(B.r, a, c);
  else if (j == 2 && k == 1) hq = -skew_entry(B.r, c, a);
  const double hN = (j > 0 && k > 0) ? cross_sq_hess(B.e1, B.e2, j - 1, k - 1, a, c) : 0.0;
  const int ia = 3 * j + a, ic = 3 * k + c;
  const double q = B.q, iN = B.iN;
  double v = 2.0 * B.gq[ia] * B.gq[ic] * iN + 2.0 * q * hq * iN;
  v -= 2.0 * q * (B.gq[ia] * B.gN[ic] + B.gN[ia] * B.gq[ic]) * iN * iN;
  v -= q * q * hN * iN * iN;
  v += 2.0 * q * q * B.gN[ia] * B.gN[ic] * iN * iN * iN;
  return v;
}

// Gradient entry A (0..11) of kappa m b(d).
TC_HD double barrier_grad_entry(const BarrierCore& B, int A) {
  return B.cs * B.gs[A] + B.cc * B.gc12[A];
}

// Unprojected Hessian entry (A, C) of kappa m b(d) in the 12 local coordinates.
TC_HD double barrier_hess_entry(const BarrierCore& B, int A, int C) {
  if (B.regime != 0) return 0.0;
  const int va = A / 3, a = A % 3, vc = C / 3, c = C % 3;
  const DistForm& f = B.f;
  double h = 0.0;
  for (int j = 0; j < f.nred; ++j) {
    if (!f.C[j][va]) continue;
    for (int k = 0; k < f.nred; ++k) {
      if (!f.C[k][vc]) continue;
      h += B.cs * f.C[j][va] * f.C[k][vc] * sqdist_reduced_hess(B, j, k, a, c);
    }
  }
  if (B.kind == KIND_EE && B.cc != 0.0) {
    // c depends on u = x1 - x0 (block 0) and v = x3 - x2 (block 1)
    const signed char Cc[2][4] = {{-1, 1, 0, 0}, {0, 0, -1, 1}};
    for (int j = 0; j < 2; ++j) {
      if (!Cc[j][va]) continue;
      for (int k = 0; k < 2; ++k) {
        if (!Cc[k][vc]) continue;
        h += B.cc * Cc[j][va] * Cc[k][vc] * cross_sq_hess(B.u, B.v, j, k, a, c);
      }
    }
  }
  h += B.cr * B.gs[A] * B.gs[C];
  if (B.kind == KIND_EE) {
    h += B.cx * (B.gs[A] * B.gc12[C] + B.gc12[A] * B.gs[C]);
    h += B.cm * B.gc12[A] * B.gc12[C];
  }
  return h;
}

// Barrier energy only (line search).  +inf if s <= 0, 0 if d >= dhat.
TC_HD double barrier_energy(int kind, const double* x12, double meps, double dhat, double kappa) {
  const double s = pair_sqdist(kind, x12, nullptr);
  if (!(s > 0.0)) return INFINITY;
  const double d = sqrt(s);
  if (d >= dhat) return 0.0;
  double b, b1, b2;
  barrier_d(d, dhat, &b, &b1, &b2);
  double m = 1.0;
  if (kind == KIND_EE) {
    const d3 u = ld(x12 + 3) - ld(x12), v = ld(x12 + 9) - ld(x12 + 6);
    const d3 n = cross(u, v);
    const double c = dot(n, n);
    if (c < meps) m = 2.0 * c / meps - c * c / (meps * meps);
  }
  return kappa * m * b;
}

// ------------------------------------------------------------------ friction (App. A.3)
// The closest-point difference c = sum_v w_v x_v of a pair's closest features (first
// primitive minus second; |c| is the distance) as weights w of the four local vertices, for
// the distance type `type` returned by classify().
TC_HD void closest_point_weights(int kind, int type, const double* x12, double* w) {
  const d3 P[4] = {ld(x12), ld(x12 + 3), ld(x12 + 6), ld(x12 + 9)};
  for (int v = 0; v < 4; ++v) w[v] = 0.0;
  if (kind == KIND_PT) {
    w[0] = 1.0;
    if (type < 3) {
      w[1 + type] = -1.0;
    } else if (type < 6) {  // edges (1,2), (2,3), (3,1)
      const int a = type - 2, b = type == 5 ? 1 : type - 1;
      const d3 e = P[b] - P[a];
      const double u = dot(P[0] - P[a], e) / dot(e, e);
      w[a] = -(1.0 - u);
      w[b] = -u;
    } else {  // projection onto the plane, in barycentric coordinates
      const d3 e1 = P[2] - P[1], e2 = P[3] - P[1], r = P[0] - P[1];
      const double a11 = dot(e1, e1), a12 = dot(e1, e2), a22 = dot(e2, e2);
      const double b1 = dot(r, e1), b2 = dot(r, e2);
      const double det = a11 * a22 - a12 * a12;
      const double l1 = (a22 * b1 - a12 * b2) / det, l2 = (a11 * b2 - a12 * b1) / det;
      w[1] = -(1.0 - l1 - l2);
      w[2] = -l1;
      w[3] = -l2;
    }
    return;
  }
  if (type < 4) {
    w[type < 2 ? 0 : 1] = 1.0;
    w[(type & 1) ? 3 : 2] = -1.0;
  } else if (type < 6) {  // a0 or a1 against edge b
    const d3 e = P[3] - P[2];
    const double t = dot(P[type - 4] - P[2], e) / dot(e, e);
    w[type - 4] = 1.0;
    w[2] = -(1.0 - t);
    w[3] = -t;
  } else if (type < 8) {  // b0 or b1 against edge a
    const d3 e = P[1] - P[0];
    const double t = dot(P[type - 4] - P[0], e) / dot(e, e);
    w[0] = 1.0 - t;
    w[1] = t;
    w[type - 4] = -1.0;
  } else {  // stationary point of |a0 + s d1 - b0 - t d2|^2
    const d3 d1 = P[1] - P[0], d2 = P[3] - P[2], r = P[0] - P[2];
    const double a = dot(d1, d1), b = dot(d1, d2), e = dot(d2, d2);
    const double c = dot(d1, r), f = dot(d2, r);
    const double den = a * e - b * b;
    const double sa = (b * f - c * e) / den, tb = (a * f - b * c) / den;
    w[0] = 1.0 - sa;
    w[1] = sa;
    w[2] = -(1.0 - tb);
    w[3] = -tb;
  }
}

// Magnitude of a pair's barrier normal force, -kappa m b'(d), at squared distance s (the
// edge-edge mollifier value m taken at x12).
TC_HD double normal_force(int kind, const double* x12, double s, double meps, double dhat,
                          double kappa) {
  double b, b1, b2;
  barrier_d(sqrt(s), dhat, &b, &b1, &b2);
  double m = 1.0;
  if (kind == KIND_EE) {
    const d3 n = cross(ld(x12 + 3) - ld(x12), ld(x12 + 9) - ld(x12 + 6));
    const double c = dot(n, n);
    if (c < meps) m = 2.0 * c / meps - c * c / (meps * meps);
  }
  return -kappa * m * b1;
}

// f0 of the friction mollifier at y = |u| with eh = eps_v h: the integral of f1 (f1(y) =
// 2y/eh - y^2/eh^2 below eh, 1 above) from eh to y, plus eh.
TC_HD double friction_f0(double y, double eh) {
  return y < eh ? y * y * (1.0 / eh - y / (3.0 * eh * eh)) + eh / 3.0 : y;
}
// f1(y)/y and f1'(y) (their common limit 2/eh at y = 0).
TC_HD void friction_f1(double y, double eh, double* f1y, double* df1) {
  if (y < eh) {
    *f1y = 2.0 / eh - y / (eh * eh);
    *df1 = 2.0 / eh - 2.0 * y / (eh * eh);
  } else {
    *f1y = 1.0 / y;
    *df1 = 0.0;
  }
}

// Tangential part u of (sum_v w_v x_v - c0) for the lagged normal n.
TC_HD d3 friction_u(const double* x12, const double* w, const d3& c0, const d3& n) {
  d3 dl = mk(0, 0, 0);
  for (int v = 0; v < 4; ++v) dl = dl + w[v] * ld(x12 + 3 * v);
  dl = dl - c0;
  return dl - dot(n, dl) * n;
}

// Gradient g[12] and Hessian H[144] of mul * f0(|u|) with u = (I - n n^T)(sum w_v x_v - c0):
// g_v = mul w_v (f1/y) u, H_ab = mul w_a w_b [ (f1/y) (I - n n^T) + (f1' - f1/y) uh uh^T ]
// (uh = u/|u|; the second term vanishes at u = 0).  Positive semidefinite: f1' >= 0 and
// f1/y > 0.  Returns the energy.
TC_HD double friction_derivs(const double* x12, const double* w, const d3& c0, const d3& n,
                             double mul, double eh, double* g, double* H) {
  const d3 u = friction_u(x12, w, c0, n);
  const double y = sqrt(dot(u, u));
  double f1y, df1;
  friction_f1(y, eh, &f1y, &df1);
  const d3 uh = y > 0.0 ? (1.0 / y) * u : mk(0, 0, 0);
  double H3[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      H3[3 * i + j] = f1y * ((i == j ? 1.0 : 0.0) - at(n, i) * at(n, j)) + (df1 - f1y) * at(uh, i) * at(uh, j);
  for (int a = 0; a < 4; ++a) {
    st(g + 3 * a, (mul * w[a] * f1y) * u);
    for (int b = 0; b < 4; ++b) {
      const double s = mul * w[a] * w[b];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) H[12 * (3 * a + i) + 3 * b + j] = s * H3[3 * i + j];
    }
  }
  return mul * friction_f0(y, eh);
}

// Additive CCD by conservative advancement: with the common mean displacement removed, the
// pair distance shrinks at most at rate lp = (largest displacement on one side) + (largest
// on the other).  Advance by a fraction of distance / lp; stop before the distance falls
// below gap_ratio * d(0), return 1 once the whole step is covered.  max_iter bounds the
// loop (the time reached so far is returned, which is still safe).
// stop_at (nullable): the running minimum over other pairs (a double's bits, non-negative);
// once t reaches it, this pair cannot lower the minimum and the loop ends early (the
// minimum over all pairs is unchanged).
TC_HD double accd(int kind, const double* x12, const double* p12, double gap_ratio, int max_iter,
                  const unsigned long long* stop_at = nullptr) {
  double q[12];
  for (int c = 0; c < 3; ++c) {
    const double mean = 0.25 * (p12[c] + p12[3 + c] + p12[6 + c] + p12[9 + c]);
    for (int v = 0; v < 4; ++v) q[3 * v + c] = p12[3 * v + c] - mean;
  }
  double len[4];
  for (int v = 0; v < 4; ++v) len[v] = sqrt(q[3 * v] * q[3 * v] + q[3 * v + 1] * q[3 * v + 1] + q[3 * v + 2] * q[3 * v + 2]);
  const double lp = kind == KIND_PT ? len[0] + fmax(len[1], fmax(len[2], len[3]))
                                    : fmax(len[0], len[1]) + fmax(len[2], len[3]);
  if (lp == 0.0) return 1.0;
  const double d0 = sqrt(pair_sqdist(kind, x12, nullptr));
  if (!(d0 > 0.0)) return 0.0;
  const double gap = gap_ratio * d0;
  double t = 0.0, step = (1.0 - gap_ratio) * d0 / lp;
  double xt[12];
  for (int it = 0; it < max_iter; ++it) {
    const double tn = t + step;
    for (int k = 0; k < 12; ++k) xt[k] = x12[k] + tn * q[k];
    const double d = sqrt(pair_sqdist(kind, xt, nullptr));
    if (it > 0 && d < gap) return t;
    t = tn;
    if (t > 1.0) return 1.0;
    step = 0.9 * d / lp;
    if (stop_at && (it & 15) == 15) {
      const unsigned long long bits = *(volatile const unsigned long long*)stop_at;
      double m;
      __builtin_memcpy(&m, &bits, sizeof(double));
      if (t >= m) return t;
    }
  }
  return t;
}

}  // namespace tc
