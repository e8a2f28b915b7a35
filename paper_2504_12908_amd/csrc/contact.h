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

// Energy kappa * m * b(d) of one pair with its 12-gradient and (unprojected) 12x12 Hessian,
// the Hessian written at H[(i*12+j)*stride].  Returns the distance type; *e = +inf when
// s <= 0 and 0 (with zero derivatives) when d >= dhat.  work: kBarrierWork doubles of
// scratch (on the GPU a slice of LDS, so the temporaries never go to private memory).
constexpr int kBarrierWork = 160;
TC_HD int barrier_pair(int kind, const double* x12, double meps, double dhat, double kappa,
                       double* e, double* g12, double* H, int stride, double* work) {
  const int type = classify(kind, x12);
  const DistForm f = dist_form(kind, type);
  for (int k = 0; k < 12; ++k) g12[k] = 0.0;
  for (int k = 0; k < 144; ++k) H[k * stride] = 0.0;
  double* gr = work;         // 9
  double* Hr = work + 9;     // 81
  double* gc12 = work + 90;  // 12
  double* Hc = work + 102;   // 36
  double* gs = work + 138;   // 12
  const double s = sqdist_reduced(f, x12, gr, Hr);
  if (!(s > 0.0)) { *e = INFINITY; return type; }
  const double d = sqrt(s);
  if (d >= dhat) { *e = 0.0; return type; }
  double b, b1, b2;
  barrier_d(d, dhat, &b, &b1, &b2);
  const double Bs = b1 / (2.0 * d), Bss = (b2 - b1 / d) / (4.0 * s);
  double m = 1.0, m1 = 0.0, m2 = 0.0;
  for (int k = 0; k < 12; ++k) gc12[k] = 0.0;
  if (kind == KIND_EE) {
    const d3 u = ld(x12 + 3) - ld(x12), v = ld(x12 + 9) - ld(x12 + 6);
    double gc[6];
    const double c = cross_sq(u, v, gc, Hc);
    if (c < meps) {
      m = 2.0 * c / meps - c * c / (meps * meps);
      m1 = 2.0 / meps - 2.0 * c / (meps * meps);
      m2 = -2.0 / (meps * meps);
    }
    for (int i = 0; i < 3; ++i) {
      gc12[i] = -gc[i];
      gc12[3 + i] = gc[i];
      gc12[6 + i] = -gc[3 + i];
      gc12[9 + i] = gc[3 + i];
    }
  }
  // grad of s in 12-space
  for (int k = 0; k < 12; ++k) gs[k] = 0.0;
  for (int j = 0; j < f.nred; ++j)
    for (int v = 0; v < 4; ++v)
      if (f.C[j][v])
        for (int i = 0; i < 3; ++i) gs[3 * v + i] += f.C[j][v] * gr[3 * j + i];
  *e = kappa * m * b;
  for (int k = 0; k < 12; ++k) g12[k] = kappa * (m * Bs * gs[k] + m1 * b * gc12[k]);
  // kappa * m * Bs * Hess(s), pulled back from reduced space
  const double cs = kappa * m * Bs;
  for (int j = 0; j < f.nred; ++j)
    for (int k = 0; k < f.nred; ++k)
      for (int v = 0; v < 4; ++v) {
        if (!f.C[j][v]) continue;
        for (int w = 0; w < 4; ++w) {
          if (!f.C[k][w]) continue;
          const double cf = cs * f.C[j][v] * f.C[k][w];
          for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c)
              H[((3 * v + a) * 12 + 3 * w + c) * stride] += cf * Hr[(j * f.nred + k) * 9 + 3 * a + c];
        }
      }
  if (kind == KIND_EE && m1 != 0.0) {
    // kappa * m1 * b * Hess(c); c depends on u = x1 - x0 (block 0) and v = x3 - x2 (block 1)
    const signed char Cc[2][4] = {{-1, 1, 0, 0}, {0, 0, -1, 1}};
    const double cc = kappa * m1 * b;
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k)
        for (int v = 0; v < 4; ++v) {
          if (!Cc[j][v]) continue;
          for (int w = 0; w < 4; ++w) {
            if (!Cc[k][w]) continue;
            const double cf = cc * Cc[j][v] * Cc[k][w];
            for (int a = 0; a < 3; ++a)
              for (int c = 0; c < 3; ++c)
                H[((3 * v + a) * 12 + 3 * w + c) * stride] += cf * Hc[(2 * j + k) * 9 + 3 * a + c];
          }
        }
  }
  for (int a = 0; a < 12; ++a)
    for (int c = 0; c < 12; ++c) {
      double v = kappa * m * Bss * gs[a] * gs[c];
      if (kind == KIND_EE) {
        v += kappa * m1 * Bs * (gs[a] * gc12[c] + gc12[a] * gs[c]);
        v += kappa * m2 * b * gc12[a] * gc12[c];
      }
      H[(a * 12 + c) * stride] += v;
    }
  return type;
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

// Additive CCD by conservative advancement: with the common mean displacement removed, the
// pair distance shrinks at most at rate lp = (largest displacement on one side) + (largest
// on the other).  Advance by a fraction of distance / lp; stop before the distance falls
// below gap_ratio * d(0), return 1 once the whole step is covered.  max_iter bounds the
// loop (the time reached so far is returned, which is still safe).
TC_HD double accd(int kind, const double* x12, const double* p12, double gap_ratio, int max_iter) {
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
  }
  return t;
}

}  // namespace tc
