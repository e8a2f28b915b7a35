// Tactile outputs (Taccel Sec. 4.2).  Markers: one thread per marker.  Depth map: one
// wavefront per triangle walks the pixels of its bounding box (a scatter with 64-bit atomic
// minima on an order-preserving key of the ray parameter, then on the triangle index), so the
// result does not depend on the order in which wavefronts run.  The coverage and depth
// arithmetic is evaluated exactly as written (FP contraction off), which makes every pixel
// decision reproducible by any IEEE FP64 evaluation of the same expressions.
#include "tactile.h"

#include <climits>
#include <cmath>

namespace tc {
namespace {

__device__ __forceinline__ int gidx() { return blockIdx.x * blockDim.x + threadIdx.x; }

__device__ __forceinline__ void project(const Camera& c, const double* p, double& u, double& v,
                                        double& t) {
#pragma clang fp contract(off)
  const double dx = p[0] - c.o[0], dy = p[1] - c.o[1], dz = p[2] - c.o[2];
  u = (dx * c.eu[0] + dy * c.eu[1]) + dz * c.eu[2];
  v = (dx * c.ev[0] + dy * c.ev[1]) + dz * c.ev[2];
  t = (dx * c.en[0] + dy * c.en[1]) + dz * c.en[2];
}

// Does the projected triangle (U, V) contain (a, b) (edges included)?  If so, *t is the ray
// parameter there, interpolated from T.
__device__ __forceinline__ bool covers(const double* U, const double* V, const double* T, double a,
                                       double b, double* t) {
#pragma clang fp contract(off)
  const double w0 = (U[1] - a) * (V[2] - b) - (U[2] - a) * (V[1] - b);
  const double w1 = (U[2] - a) * (V[0] - b) - (U[0] - a) * (V[2] - b);
  const double w2 = (U[0] - a) * (V[1] - b) - (U[1] - a) * (V[0] - b);
  const double A = (w0 + w1) + w2;
  bool in = false;
  if (A > 0.0) in = w0 >= 0.0 && w1 >= 0.0 && w2 >= 0.0;
  else if (A < 0.0) in = w0 <= 0.0 && w1 <= 0.0 && w2 <= 0.0;
  if (in) *t = ((w0 * T[0] + w1 * T[1]) + w2 * T[2]) / A;
  return in;
}

// Unsigned key with the order of the doubles (negative values below positive ones).
__device__ __forceinline__ unsigned long long order_key(double t) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(t);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}
__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
  return __longlong_as_double((long long)b);
}
constexpr unsigned long long kEmpty = ~0ull;

__global__ void k_markers(int m, const int* mnode, const double* bary, const double* x,
                          const double* xr, double* pos, double* flow) {
#pragma clang fp contract(off)
  const int k = gidx();
  if (k >= m) return;
  const int n0 = mnode[3 * k], n1 = mnode[3 * k + 1], n2 = mnode[3 * k + 2];
  const double b0 = bary[3 * k], b1 = bary[3 * k + 1], b2 = bary[3 * k + 2];
  for (int c = 0; c < 3; ++c) {
    const double p = (b0 * x[3 * n0 + c] + b1 * x[3 * n1 + c]) + b2 * x[3 * n2 + c];
    const double r = (b0 * xr[3 * n0 + c] + b1 * xr[3 * n1 + c]) + b2 * xr[3 * n2 + c];
    pos[3 * k + c] = p;
    flow[3 * k + c] = p - r;
  }
}

__global__ void k_depth_clear(int npix, unsigned long long* zkey, int* zidx) {
  const int k = gidx();
  if (k >= npix) return;
  zkey[k] = kEmpty;
  zidx[k] = INT_MAX;
}

__global__ void __launch_bounds__(64) k_depth_raster(Camera c, int ntri, const int* tnode,
                                                     const double* x, unsigned long long* zkey,
                                                     int* zidx, int pass) {
  const int tri = blockIdx.x;
  if (tri >= ntri) return;
  double U[3], V[3], T[3];
  for (int k = 0; k < 3; ++k) project(c, x + 3 * (size_t)tnode[3 * tri + k], U[k], V[k], T[k]);
  for (int k = 0; k < 3; ++k)
    if (!isfinite(U[k]) || !isfinite(V[k]) || !isfinite(T[k])) return;
  // pixels whose centre can lie in the projection, clamped to the image
  const double inv = 1.0 / c.pix;
  double jlo = floor(fmin(fmin(U[0], U[1]), U[2]) * inv - 0.5);
  double jhi = ceil(fmax(fmax(U[0], U[1]), U[2]) * inv - 0.5);
  double ilo = floor(fmin(fmin(V[0], V[1]), V[2]) * inv - 0.5);
  double ihi = ceil(fmax(fmax(V[0], V[1]), V[2]) * inv - 0.5);
  jlo = fmax(jlo, 0.0);
  ilo = fmax(ilo, 0.0);
  jhi = fmin(jhi, (double)(c.W - 1));
  ihi = fmin(ihi, (double)(c.H - 1));
  if (!(jlo <= jhi && ilo <= ihi)) return;
  const int j0 = (int)jlo, i0 = (int)ilo;
  const int nj = (int)jhi - j0 + 1, ni = (int)ihi - i0 + 1;
  const long long npx = (long long)nj * ni;
  for (long long q = threadIdx.x; q < npx; q += blockDim.x) {
    const int i = i0 + (int)(q / nj), j = j0 + (int)(q % nj);
    const double a = (j + 0.5) * c.pix, b = (i + 0.5) * c.pix;
    double t;
    if (!covers(U, V, T, a, b, &t)) continue;
    const size_t px = (size_t)i * c.W + j;
    if (pass == 0) atomicMin(zkey + px, order_key(t));
    else if (order_key(t) == zkey[px]) atomicMin(zidx + px, tri);
  }
}

__global__ void k_depth_finish(Camera c, const int* tnode, const double* x,
                               const unsigned long long* zkey, const int* zidx, double* depth,
                               double* normal) {
#pragma clang fp contract(off)
  const int px = gidx();
  if (px >= c.W * c.H) return;
  const unsigned long long key = zkey[px];
  const int tri = zidx[px];
  double* nrm = normal + 3 * (size_t)px;
  if (key == kEmpty || tri == INT_MAX) {
    depth[px] = INFINITY;
    nrm[0] = nrm[1] = nrm[2] = 0.0;
    return;
  }
  depth[px] = key_value(key);
  const double* p0 = x + 3 * (size_t)tnode[3 * tri];
  const double* p1 = x + 3 * (size_t)tnode[3 * tri + 1];
  const double* p2 = x + 3 * (size_t)tnode[3 * tri + 2];
  double e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    e1[k] = p1[k] - p0[k];
    e2[k] = p2[k] - p0[k];
  }
  double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double ln = sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
  for (int k = 0; k < 3; ++k) n[k] = n[k] / ln;
  const bool flip = (n[0] * c.en[0] + n[1] * c.en[1]) + n[2] * c.en[2] > 0.0;
  for (int k = 0; k < 3; ++k) nrm[k] = flip ? -n[k] : n[k];
}

int nblocks(long long n, int tpb) { return (int)((n + tpb - 1) / tpb); }

}  // namespace

void launch_markers(int m, const int* mnode, const double* bary, const double* x, const double* xr,
                    double* pos, double* flow, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_markers, dim3(nblocks(m, 64)), dim3(64), 0, s, m, mnode, bary, x, xr, pos, flow);
}
void launch_depth_clear(int npix, unsigned long long* zkey, int* zidx, hipStream_t s) {
  if (npix > 0) hipLaunchKernelGGL(k_depth_clear, dim3(nblocks(npix, 256)), dim3(256), 0, s, npix, zkey, zidx);
}
void launch_depth_raster(const Camera& c, int ntri, const int* tnode, const double* x,
                         unsigned long long* zkey, int* zidx, int pass, hipStream_t s) {
  if (ntri > 0) hipLaunchKernelGGL(k_depth_raster, dim3(ntri), dim3(64), 0, s, c, ntri, tnode, x, zkey, zidx, pass);
}
void launch_depth_finish(const Camera& c, const int* tnode, const double* x,
                         const unsigned long long* zkey, const int* zidx, double* depth,
                         double* normal, hipStream_t s) {
  const int npix = c.W * c.H;
  if (npix > 0) hipLaunchKernelGGL(k_depth_finish, dim3(nblocks(npix, 256)), dim3(256), 0, s, c, tnode, x, zkey, zidx, depth, normal);
}

}  // namespace tc
