// Tactile outputs of the deformed pad (Taccel Sec. 4.2): marker positions and flows, and
// depth / normal maps of the coated surface seen orthographically from an image plane.
#pragma once
#include <hip/hip_runtime.h>

namespace tc {

// Image plane: pixel (i, j) is the ray from o + (j + 1/2) pix eu + (i + 1/2) pix ev along
// en = eu x ev.
struct Camera {
  double o[3], eu[3], ev[3], en[3];
  double pix;
  int W, H;
};

// pos[k] = sum_u bary[k][u] x[node[k][u]], flow[k] = pos[k] - the same sum over xr (rest).
void launch_markers(int m, const int* mnode, const double* bary, const double* x, const double* xr,
                    double* pos, double* flow, hipStream_t s);
// Depth map in three launches over ntri triangles (node ids tnode[ntri][3], positions x):
// clear, nearest ray parameter per pixel (pass 0), lowest triangle index attaining it
// (pass 1), then depth and normal per pixel.  zkey/zidx: W*H scratch words.
void launch_depth_clear(int npix, unsigned long long* zkey, int* zidx, hipStream_t s);
void launch_depth_raster(const Camera& c, int ntri, const int* tnode, const double* x,
                         unsigned long long* zkey, int* zidx, int pass, hipStream_t s);
void launch_depth_finish(const Camera& c, const int* tnode, const double* x,
                         const unsigned long long* zkey, const int* zidx, double* depth,
                         double* normal, hipStream_t s);

}  // namespace tc
