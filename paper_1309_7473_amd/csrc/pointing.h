// Per-sample pointing computed from a boresight model (Test setup section:
// the scanning pattern plus each detector's place and polarisation angle in
// the focal plane), for scans that do not store pix / cos 2psi / sin 2psi.
//
// Flat sky in pixel units.  Boresight of sample t: (y_b, x_b), focal plane
// turned by phi(t) about the map centre (c_y, c_x) = ((ny-1)/2, (nx-1)/2).
// Detector d: offset (dy, dx) before the turn, angle psi_d.
//   ry = (y_b - c_y) + dy,  rx = (x_b - c_x) + dx
//   py = (c_y + sin(phi) rx) + cos(phi) ry,  px = (c_x + cos(phi) rx) - sin(phi) ry
//   pixel (floor(py + 1/2), floor(px + 1/2)), -1 off the map
//   weights cos 2(psi + phi) = c2psi c2phi - s2psi s2phi,
//           sin 2(psi + phi) = s2psi c2phi + c2psi s2phi
// Every operation is one rounded float64 operation in the order written (no
// contraction), so the pixel decisions are those of any other float64
// evaluation of the same expressions.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mm {

struct Bore {
  const double* b = nullptr;    // [6][n]: y_b, x_b, cos phi, sin phi, cos 2phi, sin 2phi
  const double* det = nullptr;  // [4][ndet]: dy, dx, cos 2psi, sin 2psi
  int logn = 0;                 // n = 2^logn samples per detector
  int ndet = 0;
  int ny = 0, nx = 0;
};

__device__ __forceinline__ int bore_pixel(double yb, double xb, double c, double s, double dy,
                                          double dx, int ny, int nx) {
#pragma clang fp contract(off)
  const double cy = 0.5 * double(ny - 1), cx = 0.5 * double(nx - 1);
  const double ry = (yb - cy) + dy;
  const double rx = (xb - cx) + dx;
  const double py = (cy + s * rx) + c * ry;
  const double px = (cx + c * rx) - s * ry;
  const double fy = floor(py + 0.5), fx = floor(px + 0.5);
  if (!(fy >= 0.0 && fy < double(ny) && fx >= 0.0 && fx < double(nx))) return -1;
  return int(fy) * nx + int(fx);
}

__device__ __forceinline__ void bore_weights(double c2p, double s2p, double c2f, double s2f,
                                             double* c, double* s) {
#pragma clang fp contract(off)
  *c = c2p * c2f - s2p * s2f;
  *s = s2p * c2f + c2p * s2f;
}

__device__ __forceinline__ int bore_pixel_at(const Bore& bo, int d, int64_t t) {
  const int64_t n = int64_t(1) << bo.logn;
  return bore_pixel(bo.b[t], bo.b[n + t], bo.b[2 * n + t], bo.b[3 * n + t], bo.det[d],
                    bo.det[bo.ndet + d], bo.ny, bo.nx);
}

__device__ __forceinline__ void bore_weights_at(const Bore& bo, int d, int64_t t, double* c,
                                                double* s) {
  const int64_t n = int64_t(1) << bo.logn;
  bore_weights(bo.det[2 * bo.ndet + d], bo.det[3 * bo.ndet + d], bo.b[4 * n + t],
               bo.b[5 * n + t], c, s);
}

// Sample i = d * n + t of the whole scan: stored pointing when pix is given.
__device__ __forceinline__ int sample_pixel(const int32_t* pix, const Bore& bo, int64_t i) {
  if (pix) return pix[i];
  return bore_pixel_at(bo, int(i >> bo.logn), i & ((int64_t(1) << bo.logn) - 1));
}

__device__ __forceinline__ void sample_weights(const float* c2, const float* s2, const Bore& bo,
                                               int64_t i, double* c, double* s) {
  if (c2) {
    *c = double(c2[i]);
    *s = double(s2[i]);
  } else {
    bore_weights_at(bo, int(i >> bo.logn), i & ((int64_t(1) << bo.logn) - 1), c, s);
  }
}

}  // namespace mm
