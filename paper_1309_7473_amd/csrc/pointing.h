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

// Float32 evaluation of the same pixel, for inputs Y = fl32(y_b - c_y),
// X = fl32(x_b - c_x), c, s, dy, dx rounded to float32 from their float64
// values.  Each rounding is at most u = 2^-24 relative; propagated through
// ry, rx, the products and the two sums, |p32 - p64| <= u (|c_p| + 4|rx| +
// 3|ry| + |X| + |Y| + |dx| + |dy| + |p|) on either axis (the float64
// definition's own roundings are 2^29 times smaller), plus u|p| for the
// float32 p + 1/2.  When p + 1/2 lies farther than twice that from an
// integer on both axes, floor(p32 + 1/2) equals the float64 definition's
// floor; otherwise the caller evaluates the float64 definition.  Returns
// the pixel, -1 off the map, or -2 for "not decided".
__device__ __forceinline__ int bore_pixel_f32(float Y, float X, float c, float s, float dy,
                                              float dx, int ny, int nx) {
#pragma clang fp contract(off)
  const float cy = 0.5f * float(ny - 1), cx = 0.5f * float(nx - 1);
  const float ry = Y + dy;
  const float rx = X + dx;
  const float py = (cy + s * rx) + c * ry;
  const float px = (cx + c * rx) - s * ry;
  const float com = 4.0f * (fabsf(rx) + fabsf(ry)) + fabsf(X) + fabsf(Y) + fabsf(dx) + fabsf(dy);
  const float ty = 1.1920929e-07f * (cy + com + 2.0f * fabsf(py));   // 2u (...)
  const float tx = 1.1920929e-07f * (cx + com + 2.0f * fabsf(px));
  const float vy = py + 0.5f, vx = px + 0.5f;
  const float fy = floorf(vy), fx = floorf(vx);
  const float dyy = fminf(vy - fy, fy + 1.0f - vy);
  const float dxx = fminf(vx - fx, fx + 1.0f - vx);
  if (!(dyy > ty && dxx > tx)) return -2;
  if (!(fy >= 0.0f && fy < float(ny) && fx >= 0.0f && fx < float(nx))) return -1;
  return int(fy) * nx + int(fx);
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

// The weights (c, s) = (cos, sin)(theta) as u = theta 2^32 / 2pi mod 2^32
// (angles then add exactly, mod 2^32).
__device__ __forceinline__ uint32_t weight_angle(double c, double s) {
  const double t = atan2(s, c) * (4294967296.0 / 6.283185307179586476925);
  const int64_t q = int64_t(llrint(t));          // |t| <= 2^31
  return uint32_t(q & 0xFFFFFFFFll);
}

// The float64 definition as an out-of-line call, for the rare samples the
// float32 evaluation leaves undecided (keeps the caller's registers low).
static __device__ __attribute__((noinline)) int bore_pixel_slow(Bore bo, int d, int64_t t) {
  return bore_pixel_at(bo, d, t);
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
