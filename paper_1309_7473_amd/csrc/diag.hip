// Convergence diagnostics of the Results section on the device: flat-sky
// binned auto-spectra (TT, and EE, BB for I,Q,U) of a map, and the delayed
// A-norm error estimate of PCG (host arithmetic on the recorded scalars).
//
// Spectra: the map is zero outside the active pixels (no apodisation); each
// component's unnormalised 2-D DFT X(k) comes from the map FFT kernels; for
// Q and U, E = Q cos 2phi + U sin 2phi and B = -Q sin 2phi + U cos 2phi with
// phi the wavevector angle; C_b = (pixel solid angle / pixels) times the mean
// of |X(k)|^2 over the modes with ell = 2 pi |k| / pixel in [b dell, (b+1) dell)
// (|k| in cycles per pixel).  Per-block bin sums in LDS, then a fixed-order sum
// over the blocks.
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "mm_device.h"
#include "mm_internal.h"

namespace mm {

template <int NC>
__global__ void k_spec_load(const double* __restrict__ x, const int32_t* __restrict__ mask,
                            int npix, Cx<double>* __restrict__ planes) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const bool on = mask[p] != 0;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    planes[int64_t(c) * npix + p] = cx(on ? x[int64_t(c) * npix + p] : 0.0, 0.0);
}

// part[block][bin][4] = (sum |T|^2, sum |E|^2, sum |B|^2, modes)
template <int NC>
__global__ void __launch_bounds__(256) k_spec_bin(const Cx<double>* __restrict__ planes, int logny,
                                                  int lognx, double ell_per_cycle, double inv_dell,
                                                  int nbins, double* __restrict__ part) {
  extern __shared__ double sb[];
  for (int i = threadIdx.x; i < nbins * 4; i += blockDim.x) sb[i] = 0.0;
  __syncthreads();
  const int ny = 1 << logny, nx = 1 << lognx;
  const int64_t npix = int64_t(ny) * nx;
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < npix;
       k += int64_t(gridDim.x) * blockDim.x) {
    const int y = int(k >> lognx), xx = int(k & (nx - 1));
    const double fy = double(y < ny / 2 ? y : y - ny) / double(ny);
    const double fx = double(xx < nx / 2 ? xx : xx - nx) / double(nx);
    const double ell = ell_per_cycle * sqrt(fy * fy + fx * fx);
    const int b = int(floor(ell * inv_dell));
    if (b >= nbins) continue;
    const Cx<double> t = planes[k];
    atomicAdd(&sb[4 * b + 0], t.x * t.x + t.y * t.y);
    if constexpr (NC == 3) {
      const double phi = atan2(fy, fx);
      const double c2 = cos(2.0 * phi), s2 = sin(2.0 * phi);
      const Cx<double> q = planes[npix + k], u = planes[2 * npix + k];
      const Cx<double> e = cx(q.x * c2 + u.x * s2, q.y * c2 + u.y * s2);
      const Cx<double> bm = cx(-q.x * s2 + u.x * c2, -q.y * s2 + u.y * c2);
      atomicAdd(&sb[4 * b + 1], e.x * e.x + e.y * e.y);
      atomicAdd(&sb[4 * b + 2], bm.x * bm.x + bm.y * bm.y);
    }
    atomicAdd(&sb[4 * b + 3], 1.0);
  }
  __syncthreads();
  double* out = part + int64_t(blockIdx.x) * nbins * 4;
  for (int i = threadIdx.x; i < nbins * 4; i += blockDim.x) out[i] = sb[i];
}

// out[0..2][b] = normalised mean power, out[3][b] = modes
__global__ void k_spec_final(const double* __restrict__ part, int nblocks, int nbins, double norm,
                             double* __restrict__ out) {
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nblocks; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) s[i] += part[(int64_t(k) * nbins + b) * 4 + i];
    const double c = s[3];
    for (int i = 0; i < 3; ++i) out[i * nbins + b] = c > 0 ? s[i] * norm / c : 0.0;
    out[3 * nbins + b] = c;
  }
}

static int ilog2d(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// The spectra with the scratch given: planes (ncomp x npix complex double),
// the block partials (kSpecBlocks x kSpecMaxBins x 4 double) and the result
// (4 x kSpecMaxBins double).  Every scratch element read is written first by
// the same call (the load fills the planes, each binning block writes its
// whole partial row, the final kernel writes every result it reads back), so
// nothing needs clearing between calls.
static mm_status map_spectra_into(ScanImpl* s, const double* x, double pixel_arcmin, double dell,
                                  int nbins, double* spectra, double* counts, Cx<double>* planes,
                                  double* part, double* res, hipStream_t st) {
  const int npix = s->npix, nc = s->nc;
  const int32_t* mask = s->at<int32_t>(s->lay.mask);
  const dim3 g((npix + 255) / 256), b(256);
  if (nc == 3)
    hipLaunchKernelGGL(k_spec_load<3>, g, b, 0, st, x, mask, npix, planes);
  else
    hipLaunchKernelGGL(k_spec_load<1>, g, b, 0, st, x, mask, npix, planes);
  MM_HIP(hipGetLastError());
  mm_status rc;
  if ((rc = map_fft(s, planes, nc, false, st)) != MM_OK) return rc;
  const double d = pixel_arcmin * 3.14159265358979323846 / (180.0 * 60.0);
  const double ell_per_cycle = 2.0 * 3.14159265358979323846 / d;
  int nblocks = (npix + 255) / 256;
  if (nblocks > kSpecBlocks) nblocks = kSpecBlocks;
  const size_t lds = size_t(nbins) * 4 * sizeof(double);
  if (nc == 3)
    hipLaunchKernelGGL(k_spec_bin<3>, dim3(nblocks), b, lds, st, planes, ilog2d(s->ny), ilog2d(s->nx),
                       ell_per_cycle, 1.0 / dell, nbins, part);
  else
    hipLaunchKernelGGL(k_spec_bin<1>, dim3(nblocks), b, lds, st, planes, ilog2d(s->ny), ilog2d(s->nx),
                       ell_per_cycle, 1.0 / dell, nbins, part);
  hipLaunchKernelGGL(k_spec_final, dim3(1), b, 0, st, part, nblocks, nbins, d * d / double(npix), res);
  MM_HIP(hipGetLastError());
  std::vector<double> h(size_t(4) * nbins);
  MM_HIP(hipMemcpyAsync(h.data(), res, h.size() * 8, hipMemcpyDeviceToHost, st));
  MM_HIP(hipStreamSynchronize(st));
  const int nout = nc == 3 ? 3 : 1;
  for (int i = 0; i < nout; ++i)
    for (int k = 0; k < nbins; ++k) spectra[i * nbins + k] = h[size_t(i) * nbins + k];
  if (counts)
    for (int k = 0; k < nbins; ++k) counts[k] = h[size_t(3) * nbins + k];
  return MM_OK;
}

mm_status map_spectra(ScanImpl* s, const double* x, double pixel_arcmin, double dell, int nbins,
                      double* spectra, double* counts, hipStream_t st) {
  double* part = s->at<double>(s->lay.spec);
  return map_spectra_into(s, x, pixel_arcmin, dell, nbins, spectra, counts,
                          s->at<Cx<double>>(s->lay.planes), part,
                          part + int64_t(kSpecBlocks) * kSpecMaxBins * 4, st);
}

// ------------------------------------------------ allocation-free variant
// Scratch of mm_map_spectra_noalloc: one array per device for the whole
// process, never allocated at run time.  Host code must not pass `scratch`
// itself to a kernel (on the host it names a stand-in, not device memory):
// its device address comes from hipGetSymbolAddress, once per device, with
// that device current.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static mm_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(MM_EDEVICE, "device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MM_OK;
}

size_t map_spectra_noalloc_bytes(const ScanImpl* s) {
  const size_t planes = size_t(s->nc) * size_t(s->npix) * sizeof(Cx<double>);
  const size_t tail = size_t(kSpecBlocks + 1) * kSpecMaxBins * 4 * sizeof(double);
  return ((planes + 255) & ~size_t(255)) + tail;
}

mm_status map_spectra_noalloc(ScanImpl* s, const double* x, double pixel_arcmin, double dell,
                              int nbins, double* spectra, double* counts, hipStream_t st) {
  if (map_spectra_noalloc_bytes(s) > kNoallocScratchBytes)
    return fail(MM_EINVAL, "map too large for the allocation-free spectra: ncomp * ny * nx * 16 "
                           "bytes plus 4.2 MB of partials must fit in 64 MiB");
  int dev = -1;
  MM_HIP(hipGetDevice(&dev));
  // the scan's memory must be on the current device (the scratch is per device)
  hipPointerAttribute_t attr{};
  MM_HIP(hipPointerGetAttributes(&attr, s->ws));
  if (attr.device != dev) return fail(MM_EINVAL, "call with the scan's device current");
  void* base = nullptr;
  mm_status rc;
  if ((rc = scratch_address(dev, &base)) != MM_OK) return rc;
  char* b = static_cast<char*>(base);
  const size_t planes = size_t(s->nc) * size_t(s->npix) * sizeof(Cx<double>);
  double* part = reinterpret_cast<double*>(b + ((planes + 255) & ~size_t(255)));
  return map_spectra_into(s, x, pixel_arcmin, dell, nbins, spectra, counts,
                          reinterpret_cast<Cx<double>*>(b), part,
                          part + int64_t(kSpecBlocks) * kSpecMaxBins * 4, st);
}

}  // namespace mm
