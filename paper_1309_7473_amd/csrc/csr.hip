// Pixel-major (CSR) index of each detector group's samples, built once per
// scan, so that P^T can be applied as a per-pixel gather-and-sum instead of
// an atomic scatter.
//
// For group g (detectors g*G .. g*G+G-1, G*n samples) the entries of pixel p
// are off[g][p] .. off[g][p+1]-1; entry e holds the group-relative sample
// index idx[e] = d_local*n + t and, for I,Q,U, its weights (cos 2psi,
// sin 2psi) as float32, except for boresight pointing on the float64 path,
// whose gather computes them from the index.  Runs of equal pixels inside a wavefront claim their slots with
// one atomic, so the order inside a pixel is fixed once the index is built
// (the per-pixel sum order of every later apply is then fixed too).
#include "mm_device.h"
#include "mm_internal.h"

namespace mm {

// Run structure of the keys held by the 64 lanes (a run also starts at a
// group boundary): returns the lane that heads this lane's run and the run
// length (valid on every lane).
__device__ __forceinline__ void wave_runs(int key, bool force_head, int* head_lane, int* run_len) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1);
  const bool head = (lane == 0) || (prev != key) || force_head;
  const uint64_t hm = __ballot(head);
  const uint64_t below = hm & ((lane == 63) ? ~uint64_t(0) : ((uint64_t(2) << lane) - 1));
  const int h = 63 - __clzll(below);
  const uint64_t above = (h == 63) ? 0 : (hm >> (h + 1));
  const int next = above ? (h + 1 + __ffsll(static_cast<long long>(above)) - 1) : 64;
  *head_lane = h;
  *run_len = next - h;
}

__global__ void __launch_bounds__(256) k_csr_count(const int32_t* __restrict__ pix, Bore bo,
                                                   int64_t n, int64_t total, int G, int npix,
                                                   int32_t* __restrict__ cnt) {
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t gsz = int64_t(G) * n;
  for (int64_t base = wave * 64; base < total; base += nwaves * 64) {
    const int64_t i = base + lane;
    int p = -1;
    if (i < total) {
      p = sample_pixel(pix, bo, i);
      if (unsigned(p) >= unsigned(npix)) p = -1;
    }
    int h, len;
    wave_runs(p, i < total && (i % gsz) == 0, &h, &len);
    if (lane == h && p >= 0) {
      const int64_t g = i / gsz;
      atomicAdd(cnt + g * npix + p, len);
    }
  }
}

// Exclusive scan of one group's counts (one block per group): off[0..npix],
// and the counts become fill cursors (= off[p]).
__global__ void __launch_bounds__(1024) k_csr_scan(int32_t* __restrict__ cnt,
                                                   int32_t* __restrict__ off, int npix) {
  const int g = blockIdx.x;
  int32_t* c = cnt + int64_t(g) * npix;
  int32_t* o = off + int64_t(g) * (npix + 1);
  const int nt = blockDim.x;
  const int chunk = (npix + nt - 1) / nt;
  const int a = threadIdx.x * chunk;
  const int b = (a + chunk < npix) ? a + chunk : npix;
  int64_t s = 0;
  for (int p = a; p < b; ++p) s += c[p];
  __shared__ int64_t part[1024];
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off2 = 1; off2 < nt; off2 <<= 1) {
    const int64_t v = (threadIdx.x >= off2) ? part[threadIdx.x - off2] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int64_t run = part[threadIdx.x] - s;
  for (int p = a; p < b; ++p) {
    const int32_t cp = c[p];
    o[p] = int32_t(run);
    c[p] = int32_t(run);
    run += cp;
  }
  if (threadIdx.x == nt - 1) o[npix] = int32_t(part[nt - 1]);
}

// Counts on-map samples whose weights (stored, or from the boresight model)
// are not of unit norm (|c^2 + s^2 - 1| > 1e-6 in float64, or not finite).
__global__ void k_unit_weights(const int32_t* __restrict__ pix, Bore bo,
                               const float* __restrict__ c2, const float* __restrict__ s2,
                               int64_t total, int npix, int* __restrict__ bad) {
  int cnt = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total; i += stride) {
    if (unsigned(sample_pixel(pix, bo, i)) >= unsigned(npix)) continue;
    double c, s;
    sample_weights(c2, s2, bo, i, &c, &s);
    const double r = c * c + s * s - 1.0;
    cnt += (r <= 1e-6 && r >= -1e-6) ? 0 : 1;
  }
  if (cnt) atomicAdd(bad, cnt);
}

__global__ void k_angles_t(const float* __restrict__ c2, const float* __restrict__ s2,
                           int64_t total, uint32_t* __restrict__ ang) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total; i += stride)
    ang[i] = weight_angle(c2[i], s2[i]);
}

template <int NC>
__global__ void __launch_bounds__(256) k_csr_fill(const int32_t* __restrict__ pix, Bore bo,
                                                  const float* __restrict__ c2,
                                                  const float* __restrict__ s2, int64_t n,
                                                  int64_t total, int G, int npix,
                                                  int32_t* __restrict__ cursor,
                                                  int32_t* __restrict__ idx,
                                                  float2* __restrict__ w,
                                                  int2* __restrict__ ia) {
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t gsz = int64_t(G) * n;
  for (int64_t base = wave * 64; base < total; base += nwaves * 64) {
    const int64_t i = base + lane;
    int p = -1;
    if (i < total) {
      p = sample_pixel(pix, bo, i);
      if (unsigned(p) >= unsigned(npix)) p = -1;
    }
    int h, len;
    wave_runs(p, i < total && (i % gsz) == 0, &h, &len);
    const int64_t g = (i < total) ? i / gsz : 0;
    int slot0 = 0;
    if (lane == h && p >= 0) slot0 = atomicAdd(cursor + g * npix + p, len);
    slot0 = __shfl(slot0, h);
    if (p >= 0) {
      const int64_t e = g * gsz + slot0 + (lane - h);
      idx[e] = int32_t(i - g * gsz);
      if constexpr (NC == 3) {
        if (ia) {            // unit-norm weights: (index, angle) in 8 B
          double c, sn;
          sample_weights(c2, s2, bo, i, &c, &sn);
          ia[e] = make_int2(int32_t(i - g * gsz), int32_t(weight_angle(c, sn)));
        } else if (w) {      // NULL: the gather computes the weights from the boresight model
          double c, sn;
          sample_weights(c2, s2, bo, i, &c, &sn);
          w[e] = make_float2(float(c), float(sn));
        }
      }
    }
  }
}

#ifndef MM_ANGLE_WEIGHTS
#define MM_ANGLE_WEIGHTS 1
#endif
constexpr bool kAngleWeights = MM_ANGLE_WEIGHTS != 0;

mm_status csr_setup(ScanImpl* s, hipStream_t st) {
  const Layout& L = s->lay;
  const int npix = s->npix;
  const int G = s->plan.G;
  const int ngroups = (s->ndet + G - 1) / G;
  const int64_t total = int64_t(s->ndet) * s->n;
  int32_t* cnt = s->at<int32_t>(L.csr_cnt);
  mm_status r;
  if ((r = fill_zero(cnt, size_t(ngroups) * npix * 4, st)) != MM_OK) return r;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  const Bore bo = scan_bore(s);
  hipLaunchKernelGGL(k_csr_count, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo, s->n,
                     total, G, npix, cnt);
  hipLaunchKernelGGL(k_csr_scan, dim3(ngroups), dim3(1024), 0, st, cnt, s->at<int32_t>(L.csr_off),
                     npix);
  // weights of unit norm on the float32 and bfloat16 paths go into the index
  // as 4-byte angles instead of 8-byte float32 pairs
  s->csr_ang = false;
  if (s->nc == 3 && s->plan.csr_w && !s->plan.f64 && kAngleWeights) {
    int* bad = s->at<int>(L.misc);
    if ((r = fill_zero(bad, 4, st)) != MM_OK) return r;
    hipLaunchKernelGGL(k_unit_weights, dim3(2048), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, total, npix, bad);
    MM_HIP(hipGetLastError());
    int h = 0;
    MM_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    s->csr_ang = h == 0;
  }
  // a time-major copy of the angles for pass 1 (8 B of pointing a sample)
  s->ang_t_ready = false;
  if (s->csr_ang && !s->plan.otf && !s->plan.f64) {   // the region plan_and_layout sized
    hipLaunchKernelGGL(k_angles_t, dim3(2048), dim3(256), 0, st, s->d.cos2psi, s->d.sin2psi,
                       total, s->at<uint32_t>(L.ang_t));
    MM_HIP(hipGetLastError());
    s->ang_t_ready = true;
  }
  if (s->nc == 3)
    hipLaunchKernelGGL(k_csr_fill<3>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, s->n, total, G, npix, cnt,
                       s->at<int32_t>(L.csr_idx),
                       s->plan.csr_w && !s->csr_ang ? s->at<float2>(L.csr_w)
                                                    : static_cast<float2*>(nullptr),
                       s->csr_ang ? s->at<int2>(L.csr_w) : static_cast<int2*>(nullptr));
  else
    hipLaunchKernelGGL(k_csr_fill<1>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, s->n, total, G, npix, cnt,
                       s->at<int32_t>(L.csr_idx), static_cast<float2*>(nullptr),
                       static_cast<int2*>(nullptr));
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
