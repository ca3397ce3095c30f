// Pixel-major (CSR) index of each detector group's samples, built once per
// scan, so that P^T can be applied as a per-pixel gather-and-sum instead of
// an atomic scatter.
//
// Run-length form (plan.rle, groups of at most 2^28 samples): a raster scan
// steps a quarter pixel a sample, so a detector stays about four consecutive
// samples in one pixel.  The entries of pixel p are then runs of consecutive
// group-relative samples, one uint32 each: (first sample << 4) | length,
// length 1..4 (longer runs are split), in time order.  The gather reads a run's timestream
// and its time-major weights as consecutive samples, so the index costs about
// 1 byte a sample instead of 4 (plus 4-8 of pixel-major weights).
//
// Per-sample form (larger groups):
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

// samples per run entry of the run-length index: the gather reads a run as
// one vector of four samples, so longer runs are split into pieces of four
// (a raster scan at a quarter pixel a sample gives runs of four, rarely five)
constexpr int kRunMax = 4;

// Entries a wave run of `len` samples takes: one per sample, or one per
// kRunMax-sample piece in the run-length form; the lanes heading a piece.
template <bool RLE>
__device__ __forceinline__ int run_entries(int len) {
  return RLE ? (len + kRunMax - 1) / kRunMax : len;
}

template <bool RLE>
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
      atomicAdd(cnt + g * npix + p, run_entries<RLE>(len));
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

// Chunk-coded pointing for pass 1, for each kPtcChunk-sample chunk of
// one detector.  Header: the smallest on-map pixel of the chunk (0 if none),
// and the chunk's angle trend u0 + slope * i through its first and last
// on-map samples (i the sample's place in the chunk; slope 0 with fewer than
// two), stored as base = u0 - 2^15 and slope.  Each sample is (pixel - lowest)
// | (angle - base - slope * i) << 16 (mod 2^32), with 0xFFFF in the low half
// for a sample off the map (pixel outside [0, npix)).  Pass 1 decodes exactly
// the stored pixel and angle.  A chunk whose on-map pixels span more than
// 65534 ids, or whose on-map angles stray 2^15 or more from the trend, sets
// *bad, and the scan keeps the uncoded form.
__global__ void __launch_bounds__(256) k_ptc_encode(const int32_t* __restrict__ pix,
                                                    const uint32_t* __restrict__ ang,
                                                    int64_t nchunks, int npix,
                                                    int4* __restrict__ hdr,
                                                    uint32_t* __restrict__ code,
                                                    int* __restrict__ bad) {
  // one wavefront per chunk, one lane per sample (coalesced loads and stores;
  // the chunk's extremes and first and last on-map samples by wave reductions)
  static_assert(kPtcChunk == 64, "one lane per sample of a chunk");
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
  for (int64_t c = wave; c < nchunks; c += nwaves) {
    const int64_t i = c * kPtcChunk + lane;
    const int q = pix[i];
    const uint32_t u = ang[i];
    const bool on = unsigned(q) < unsigned(npix);
    int lo = on ? q : npix, hi = on ? q : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int lo2 = __shfl_xor(lo, off), hi2 = __shfl_xor(hi, off);
      lo = lo2 < lo ? lo2 : lo;
      hi = hi2 > hi ? hi2 : hi;
    }
    if (hi < 0) lo = 0;
    const unsigned long long onm = __ballot(on);
    const int i0 = onm ? __ffsll(onm) - 1 : -1;
    const int i1 = onm ? 63 - __clzll(onm) : -1;
    const uint32_t ua = __shfl(u, i0 < 0 ? 0 : i0), ue = __shfl(u, i1 < 0 ? 0 : i1);
    // the trend: a signed angle step per sample, rounded to the nearest
    int32_t slope = 0;
    uint32_t u0 = 0;
    if (i0 >= 0) {
      if (i1 > i0) {
        const int64_t du = int64_t(int32_t(ue - ua));
        const int64_t span = i1 - i0;
        slope = int32_t(du >= 0 ? (du + span / 2) / span : -((-du + span / 2) / span));
      }
      u0 = ua - uint32_t(slope) * uint32_t(i0);
    }
    const uint32_t ub = u0 - 32768u;
    const uint32_t r = u - ub - uint32_t(slope) * uint32_t(lane);
    const bool fits = !on || r <= 65535u;
    const bool ok = hi - lo <= 65534 && __ballot(!fits) == 0ull;
    code[i] = on ? (uint32_t(q - lo) | (r << 16)) : 0xFFFFu;
    if (lane == 0) {
      hdr[c] = make_int4(lo, int(ub), slope, 0);
      if (!ok) atomicOr(bad, 1);
    }
  }
}

// Run-length entries: the lane heading each kRunMax-sample piece of a wave run
// writes (first sample << 4) | length into the pixel's next free slot.
__global__ void __launch_bounds__(256) k_rle_fill(const int32_t* __restrict__ pix, Bore bo,
                                                  int64_t total, int64_t gsz, int npix,
                                                  int32_t* __restrict__ cursor,
                                                  uint32_t* __restrict__ hdr) {
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
  const int lane = threadIdx.x & 63;
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
    if (lane == h && p >= 0) slot0 = atomicAdd(cursor + g * npix + p, run_entries<true>(len));
    slot0 = __shfl(slot0, h);
    const int off = lane - h;
    if (p >= 0 && off % kRunMax == 0) {
      const int piece = len - off < kRunMax ? len - off : kRunMax;
      const uint32_t first = uint32_t(i - g * gsz);
      hdr[g * gsz + slot0 + off / kRunMax] = (first << 4) | uint32_t(piece);
    }
  }
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

// Each pixel's runs in time order (by first sample; runs of one pixel never
// overlap, so the entries are distinct).  Pixels next to each other along a
// sweep are then visited by the same detector passes in the same order, so
// the gather's lanes for neighbouring pixels (one wave holds four) read
// neighbouring pieces of the same timestream lines, and the index no longer
// depends on the order the fill's atomics happened to claim slots in.  One
// wavefront per pixel and group: the entries go to LDS and each is written
// back at its rank, the number of smaller entries, which the lanes count from
// LDS.  A pixel with more than kSortCap entries is sorted in place by one lane
// (insertion sort).
constexpr int kSortCap = 2048;

__global__ void __launch_bounds__(256) k_rle_sort(const int32_t* __restrict__ roff_all, int npix,
                                                  int ngroups, int64_t gsz,
                                                  uint32_t* __restrict__ hdr_all) {
  __shared__ uint32_t keys[4][kSortCap];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t item = int64_t(blockIdx.x) * 4 + w;
  const bool valid = item < int64_t(npix) * ngroups;
  int b = 0, k = 0;
  uint32_t* h = hdr_all;
  if (valid) {
    const int g = int(item / npix), p = int(item % npix);
    const int32_t* roff = roff_all + int64_t(g) * (npix + 1);
    h = hdr_all + int64_t(g) * gsz;
    b = roff[p];
    k = roff[p + 1] - b;
  }
  const bool ranked = k > 1 && k <= kSortCap;
  if (ranked)
    for (int t = lane; t < k; t += 64) keys[w][t] = h[b + t];
  __syncthreads();
  if (ranked) {
    for (int t = lane; t < k; t += 64) {
      const uint32_t v = keys[w][t];
      int r = 0;
      for (int j = 0; j < k; ++j) {
        const uint32_t kj = keys[w][j];
        r += (kj < v || (kj == v && j < t)) ? 1 : 0;   // ties (none expected) keep their order
      }
      h[b + r] = v;
    }
  } else if (k > kSortCap && lane == 0) {
    for (int q = b + 1; q < b + k; ++q) {
      const uint32_t v = h[q];
      int j = q - 1;
      while (j >= b && h[j] > v) {
        h[j + 1] = h[j];
        --j;
      }
      h[j + 1] = v;
    }
  }
}

// The run-length index's angle-coded weights in gather order: each pixel's
// runs are expanded exactly as the gather does (16 lanes, batches of 16 runs,
// lane l taking samples l, l + 16, ... of a batch) and sample q of the pixel
// gets the time-major angle of its sample (ang_t), or with boresight
// pointing (ang_t NULL) the angle of the model's float64 weights, as the
// per-sample index stores it.  blockIdx.y is the group.
__global__ void __launch_bounds__(256) k_rle_angles(const int32_t* __restrict__ roff_all,
                                                    const int32_t* __restrict__ soff_all,
                                                    const uint32_t* __restrict__ hdr_all,
                                                    const uint32_t* __restrict__ ang_t, Bore bo,
                                                    int npix, int64_t gsz,
                                                    uint32_t* __restrict__ pa_all) {
  constexpr int LPP = 16;
  const int g = blockIdx.y;
  const int l = threadIdx.x % LPP;
  const int p = blockIdx.x * (256 / LPP) + threadIdx.x / LPP;
  if (p >= npix) return;               // whole 16-lane groups leave together
  const int32_t* roff = roff_all + int64_t(g) * (npix + 1);
  const uint32_t* hdr = hdr_all + int64_t(g) * gsz;
  const uint32_t* ang = ang_t ? ang_t + int64_t(g) * gsz : nullptr;
  uint32_t* pa = pa_all + int64_t(g) * gsz + soff_all[int64_t(g) * (npix + 1) + p];
  const int b = roff[p], e = roff[p + 1];
  for (int kb = b; kb < e; kb += LPP) {
    const int k = kb + l;
    const uint32_t h = k < e ? hdr[k] : 0u;
    const int first = int(h >> 4), len = int(h & 15u);
    int incl = len;
#pragma unroll
    for (int off = 1; off < LPP; off <<= 1) {
      const int v = __shfl_up(incl, off, LPP);
      if (l >= off) incl += v;
    }
    const int excl = incl - len;
    const int total = __shfl(incl, LPP - 1, LPP);
    for (int q0 = 0; q0 < total; q0 += LPP) {
      const int q = q0 + l;
      int r = 0;
#pragma unroll
      for (int step = LPP / 2; step > 0; step >>= 1)
        if (__shfl(excl, r + step, LPP) <= q) r += step;
      const int ik = __shfl(first, r, LPP) + (q - __shfl(excl, r, LPP));
      if (q < total) {
        if (ang) {
          pa[q] = ang[ik];
        } else {
          double c, sn;
          sample_weights(nullptr, nullptr, bo, int64_t(g) * gsz + ik, &c, &sn);
          pa[q] = weight_angle(c, sn);
        }
      }
    }
    pa += total;
  }
}

mm_status csr_setup(ScanImpl* s, hipStream_t st) {
  const Layout& L = s->lay;
  const int npix = s->npix;
  const int G = s->plan.G;
  const int ngroups = (s->ndet + G - 1) / G;
  const int64_t total = int64_t(s->ndet) * s->n;
  const int64_t gsz = int64_t(G) * s->n;
  int32_t* cnt = s->at<int32_t>(L.csr_cnt);
  mm_status r;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  const Bore bo = scan_bore(s);
  // weights of unit norm on the float32 and bfloat16 paths are stored as
  // 4-byte angles instead of 8-byte float32 pairs
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
  // pass 1's chunk-coded copy of the pixels and angles, if every chunk fits
  s->ptc_ready = false;
  if (s->ang_t_ready && s->plan.ptc && s->d.pix) {
    int* bad = s->at<int>(L.misc);
    if ((r = fill_zero(bad, 4, st)) != MM_OK) return r;
    const int64_t nchunks = total / kPtcChunk;   // one wavefront each, four a block
    int64_t cb = (nchunks + 3) / 4;
    if (cb > 65536) cb = 65536;
    hipLaunchKernelGGL(k_ptc_encode, dim3(unsigned(cb)), dim3(256), 0, st, s->d.pix,
                       s->at<uint32_t>(L.ang_t), nchunks, npix, s->at<int4>(L.ptc_h),
                       s->at<uint32_t>(L.ptc), bad);
    MM_HIP(hipGetLastError());
    int h = 0;
    MM_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    s->ptc_ready = h == 0;
  }
  // run-length index with angle-coded weights: the angles also go pixel-major
  // in gather order, for which each pixel's sample offsets come first
  // (boresight pointing: the angles come from the model, no time-major copy)
  s->rle_pa = s->plan.rle && (s->ang_t_ready || (s->plan.otf && s->csr_ang));
  if (s->rle_pa) {
    if ((r = fill_zero(cnt, size_t(ngroups) * npix * 4, st)) != MM_OK) return r;
    hipLaunchKernelGGL(k_csr_count<false>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->n, total, G, npix, cnt);
    hipLaunchKernelGGL(k_csr_scan, dim3(ngroups), dim3(1024), 0, st, cnt,
                       s->at<int32_t>(L.csr_soff), npix);
    MM_HIP(hipGetLastError());
  }
  if ((r = fill_zero(cnt, size_t(ngroups) * npix * 4, st)) != MM_OK) return r;
  if (s->plan.rle)
    hipLaunchKernelGGL(k_csr_count<true>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->n, total, G, npix, cnt);
  else
    hipLaunchKernelGGL(k_csr_count<false>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->n, total, G, npix, cnt);
  hipLaunchKernelGGL(k_csr_scan, dim3(ngroups), dim3(1024), 0, st, cnt, s->at<int32_t>(L.csr_off),
                     npix);
  if (s->plan.rle) {
    hipLaunchKernelGGL(k_rle_fill, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo, total,
                       gsz, npix, cnt, s->at<uint32_t>(L.csr_idx));
    const int64_t nsort = int64_t(npix) * ngroups;   // one wavefront each, four a block
    hipLaunchKernelGGL(k_rle_sort, dim3(unsigned((nsort + 3) / 4)), dim3(256), 0, st,
                       s->at<int32_t>(L.csr_off), npix, ngroups, gsz, s->at<uint32_t>(L.csr_idx));
    if (s->rle_pa)
      hipLaunchKernelGGL(k_rle_angles, dim3(unsigned((npix + 15) / 16), unsigned(ngroups)),
                         dim3(256), 0, st, s->at<int32_t>(L.csr_off), s->at<int32_t>(L.csr_soff),
                         s->at<uint32_t>(L.csr_idx),
                         s->ang_t_ready ? s->at<uint32_t>(L.ang_t) : static_cast<uint32_t*>(nullptr),
                         bo, npix, gsz, s->at<uint32_t>(L.csr_w));
  } else if (s->nc == 3) {
    hipLaunchKernelGGL(k_csr_fill<3>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, s->n, total, G, npix, cnt,
                       s->at<int32_t>(L.csr_idx),
                       s->plan.csr_w && !s->csr_ang ? s->at<float2>(L.csr_w)
                                                    : static_cast<float2*>(nullptr),
                       s->csr_ang ? s->at<int2>(L.csr_w) : static_cast<int2*>(nullptr));
  } else {
    hipLaunchKernelGGL(k_csr_fill<1>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, s->n, total, G, npix, cnt,
                       s->at<int32_t>(L.csr_idx), static_cast<float2*>(nullptr),
                       static_cast<int2*>(nullptr));
  }
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
