// Binned (eq. 3-4) and Jacobi (eq. 5) preconditioners, the active-pixel mask
// and the per-pixel Sigma^-1 = B^(-1/2) used by the circulant preconditioner
// (eq. 7).
//
// w_d = (N^-1)_tt = (iN_0 + 2 sum_{k=1}^{n/2-1} iN_k + iN_{n/2}) / n is the
// diagonal of detector d's circulant inverse covariance.  The binned block of
// pixel p is B_p = sum_{samples in p} w_d u u^T, u = (1, cos 2psi, sin 2psi);
// the Jacobi block uses w_d = 1.  Both are accumulated in one pass over the
// pointing with the same wave-level run pre-sum as the scatter of A.
#include "linalg_small.h"
#include <type_traits>

#include "mm_device.h"
#include "mm_internal.h"

namespace mm {

__global__ void k_fill_zero(uint32_t* __restrict__ p, size_t nwords) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < nwords;
       i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

mm_status fill_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return MM_OK;
  const size_t words = (bytes + 3) / 4;
  size_t blocks = (words + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_zero, dim3(unsigned(blocks)), dim3(256), 0, st,
                     static_cast<uint32_t*>(p), words);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

__global__ void k_det_weights(const float* __restrict__ iN, int64_t n, double* __restrict__ w) {
  const int d = blockIdx.x;
  const int64_t M = n / 2;
  const float* row = iN + int64_t(d) * (M + 1);
  double v[1] = {0.0};
  for (int64_t k = threadIdx.x; k <= M; k += blockDim.x) {
    const double x = double(row[k]);
    v[0] += (k == 0 || k == M) ? x : 2.0 * x;
  }
  __shared__ double sm[16];
  block_sum<1>(v, sm);
  if (threadIdx.x == 0) w[d] = v[0] / double(n);
}

// With inter-detector correlations the diagonal of N^-1(k) is
// iN_d(k) - sum_j V_b[d][j]^2: subtract its mean over the n two-sided
// frequencies (bin b holds 2 (e1 - e0) of them, less k = 0 and k = n/2).
__global__ void k_det_weights_corr(const float* __restrict__ V, const int32_t* __restrict__ edges,
                                   int nbins, int rank, int ndet, int64_t n,
                                   double* __restrict__ w) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= ndet) return;
  double s = 0.0;
  for (int b = 0; b < nbins; ++b) {
    const int64_t e0 = edges[b], e1 = edges[b + 1];
    const int64_t cnt = 2 * (e1 - e0) - (e0 == 0 ? 1 : 0) - (e1 == n / 2 + 1 ? 1 : 0);
    double v2 = 0.0;
    for (int j = 0; j < rank; ++j) {
      const double v = double(V[(int64_t(b) * ndet + d) * rank + j]);
      v2 += v * v;
    }
    s += double(cnt) * v2;
  }
  w[d] -= s / double(n);
}

__global__ void k_validate_finite(const float* __restrict__ v, int64_t count, int* __restrict__ bad) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    if (!isfinite(v[i])) atomicOr(bad, 1);
}

// One lane per sample; every lane of a wave takes the same number of trips.
template <int NC>
__global__ void __launch_bounds__(256) k_binned_accum(const int32_t* __restrict__ pix, Bore bo,
                                                      const float* __restrict__ c2,
                                                      const float* __restrict__ s2,
                                                      const double* __restrict__ detw,
                                                      int64_t n, int64_t total, int npix,
                                                      double* __restrict__ hits,
                                                      double* __restrict__ Bb,
                                                      double* __restrict__ Bj) {
  constexpr int NU = (NC == 3) ? 6 : 1;
  constexpr int NV = 1 + 2 * NU;
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
  const int lane = threadIdx.x & 63;
  for (int64_t base = wave * 64; base < total; base += nwaves * 64) {
    const int64_t i = base + lane;
    int p = -1;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    if (i < total) {
      p = sample_pixel(pix, bo, i);
      if (unsigned(p) >= unsigned(npix)) p = -1;
      if (p >= 0) {
        const double wd = detw[i / n];
        double u[NU];
        if constexpr (NC == 3) {
          double c, s;
          sample_weights(c2, s2, bo, i, &c, &s);
          u[0] = 1.0; u[1] = c; u[2] = s; u[3] = c * c; u[4] = c * s; u[5] = s * s;
        } else {
          u[0] = 1.0;
        }
        v[0] = 1.0;
#pragma unroll
        for (int k = 0; k < NU; ++k) {
          v[1 + k] = u[k];
          v[1 + NU + k] = wd * u[k];
        }
      }
    }
    if (wave_segmented_sum<3, NV>(p, v)) {
      atomic_add_f64(hits + p, v[0]);
#pragma unroll
      for (int k = 0; k < NU; ++k) {
        atomic_add_f64(Bj + 6 * int64_t(p) + k, v[1 + k]);
        atomic_add_f64(Bb + 6 * int64_t(p) + k, v[1 + NU + k]);
      }
    }
  }
}

// The same sums as k_binned_accum through the pixel-major index (when the
// scan has one): 16 lanes per pixel run over the pixel's entries of every
// detector group in a fixed order, so no atomics and a deterministic result.
// Entry ik of group g is detector g * G + ik / n, sample ik mod n.
// RLE: the entries are runs (first sample << 4 | length) of consecutive
// group-relative samples.
template <int NC, bool RLE>
__global__ void __launch_bounds__(256) k_binned_gather(const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ idx,
                                                       const float2* __restrict__ w,
                                                       const float* __restrict__ c2,
                                                       const float* __restrict__ s2, Bore bo,
                                                       const double* __restrict__ detw,
                                                       int ngroups, int G, int n, int npix,
                                                       double* __restrict__ hits,
                                                       double* __restrict__ Bb,
                                                       double* __restrict__ Bj) {
  constexpr int LPP = 16;
  constexpr int NU = (NC == 3) ? 6 : 1;
  constexpr int NV = 1 + 2 * NU;
  const int l = threadIdx.x % LPP;
  const int p = blockIdx.x * (256 / LPP) + threadIdx.x / LPP;
  if (p >= npix) return;               // whole 16-lane groups leave together
  const int64_t gsz = int64_t(G) * n;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    const int32_t* o = off + int64_t(g) * (npix + 1);
    const int b = o[p], e = o[p + 1];
    for (int k = b + l; k < e; k += LPP) {
      int first, len;
      if constexpr (RLE) {
        const uint32_t h = reinterpret_cast<const uint32_t*>(idx)[int64_t(g) * gsz + k];
        first = int(h >> 4);
        len = int(h & 15u);
      } else {
        first = idx[int64_t(g) * gsz + k];
        len = 1;
      }
      for (int jj = 0; jj < len; ++jj) {
        const int ik = first + jj;
        const int d = g * G + ik / n;
        const double wd = detw[d];
        double u[NU];
        u[0] = 1.0;
        if constexpr (NC == 3) {
          double c, sn;
          if (w) {
            const float2 cs = w[int64_t(g) * gsz + k];
            c = double(cs.x);
            sn = double(cs.y);
          } else if (c2) {   // the stored time-major weights, sample g G n + ik
            c = double(c2[int64_t(g) * gsz + ik]);
            sn = double(s2[int64_t(g) * gsz + ik]);
          } else {
            bore_weights_at(bo, d, ik % n, &c, &sn);
          }
          u[1] = c; u[2] = sn; u[3] = c * c; u[4] = c * sn; u[5] = sn * sn;
        }
        v[0] += 1.0;
#pragma unroll
        for (int j = 0; j < NU; ++j) {
          v[1 + j] += u[j];
          v[1 + NU + j] += wd * u[j];
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int o2 = LPP / 2; o2 > 0; o2 >>= 1) v[k] += __shfl_xor(v[k], o2, LPP);
  if (l == 0) {
    hits[p] = v[0];
#pragma unroll
    for (int j = 0; j < NU; ++j) {
      Bj[6 * int64_t(p) + j] = v[1 + j];
      Bb[6 * int64_t(p) + j] = v[1 + NU + j];
    }
  }
}

// Mask, inverse blocks and Sigma^-1 per pixel.
template <int NC>
__global__ void k_binned_finalize(const double* __restrict__ hits, const double* __restrict__ Bb,
                                  const double* __restrict__ Bj, int npix, double rcond,
                                  int32_t* __restrict__ mask, double* __restrict__ binv_b,
                                  double* __restrict__ binv_j, double* __restrict__ siginv,
                                  double* __restrict__ sigma) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  double ob[6] = {0, 0, 0, 0, 0, 0}, oj[6] = {0, 0, 0, 0, 0, 0}, os[6] = {0, 0, 0, 0, 0, 0};
  double oq[6] = {0, 0, 0, 0, 0, 0};
  int on = 0;
  if (NC == 1) {
    const double b = Bb[6 * int64_t(p)], j = Bj[6 * int64_t(p)];
    if (hits[p] > 0.0 && b > 0.0 && j > 0.0) {
      on = 1;
      ob[0] = 1.0 / b;
      oj[0] = 1.0 / j;
      os[0] = 1.0 / sqrt(b);
      oq[0] = sqrt(b);
    }
  } else if (hits[p] > 0.0) {
    double A[3][3], V[3][3];
    unpack_sym3(Bb + 6 * int64_t(p), A);
    jacobi_eig<3>(A, V);
    double lam[3] = {A[0][0], A[1][1], A[2][2]};
    double lmin = lam[0], lmax = lam[0];
    for (int i = 1; i < 3; ++i) {
      lmin = fmin(lmin, lam[i]);
      lmax = fmax(lmax, lam[i]);
    }
    if (lmax > 0.0 && lmin / lmax >= rcond) {
      double out[3][3];
      sym3_func(V, lam, [](double l) { return 1.0 / l; }, out);
      pack_sym3(out, ob);
      sym3_func(V, lam, [](double l) { return 1.0 / sqrt(l); }, out);
      pack_sym3(out, os);
      sym3_func(V, lam, [](double l) { return sqrt(l); }, out);
      pack_sym3(out, oq);
      double Aj[3][3], Vj[3][3];
      unpack_sym3(Bj + 6 * int64_t(p), Aj);
      jacobi_eig<3>(Aj, Vj);
      double lj[3] = {Aj[0][0], Aj[1][1], Aj[2][2]};
      if (fmin(fmin(lj[0], lj[1]), lj[2]) > 0.0) {
        on = 1;
        sym3_func(Vj, lj, [](double l) { return 1.0 / l; }, out);
        pack_sym3(out, oj);
      } else {
        for (int k = 0; k < 6; ++k) ob[k] = os[k] = oq[k] = 0.0;
      }
    }
  }
  mask[p] = on;
  for (int k = 0; k < 6; ++k) {
    binv_b[6 * int64_t(p) + k] = ob[k];
    binv_j[6 * int64_t(p) + k] = oj[k];
    siginv[6 * int64_t(p) + k] = os[k];
    sigma[6 * int64_t(p) + k] = oq[k];
  }
}

template <int NC>
__global__ void k_binned_apply(const double* __restrict__ binv, const int32_t* __restrict__ mask,
                               const double* __restrict__ r, double* __restrict__ z, int npix) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const double* b = binv + 6 * int64_t(p);
  if (NC == 1) {
    z[p] = mask[p] ? b[0] * r[p] : 0.0;
  } else {
    const double r0 = r[p], r1 = r[npix + p], r2 = r[2 * npix + p];
    const bool on = mask[p] != 0;
    z[p] = on ? b[0] * r0 + b[1] * r1 + b[2] * r2 : 0.0;
    z[npix + p] = on ? b[1] * r0 + b[3] * r1 + b[4] * r2 : 0.0;
    z[2 * npix + p] = on ? b[2] * r0 + b[4] * r1 + b[5] * r2 : 0.0;
  }
}

// counts pixel ids outside [-1, npix) (stored pointing), non-finite boresight
// values, and non-finite or negative 1/N(f)
__global__ void k_validate(const int32_t* __restrict__ pix, int64_t total, int npix,
                           const double* __restrict__ bore, int64_t nbore,
                           const float* __restrict__ iN, int64_t niN, int* __restrict__ bad) {
  int c = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  if (pix) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total; i += stride) {
      const int p = pix[i];
      c += (p < -1 || p >= npix) ? 1 : 0;
    }
  }
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < nbore; i += stride)
    c += isfinite(bore[i]) ? 0 : 1;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < niN; i += stride) {
    const float v = iN[i];
    c += (!(v >= 0.0f) || isinf(v)) ? 1 : 0;
  }
  if (c) atomicAdd(bad, c);
}

__global__ void k_count_active(const int32_t* __restrict__ mask, int npix, int* __restrict__ out) {
  int c = 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += gridDim.x * blockDim.x)
    c += mask[p];
  atomicAdd(out, c);
}

mm_status binned_setup(ScanImpl* s, hipStream_t st) {
  const Layout& L = s->lay;
  const int npix = s->npix;
  {
    int* bad = s->at<int>(L.misc);
    mm_status r0;
    if ((r0 = fill_zero(bad, 4, st)) != MM_OK) return r0;
    const int64_t total = int64_t(s->ndet) * s->n;
    const int64_t niN = int64_t(s->ndet) * (s->n / 2 + 1);
    const bool otf = s->plan.otf;
    hipLaunchKernelGGL(k_validate, dim3(2048), dim3(256), 0, st, otf ? nullptr : s->d.pix, total,
                       npix, otf ? s->d.bore : nullptr, otf ? int64_t(6) * s->n : 0,
                       s->d.inv_noise, niN, bad);
    if (otf)
      hipLaunchKernelGGL(k_validate, dim3(1), dim3(256), 0, st, nullptr, 0, npix, s->d.det_off,
                         int64_t(4) * s->ndet, nullptr, 0, bad);
    if (s->plan.corr_rank > 0)
      hipLaunchKernelGGL(k_validate_finite, dim3(256), dim3(256), 0, st, s->d.corr_V,
                         int64_t(s->plan.corr_nbins) * s->ndet * s->plan.corr_rank, bad);
    MM_HIP(hipGetLastError());
    int h = 0;
    MM_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    if (h)
      return fail(MM_EINVAL,
                  "pix outside [-1, ny*nx), bore / det_off non-finite, inv_noise negative / "
                  "non-finite or corr_V non-finite");
  }
  hipLaunchKernelGGL(k_det_weights, dim3(s->ndet), dim3(256), 0, st, s->d.inv_noise, s->n,
                     s->at<double>(L.detw));
  if (s->plan.corr_rank > 0)
    hipLaunchKernelGGL(k_det_weights_corr, dim3((s->ndet + 255) / 256), dim3(256), 0, st,
                       s->d.corr_V, s->at<int32_t>(L.corr_edges), s->plan.corr_nbins,
                       s->plan.corr_rank, s->ndet, s->n, s->at<double>(L.detw));
  mm_status r;
  if ((r = fill_zero(s->ws + L.hits, size_t(npix) * 8, st)) != MM_OK) return r;
  if ((r = fill_zero(s->ws + L.bb, size_t(npix) * 6 * 8, st)) != MM_OK) return r;
  if ((r = fill_zero(s->ws + L.bj, size_t(npix) * 6 * 8, st)) != MM_OK) return r;
  const int64_t total = int64_t(s->ndet) * s->n;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  const Bore bo = scan_bore(s);
  if (s->plan.csr) {
    // build the pixel-major index first, then sum through it
    if ((r = csr_setup(s, st)) != MM_OK) return r;
    const int G = s->plan.G, ngroups = (s->ndet + G - 1) / G;
    // boresight pointing: float64 weights from the model, not the index's float32
    // copy; angle-coded index: the stored time-major weights themselves
    // (the run-length index keeps no weights: the time-major ones always)
    const bool rle = s->plan.rle;
    const float2* w = s->plan.csr_w && !s->plan.otf && !s->csr_ang && !rle
                          ? s->at<float2>(L.csr_w)
                          : nullptr;
    const bool tm = (s->csr_ang || rle) && !s->plan.otf;
    const float* c2 = tm ? s->d.cos2psi : nullptr;
    const float* s2 = tm ? s->d.sin2psi : nullptr;
    const dim3 gg((npix + 15) / 16);
    auto go = [&](auto nc, auto rl) {
      constexpr int NC_ = decltype(nc)::value;
      constexpr bool R_ = decltype(rl)::value;
      hipLaunchKernelGGL((k_binned_gather<NC_, R_>), gg, dim3(256), 0, st,
                         s->at<int32_t>(L.csr_off), s->at<int32_t>(L.csr_idx), w, c2, s2, bo,
                         s->at<double>(L.detw), ngroups, G, int(s->n), npix,
                         s->at<double>(L.hits), s->at<double>(L.bb), s->at<double>(L.bj));
    };
    using N3 = std::integral_constant<int, 3>;
    using N1 = std::integral_constant<int, 1>;
    if (s->nc == 3) {
      if (rle) go(N3{}, std::true_type{}); else go(N3{}, std::false_type{});
    } else {
      if (rle) go(N1{}, std::true_type{}); else go(N1{}, std::false_type{});
    }
  } else if (s->nc == 3)
    hipLaunchKernelGGL(k_binned_accum<3>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, s->at<double>(L.detw), s->n, total, npix,
                       s->at<double>(L.hits), s->at<double>(L.bb), s->at<double>(L.bj));
  else
    hipLaunchKernelGGL(k_binned_accum<1>, dim3(unsigned(blocks)), dim3(256), 0, st, s->d.pix, bo,
                       s->d.cos2psi, s->d.sin2psi, s->at<double>(L.detw), s->n, total, npix,
                       s->at<double>(L.hits), s->at<double>(L.bb), s->at<double>(L.bj));
  const dim3 g((npix + 255) / 256), b(256);
  const double rc = s->d.mask_rcond > 0 ? s->d.mask_rcond : 1e-3;
  if (s->nc == 3)
    hipLaunchKernelGGL(k_binned_finalize<3>, g, b, 0, st, s->at<double>(L.hits),
                       s->at<double>(L.bb), s->at<double>(L.bj), npix, rc, s->at<int32_t>(L.mask),
                       s->at<double>(L.binv_b), s->at<double>(L.binv_j), s->at<double>(L.siginv),
                       s->at<double>(L.sigma));
  else
    hipLaunchKernelGGL(k_binned_finalize<1>, g, b, 0, st, s->at<double>(L.hits),
                       s->at<double>(L.bb), s->at<double>(L.bj), npix, rc, s->at<int32_t>(L.mask),
                       s->at<double>(L.binv_b), s->at<double>(L.binv_j), s->at<double>(L.siginv),
                       s->at<double>(L.sigma));
  int* cnt = s->at<int>(L.misc);
  if ((r = fill_zero(cnt, 4, st)) != MM_OK) return r;
  hipLaunchKernelGGL(k_count_active, dim3(64), dim3(256), 0, st, s->at<int32_t>(L.mask), npix, cnt);
  MM_HIP(hipGetLastError());
  int h = 0;
  MM_HIP(hipMemcpyAsync(&h, cnt, 4, hipMemcpyDeviceToHost, st));
  MM_HIP(hipStreamSynchronize(st));
  s->n_active = h;
  return MM_OK;
}

mm_status binned_apply(ScanImpl* s, int jacobi, const double* r, double* z, hipStream_t st) {
  const Layout& L = s->lay;
  const double* binv = s->at<double>(jacobi ? L.binv_j : L.binv_b);
  const dim3 g((s->npix + 255) / 256), b(256);
  if (s->nc == 3)
    hipLaunchKernelGGL(k_binned_apply<3>, g, b, 0, st, binv, s->at<int32_t>(L.mask), r, z, s->npix);
  else
    hipLaunchKernelGGL(k_binned_apply<1>, g, b, 0, st, binv, s->at<int32_t>(L.mask), r, z, s->npix);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
