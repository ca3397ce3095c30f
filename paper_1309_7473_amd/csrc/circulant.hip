// The circulant ("constant correlation") preconditioner (paper eq. 7-13).
//
// Build (once per solve):
//   r      = active pixel nearest (ny/2, nx/2), smallest id on ties;
//   c_g    = A e_(r,g), g < ncomp: one row of A per Stokes component (eq. 6);
//   q(d)   = Sigma_r^-T C_j Sigma_j^-1, j = r + d mod (ny, nx), (C_j)_gb =
//            c_g[b, j], zero for inactive j (eq. 10, eq. 13);
//   q(d)  *= exp(-|d~|^2 / 2 sigma^2) (minimal-image d~, Regularization);
//   q(d)   = (q(d) + q(-d)^T) / 2 (optional);
//   K(k)   = conj(FFT2 q)(k) (eq. 11), a Hermitian ncomp x ncomp block per
//            wavenumber; eigenvalues floored at eps * max over all k; K^-1.
// Apply: z = Sigma^-1 F^-1 K^-1 F Sigma^-T r (eq. 12).
//
// Everything map-sized runs in float64.  The 2-D FFTs are row and column
// passes of the LDS Stockham FFT over complex planes [plane][ny][nx].
#include "fft_lds.h"
#include "linalg_small.h"
#include "mm_internal.h"

namespace mm {

__global__ void k_ref_key(const int32_t* __restrict__ mask, int ny, int nx,
                          unsigned long long* __restrict__ key) {
  const int cy = ny / 2, cx_ = nx / 2;
  unsigned long long best = ~0ull;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < ny * nx; p += gridDim.x * blockDim.x) {
    if (!mask[p]) continue;
    const long long dy = p / nx - cy, dx = p % nx - cx_;
    const unsigned long long k =
        (static_cast<unsigned long long>(dy * dy + dx * dx) << 32) | static_cast<unsigned>(p);
    best = k < best ? k : best;
  }
  atomicMin(key, best);
}

__global__ void k_set_unit(double* __restrict__ e, int64_t idx) { e[idx] = 1.0; }

// q planes: out[(a*nc+b)][d] = complex(q_ab(d), 0)
template <int NC>
__device__ __forceinline__ void q_raw(int dy, int dx, int ry, int rx, int ny, int nx,
                                      const int32_t* mask, const double* probe,
                                      const double* siginv, double (&q)[NC][NC]) {
  const int npix = ny * nx;
  const int jy = (ry + dy) % ny, jx = (rx + dx) % nx;
  const int j = jy * nx + jx;
  const int r = ry * nx + rx;
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) q[a][b] = 0.0;
  if (!mask[j]) return;
  double Sr[NC][NC], Sj[NC][NC], Cm[NC][NC];
  if constexpr (NC == 3) {
    unpack_sym3(siginv + 6 * int64_t(r), Sr);
    unpack_sym3(siginv + 6 * int64_t(j), Sj);
  } else {
    Sr[0][0] = siginv[6 * int64_t(r)];
    Sj[0][0] = siginv[6 * int64_t(j)];
  }
#pragma unroll
  for (int g = 0; g < NC; ++g)
#pragma unroll
    for (int b = 0; b < NC; ++b) Cm[g][b] = probe[(int64_t(g) * NC + b) * npix + j];
  // q = Sr^T Cm Sj
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      double s = 0.0;
#pragma unroll
      for (int g = 0; g < NC; ++g)
#pragma unroll
        for (int h = 0; h < NC; ++h) s += Sr[g][a] * Cm[g][h] * Sj[h][b];
      q[a][b] = s;
    }
}

template <int NC>
__global__ void k_q_assemble(const int32_t* __restrict__ mask, const double* __restrict__ probe,
                             const double* __restrict__ siginv, int ny, int nx, int ref,
                             double sigma, int symmetrize, Cx<double>* __restrict__ planes) {
  const int npix = ny * nx;
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= npix) return;
  const int dy = d / nx, dx = d % nx;
  const int ry = ref / nx, rx = ref % nx;
  double q[NC][NC];
  q_raw<NC>(dy, dx, ry, rx, ny, nx, mask, probe, siginv, q);
  double g = 1.0;
  if (sigma > 0.0) {
    const int my = dy > ny / 2 ? dy - ny : dy;
    const int mx = dx > nx / 2 ? dx - nx : dx;
    g = exp(-double(my * my + mx * mx) / (2.0 * sigma * sigma));
  }
  if (symmetrize) {
    double qm[NC][NC];
    q_raw<NC>((ny - dy) % ny, (nx - dx) % nx, ry, rx, ny, nx, mask, probe, siginv, qm);
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int b = 0; b < NC; ++b) q[a][b] = 0.5 * (q[a][b] + qm[b][a]);
  }
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      Cx<double> v;
      v.x = g * q[a][b];
      v.y = 0.0;
      planes[int64_t(a * NC + b) * npix + d] = v;
    }
}

// ------------------------------------------------------------ 2-D FFT
template <bool INV>
__global__ void __launch_bounds__(kNT) k_map_rows(Cx<double>* __restrict__ planes, int logny,
                                                  int lognx, int logRB, int logLmax,
                                                  const Cx<double>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx;
  const int cnt = nx << logRB;
  Cx<double>* base = planes + (int64_t(blockIdx.y) << (logny + lognx)) + (int64_t(blockIdx.x) * cnt);
  for (int e = threadIdx.x; e < cnt; e += kNT) buf[e] = base[e];
  __syncthreads();
  FftShape sh{lognx, logRB, 1, nx, false, logLmax};
  lds_fft<double, kNT, kMapE, INV>(buf, sh, tw);
  for (int e = threadIdx.x; e < cnt; e += kNT) base[e] = buf[e];
}

template <bool INV>
__global__ void __launch_bounds__(kNT) k_map_cols(Cx<double>* __restrict__ planes, int logny,
                                                  int lognx, int logCB, int logLmax,
                                                  const Cx<double>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx, ny = 1 << logny, CB = 1 << logCB;
  Cx<double>* base = planes + (int64_t(blockIdx.y) << (logny + lognx)) + int64_t(blockIdx.x) * CB;
  const int cnt = CB * ny;
  for (int e = threadIdx.x; e < cnt; e += kNT) {
    const int y = e >> logCB, c = e & (CB - 1);
    buf[e] = base[int64_t(y) * nx + c];
  }
  __syncthreads();
  FftShape sh{logny, logCB, CB, 1, true, logLmax};
  lds_fft<double, kNT, kMapE, INV>(buf, sh, tw);
  for (int e = threadIdx.x; e < cnt; e += kNT) {
    const int y = e >> logCB, c = e & (CB - 1);
    base[int64_t(y) * nx + c] = buf[e];
  }
}

static int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

mm_status map_fft(ScanImpl* s, Cx<double>* planes, int nplanes, bool inv, hipStream_t st) {
  const int logny = ilog2i(s->ny), lognx = ilog2i(s->nx);
  const int cap = kMapE * kNT;  // complex elements per block
  int logRB = ilog2i(cap) - lognx;
  if (logRB > logny) logRB = logny;
  if (logRB < 0) logRB = 0;
  int logCB = ilog2i(cap) - logny;
  if (logCB > lognx) logCB = lognx;
  if (logCB < 0) logCB = 0;
  const Cx<double>* tw = s->at<Cx<double>>(s->lay.tw_map);
  const int logL = s->plan.logMapL;
  const size_t ldsr = (size_t(s->nx) << logRB) * sizeof(Cx<double>);
  const size_t ldsc = (size_t(s->ny) << logCB) * sizeof(Cx<double>);
  const dim3 gr(unsigned(s->ny >> logRB), unsigned(nplanes));
  const dim3 gc(unsigned(s->nx >> logCB), unsigned(nplanes));
  if (!inv) {
    hipLaunchKernelGGL(k_map_rows<false>, gr, dim3(kNT), ldsr, st, planes, logny, lognx, logRB, logL, tw);
    hipLaunchKernelGGL(k_map_cols<false>, gc, dim3(kNT), ldsc, st, planes, logny, lognx, logCB, logL, tw);
  } else {
    hipLaunchKernelGGL(k_map_cols<true>, gc, dim3(kNT), ldsc, st, planes, logny, lognx, logCB, logL, tw);
    hipLaunchKernelGGL(k_map_rows<true>, gr, dim3(kNT), ldsr, st, planes, logny, lognx, logRB, logL, tw);
  }
  MM_HIP(hipGetLastError());
  return MM_OK;
}

// ------------------------------------------------- per-wavenumber inverse
// Real embedding of the Hermitian part of K = conj(qhat): R = [[Re, -Im], [Im, Re]].
template <int NC>
__device__ __forceinline__ void embed_K(const Cx<double>* qhat, int64_t npix, int64_t k,
                                        double (&R)[2 * NC][2 * NC]) {
  double re[NC][NC], im[NC][NC];
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      const Cx<double> v = qhat[int64_t(a * NC + b) * npix + k];
      re[a][b] = v.x;
      im[a][b] = -v.y;  // conj
    }
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      const double hr = 0.5 * (re[a][b] + re[b][a]);
      const double hi = 0.5 * (im[a][b] - im[b][a]);
      R[a][b] = hr;
      R[NC + a][NC + b] = hr;
      R[NC + a][b] = hi;
      R[a][NC + b] = -hi;
    }
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long* addr, double v) {
  if (v > 0.0) atomicMax(addr, static_cast<unsigned long long>(__double_as_longlong(v)));
}

template <int NC>
__global__ void k_kinv_lmax(const Cx<double>* __restrict__ qhat, int npix,
                            unsigned long long* __restrict__ lmax_bits) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (k < npix) {
    double R[2 * NC][2 * NC], V[2 * NC][2 * NC];
    embed_K<NC>(qhat, npix, k, R);
    jacobi_eig<2 * NC>(R, V);
#pragma unroll
    for (int i = 0; i < 2 * NC; ++i) m = fmax(m, R[i][i]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomic_max_pos(lmax_bits, m);
}

template <int NC>
__global__ void k_kinv_floor(const Cx<double>* __restrict__ qhat, int npix,
                             const unsigned long long* __restrict__ lmax_bits, double eps,
                             Cx<double>* __restrict__ kinv, int* __restrict__ nfloor) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npix) return;
  const double lmax = __longlong_as_double(static_cast<long long>(*lmax_bits));
  const double floor_v = eps * lmax;
  double R[2 * NC][2 * NC], V[2 * NC][2 * NC];
  embed_K<NC>(qhat, npix, k, R);
  jacobi_eig<2 * NC>(R, V);
  double f[2 * NC];
  int nf = 0;
#pragma unroll
  for (int i = 0; i < 2 * NC; ++i) {
    double l = R[i][i];
    if (l < floor_v) {
      l = floor_v;
      ++nf;
    }
    f[i] = 1.0 / l;
  }
  if (nf) atomicAdd(nfloor, nf);  // every eigenvalue of K is counted twice
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int i = 0; i < 2 * NC; ++i) {
        sr += V[a][i] * f[i] * V[b][i];
        si += V[NC + a][i] * f[i] * V[b][i];
      }
      Cx<double> v;
      v.x = sr;
      v.y = si;
      kinv[int64_t(k) * NC * NC + a * NC + b] = v;
    }
}

// eq. 12 literally: general complex inverse of K = conj(qhat), no floor.
template <int NC>
__global__ void k_kinv_general(const Cx<double>* __restrict__ qhat, int npix,
                               Cx<double>* __restrict__ kinv) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npix) return;
  Cx<double> K[NC][NC];
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) K[a][b] = conj(qhat[int64_t(a * NC + b) * npix + k]);
  Cx<double>* out = kinv + int64_t(k) * NC * NC;
  if constexpr (NC == 1) {
    const double den = K[0][0].x * K[0][0].x + K[0][0].y * K[0][0].y;
    out[0] = cx(K[0][0].x / den, -K[0][0].y / den);
  } else {
    // adjugate / determinant
    Cx<double> adj[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int r0 = (b + 1) % 3, r1 = (b + 2) % 3, c0 = (a + 1) % 3, c1 = (a + 2) % 3;
        adj[a][b] = K[r0][c0] * K[r1][c1] - K[r0][c1] * K[r1][c0];
      }
    Cx<double> det = K[0][0] * adj[0][0] + K[0][1] * adj[1][0] + K[0][2] * adj[2][0];
    const double dd = det.x * det.x + det.y * det.y;
    const Cx<double> inv = cx(det.x / dd, -det.y / dd);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) out[a * 3 + b] = adj[a][b] * inv;
  }
}

// ------------------------------------------------------------ apply
template <int NC>
__global__ void k_circ_pre(const double* __restrict__ r, const double* __restrict__ siginv,
                           const int32_t* __restrict__ mask, int npix,
                           Cx<double>* __restrict__ planes) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const double* S = siginv + 6 * int64_t(p);
  double u[NC];
  if constexpr (NC == 1) {
    u[0] = mask[p] ? S[0] * r[p] : 0.0;
  } else {
    const bool on = mask[p] != 0;
    const double r0 = on ? r[p] : 0.0, r1 = on ? r[npix + p] : 0.0, r2 = on ? r[2 * npix + p] : 0.0;
    u[0] = S[0] * r0 + S[1] * r1 + S[2] * r2;
    u[1] = S[1] * r0 + S[3] * r1 + S[4] * r2;
    u[2] = S[2] * r0 + S[4] * r1 + S[5] * r2;
  }
#pragma unroll
  for (int a = 0; a < NC; ++a) planes[int64_t(a) * npix + p] = cx(u[a], 0.0);
}

template <int NC>
__global__ void k_circ_kmul(Cx<double>* __restrict__ planes, const Cx<double>* __restrict__ kinv,
                            int npix, double scale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npix) return;
  Cx<double> u[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) u[a] = planes[int64_t(a) * npix + k];
  const Cx<double>* Ki = kinv + int64_t(k) * NC * NC;
#pragma unroll
  for (int a = 0; a < NC; ++a) {
    Cx<double> s = cx(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < NC; ++b) s = s + Ki[a * NC + b] * u[b];
    planes[int64_t(a) * npix + k] = scale * s;
  }
}

template <int NC>
__global__ void k_circ_post(const Cx<double>* __restrict__ planes, const double* __restrict__ siginv,
                            const int32_t* __restrict__ mask, int npix, double* __restrict__ z) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const double* S = siginv + 6 * int64_t(p);
  const bool on = mask[p] != 0;
  if constexpr (NC == 1) {
    z[p] = on ? S[0] * planes[p].x : 0.0;
  } else {
    const double v0 = planes[p].x, v1 = planes[npix + p].x, v2 = planes[2 * int64_t(npix) + p].x;
    z[p] = on ? S[0] * v0 + S[1] * v1 + S[2] * v2 : 0.0;
    z[npix + p] = on ? S[1] * v0 + S[3] * v1 + S[4] * v2 : 0.0;
    z[2 * int64_t(npix) + p] = on ? S[2] * v0 + S[4] * v1 + S[5] * v2 : 0.0;
  }
}

// ------------------------------------------------------------ host
struct Misc {
  unsigned long long ref_key;
  unsigned long long lmax_bits;
  int nfloor;
  int active;
};

template <int NC>
static mm_status build_t(ScanImpl* s, const mm_precon_opts* o, hipStream_t st) {
  const Layout& L = s->lay;
  const int npix = s->npix, ny = s->ny, nx = s->nx;
  const dim3 g((npix + 255) / 256), b(256);
  Misc* misc = s->at<Misc>(L.misc + 64);
  const int32_t* mask = s->at<int32_t>(L.mask);
  int ref;
  if (o && o->ref_y >= 0 && o->ref_x >= 0) {
    ref = o->ref_y * nx + o->ref_x;
  } else {
    Misc init{};
    init.ref_key = ~0ull;
    MM_HIP(hipMemcpyAsync(misc, &init, sizeof(Misc), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_ref_key, dim3(64), dim3(256), 0, st, mask, ny, nx, &misc->ref_key);
    MM_HIP(hipGetLastError());
    Misc h{};
    MM_HIP(hipMemcpyAsync(&h, misc, sizeof(Misc), hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    if (h.ref_key == ~0ull) return fail(MM_EINVAL, "no active pixel to probe");
    ref = int(h.ref_key & 0xffffffffull);
  }
  {
    int32_t mref = 0;
    MM_HIP(hipMemcpyAsync(&mref, mask + ref, 4, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    if (!mref) return fail(MM_EINVAL, "reference pixel is not active");
  }
  s->ref_pixel = ref;
  // probes c_g = A e_(r, g)
  double* probe = s->at<double>(L.probe);
  double* e = s->at<double>(L.vec) + 4 * int64_t(NC) * npix;  // the spare CG vector
  for (int gi = 0; gi < NC; ++gi) {
    mm_status r;
    if ((r = fill_zero(e, size_t(NC) * npix * 8, st)) != MM_OK) return r;
    hipLaunchKernelGGL(k_set_unit, dim3(1), dim3(1), 0, st, e, int64_t(gi) * npix + ref);
    MM_HIP(hipGetLastError());
    if ((r = filter_pipeline(s, 0, nullptr, e, probe + int64_t(gi) * NC * npix, st)) != MM_OK)
      return r;
  }
  const double sigma = o ? o->gauss_sigma_px : 0.0;
  const int sym = o ? (o->symmetrize != 0) : 1;
  double eps = o ? o->eig_floor_rel : 1e-6;
  if (!(eps > 0.0)) eps = 1e-6;
  Cx<double>* planes = s->at<Cx<double>>(L.planes);
  hipLaunchKernelGGL(k_q_assemble<NC>, g, b, 0, st, mask, probe, s->at<double>(L.siginv), ny, nx,
                     ref, sigma, sym, planes);
  MM_HIP(hipGetLastError());
  mm_status r;
  if ((r = map_fft(s, planes, NC * NC, false, st)) != MM_OK) return r;
  Cx<double>* kinv = s->at<Cx<double>>(L.kinv);
  Misc h{};
  if (sym) {
    Misc init{};
    init.ref_key = h.ref_key;
    MM_HIP(hipMemcpyAsync(misc, &init, sizeof(Misc), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_kinv_lmax<NC>, g, b, 0, st, planes, npix, &misc->lmax_bits);
    hipLaunchKernelGGL(k_kinv_floor<NC>, g, b, 0, st, planes, npix, &misc->lmax_bits, eps, kinv,
                       &misc->nfloor);
    MM_HIP(hipGetLastError());
    MM_HIP(hipMemcpyAsync(&h, misc, sizeof(Misc), hipMemcpyDeviceToHost, st));
  } else {
    hipLaunchKernelGGL(k_kinv_general<NC>, g, b, 0, st, planes, npix, kinv);
    MM_HIP(hipGetLastError());
  }
  MM_HIP(hipStreamSynchronize(st));
  if (sym && h.lmax_bits == 0) return fail(MM_EINVAL, "circulant kernel has no positive eigenvalue");
  s->n_floored = sym ? h.nfloor / 2 : 0;
  s->circ_built = true;
  s->circ_sym = sym;
  return MM_OK;
}

mm_status circulant_build(ScanImpl* s, const mm_precon_opts* o, hipStream_t st) {
  s->circ_built = false;
  return s->nc == 3 ? build_t<3>(s, o, st) : build_t<1>(s, o, st);
}

template <int NC>
static mm_status apply_t(ScanImpl* s, const double* r, double* z, hipStream_t st) {
  const Layout& L = s->lay;
  const int npix = s->npix;
  const dim3 g((npix + 255) / 256), b(256);
  Cx<double>* planes = s->at<Cx<double>>(L.planes);
  hipLaunchKernelGGL(k_circ_pre<NC>, g, b, 0, st, r, s->at<double>(L.siginv),
                     s->at<int32_t>(L.mask), npix, planes);
  MM_HIP(hipGetLastError());
  mm_status rc;
  if ((rc = map_fft(s, planes, NC, false, st)) != MM_OK) return rc;
  hipLaunchKernelGGL(k_circ_kmul<NC>, g, b, 0, st, planes, s->at<Cx<double>>(L.kinv), npix,
                     1.0 / double(npix));
  MM_HIP(hipGetLastError());
  if ((rc = map_fft(s, planes, NC, true, st)) != MM_OK) return rc;
  hipLaunchKernelGGL(k_circ_post<NC>, g, b, 0, st, planes, s->at<double>(L.siginv),
                     s->at<int32_t>(L.mask), npix, z);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

mm_status circulant_apply(ScanImpl* s, const double* r, double* z, hipStream_t st) {
  if (!s->circ_built) return fail(MM_ENOTBUILT, "circulant preconditioner not built");
  return s->nc == 3 ? apply_t<3>(s, r, z, st) : apply_t<1>(s, r, z, st);
}

}  // namespace mm
