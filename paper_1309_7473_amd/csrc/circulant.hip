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
#include <cmath>
#include <vector>

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
template <bool INV, int NT, int E>
__global__ void __launch_bounds__(NT) k_map_rows(Cx<double>* __restrict__ planes, int logny,
                                                  int lognx, int logRB, int logLmax,
                                                  const Cx<double>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx;
  const int cnt = nx << logRB;
  Cx<double>* base = planes + (int64_t(blockIdx.y) << (logny + lognx)) + (int64_t(blockIdx.x) * cnt);
  for (int e = threadIdx.x; e < cnt; e += NT) buf[e] = base[e];
  __syncthreads();
  FftShape sh{lognx, logRB, 1, nx, false, logLmax};
  lds_fft<double, NT, E, INV>(buf, sh, tw);
  for (int e = threadIdx.x; e < cnt; e += NT) base[e] = buf[e];
}

template <bool INV, int NT, int E>
__global__ void __launch_bounds__(NT) k_map_cols(Cx<double>* __restrict__ planes, int logny,
                                                  int lognx, int logCB, int logLmax,
                                                  const Cx<double>* __restrict__ tw) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx, ny = 1 << logny, CB = 1 << logCB;
  Cx<double>* base = planes + (int64_t(blockIdx.y) << (logny + lognx)) + int64_t(blockIdx.x) * CB;
  const int cnt = CB * ny;
  for (int e = threadIdx.x; e < cnt; e += NT) {
    const int y = e >> logCB, c = e & (CB - 1);
    buf[e] = base[int64_t(y) * nx + c];
  }
  __syncthreads();
  FftShape sh{logny, logCB, CB, 1, true, logLmax};
  lds_fft<double, NT, E, INV>(buf, sh, tw);
  for (int e = threadIdx.x; e < cnt; e += NT) {
    const int y = e >> logCB, c = e & (CB - 1);
    base[int64_t(y) * nx + c] = buf[e];
  }
}

static int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

static mm_status map_fft_dims(ScanImpl* s, Cx<double>* planes, int logny, int lognx, int nplanes,
                              bool inv, hipStream_t st);

mm_status map_fft(ScanImpl* s, Cx<double>* planes, int nplanes, bool inv, hipStream_t st) {
  return map_fft_dims(s, planes, ilog2i(s->ny), ilog2i(s->nx), nplanes, inv, st);
}

// nplanes [2^logny][2^lognx] planes (sides up to the map's), with blocks of
// NT threads holding E elements each; parts: 1 the row transforms, 2 the
// column transforms, 3 both
template <int NT, int E>
static mm_status map_fft_blocks(ScanImpl* s, Cx<double>* planes, int logny, int lognx,
                                int nplanes, bool inv, hipStream_t st, int parts = 3) {
  const int ny = 1 << logny, nx = 1 << lognx;
  const int cap = E * NT;  // complex elements per block
  int logRB = ilog2i(cap) - lognx;
  if (logRB > logny) logRB = logny;
  if (logRB < 0) logRB = 0;
  int logCB = ilog2i(cap) - logny;
  if (logCB > lognx) logCB = lognx;
  if (logCB < 0) logCB = 0;
  const Cx<double>* tw = s->at<Cx<double>>(s->lay.tw_map);
  const int logL = s->plan.logMapL;
  const size_t ldsr = (size_t(nx) << logRB) * sizeof(Cx<double>);
  const size_t ldsc = (size_t(ny) << logCB) * sizeof(Cx<double>);
  // planes go in chunks of at most 65535 (the grid's y limit)
  for (int p0 = 0; p0 < nplanes; p0 += 65535) {
    const int np = nplanes - p0 < 65535 ? nplanes - p0 : 65535;
    Cx<double>* pl = planes + (int64_t(p0) << (logny + lognx));
    const dim3 gr(unsigned(ny >> logRB), unsigned(np));
    const dim3 gc(unsigned(nx >> logCB), unsigned(np));
    if (!inv) {
      if (parts & 1)
        hipLaunchKernelGGL((k_map_rows<false, NT, E>), gr, dim3(NT), ldsr, st, pl, logny, lognx, logRB, logL, tw);
      if (parts & 2)
        hipLaunchKernelGGL((k_map_cols<false, NT, E>), gc, dim3(NT), ldsc, st, pl, logny, lognx, logCB, logL, tw);
    } else {
      if (parts & 2)
        hipLaunchKernelGGL((k_map_cols<true, NT, E>), gc, dim3(NT), ldsc, st, pl, logny, lognx, logCB, logL, tw);
      if (parts & 1)
        hipLaunchKernelGGL((k_map_rows<true, NT, E>), gr, dim3(NT), ldsr, st, pl, logny, lognx, logRB, logL, tw);
    }
    MM_HIP(hipGetLastError());
  }
  return MM_OK;
}

static mm_status map_fft_dims(ScanImpl* s, Cx<double>* planes, int logny, int lognx, int nplanes,
                              bool inv, hipStream_t st) {
  // sides up to 1024: smaller blocks (16 or 32 KB of LDS) put more of them
  // on the chip; larger sides need the 64 KB block
  const int side = (logny > lognx ? logny : lognx);
  if (side <= 10) return map_fft_blocks<128, 8>(s, planes, logny, lognx, nplanes, inv, st);
  return map_fft_blocks<kNT, kMapE>(s, planes, logny, lognx, nplanes, inv, st);
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

// blockIdx.y batches independent kernels (the tiles of the tiled
// preconditioner): planes, inverses and the maximum advance by one kernel.
template <int NC>
__global__ void k_kinv_lmax(const Cx<double>* __restrict__ qhat, int npix,
                            unsigned long long* __restrict__ lmax_bits) {
  qhat += int64_t(blockIdx.y) * NC * NC * npix;
  lmax_bits += blockIdx.y;
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
                             Cx<double>* __restrict__ kinv, int* __restrict__ nfloor,
                             const int32_t* __restrict__ skip = nullptr) {
  qhat += int64_t(blockIdx.y) * NC * NC * npix;
  kinv += int64_t(blockIdx.y) * NC * NC * npix;
  lmax_bits += blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= npix) return;
  const double lmax = __longlong_as_double(static_cast<long long>(*lmax_bits));
  // a tile without active pixels (or without a positive eigenvalue) adds nothing
  if (skip && (skip[blockIdx.y] < 0 || !(lmax > 0.0))) {
#pragma unroll
    for (int i = 0; i < NC * NC; ++i) kinv[int64_t(k) * NC * NC + i] = cx(0.0, 0.0);
    return;
  }
  const double floor_v = eps * lmax;
  double R[2 * NC][2 * NC], V[2 * NC][2 * NC];
  embed_K<NC>(qhat, npix, k, R);
  jacobi_eig<2 * NC>(R, V);
  // The real embedding holds every eigenvalue of the Hermitian K twice; in
  // ascending order the copies are neighbours (ranks 2m and 2m+1).  Each
  // pair is taken as one eigenvalue (the mean of its two rounded copies),
  // floored as one and counted once, so both copies always get the same
  // 1/lambda and the floored count is that of K itself.
  int rank[2 * NC];
#pragma unroll
  for (int i = 0; i < 2 * NC; ++i) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < 2 * NC; ++j)
      c += (R[j][j] < R[i][i] || (R[j][j] == R[i][i] && j < i)) ? 1 : 0;
    rank[i] = c;
  }
  double f[2 * NC];
  int nf = 0;
#pragma unroll
  for (int i = 0; i < 2 * NC; ++i) {
    double partner = R[i][i];
#pragma unroll
    for (int j = 0; j < 2 * NC; ++j)
      if (rank[j] == (rank[i] ^ 1)) partner = R[j][j];
    double l = 0.5 * (R[i][i] + partner);
    if (l < floor_v) {
      l = floor_v;
      nf += (rank[i] & 1) ? 0 : 1;
    }
    f[i] = 1.0 / l;
  }
  if (nf) atomicAdd(nfloor, nf);
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
  planes += int64_t(blockIdx.y) * NC * npix;
  kinv += int64_t(blockIdx.y) * NC * NC * npix;
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

// ---------------------------------------------- fused apply (sides <= 1024)
// The seven steps of the apply (Sigma^-T, forward rows, forward columns, K^-1,
// inverse columns, inverse rows, Sigma^-1) in three kernels whose blocks hold
// the same pixels of all NC planes: the symmetric Sigma^-1 blocks and the
// per-wavenumber NC x NC products need every component at a pixel.  The NC
// planes of a block are transformed together as one batch (padded to NP = 4
// planes for I,Q,U, so that the batch count stays a power of two; the pad
// plane is zero and never stored), 128 threads a plane.  The transforms are
// the same Stockham stages as map_fft's; results agree with the seven-kernel
// path to rounding (the compiler may fuse multiply-adds differently).
constexpr int kFuseE = 8, kFuseCapLog = 10;   // 1024 complex elements a plane a block
template <int NC>
struct Fuse {
  static constexpr int NP = NC == 3 ? 4 : 1, LOGNP = NC == 3 ? 2 : 0;
  static constexpr int NT = (1 << kFuseCapLog) / kFuseE * NP;
};

// Sigma^-T r on RB rows, then the forward row transforms.  LDS [NP][RB][nx].
template <int NC>
__global__ void __launch_bounds__(Fuse<NC>::NT) k_circ_rows_pre(
    const double* __restrict__ r, const double* __restrict__ siginv,
    const int32_t* __restrict__ mask, int logny, int lognx, int logRB, int logLmax,
    const Cx<double>* __restrict__ tw, Cx<double>* __restrict__ planes) {
  constexpr int NT = Fuse<NC>::NT;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx;
  const int npix = 1 << (logny + lognx);
  const int cnt = nx << logRB;
  const int p0 = blockIdx.x * cnt;
  for (int e = threadIdx.x; e < cnt; e += NT) {
    const int p = p0 + e;
    const double* S = siginv + 6 * int64_t(p);
    const bool on = mask[p] != 0;
    if constexpr (NC == 1) {
      buf[e] = cx(on ? S[0] * r[p] : 0.0, 0.0);
    } else {
      const double r0 = on ? r[p] : 0.0, r1 = on ? r[npix + p] : 0.0,
                   r2 = on ? r[2 * npix + p] : 0.0;
      buf[e] = cx(S[0] * r0 + S[1] * r1 + S[2] * r2, 0.0);
      buf[cnt + e] = cx(S[1] * r0 + S[3] * r1 + S[4] * r2, 0.0);
      buf[2 * cnt + e] = cx(S[2] * r0 + S[4] * r1 + S[5] * r2, 0.0);
      buf[3 * cnt + e] = cx(0.0, 0.0);
    }
  }
  __syncthreads();
  FftShape sh{lognx, logRB + Fuse<NC>::LOGNP, 1, nx, false, logLmax};
  lds_fft<double, NT, kFuseE, false>(buf, sh, tw);
  for (int e = threadIdx.x; e < NC * cnt; e += NT) {
    const int a = e / cnt, i = e - a * cnt;
    planes[int64_t(a) * npix + p0 + i] = buf[e];
  }
}

// CB columns: forward column transforms, scale * K^-1(k) per wavenumber,
// inverse column transforms.  LDS [ny][NP][CB]: one batch of NP * CB columns.
template <int NC>
__global__ void __launch_bounds__(Fuse<NC>::NT) k_circ_cols_kmul(
    Cx<double>* __restrict__ planes, const Cx<double>* __restrict__ kinv, int logny, int lognx,
    int logCB, int logLmax, const Cx<double>* __restrict__ tw, double scale) {
  constexpr int NT = Fuse<NC>::NT, NP = Fuse<NC>::NP, LOGNP = Fuse<NC>::LOGNP;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx, CB = 1 << logCB;
  const int npix = 1 << (logny + lognx);
  // blockIdx.y: one of a batch of NC-plane sets (the tiles of the tiled apply)
  planes += int64_t(blockIdx.y) * NC * npix;
  kinv += int64_t(blockIdx.y) * NC * NC * npix;
  const int logW = logCB + LOGNP;             // LDS row: NP * CB elements
  const int tot = 1 << (logny + logW);
  const int x0 = blockIdx.x * CB;
  for (int e = threadIdx.x; e < tot; e += NT) {
    const int y = e >> logW, a = (e >> logCB) & (NP - 1), c = e & (CB - 1);
    buf[e] = a < NC ? planes[int64_t(a) * npix + int64_t(y) * nx + x0 + c] : cx(0.0, 0.0);
  }
  __syncthreads();
  FftShape sh{logny, logW, 1 << logW, 1, true, logLmax};
  lds_fft<double, NT, kFuseE, false>(buf, sh, tw);
  for (int e = threadIdx.x; e < (tot >> LOGNP); e += NT) {
    const int y = e >> logCB, c = e & (CB - 1);
    const int64_t k = int64_t(y) * nx + x0 + c;
    const Cx<double>* Ki = kinv + k * NC * NC;
    const int b0 = (y << logW) + c;
    Cx<double> u[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) u[a] = buf[b0 + a * CB];
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      Cx<double> t = cx(0.0, 0.0);
#pragma unroll
      for (int b = 0; b < NC; ++b) t = t + Ki[a * NC + b] * u[b];
      buf[b0 + a * CB] = scale * t;
    }
  }
  __syncthreads();
  lds_fft<double, NT, kFuseE, true>(buf, sh, tw);
  for (int e = threadIdx.x; e < tot; e += NT) {
    const int y = e >> logW, a = (e >> logCB) & (NP - 1), c = e & (CB - 1);
    if (a < NC) planes[int64_t(a) * npix + int64_t(y) * nx + x0 + c] = buf[e];
  }
}

// inverse row transforms on RB rows, then Sigma^-1 on the real parts.
// LDS [NP][RB][nx].
template <int NC>
__global__ void __launch_bounds__(Fuse<NC>::NT) k_circ_rows_post(
    const Cx<double>* __restrict__ planes, const double* __restrict__ siginv,
    const int32_t* __restrict__ mask, int logny, int lognx, int logRB, int logLmax,
    const Cx<double>* __restrict__ tw, double* __restrict__ z) {
  constexpr int NT = Fuse<NC>::NT, NP = Fuse<NC>::NP;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* buf = reinterpret_cast<Cx<double>*>(smem);
  const int nx = 1 << lognx;
  const int npix = 1 << (logny + lognx);
  const int cnt = nx << logRB;
  const int p0 = blockIdx.x * cnt;
  for (int e = threadIdx.x; e < NP * cnt; e += NT) {
    const int a = e / cnt, i = e - a * cnt;
    buf[e] = a < NC ? planes[int64_t(a) * npix + p0 + i] : cx(0.0, 0.0);
  }
  __syncthreads();
  FftShape sh{lognx, logRB + Fuse<NC>::LOGNP, 1, nx, false, logLmax};
  lds_fft<double, NT, kFuseE, true>(buf, sh, tw);
  for (int e = threadIdx.x; e < cnt; e += NT) {
    const int p = p0 + e;
    const double* S = siginv + 6 * int64_t(p);
    const bool on = mask[p] != 0;
    if constexpr (NC == 1) {
      z[p] = on ? S[0] * buf[e].x : 0.0;
    } else {
      const double v0 = buf[e].x, v1 = buf[cnt + e].x, v2 = buf[2 * cnt + e].x;
      z[p] = on ? S[0] * v0 + S[1] * v1 + S[2] * v2 : 0.0;
      z[npix + p] = on ? S[1] * v0 + S[3] * v1 + S[4] * v2 : 0.0;
      z[2 * int64_t(npix) + p] = on ? S[2] * v0 + S[4] * v1 + S[5] * v2 : 0.0;
    }
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
  s->n_floored = sym ? h.nfloor : 0;
  s->circ_built = true;
  s->circ_sym = sym;
  return MM_OK;
}

mm_status circulant_build(ScanImpl* s, const mm_precon_opts* o, hipStream_t st) {
  s->circ_built = false;
  return s->nc == 3 ? build_t<3>(s, o, st) : build_t<1>(s, o, st);
}

#ifndef MM_CIRC_FUSED
#define MM_CIRC_FUSED 1
#endif

template <int NC>
static mm_status apply_t(ScanImpl* s, const double* r, double* z, hipStream_t st) {
  const Layout& L = s->lay;
  const int npix = s->npix;
  const int logny = ilog2i(s->ny), lognx = ilog2i(s->nx);
  constexpr int kCapLog = kFuseCapLog;
  constexpr int NP = Fuse<NC>::NP, NT = Fuse<NC>::NT;
  if (MM_CIRC_FUSED && logny <= kCapLog && lognx <= kCapLog && (1 << logny) == s->ny &&
      (1 << lognx) == s->nx) {
    const int logRB = (kCapLog - lognx < logny) ? kCapLog - lognx : logny;
    const int logCB = (kCapLog - logny < lognx) ? kCapLog - logny : lognx;
    const size_t lds_r = size_t(NP) * (size_t(s->nx) << logRB) * sizeof(Cx<double>);
    const size_t lds_c = size_t(NP) * (size_t(s->ny) << logCB) * sizeof(Cx<double>);
    const Cx<double>* tw = s->at<Cx<double>>(L.tw_map);
    const int logL = s->plan.logMapL;
    Cx<double>* planes = s->at<Cx<double>>(L.planes);
    hipLaunchKernelGGL(k_circ_rows_pre<NC>, dim3(unsigned(s->ny >> logRB)), dim3(NT), lds_r,
                       st, r, s->at<double>(L.siginv), s->at<int32_t>(L.mask), logny, lognx,
                       logRB, logL, tw, planes);
    hipLaunchKernelGGL(k_circ_cols_kmul<NC>, dim3(unsigned(s->nx >> logCB)), dim3(NT),
                       lds_c, st, planes, s->at<Cx<double>>(L.kinv), logny, lognx, logCB, logL,
                       tw, 1.0 / double(npix));
    hipLaunchKernelGGL(k_circ_rows_post<NC>, dim3(unsigned(s->ny >> logRB)), dim3(NT),
                       lds_r, st, planes, s->at<double>(L.siginv), s->at<int32_t>(L.mask), logny,
                       lognx, logRB, logL, tw, z);
    MM_HIP(hipGetLastError());
    return MM_OK;
  }
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


// ====================================================== tiled preconditioner
// The position-dependent variant the Summary section proposes: T x T tiles at
// stride T/2, each with its own constant-correlation kernel K_t built like
// K but from a probe at the tile's reference pixel and on the tile's own
// periodic T x T displacement grid, merged by a sin^2 partition of unity:
//   M_T r = Sigma^-1 [ sum_t sqrt(W_t) F_t^-1 K_t^-1 F_t sqrt(W_t) ] Sigma^-T r.
// By default every tile's reference pixel is probed on its own (ncomp
// A-applies per tile), which is the definition.  With probe_sets = s >= 2 the
// tiles whose tile row and column agree modulo s share one A-apply per
// component (s^2 sets, same-set references at least s T/2 pixels apart): a
// cheaper set-up whose q_t also picks up the other references' responses,
// damped only by their distance and the taper.  Each probe response is cut
// down at once to the T x T window of displacements each of its tiles uses
// (held in the K^-1 area until the inverses are formed).

struct TiledLayout {
  size_t kinv, planes, probes, tref, tlist, swy, swx, lmax, nfloor, total;
};

static TiledLayout tiled_layout(const ScanImpl* s, int T) {
  const int nc = s->nc;
  const int nty = 2 * s->ny / T - 1, ntx = 2 * s->nx / T - 1;
  const size_t nt = size_t(nty) * ntx, TT = size_t(T) * T;
  TiledLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (b + 255) & ~size_t(255);
    return o;
  };
  L.kinv = take(nt * TT * nc * nc * 16);
  L.planes = take(nt * TT * nc * nc * 16);
  L.probes = take(size_t(nc) * s->npix * 8);   // one probe response
  L.tref = take(nt * 4);
  L.tlist = take(nt * 4);
  L.swy = take(size_t(nty) * T * 8);
  L.swx = take(size_t(ntx) * T * 8);
  L.lmax = take(nt * 8);
  L.nfloor = take(8);
  L.total = off;
  return L;
}

// T a power of two in [8, map side]; the tile count fits a grid dimension
bool tiled_size_ok(const ScanImpl* s, int T) {
  if (T < 8 || (T & (T - 1)) != 0 || T > s->ny || T > s->nx) return false;
  const long nt = long(2 * s->ny / T - 1) * (2 * s->nx / T - 1);
  return nt <= 65535;
}

size_t tiled_workspace_bytes(const ScanImpl* s, int T) {
  return tiled_size_ok(s, T) ? tiled_layout(s, T).total : 0;
}

// sqrt of the 1-D merge weight of tile i (of nt) at offset u
static double tile_sqrt_weight(int i, int nt, int T, int u) {
  if (nt == 1) return 1.0;
  if ((i == 0 && u < T / 2) || (i == nt - 1 && u >= T / 2)) return 1.0;
  const double sn = std::sin(3.14159265358979323846 * (u + 0.5) / T);
  return std::fabs(sn);
}

// The T x T window of one probe response around each listed tile's
// reference pixel: win[t][g*NC+b][y][x] = resp[b][r_t + d] with d the
// minimal image of (y, x) on the tile, r_t + d taken modulo the map.
template <int NC>
__global__ void k_tile_window(const double* __restrict__ resp, int ny, int nx, int logT,
                              const int32_t* __restrict__ tref, const int32_t* __restrict__ tlist,
                              int g, double* __restrict__ win) {
  const int T = 1 << logT, TT = T * T;
  const int t = tlist[blockIdx.y];
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= TT) return;
  const int ref = tref[t];
  const int y = e >> logT, x = e & (T - 1);
  const int my = y > T / 2 ? y - T : y, mx = x > T / 2 ? x - T : x;
  const int jy = (ref / nx + my + ny) % ny, jx = (ref % nx + mx + nx) % nx;
  const int64_t j = int64_t(jy) * nx + jx, npix = int64_t(ny) * nx;
#pragma unroll
  for (int b = 0; b < NC; ++b)
    win[(int64_t(t) * NC * NC + g * NC + b) * TT + e] = resp[b * npix + j];
}

// q_t(d) = Sigma_r^-T C(d) Sigma_j^-1 from a tile's probe window (zero if
// the pixel j = r + d is inactive)
template <int NC>
__device__ __forceinline__ void q_window(const double* win, int TT, int e, int64_t j,
                                         const double (&Sr)[NC][NC], const int32_t* mask,
                                         const double* siginv, double (&q)[NC][NC]) {
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) q[a][b] = 0.0;
  if (!mask[j]) return;
  double Sj[NC][NC], Cm[NC][NC];
  if constexpr (NC == 3) {
    unpack_sym3(siginv + 6 * j, Sj);
  } else {
    Sj[0][0] = siginv[6 * j];
  }
#pragma unroll
  for (int g = 0; g < NC; ++g)
#pragma unroll
    for (int b = 0; b < NC; ++b) Cm[g][b] = win[int64_t(g * NC + b) * TT + e];
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

// planes[t][a*NC+b][y][x] = taper * sym q_t(d), d the minimal image of (y, x) on the tile
template <int NC>
__global__ void k_tq_assemble(const int32_t* __restrict__ mask, const double* __restrict__ win,
                              const double* __restrict__ siginv, int ny, int nx, int logT,
                              const int32_t* __restrict__ tref, double sigma,
                              Cx<double>* __restrict__ planes) {
  const int T = 1 << logT, TT = T * T;
  const int t = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= TT) return;
  Cx<double>* out = planes + int64_t(t) * NC * NC * TT + e;
  const int ref = tref[t];
  if (ref < 0) {
#pragma unroll
    for (int i = 0; i < NC * NC; ++i) out[int64_t(i) * TT] = cx(0.0, 0.0);
    return;
  }
  win += int64_t(t) * NC * NC * TT;
  const int y = e >> logT, x = e & (T - 1);
  // d and -d on the tile's grid (both T/2 at the Nyquist index)
  const int ym = (T - y) & (T - 1), xm = (T - x) & (T - 1);
  const int em = (ym << logT) | xm;
  const int my = y > T / 2 ? y - T : y, mx = x > T / 2 ? x - T : x;
  const int mym = ym > T / 2 ? ym - T : ym, mxm = xm > T / 2 ? xm - T : xm;
  const int ry = ref / nx, rx = ref % nx;
  const int64_t j = int64_t((ry + my + ny) % ny) * nx + (rx + mx + nx) % nx;
  const int64_t jm = int64_t((ry + mym + ny) % ny) * nx + (rx + mxm + nx) % nx;
  double Sr[NC][NC];
  if constexpr (NC == 3) {
    unpack_sym3(siginv + 6 * int64_t(ref), Sr);
  } else {
    Sr[0][0] = siginv[6 * int64_t(ref)];
  }
  double q[NC][NC], qm[NC][NC];
  q_window<NC>(win, TT, e, j, Sr, mask, siginv, q);
  q_window<NC>(win, TT, em, jm, Sr, mask, siginv, qm);
  double g = 1.0;
  if (sigma > 0.0) g = exp(-double(my * my + mx * mx) / (2.0 * sigma * sigma));
#pragma unroll
  for (int a = 0; a < NC; ++a)
#pragma unroll
    for (int b = 0; b < NC; ++b) out[int64_t(a * NC + b) * TT] = cx(g * 0.5 * (q[a][b] + qm[b][a]), 0.0);
}

__global__ void k_set_units(double* __restrict__ e, const int32_t* __restrict__ idx, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) e[idx[i]] = 1.0;
}

// tile planes[t][a][y][x] = sqrt(W_t) * u_a(oy + y, ox + x), u = Sigma^-T r (global planes)
template <int NC>
__global__ void k_tile_gather(const Cx<double>* __restrict__ u, int ny, int nx, int logT, int ntx,
                              const double* __restrict__ swy, const double* __restrict__ swx,
                              Cx<double>* __restrict__ tp) {
  const int T = 1 << logT, TT = T * T;
  const int t = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= TT) return;
  const int iy = t / ntx, ix = t % ntx;
  const int y = e >> logT, x = e & (T - 1);
  const int p = (iy * (T / 2) + y) * nx + ix * (T / 2) + x;
  const double w = swy[iy * T + y] * swx[ix * T + x];
  const int npix = ny * nx;
#pragma unroll
  for (int a = 0; a < NC; ++a)
    tp[(int64_t(t) * NC + a) * TT + e] = cx(w * u[int64_t(a) * npix + p].x, 0.0);
}

// z = Sigma^-1 sum_t sqrt(W_t) v_t / T^2 over the (<= 4) tiles covering each pixel
template <int NC>
__global__ void k_tile_post(const Cx<double>* __restrict__ tp, const double* __restrict__ siginv,
                            const int32_t* __restrict__ mask, int ny, int nx, int logT, int nty,
                            int ntx, const double* __restrict__ swy, const double* __restrict__ swx,
                            double* __restrict__ z) {
  const int npix = ny * nx;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const int T = 1 << logT, TT = T * T, h = T / 2;
  const int y = p / nx, x = p % nx;
  double v[NC];
#pragma unroll
  for (int a = 0; a < NC; ++a) v[a] = 0.0;
  for (int iy = y / h - 1; iy <= y / h; ++iy) {
    if (iy < 0 || iy >= nty) continue;
    const int uy = y - iy * h;
    if (uy >= T) continue;
    for (int ix = x / h - 1; ix <= x / h; ++ix) {
      if (ix < 0 || ix >= ntx) continue;
      const int ux = x - ix * h;
      if (ux >= T) continue;
      const int t = iy * ntx + ix;
      const double w = swy[iy * T + uy] * swx[ix * T + ux];
#pragma unroll
      for (int a = 0; a < NC; ++a) v[a] += w * tp[(int64_t(t) * NC + a) * TT + uy * T + ux].x;
    }
  }
  const double sc = 1.0 / double(TT);
  const double* S = siginv + 6 * int64_t(p);
  const bool on = mask[p] != 0;
  if constexpr (NC == 1) {
    z[p] = on ? S[0] * v[0] * sc : 0.0;
  } else {
    z[p] = on ? (S[0] * v[0] + S[1] * v[1] + S[2] * v[2]) * sc : 0.0;
    z[npix + p] = on ? (S[1] * v[0] + S[3] * v[1] + S[4] * v[2]) * sc : 0.0;
    z[2 * int64_t(npix) + p] = on ? (S[2] * v[0] + S[4] * v[1] + S[5] * v[2]) * sc : 0.0;
  }
}

template <int NC>
static mm_status tiled_build_t(ScanImpl* s, const mm_precon_opts* o, hipStream_t st) {
  const int T = o->tile, logT = ilog2i(T), TT = T * T;
  const int ny = s->ny, nx = s->nx, npix = s->npix, h = T / 2;
  const int nty = 2 * ny / T - 1, ntx = 2 * nx / T - 1, nt = nty * ntx;
  char* tws = static_cast<char*>(o->tiled_workspace);
  const TiledLayout TL = tiled_layout(s, T);
  auto at = [&](size_t off) { return tws + off; };
  // reference pixel per tile: the active pixel nearest the tile centre
  std::vector<int32_t> mask(npix);
  MM_HIP(hipMemcpyAsync(mask.data(), s->at<int32_t>(s->lay.mask), size_t(npix) * 4,
                        hipMemcpyDeviceToHost, st));
  MM_HIP(hipStreamSynchronize(st));
  // probe sets: 0 = every tile alone (the definition); s >= 2 = tiles whose
  // tile row and column agree modulo s
  const int ps = o->probe_sets;
  std::vector<int32_t> tref(nt, -1), tset(nt);
  for (int iy = 0; iy < nty; ++iy)
    for (int ix = 0; ix < ntx; ++ix) {
      const int oy = iy * h, ox = ix * h, cy = oy + h, cxp = ox + h;
      int best = -1;
      long bd = 0;
      for (int y = oy; y < oy + T; ++y)
        for (int x = ox; x < ox + T; ++x) {
          const int p = y * nx + x;
          if (!mask[p]) continue;
          const long d = long(y - cy) * (y - cy) + long(x - cxp) * (x - cxp);
          if (best < 0 || d < bd || (d == bd && p < best)) {
            best = p;
            bd = d;
          }
        }
      tref[iy * ntx + ix] = best;
      tset[iy * ntx + ix] = ps >= 2 ? (iy % ps) * ps + (ix % ps) : iy * ntx + ix;
    }
  const int nsets = ps >= 2 ? ps * ps : nt;
  std::vector<double> swy(size_t(nty) * T), swx(size_t(ntx) * T);
  for (int i = 0; i < nty; ++i)
    for (int u = 0; u < T; ++u) swy[size_t(i) * T + u] = tile_sqrt_weight(i, nty, T, u);
  for (int i = 0; i < ntx; ++i)
    for (int u = 0; u < T; ++u) swx[size_t(i) * T + u] = tile_sqrt_weight(i, ntx, T, u);
  MM_HIP(hipMemcpyAsync(at(TL.tref), tref.data(), size_t(nt) * 4, hipMemcpyHostToDevice, st));
  MM_HIP(hipMemcpyAsync(at(TL.swy), swy.data(), swy.size() * 8, hipMemcpyHostToDevice, st));
  MM_HIP(hipMemcpyAsync(at(TL.swx), swx.data(), swx.size() * 8, hipMemcpyHostToDevice, st));
  // probes: per set and component one A-apply with a unit at every reference
  // of the set, cut at once into the set's tile windows (in the K^-1 area)
  double* resp = reinterpret_cast<double*>(at(TL.probes));
  double* win = reinterpret_cast<double*>(at(TL.kinv));
  double* e = s->at<double>(s->lay.vec) + 4 * int64_t(NC) * npix;   // the spare CG vector
  int32_t* idx = reinterpret_cast<int32_t*>(at(TL.lmax));   // scratch until the floor
  int32_t* tlist = reinterpret_cast<int32_t*>(at(TL.tlist));
  mm_status r;
  std::vector<std::vector<int32_t>> members(nsets);
  for (int t = 0; t < nt; ++t)
    if (tref[t] >= 0) members[tset[t]].push_back(t);
  for (int set = 0; set < nsets; ++set) {
    const std::vector<int32_t>& mt = members[set];
    if (mt.empty()) continue;
    MM_HIP(hipMemcpyAsync(tlist, mt.data(), mt.size() * 4, hipMemcpyHostToDevice, st));
    for (int g = 0; g < NC; ++g) {
      std::vector<int32_t> units(mt.size());
      for (size_t i = 0; i < mt.size(); ++i) units[i] = g * npix + tref[mt[i]];
      if ((r = fill_zero(e, size_t(NC) * npix * 8, st)) != MM_OK) return r;
      MM_HIP(hipMemcpyAsync(idx, units.data(), units.size() * 4, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_set_units, dim3(unsigned((units.size() + 255) / 256)), dim3(256), 0, st,
                         e, idx, int(units.size()));
      MM_HIP(hipGetLastError());
      if ((r = filter_pipeline(s, 0, nullptr, e, resp, st)) != MM_OK) return r;
      hipLaunchKernelGGL(k_tile_window<NC>, dim3(unsigned((TT + 255) / 256), unsigned(mt.size())),
                         dim3(256), 0, st, resp, ny, nx, logT,
                         reinterpret_cast<const int32_t*>(at(TL.tref)), tlist, g, win);
      MM_HIP(hipGetLastError());
      MM_HIP(hipStreamSynchronize(st));   // idx (and tlist) are reused by the next probe
    }
  }
  Cx<double>* planes = reinterpret_cast<Cx<double>*>(at(TL.planes));
  const dim3 gt((TT + 255) / 256, nt), b(256);
  hipLaunchKernelGGL(k_tq_assemble<NC>, gt, b, 0, st, s->at<int32_t>(s->lay.mask), win,
                     s->at<double>(s->lay.siginv), ny, nx, logT,
                     reinterpret_cast<const int32_t*>(at(TL.tref)), o->gauss_sigma_px, planes);
  MM_HIP(hipGetLastError());
  if ((r = map_fft_dims(s, planes, logT, logT, nt * NC * NC, false, st)) != MM_OK) return r;
  double eps = o->eig_floor_rel;
  if (!(eps > 0.0)) eps = 1e-6;
  unsigned long long* lmax = reinterpret_cast<unsigned long long*>(at(TL.lmax));
  int* nfl = reinterpret_cast<int*>(at(TL.nfloor));
  if ((r = fill_zero(lmax, size_t(nt) * 8, st)) != MM_OK) return r;
  if ((r = fill_zero(nfl, 8, st)) != MM_OK) return r;
  hipLaunchKernelGGL(k_kinv_lmax<NC>, gt, b, 0, st, planes, TT, lmax);
  hipLaunchKernelGGL(k_kinv_floor<NC>, gt, b, 0, st, planes, TT, lmax, eps,
                     reinterpret_cast<Cx<double>*>(at(TL.kinv)), nfl,
                     reinterpret_cast<const int32_t*>(at(TL.tref)));
  MM_HIP(hipGetLastError());
  MM_HIP(hipStreamSynchronize(st));
  s->tiled_T = T;
  s->tiled_ws = tws;
  s->tiled_built = true;
  return MM_OK;
}

mm_status tiled_build(ScanImpl* s, const mm_precon_opts* o, hipStream_t st) {
  s->tiled_built = false;
  return s->nc == 3 ? tiled_build_t<3>(s, o, st) : tiled_build_t<1>(s, o, st);
}

template <int NC>
static mm_status tiled_apply_t(ScanImpl* s, const double* rv, double* z, hipStream_t st) {
  const int T = s->tiled_T, logT = ilog2i(T), TT = T * T;
  const int ny = s->ny, nx = s->nx, npix = s->npix;
  const int nty = 2 * ny / T - 1, ntx = 2 * nx / T - 1, nt = nty * ntx;
  const TiledLayout TL = tiled_layout(s, T);
  char* tws = s->tiled_ws;
  Cx<double>* u = s->at<Cx<double>>(s->lay.planes);
  Cx<double>* tp = reinterpret_cast<Cx<double>*>(tws + TL.planes);
  const double* swy = reinterpret_cast<const double*>(tws + TL.swy);
  const double* swx = reinterpret_cast<const double*>(tws + TL.swx);
  const dim3 g((npix + 255) / 256), b(256), gt((TT + 255) / 256, nt);
  hipLaunchKernelGGL(k_circ_pre<NC>, g, b, 0, st, rv, s->at<double>(s->lay.siginv),
                     s->at<int32_t>(s->lay.mask), npix, u);
  hipLaunchKernelGGL(k_tile_gather<NC>, gt, b, 0, st, u, ny, nx, logT, ntx, swy, swx, tp);
  MM_HIP(hipGetLastError());
  mm_status r;
  const Cx<double>* kinv_t = reinterpret_cast<const Cx<double>*>(tws + TL.kinv);
  if (MM_CIRC_FUSED && logT <= kFuseCapLog && nt <= 65535) {
    // row transforms, then the three-step column kernel of the circulant
    // apply with one grid row per tile, then the inverse row transforms
    if ((r = map_fft_blocks<128, 8>(s, tp, logT, logT, nt * NC, false, st, 1)) != MM_OK) return r;
    const int logCB = (kFuseCapLog - logT < logT) ? kFuseCapLog - logT : logT;
    const size_t lds_c = size_t(Fuse<NC>::NP) * (size_t(T) << logCB) * sizeof(Cx<double>);
    hipLaunchKernelGGL(k_circ_cols_kmul<NC>, dim3(unsigned(T >> logCB), unsigned(nt)),
                       dim3(Fuse<NC>::NT), lds_c, st, tp, kinv_t, logT, logT, logCB,
                       s->plan.logMapL, s->at<Cx<double>>(s->lay.tw_map), 1.0);
    MM_HIP(hipGetLastError());
    if ((r = map_fft_blocks<128, 8>(s, tp, logT, logT, nt * NC, true, st, 1)) != MM_OK) return r;
  } else {
    if ((r = map_fft_dims(s, tp, logT, logT, nt * NC, false, st)) != MM_OK) return r;
    hipLaunchKernelGGL(k_circ_kmul<NC>, gt, b, 0, st, tp, kinv_t, TT, 1.0);
    MM_HIP(hipGetLastError());
    if ((r = map_fft_dims(s, tp, logT, logT, nt * NC, true, st)) != MM_OK) return r;
  }
  hipLaunchKernelGGL(k_tile_post<NC>, g, b, 0, st, tp, s->at<double>(s->lay.siginv),
                     s->at<int32_t>(s->lay.mask), ny, nx, logT, nty, ntx, swy, swx, z);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

mm_status tiled_apply(ScanImpl* s, const double* r, double* z, hipStream_t st) {
  if (!s->tiled_built) return fail(MM_ENOTBUILT, "tiled preconditioner not built");
  return s->nc == 3 ? tiled_apply_t<3>(s, r, z, st) : tiled_apply_t<1>(s, r, z, st);
}

}  // namespace mm
