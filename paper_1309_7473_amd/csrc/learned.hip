// The learned linear correction to the circulant preconditioner:
//   M_L r = M_C r + Sigma^-1 H^T H Sigma^-T r,   H = C2 o C1,
// C1 (3 -> 16 channels) and C2 (16 -> 16) 5x5 "same" correlations with zero
// padding and no bias; H^T = C1^T o C2^T (flipped taps, swapped channels).
// Weight tying keeps M_L symmetric and M_L - M_C positive semi-definite.
//
// Convolutions are implicit GEMMs on bf16 MFMA with float32 accumulation
// (v_mfma_f32_16x16x16bf16_1k): pixels x (Cin*25) x Cout, the input patch and
// the weights staged in LDS as bf16.  Weight gradients are GEMMs over the
// pixel dimension, summed per block and then over blocks in a fixed order.
// Training (Adam, float32 master weights) runs on pairs (r_w, t, ||e_w||^2)
// built on the GPU from PCG iterates: e = x_f - x_k, r = A e, r_w = Sigma^-T r,
// t = Sigma e - Sigma M_C r.
#include <cmath>
#include <new>
#include <vector>

#include "linalg_small.h"
#include "mm_device.h"
#include "mm_internal.h"

namespace mm {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bf16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return short((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return short(u >> 16);
}

constexpr int kTX = 64;  // pixels of a row per conv block (4 waves x 16)
constexpr int kTR = 4;   // rows per conv block

// out[b][co][y][x] = sum_{ci,u,v} Wk(co,ci,u,v) in[b][ci][y+dy][x+dx]
//   !TRANS: W is [CO][CI][5][5], Wk = W[co][ci][u][v], (dy,dx) = (u-2, v-2)
//    TRANS: W is [CI][CO][5][5], Wk = W[ci][co][u][v], (dy,dx) = (2-u, 2-v)
template <int CI, int CO, bool TRANS>
__global__ void __launch_bounds__(256) k_conv(const float* __restrict__ in,
                                              const float* __restrict__ W,
                                              float* __restrict__ out, int H, int Wd) {
  constexpr int K = CI * 25;
  constexpr int KT = (K + 15) / 16;
  constexpr int PR = kTR + 4, PC = kTX + 4;
  __shared__ short sW[KT * 16 * 16];
  __shared__ short sIn[CI * PR * PC];
  __shared__ int sOff[KT * 16];
  const int ntx = (Wd + kTX - 1) / kTX, nty = (H + kTR - 1) / kTR;
  int bid = blockIdx.x;
  const int tx = bid % ntx;
  bid /= ntx;
  const int ty = bid % nty;
  const int b = bid / nty;
  const int x0 = tx * kTX, y0 = ty * kTR;
  for (int i = threadIdx.x; i < KT * 16 * 16; i += 256) {
    const int k = i >> 4, co = i & 15;
    float w = 0.f;
    if (k < K && co < CO) {
      const int ci = k / 25, u = (k % 25) / 5, v = k % 5;
      w = TRANS ? W[((ci * CO + co) * 5 + u) * 5 + v] : W[((co * CI + ci) * 5 + u) * 5 + v];
    }
    sW[i] = f2bf(w);
  }
  for (int k = threadIdx.x; k < KT * 16; k += 256) {
    int off = 0;
    if (k < K) {
      const int ci = k / 25, u = (k % 25) / 5, v = k % 5;
      off = ci * PR * PC + (TRANS ? 4 - u : u) * PC + (TRANS ? 4 - v : v);
    }
    sOff[k] = off;
  }
  const float* inb = in + int64_t(b) * CI * H * Wd;
  for (int i = threadIdx.x; i < CI * PR * PC; i += 256) {
    const int c = i / (PR * PC), rem = i % (PR * PC), r = rem / PC, q = rem % PC;
    const int y = y0 + r - 2, x = x0 + q - 2;
    const float v = (y >= 0 && y < H && x >= 0 && x < Wd) ? inb[(int64_t(c) * H + y) * Wd + x] : 0.f;
    sIn[i] = f2bf(v);
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, kg = lane >> 4;
  for (int rr = 0; rr < kTR; ++rr) {
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int base = rr * PC + wave * 16 + m;
#pragma unroll 5
    for (int kt = 0; kt < KT; ++kt) {
      v4s a, bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kt * 16 + kg * 4 + j;
        a[j] = (k < K) ? sIn[sOff[k] + base] : short(0);
        bv[j] = sW[k * 16 + m];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc, 0, 0, 0);
    }
    const int y = y0 + rr;
    if (y < H && m < CO) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + wave * 16 + kg * 4 + i;
        if (x < Wd) out[((int64_t(b) * CO + m) * H + y) * Wd + x] = acc[i];
      }
    }
  }
}

constexpr int kGR = 16;  // rows per weight-gradient block (x kTX columns)

// part[blk][o][n] = sum over this block's pixels of P[b][o][y][x] * Q[b][c][y+u-2][x+v-2],
// n = c*25 + u*5 + v (o < 16: P always has 16 channels).
template <int CQ>
__global__ void __launch_bounds__(256) k_wgrad_part(const float* __restrict__ P,
                                                    const float* __restrict__ Q,
                                                    float* __restrict__ part, int H, int Wd) {
  constexpr int N = CQ * 25;
  constexpr int NT = (N + 15) / 16;
  constexpr int PR = kGR + 4, PC = kTX + 4;
  extern __shared__ __align__(16) unsigned char smem[];
  short* sP = reinterpret_cast<short*>(smem);             // [16][kGR][kTX]
  short* sQ = sP + 16 * kGR * kTX;                        // [CQ][PR][PC]
  int* sOff = reinterpret_cast<int*>(sQ + CQ * PR * PC);  // [NT*16]
  float* sAcc = reinterpret_cast<float*>(sOff + NT * 16); // [16][NT*16]
  const int ntx = (Wd + kTX - 1) / kTX, nty = (H + kGR - 1) / kGR;
  int bid = blockIdx.x;
  const int tx = bid % ntx;
  bid /= ntx;
  const int ty = bid % nty;
  const int b = bid / nty;
  const int x0 = tx * kTX, y0 = ty * kGR;
  const float* Pb = P + int64_t(b) * 16 * H * Wd;
  const float* Qb = Q + int64_t(b) * CQ * H * Wd;
  for (int i = threadIdx.x; i < 16 * kGR * kTX; i += 256) {
    const int o = i / (kGR * kTX), rem = i % (kGR * kTX), r = rem / kTX, q = rem % kTX;
    const int y = y0 + r, x = x0 + q;
    const float v = (y < H && x < Wd) ? Pb[(int64_t(o) * H + y) * Wd + x] : 0.f;
    sP[i] = f2bf(v);
  }
  for (int i = threadIdx.x; i < CQ * PR * PC; i += 256) {
    const int c = i / (PR * PC), rem = i % (PR * PC), r = rem / PC, q = rem % PC;
    const int y = y0 + r - 2, x = x0 + q - 2;
    const float v = (y >= 0 && y < H && x >= 0 && x < Wd) ? Qb[(int64_t(c) * H + y) * Wd + x] : 0.f;
    sQ[i] = f2bf(v);
  }
  for (int n = threadIdx.x; n < NT * 16; n += 256) {
    int off = 0;
    if (n < N) {
      const int c = n / 25, u = (n % 25) / 5, v = n % 5;
      off = c * PR * PC + u * PC + v;
    }
    sOff[n] = off;
  }
  for (int i = threadIdx.x; i < 16 * NT * 16; i += 256) sAcc[i] = 0.f;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m = lane & 15, kg = lane >> 4;
  v4f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
  // K steps: 16 pixels (one row, 16 columns); wave w takes rows w, w+4, ...
  for (int rr = wave; rr < kGR; rr += 4) {
    for (int c0 = 0; c0 < kTX; c0 += 16) {
      v4s a;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = sP[(m * kGR + rr) * kTX + c0 + kg * 4 + j];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        v4s bv;
        const int off = sOff[t * 16 + m] + rr * PC + c0 + kg * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = (t * 16 + m < N) ? sQ[off + j] : short(0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bv, acc[t], 0, 0, 0);
      }
    }
  }
  // D[o = 4*kg + i][n = t*16 + m]; sum the four waves in LDS in a fixed order
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) sAcc[(kg * 4 + i) * (NT * 16) + t * 16 + m] += acc[t][i];
    }
    __syncthreads();
  }
  float* pb = part + int64_t(blockIdx.x) * 16 * N;
  for (int i = threadIdx.x; i < 16 * N; i += 256) {
    const int o = i / N, n = i % N;
    pb[i] = sAcc[o * (NT * 16) + n];
  }
}

// dW[o][c][u][v] (+)= sum over blocks of part (fixed order, float64 sums)
__global__ void k_wgrad_sum(const float* __restrict__ part, int nblk, int n, float* __restrict__ dW,
                            int accumulate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += part[int64_t(k) * n + i];
  dW[i] = accumulate ? dW[i] + float(s) : float(s);
}

// loss terms and output gradient: d = y - t; gy = (2/B) d / e2[b]
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                            const float* __restrict__ e2, int64_t per, int B,
                            float* __restrict__ gy, double* __restrict__ lpart) {
  double acc[1] = {0.0};
  const int64_t total = per * B;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int b = int(i / per);
    const float d = y[i] - t[i];
    acc[0] += double(d) * double(d) / double(e2[b]);
    gy[i] = (2.0f / float(B)) * d / e2[b];
  }
  __shared__ double sm[16];
  block_sum<1>(acc, sm);
  if (threadIdx.x == 0) lpart[blockIdx.x] = acc[0];
}

__global__ void k_adam(float* __restrict__ W, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------- per-pixel Sigma maps
// img[c][p] = (Sigma^-T r)_c (active pixels, else 0), float32 image
template <int NC>
__global__ void k_whiten(const double* __restrict__ r, const double* __restrict__ siginv,
                         const int32_t* __restrict__ mask, int npix, float* __restrict__ img) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const double* S = siginv + 6 * int64_t(p);
  const bool on = mask[p] != 0;
  if constexpr (NC == 1) {
    img[p] = on ? float(S[0] * r[p]) : 0.f;
  } else {
    const double r0 = on ? r[p] : 0.0, r1 = on ? r[npix + p] : 0.0, r2 = on ? r[2 * npix + p] : 0.0;
    img[p] = float(S[0] * r0 + S[1] * r1 + S[2] * r2);
    img[npix + p] = float(S[1] * r0 + S[3] * r1 + S[4] * r2);
    img[2 * npix + p] = float(S[2] * r0 + S[4] * r1 + S[5] * r2);
  }
}

// z[c][p] += (Sigma^-1 y)_c on active pixels
template <int NC>
__global__ void k_unwhiten_add(const float* __restrict__ y, const double* __restrict__ siginv,
                               const int32_t* __restrict__ mask, int npix, double* __restrict__ z) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix || !mask[p]) return;
  const double* S = siginv + 6 * int64_t(p);
  if constexpr (NC == 1) {
    z[p] += S[0] * double(y[p]);
  } else {
    const double y0 = y[p], y1 = y[npix + p], y2 = y[2 * npix + p];
    z[p] += S[0] * y0 + S[1] * y1 + S[2] * y2;
    z[npix + p] += S[1] * y0 + S[3] * y1 + S[4] * y2;
    z[2 * npix + p] += S[2] * y0 + S[4] * y1 + S[5] * y2;
  }
}

// pair pieces: e = x_f - x_k (masked); sigma_e = Sigma e; then t = Sigma (e - M_C r)
__global__ void k_sub_masked(const double* __restrict__ a, const double* __restrict__ b,
                             const int32_t* __restrict__ mask, int npix, int nc,
                             double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  for (int c = 0; c < nc; ++c) {
    const int64_t i = int64_t(c) * npix + p;
    out[i] = mask[p] ? a[i] - b[i] : 0.0;
  }
}

template <int NC>
__global__ void k_sigma_img(const double* __restrict__ x, const double* __restrict__ sigma,
                            int npix, float* __restrict__ img, double* __restrict__ e2part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (p < npix) {
    const double* S = sigma + 6 * int64_t(p);
    if constexpr (NC == 1) {
      const double v = S[0] * x[p];
      img[p] = float(v);
      acc[0] = v * v;
    } else {
      const double x0 = x[p], x1 = x[npix + p], x2 = x[2 * npix + p];
      const double v0 = S[0] * x0 + S[1] * x1 + S[2] * x2;
      const double v1 = S[1] * x0 + S[3] * x1 + S[4] * x2;
      const double v2 = S[2] * x0 + S[4] * x1 + S[5] * x2;
      img[p] = float(v0);
      img[npix + p] = float(v1);
      img[2 * npix + p] = float(v2);
      acc[0] = v0 * v0 + v1 * v1 + v2 * v2;
    }
  }
  if (e2part) {
    __shared__ double sm[16];
    block_sum<1>(acc, sm);
    if (threadIdx.x == 0) e2part[blockIdx.x] = acc[0];
  }
}

__global__ void k_sum_to_float(const double* __restrict__ part, int n, float* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  *out = float(s);
}

// ------------------------------------------------------------- host side
struct Learned {
  uint64_t magic;
  int nc, ny, nx, batch;
  char* ws;
  size_t ws_bytes;
  // offsets
  size_t w1, w2, g1, g2, m1, m2, v1, v2;   // float weights / grads / Adam state
  size_t act;                                // activation buffers (batch)
  size_t part, lpart, e2p;
  int64_t nact;                              // floats per 16-channel batch buffer
  int step = 0;
  float* at(size_t off) const { return reinterpret_cast<float*>(ws + off); }
};

static constexpr uint64_t kLearnedMagic = 0x6d6d5f6c726e6431ull;
constexpr int kW1 = 16 * 3 * 25, kW2 = 16 * 16 * 25;

static int conv_blocks(int B, int H, int W) {
  return B * ((H + kTR - 1) / kTR) * ((W + kTX - 1) / kTX);
}
static int wgrad_blocks(int B, int H, int W) {
  return B * ((H + kGR - 1) / kGR) * ((W + kTX - 1) / kTX);
}
static size_t wgrad_lds(int CQ) {
  const int N = CQ * 25, NT = (N + 15) / 16;
  return size_t(16 * kGR * kTX + CQ * (kGR + 4) * (kTX + 4)) * 2 + size_t(NT * 16) * 4 +
         size_t(16 * NT * 16) * 4;
}

static size_t learned_layout(int nc, int ny, int nx, int batch, Learned* L) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const int w1n = 16 * nc * 25;
  L->w1 = take(w1n * 4);
  L->w2 = take(kW2 * 4);
  L->g1 = take(w1n * 4);
  L->g2 = take(kW2 * 4);
  L->m1 = take(w1n * 4);
  L->m2 = take(kW2 * 4);
  L->v1 = take(w1n * 4);
  L->v2 = take(kW2 * 4);
  const int64_t npix = int64_t(ny) * nx;
  L->nact = int64_t(batch) * 16 * npix;
  // R, T (nc ch), a1, a2, a3 (16), y, gy (nc), g_a3, g_a2, g_a1 (16) + e2 batch
  L->act = take(size_t(batch) * npix * 4 * (4 * nc + 6 * 16) + size_t(batch) * 4);
  const int nb = wgrad_blocks(batch, ny, nx);
  L->part = take(size_t(nb) * 16 * 16 * 25 * 4);
  L->lpart = take(size_t(2048) * 8);
  L->e2p = take(size_t((npix + 255) / 256) * 8);
  return off;
}

struct Act {
  float *R, *T, *a1, *a2, *a3, *y, *gy, *ga3, *ga2, *ga1, *e2;
};

static Act acts(const Learned* L) {
  const int64_t npix = int64_t(L->ny) * L->nx;
  const int64_t cn = int64_t(L->batch) * L->nc * npix, c16 = int64_t(L->batch) * 16 * npix;
  float* p = L->at(L->act);
  Act a;
  a.R = p; p += cn;
  a.T = p; p += cn;
  a.y = p; p += cn;
  a.gy = p; p += cn;
  a.a1 = p; p += c16;
  a.a2 = p; p += c16;
  a.a3 = p; p += c16;
  a.ga3 = p; p += c16;
  a.ga2 = p; p += c16;
  a.ga1 = p; p += c16;
  a.e2 = p;
  return a;
}

template <int CI, int CO, bool TRANS>
static void conv(const float* in, const float* W, float* out, int B, int H, int Wd, hipStream_t st) {
  hipLaunchKernelGGL((k_conv<CI, CO, TRANS>), dim3(conv_blocks(B, H, Wd)), dim3(256), 0, st, in, W,
                     out, H, Wd);
}

// H^T H x for B images of nc channels; x in a.R-like buffer, result in y
static void hth(const Learned* L, const Act& a, const float* x, float* y, int B, hipStream_t st) {
  const float* W1 = L->at(L->w1);
  const float* W2 = L->at(L->w2);
  const int H = L->ny, Wd = L->nx;
  if (L->nc == 3) {
    conv<3, 16, false>(x, W1, a.a1, B, H, Wd, st);
    conv<16, 16, false>(a.a1, W2, a.a2, B, H, Wd, st);
    conv<16, 16, true>(a.a2, W2, a.a3, B, H, Wd, st);
    conv<16, 3, true>(a.a3, W1, y, B, H, Wd, st);
  } else {
    conv<1, 16, false>(x, W1, a.a1, B, H, Wd, st);
    conv<16, 16, false>(a.a1, W2, a.a2, B, H, Wd, st);
    conv<16, 16, true>(a.a2, W2, a.a3, B, H, Wd, st);
    conv<16, 1, true>(a.a3, W1, y, B, H, Wd, st);
  }
}

template <int CQ>
static mm_status wgrad(const Learned* L, const float* P, const float* Q, float* dW, int accumulate,
                       int B, hipStream_t st) {
  const int nb = wgrad_blocks(B, L->ny, L->nx);
  const size_t lds = wgrad_lds(CQ);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_wgrad_part<CQ>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  float* part = L->at(L->part);
  hipLaunchKernelGGL(k_wgrad_part<CQ>, dim3(nb), dim3(256), lds, st, P, Q, part, L->ny, L->nx);
  const int n = 16 * CQ * 25;
  hipLaunchKernelGGL(k_wgrad_sum, dim3((n + 255) / 256), dim3(256), 0, st, part, nb, n, dW, accumulate);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

static Learned* getL(mm_learned h) {
  Learned* L = reinterpret_cast<Learned*>(h);
  return (L && L->magic == kLearnedMagic) ? L : nullptr;
}

mm_status learned_apply(ScanImpl* s, const double* r, double* z, hipStream_t st) {
  Learned* L = getL(s->learned);
  if (!L) return fail(MM_ENOTBUILT, "no learned correction attached");
  mm_status rc = circulant_apply(s, r, z, st);
  if (rc != MM_OK) return rc;
  const Act a = acts(L);
  const dim3 g((s->npix + 255) / 256), b(256);
  if (s->nc == 3)
    hipLaunchKernelGGL(k_whiten<3>, g, b, 0, st, r, s->at<double>(s->lay.siginv),
                       s->at<int32_t>(s->lay.mask), s->npix, a.R);
  else
    hipLaunchKernelGGL(k_whiten<1>, g, b, 0, st, r, s->at<double>(s->lay.siginv),
                       s->at<int32_t>(s->lay.mask), s->npix, a.R);
  hth(L, a, a.R, a.y, 1, st);
  if (s->nc == 3)
    hipLaunchKernelGGL(k_unwhiten_add<3>, g, b, 0, st, a.y, s->at<double>(s->lay.siginv),
                       s->at<int32_t>(s->lay.mask), s->npix, z);
  else
    hipLaunchKernelGGL(k_unwhiten_add<1>, g, b, 0, st, a.y, s->at<double>(s->lay.siginv),
                       s->at<int32_t>(s->lay.mask), s->npix, z);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

mm_status learned_make_pair(ScanImpl* s, const double* xf, const double* xk, float* rw, float* t,
                            float* e2, hipStream_t st) {
  if (!s->circ_built) return fail(MM_ENOTBUILT, "circulant preconditioner not built");
  const int npix = s->npix, nc = s->nc;
  const int64_t N = int64_t(nc) * npix;
  double* vec = s->at<double>(s->lay.vec);
  double* e = vec + 4 * N;   // spare vectors (not used outside a solve)
  double* r = vec + 3 * N;
  double* mcr = vec + 2 * N;
  const dim3 g((npix + 255) / 256), b(256);
  hipLaunchKernelGGL(k_sub_masked, g, b, 0, st, xf, xk, s->at<int32_t>(s->lay.mask), npix, nc, e);
  MM_HIP(hipGetLastError());
  mm_status rc;
  if ((rc = filter_pipeline(s, 0, nullptr, e, r, st)) != MM_OK) return rc;
  if ((rc = circulant_apply(s, r, mcr, st)) != MM_OK) return rc;
  const double* sig = s->at<double>(s->lay.sigma);
  double* e2p = s->at<double>(s->lay.partials);
  // r_w = Sigma^-T r
  if (nc == 3)
    hipLaunchKernelGGL(k_whiten<3>, g, b, 0, st, r, s->at<double>(s->lay.siginv),
                       s->at<int32_t>(s->lay.mask), npix, rw);
  else
    hipLaunchKernelGGL(k_whiten<1>, g, b, 0, st, r, s->at<double>(s->lay.siginv),
                       s->at<int32_t>(s->lay.mask), npix, rw);
  // ||Sigma e||^2, then t = Sigma (e - M_C r)
  if (nc == 3)
    hipLaunchKernelGGL(k_sigma_img<3>, g, b, 0, st, e, sig, npix, t, e2p);
  else
    hipLaunchKernelGGL(k_sigma_img<1>, g, b, 0, st, e, sig, npix, t, e2p);
  hipLaunchKernelGGL(k_sum_to_float, dim3(1), dim3(64), 0, st, e2p, int(g.x), e2);
  hipLaunchKernelGGL(k_sub_masked, g, b, 0, st, e, mcr, s->at<int32_t>(s->lay.mask), npix, nc, e);
  if (nc == 3)
    hipLaunchKernelGGL(k_sigma_img<3>, g, b, 0, st, e, sig, npix, t, static_cast<double*>(nullptr));
  else
    hipLaunchKernelGGL(k_sigma_img<1>, g, b, 0, st, e, sig, npix, t, static_cast<double*>(nullptr));
  MM_HIP(hipGetLastError());
  return MM_OK;
}

size_t learned_workspace_bytes(int nc, int ny, int nx, int batch) {
  Learned L{};
  return learned_layout(nc, ny, nx, batch, &L);
}

mm_status learned_create(int nc, int ny, int nx, int batch, void* ws, size_t ws_bytes,
                         const float* w1, const float* w2, hipStream_t st, mm_learned* out) {
  Learned* L = new (std::nothrow) Learned{};
  if (!L) return fail(MM_ENOMEM, "host allocation failed");
  L->magic = kLearnedMagic;
  L->nc = nc;
  L->ny = ny;
  L->nx = nx;
  L->batch = batch;
  L->ws = static_cast<char*>(ws);
  L->ws_bytes = ws_bytes;
  learned_layout(nc, ny, nx, batch, L);
  const int w1n = 16 * nc * 25;
  mm_status rc;
  if ((rc = fill_zero(L->ws, L->act, st)) != MM_OK) {
    delete L;
    return rc;
  }
  hipError_t e1 = hipMemcpyAsync(L->at(L->w1), w1, size_t(w1n) * 4, hipMemcpyHostToDevice, st);
  hipError_t e2 = hipMemcpyAsync(L->at(L->w2), w2, size_t(kW2) * 4, hipMemcpyHostToDevice, st);
  hipError_t e3 = hipStreamSynchronize(st);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    delete L;
    return hip_check(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3), "learned weights upload");
  }
  *out = reinterpret_cast<mm_learned>(L);
  return MM_OK;
}

void learned_destroy(mm_learned h) {
  Learned* L = getL(h);
  if (!L) return;
  L->magic = 0;
  delete L;
}

mm_status learned_get(mm_learned h, float* w1, float* w2) {
  Learned* L = getL(h);
  if (!L) return fail(MM_EINVAL, "invalid learned handle");
  MM_HIP(hipMemcpy(w1, L->at(L->w1), size_t(16) * L->nc * 25 * 4, hipMemcpyDeviceToHost));
  MM_HIP(hipMemcpy(w2, L->at(L->w2), size_t(kW2) * 4, hipMemcpyDeviceToHost));
  return MM_OK;
}

mm_status learned_check(mm_learned h, int nc, int ny, int nx) {
  Learned* L = getL(h);
  if (!L) return fail(MM_EINVAL, "invalid learned handle");
  if (L->nc != nc || L->ny != ny || L->nx != nx)
    return fail(MM_EINVAL, "learned correction built for another map shape");
  return MM_OK;
}

// One optimisation step on B pairs whose data sit in a.R, a.T, a.e2.  Writes
// the batch loss partials (k_loss_grad blocks) to lpart.
static mm_status train_step(Learned* L, const Act& a, int B, const mm_train_opts* o,
                            hipStream_t st, int* nlpart) {
  const int H = L->ny, Wd = L->nx;
  const int64_t per = int64_t(L->nc) * H * Wd;
  hth(L, a, a.R, a.y, B, st);
  int lb = int((per * B + 255) / 256);
  if (lb > 2048) lb = 2048;
  hipLaunchKernelGGL(k_loss_grad, dim3(lb), dim3(256), 0, st, a.y, a.T, a.e2, per, B, a.gy,
                     reinterpret_cast<double*>(L->ws + L->lpart));
  *nlpart = lb;
  const float* W1 = L->at(L->w1);
  const float* W2 = L->at(L->w2);
  float* g1 = L->at(L->g1);
  float* g2 = L->at(L->g2);
  mm_status rc;
  if (L->nc == 3) {
    conv<3, 16, false>(a.gy, W1, a.ga3, B, H, Wd, st);   // adjoint of C1^T
    conv<16, 16, false>(a.ga3, W2, a.ga2, B, H, Wd, st);  // adjoint of C2^T
    conv<16, 16, true>(a.ga2, W2, a.ga1, B, H, Wd, st);   // adjoint of C2
    if ((rc = wgrad<3>(L, a.ga1, a.R, g1, 0, B, st)) != MM_OK) return rc;
    if ((rc = wgrad<3>(L, a.a3, a.gy, g1, 1, B, st)) != MM_OK) return rc;
  } else {
    conv<1, 16, false>(a.gy, W1, a.ga3, B, H, Wd, st);
    conv<16, 16, false>(a.ga3, W2, a.ga2, B, H, Wd, st);
    conv<16, 16, true>(a.ga2, W2, a.ga1, B, H, Wd, st);
    if ((rc = wgrad<1>(L, a.ga1, a.R, g1, 0, B, st)) != MM_OK) return rc;
    if ((rc = wgrad<1>(L, a.a3, a.gy, g1, 1, B, st)) != MM_OK) return rc;
  }
  if ((rc = wgrad<16>(L, a.ga2, a.a1, g2, 0, B, st)) != MM_OK) return rc;
  if ((rc = wgrad<16>(L, a.a2, a.ga3, g2, 1, B, st)) != MM_OK) return rc;
  L->step += 1;
  const float c1 = float(1.0 - std::pow(double(o->beta1), L->step));
  const float c2 = float(1.0 - std::pow(double(o->beta2), L->step));
  const int w1n = 16 * L->nc * 25;
  hipLaunchKernelGGL(k_adam, dim3((w1n + 255) / 256), dim3(256), 0, st, L->at(L->w1), g1,
                     L->at(L->m1), L->at(L->v1), w1n, float(o->lr), float(o->beta1),
                     float(o->beta2), float(o->eps), c1, c2);
  hipLaunchKernelGGL(k_adam, dim3((kW2 + 255) / 256), dim3(256), 0, st, L->at(L->w2), g2,
                     L->at(L->m2), L->at(L->v2), kW2, float(o->lr), float(o->beta1),
                     float(o->beta2), float(o->eps), c1, c2);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

static uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

mm_status learned_train(mm_learned h, const float* rw, const float* t, const float* e2,
                        int64_t npairs, const mm_train_opts* o, double* loss_hist,
                        hipStream_t st) {
  Learned* L = getL(h);
  if (!L) return fail(MM_EINVAL, "invalid learned handle");
  const int B = o->batch;
  if (B < 1 || B > L->batch) return fail(MM_EINVAL, "batch must be in [1, the batch of mm_learned_create]");
  if (npairs < 1) return fail(MM_EINVAL, "npairs must be >= 1");
  const Act a = acts(L);
  const int64_t per = int64_t(L->nc) * L->ny * L->nx;
  std::vector<int64_t> perm(npairs);
  uint64_t seed = o->seed;
  std::vector<double> lp(2048);
  for (int ep = 0; ep < o->epochs; ++ep) {
    for (int64_t i = 0; i < npairs; ++i) perm[i] = i;
    if (o->shuffle)
      for (int64_t i = npairs - 1; i > 0; --i) {
        const int64_t j = int64_t(splitmix(seed) % uint64_t(i + 1));
        std::swap(perm[i], perm[j]);
      }
    double ep_loss = 0.0;
    int64_t nb = 0;
    for (int64_t s0 = 0; s0 + (o->drop_last ? B : 1) <= npairs; s0 += B) {
      const int bsz = int((npairs - s0 < B) ? (npairs - s0) : B);
      for (int k = 0; k < bsz; ++k) {
        const int64_t pi = perm[s0 + k];
        MM_HIP(hipMemcpyAsync(a.R + k * per, rw + pi * per, per * 4, hipMemcpyDeviceToDevice, st));
        MM_HIP(hipMemcpyAsync(a.T + k * per, t + pi * per, per * 4, hipMemcpyDeviceToDevice, st));
        MM_HIP(hipMemcpyAsync(a.e2 + k, e2 + pi, 4, hipMemcpyDeviceToDevice, st));
      }
      int nlp = 0;
      mm_status rc = train_step(L, a, bsz, o, st, &nlp);
      if (rc != MM_OK) return rc;
      MM_HIP(hipMemcpyAsync(lp.data(), L->ws + L->lpart, size_t(nlp) * 8, hipMemcpyDeviceToHost, st));
      MM_HIP(hipStreamSynchronize(st));
      double bl = 0.0;
      for (int k = 0; k < nlp; ++k) bl += lp[k];
      ep_loss += bl / bsz;
      ++nb;
    }
    if (loss_hist) loss_hist[ep] = nb ? ep_loss / nb : 0.0;
  }
  return MM_OK;
}

mm_status learned_loss(mm_learned h, const float* rw, const float* t, const float* e2,
                       int64_t npairs, double* loss, hipStream_t st) {
  Learned* L = getL(h);
  if (!L) return fail(MM_EINVAL, "invalid learned handle");
  const Act a = acts(L);
  const int64_t per = int64_t(L->nc) * L->ny * L->nx;
  std::vector<double> lp(2048);
  double tot = 0.0;
  for (int64_t s0 = 0; s0 < npairs; s0 += L->batch) {
    const int bsz = int((npairs - s0 < L->batch) ? (npairs - s0) : L->batch);
    MM_HIP(hipMemcpyAsync(a.R, rw + s0 * per, bsz * per * 4, hipMemcpyDeviceToDevice, st));
    MM_HIP(hipMemcpyAsync(a.T, t + s0 * per, bsz * per * 4, hipMemcpyDeviceToDevice, st));
    MM_HIP(hipMemcpyAsync(a.e2, e2 + s0, bsz * 4, hipMemcpyDeviceToDevice, st));
    hth(L, a, a.R, a.y, bsz, st);
    int lb = int((per * bsz + 255) / 256);
    if (lb > 2048) lb = 2048;
    hipLaunchKernelGGL(k_loss_grad, dim3(lb), dim3(256), 0, st, a.y, a.T, a.e2, per, bsz, a.gy,
                       reinterpret_cast<double*>(L->ws + L->lpart));
    MM_HIP(hipGetLastError());
    MM_HIP(hipMemcpyAsync(lp.data(), L->ws + L->lpart, size_t(lb) * 8, hipMemcpyDeviceToHost, st));
    MM_HIP(hipStreamSynchronize(st));
    for (int k = 0; k < lb; ++k) tot += lp[k];
  }
  *loss = tot / double(npairs);
  return MM_OK;
}

// Test hook: one H^T H (and its parts) on B images already in device memory.
mm_status learned_forward(mm_learned h, const float* x, int B, float* y, float* a1, float* a2,
                          float* a3, hipStream_t st) {
  Learned* L = getL(h);
  if (!L) return fail(MM_EINVAL, "invalid learned handle");
  if (B < 1 || B > L->batch) return fail(MM_EINVAL, "B out of range");
  const Act a = acts(L);
  const int64_t per = int64_t(L->nc) * L->ny * L->nx, p16 = int64_t(16) * L->ny * L->nx;
  MM_HIP(hipMemcpyAsync(a.R, x, B * per * 4, hipMemcpyDeviceToDevice, st));
  hth(L, a, a.R, a.y, B, st);
  MM_HIP(hipGetLastError());
  MM_HIP(hipMemcpyAsync(y, a.y, B * per * 4, hipMemcpyDeviceToDevice, st));
  if (a1) MM_HIP(hipMemcpyAsync(a1, a.a1, B * p16 * 4, hipMemcpyDeviceToDevice, st));
  if (a2) MM_HIP(hipMemcpyAsync(a2, a.a2, B * p16 * 4, hipMemcpyDeviceToDevice, st));
  if (a3) MM_HIP(hipMemcpyAsync(a3, a.a3, B * p16 * 4, hipMemcpyDeviceToDevice, st));
  return MM_OK;
}

// Test hook: the loss and the weight gradients (no update) for B pairs.
mm_status learned_grad(mm_learned h, const float* rw, const float* t, const float* e2, int B,
                       double* loss, float* g1, float* g2, hipStream_t st) {
  Learned* L = getL(h);
  if (!L) return fail(MM_EINVAL, "invalid learned handle");
  if (B < 1 || B > L->batch) return fail(MM_EINVAL, "B out of range");
  const Act a = acts(L);
  const int64_t per = int64_t(L->nc) * L->ny * L->nx;
  MM_HIP(hipMemcpyAsync(a.R, rw, B * per * 4, hipMemcpyDeviceToDevice, st));
  MM_HIP(hipMemcpyAsync(a.T, t, B * per * 4, hipMemcpyDeviceToDevice, st));
  MM_HIP(hipMemcpyAsync(a.e2, e2, B * 4, hipMemcpyDeviceToDevice, st));
  mm_train_opts o{};
  o.lr = 0.0;  // no update: a zero step leaves the weights unchanged
  o.beta1 = 0.9;
  o.beta2 = 0.999;
  o.eps = 1e-8;
  const int saved = L->step;
  // save Adam state so the hook has no side effects
  const int w1n = 16 * L->nc * 25;
  std::vector<float> sm1(w1n), sv1(w1n), sm2(kW2), sv2(kW2);
  MM_HIP(hipMemcpy(sm1.data(), L->at(L->m1), w1n * 4, hipMemcpyDeviceToHost));
  MM_HIP(hipMemcpy(sv1.data(), L->at(L->v1), w1n * 4, hipMemcpyDeviceToHost));
  MM_HIP(hipMemcpy(sm2.data(), L->at(L->m2), kW2 * 4, hipMemcpyDeviceToHost));
  MM_HIP(hipMemcpy(sv2.data(), L->at(L->v2), kW2 * 4, hipMemcpyDeviceToHost));
  int nlp = 0;
  mm_status rc = train_step(L, a, B, &o, st, &nlp);
  if (rc != MM_OK) return rc;
  L->step = saved;
  std::vector<double> lp(nlp);
  MM_HIP(hipMemcpyAsync(lp.data(), L->ws + L->lpart, size_t(nlp) * 8, hipMemcpyDeviceToHost, st));
  MM_HIP(hipMemcpyAsync(g1, L->at(L->g1), w1n * 4, hipMemcpyDeviceToHost, st));
  MM_HIP(hipMemcpyAsync(g2, L->at(L->g2), kW2 * 4, hipMemcpyDeviceToHost, st));
  MM_HIP(hipStreamSynchronize(st));
  MM_HIP(hipMemcpy(L->at(L->m1), sm1.data(), w1n * 4, hipMemcpyHostToDevice));
  MM_HIP(hipMemcpy(L->at(L->v1), sv1.data(), w1n * 4, hipMemcpyHostToDevice));
  MM_HIP(hipMemcpy(L->at(L->m2), sm2.data(), kW2 * 4, hipMemcpyHostToDevice));
  MM_HIP(hipMemcpy(L->at(L->v2), sv2.data(), kW2 * 4, hipMemcpyHostToDevice));
  double tot = 0.0;
  for (double v : lp) tot += v;
  *loss = tot / B;
  return MM_OK;
}

}  // namespace mm
