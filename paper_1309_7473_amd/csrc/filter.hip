// The per-iteration operator A = P^T N^-1 P and the right-hand side
// b = P^T N^-1 d (paper eq. 2) on gfx950.
//
// Per detector the real timestream t (n samples) is viewed as n/2 packed
// complex values z[j] = t[2j] + i t[2j+1], so the data never moves to be
// packed.  The length-M = n/2 complex FFT of z gives the real spectrum
// X[k], k = 0..M, through the Hermitian pair (k, M-k):
//   E = (Z[k] + conj Z[M-k]) / 2,  O = (Z[k] - conj Z[M-k]) / (2i),
//   X[k] = E + W_n^k O,  X[M-k] = conj(E - W_n^k O).
// After Y = X / N(f) the same pair gives the packed spectrum of the filtered
// timestream, and the inverse length-M FFT (scaled by 1/M) returns it packed.
// Each pair (k, M-k) is filtered where both ends sit in LDS.
//
// Small n (M <= 8192 complex): one block per detector does gather, FFT,
// filter, inverse FFT and scatter in LDS (one kernel, no timestream traffic).
// Large n: four-step split M = M1 * M2 (index j = j1*M2 + j2, frequency
// k = k1 + M1*k2) in three kernels per group of detectors:
//   pass 1: gather P x (or read d) into C columns x M1 rows, length-M1 FFTs
//           down the columns, store;
//   pass 2: rows k1 and M1-k1 together: twiddle W_M^{k1 j2}, length-M2 FFTs,
//           pair filter (the partner of (k1,k2) is (M1-k1, M2-1-k2)), inverse
//           FFTs, conjugate twiddle, store;
//   pass 3: inverse length-M1 column FFTs, then scatter P^T back to pixels.
// The scatter pre-sums runs of equal pixels across the lanes of a wavefront
// and accumulates with float64 atomics into a [npix][4] accumulator.
//
// Storage: the timestream d and the pass buffers hold the math type (float
// or double), or bfloat16 under float math (MM_BF16): every value is rounded
// to nearest-even as it is stored and widened exactly as it is loaded, so
// only the stores between passes lose precision.
#include <type_traits>
#include <vector>
#include <cmath>

#include "fft_lds.h"
#include "fft_mixed.h"
#include "mm_internal.h"

namespace mm {

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};

struct Bf16 {};  // storage tag: bfloat16 pass buffers under float math

template <typename T, typename S>
struct Sto {  // storage in the math type itself
  using W = Cx<T>;  // one complex of the pass buffer
  using R = T;      // one real timestream sample
  static __device__ __forceinline__ Cx<T> ld(const W* p) { return *p; }
  static __device__ __forceinline__ void st(W* p, Cx<T> v) { *p = v; }
  static __device__ __forceinline__ T ldr(const R* p) { return *p; }
  static __device__ __forceinline__ T up_r(R v) { return v; }   // a loaded sample
};

template <>
struct Sto<float, Bf16> {
  using W = uint32_t;  // real part in the low half, imaginary in the high
  using R = uint16_t;
  static __device__ __forceinline__ float up(uint32_t h) { return __uint_as_float(h << 16); }
  static __device__ __forceinline__ uint32_t down(float f) {  // round to nearest even
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // NaN stays NaN
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  }
  static __device__ __forceinline__ Cx<float> ld(const W* p) {
    const uint32_t v = *p;
    return cx(__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u));
  }
  static __device__ __forceinline__ void st(W* p, Cx<float> v) {
    *p = down(v.x) | (down(v.y) << 16);
  }
  static __device__ __forceinline__ float ldr(const R* p) { return up(*p); }
  static __device__ __forceinline__ float up_r(R v) { return up(v); }
};

template <typename T, typename S>
struct PassArgs {
  using W = typename Sto<T, S>::W;
  using R = typename Sto<T, S>::R;
  const int32_t* pix;   // group base [G][n]
  const float* c2;
  const float* s2;
  const float* iN;      // group base [G][M+1]
  const R* tod;         // group base [G][n] (rhs source)
  const V4<T>* gmap;    // [npix + 1], entry npix = 0
  double* acc;          // [npix][4]
  W* work;              // [G][M] pass buffer
  const Cx<T>* tw;      // Stockham table W_Lmax^m
  TwoLevel<T> wn;       // W_n^m
  const int32_t* csr_off;  // group [npix+1]
  const int32_t* csr_idx;  // group entries
  const float2* csr_w;     // group entries (I,Q,U weights)
  const int2* csr_ia;      // group entries: (index, weights as a fixed-point angle)
  const uint32_t* rle;     // group run entries: first sample << 4 | length
  const int32_t* rle_soff; // group [npix+1]: each pixel's first sample in rle_ang
  const uint32_t* rle_ang; // group samples pixel-major: the weights as angles
  const float2* ang_tab;   // (cos, sin)(2 pi k / 256), k < 256
  const uint32_t* ang_t;   // group base [G][n]: the weights as angles, time-major
  const int4* ptc_h;       // group base [G][n/64]: chunk-coded pointing, chunk headers
  const uint32_t* ptc;     // group base [G][n]: chunk-coded pointing, samples
  const float4* bore_f;    // boresight in float32: [n] (y_b - c_y, x_b - c_x, cos phi, sin phi)
  const uint32_t* bore_a;  // [n] angle of (cos 2phi, sin 2phi)
  const float2* det_f;     // [ndet] (dy, dx) in float32
  const uint32_t* det_a;   // [ndet] angle of (cos 2psi, sin 2psi)
  const int32_t* mask;
  const float* iNt;        // group base [G][M+1], four-step order
  const Cx<T>* tw2;        // W_{2 M2}^k2, k2 < M2
  Bore bo;                 // boresight model (SRC 2, and the gather's weights)
  int det0;                // first detector of the group
  int Mi;                  // M = n/2
  int M1i;                 // four-step column length (2^a 3^b 5^c)
  uint32_t mix_code;       // stage radices of the mixed-radix LDS transform: M on the
                           // one-kernel path, M1 in passes 1 and 3 (0: a power of two)
  const Cx<T>* twm;        // W_M1^m, m < M1 (mixed-radix columns)
  int64_t n;
  int npix;
  int logM, logM1, logM2, logC, logLmax;
  T scale;              // 1/M
  double* y_out;        // non-null on the last group's gather: write acc + this
                        // group's sums to y ([ncomp][npix], zeros off the mask)
};

// Inter-detector correlated inverse noise (pass 2 in three steps).
constexpr int kMaxCorrRank = 16;

struct CorrArgs {
  const float* V;          // [nbins][ndet][rank]
  const int16_t* bin;      // [M + 1] bin of each four-step slot (entry M: bin of k = M)
  void* t;                 // [rank][M] complex: the projections sum_d V_b[d][j] X_d
  int rank, ndet;
};

// Weights (cos, sin)(theta) coded as u = theta 2^32 / 2pi (mod 2^32): with
// k = u >> 24 and d = (u mod 2^24) 2pi / 2^32 < 2pi/256, they are the table
// entry (cos, sin)(2pi k / 256) turned by d, whose cos and sin are Taylor
// polynomials to d^4 and d^5 (truncation below 1e-12); within one float32
// ulp of the weights the angle was made from.
__device__ __forceinline__ void angle_cs(uint32_t u, const float2* tab, float* c, float* sn) {
  const float2 t = tab[u >> 24];
  const float d = float(u & 0xFFFFFFu) * 1.4629180792671596e-09f;   // 2 pi / 2^32
  const float d2 = d * d;
  const float cd = 1.0f - d2 * (0.5f - d2 * (1.0f / 24.0f));
  const float sd = d * (1.0f - d2 * (1.0f / 6.0f - d2 * (1.0f / 120.0f)));
  *c = t.x * cd - t.y * sd;
  *sn = t.y * cd + t.x * sd;
}

// --------------------------------------------------------------- samples
// SRC 0: stored pointing; 1: a timestream; 2: the boresight model; 3: stored
// pixels with the weights as angles (a time-major copy made at set-up); 4:
// the boresight model from float32 copies (pass 1 of the float paths; the
// float64 definition decides the pixels the float32 evaluation cannot); 5:
// the pixels and angles of SRC 3 chunk-coded (4 B a sample, 16 B a chunk).
template <typename T, typename S, int NC, int SRC>
__device__ __forceinline__ T source_sample(const PassArgs<T, S>& a, int64_t s) {
  if constexpr (SRC == 1) {
    return Sto<T, S>::ldr(a.tod + s);
  } else if constexpr (SRC == 2 || SRC == 4) {
    // pointing from the boresight model: s = d_local * n + t
    const int d = a.det0 + int(s >> a.bo.logn);
    const int64_t t = s & ((int64_t(1) << a.bo.logn) - 1);
    const int p = bore_pixel_at(a.bo, d, t);
    const V4<T> m = a.gmap[p >= 0 ? p : a.npix];
    if constexpr (NC == 3) {
      double c, sn;
      bore_weights_at(a.bo, d, t, &c, &sn);
      return m.x + T(c) * m.y + T(sn) * m.z;
    } else {
      return m.x;
    }
  } else if constexpr (SRC == 3) {
    const int p = a.pix[s];
    const V4<T> m = a.gmap[unsigned(p) < unsigned(a.npix) ? p : a.npix];
    float c, sn;
    angle_cs(a.ang_t[s], a.ang_tab, &c, &sn);
    return m.x + T(c) * m.y + T(sn) * m.z;
  } else if constexpr (SRC == 5) {
    const int4 h = a.ptc_h[s >> kPtcLog];
    const uint32_t w = a.ptc[s];
    const uint32_t dp = w & 0xFFFFu;
    const V4<T> m = a.gmap[dp == 0xFFFFu ? a.npix : h.x + int(dp)];
    float c, sn;
    const uint32_t i = uint32_t(s & (kPtcChunk - 1));
    angle_cs(uint32_t(h.y) + uint32_t(h.z) * i + (w >> 16), a.ang_tab, &c, &sn);
    return m.x + T(c) * m.y + T(sn) * m.z;
  } else {
    const int p = a.pix[s];
    // off-map samples read the zero entry gmap[npix]: no branch around the gather
    const V4<T> m = a.gmap[unsigned(p) < unsigned(a.npix) ? p : a.npix];
    if constexpr (NC == 3) {
      return m.x + T(a.c2[s]) * m.y + T(a.s2[s]) * m.z;
    } else {
      return m.x;
    }
  }
}

// Scatter one sample per lane; must be reached by every lane of the wave
// (inactive lanes pass s < 0).
template <typename T, int NC, typename A>
__device__ __forceinline__ void scatter_sample(const A& a, int64_t s, T u) {
  int p = -1;
  double v[NC];
  v[0] = 0.0;
  if constexpr (NC == 3) {
    v[1] = 0.0;
    v[2] = 0.0;
  }
  if (s >= 0) {
    p = a.pix[s];
    if (unsigned(p) >= unsigned(a.npix)) p = -1;
    const double ud = double(u);
    v[0] = ud;
    if constexpr (NC == 3) {
      v[1] = double(a.c2[s]) * ud;
      v[2] = double(a.s2[s]) * ud;
    }
  }
  if (wave_segmented_sum<3, NC>(p, v)) {
    double* dst = a.acc + 4 * int64_t(p);
    atomic_add_f64(dst + 0, v[0]);
    if constexpr (NC == 3) {
      atomic_add_f64(dst + 1, v[1]);
      atomic_add_f64(dst + 2, v[2]);
    }
  }
}

// Filter the Hermitian pair (Z[k], Z[M-k]) in place; W = W_n^k, a = iN[k]/(4M),
// b = iN[M-k]/(4M).  The unpack's two factors 1/2 (on the even and odd
// parts and on the gains' sum and difference) ride in the gains' 1/4: as
// powers of two they change no rounding, so the result is the same bit for
// bit as with the halves applied one by one.
template <typename T>
__device__ __forceinline__ void pair_filter(Cx<T>& Zk, Cx<T>& Zmk, Cx<T> W, T a, T b) {
  const Cx<T> E = cx(Zk.x + Zmk.x, Zk.y - Zmk.y);
  const Cx<T> D = cx(Zk.x - Zmk.x, Zk.y + Zmk.y);
  const Cx<T> O = cx(D.y, -D.x);
  const Cx<T> WO = W * O;
  const T sp = a + b, sm = a - b;
  const Cx<T> Ep = cx(sp * E.x + sm * WO.x, sp * E.y + sm * WO.y);
  const Cx<T> Op = cx(sm * E.x + sp * WO.x, sm * E.y + sp * WO.y) * conj(W);
  Zk = cx(Ep.x - Op.y, Ep.y + Op.x);
  Zmk = cx(Ep.x + Op.y, Op.x - Ep.y);
}

// DC / Nyquist bin: Z[0] carries X[0] = Re+Im and X[M] = Re-Im; gains as in
// pair_filter, a0 = iN[0]/(4M), aM = iN[M]/(4M).
template <typename T>
__device__ __forceinline__ Cx<T> dc_filter(Cx<T> Z0, T a0, T aM) {
  const T y0 = a0 * (Z0.x + Z0.y);
  const T yM = aM * (Z0.x - Z0.y);
  return cx(T(2) * (y0 + yM), T(2) * (y0 - yM));
}

// The two halves of pair_filter, for a filter that mixes detectors:
// unpack (Z[k], Z[M-k]) into the real-input spectrum (X[k], X[M-k]), and
// repack a filtered (Y[k], Y[M-k]) into the packed pair.  pair_filter(a/4, b/4)
// equals pair_repack(a X[k], b X[M-k]).
template <typename T>
__device__ __forceinline__ void pair_unpack(Cx<T>& Zk, Cx<T>& Zmk, Cx<T> W) {
  const T h = T(0.5);
  const Cx<T> E = cx(h * (Zk.x + Zmk.x), h * (Zk.y - Zmk.y));
  const Cx<T> D = cx(h * (Zk.x - Zmk.x), h * (Zk.y + Zmk.y));
  const Cx<T> WO = W * cx(D.y, -D.x);
  Zk = E + WO;
  Zmk = conj(E - WO);
}

template <typename T>
__device__ __forceinline__ void pair_repack(Cx<T>& Yk, Cx<T>& Ymk, Cx<T> W) {
  const T h = T(0.5);
  const Cx<T> E = cx(h * (Yk.x + Ymk.x), h * (Yk.y - Ymk.y));
  const Cx<T> O = cx(h * (Yk.x - Ymk.x), h * (Yk.y + Ymk.y)) * conj(W);
  Yk = cx(E.x - O.y, E.y + O.x);
  Ymk = cx(E.x + O.y, O.x - E.y);
}

// slot 0: Z[0] <-> (X[0], X[M]) as (re, im), both real
template <typename T>
__device__ __forceinline__ Cx<T> dc_unpack(Cx<T> Z0) {
  return cx(Z0.x + Z0.y, Z0.x - Z0.y);
}
template <typename T>
__device__ __forceinline__ Cx<T> dc_repack(Cx<T> Y) {
  return cx(T(0.5) * (Y.x + Y.y), T(0.5) * (Y.x - Y.y));
}

// ------------------------------------------------------ prologue / epilogue
template <typename T>
__global__ void k_prologue(const double* __restrict__ x, const int32_t* __restrict__ mask,
                           V4<T>* __restrict__ gmap, double* __restrict__ acc, int npix, int nc) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > npix) return;
  if (p == npix) {   // zero entry read by off-map samples
    V4<T> z;
    z.x = z.y = z.z = z.w = T(0);
    gmap[npix] = z;
    return;
  }
  const bool on = mask[p] != 0;
  V4<T> g;
  g.x = on ? T(x[p]) : T(0);
  g.y = (on && nc == 3) ? T(x[npix + p]) : T(0);
  g.z = (on && nc == 3) ? T(x[2 * npix + p]) : T(0);
  g.w = T(0);
  gmap[p] = g;
  double4 z;
  z.x = z.y = z.z = z.w = 0.0;
  reinterpret_cast<double4*>(acc)[p] = z;
}

__global__ void k_zero_acc(double* __restrict__ acc, int npix) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  double4 z;
  z.x = z.y = z.z = z.w = 0.0;
  reinterpret_cast<double4*>(acc)[p] = z;
}

// cf: the accumulator holds float-float pairs (hi, lo) instead of doubles
__global__ void k_epilogue(const double* __restrict__ acc, const int32_t* __restrict__ mask,
                           double* __restrict__ y, int npix, int nc, int cf) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const bool on = mask[p] != 0;
  double4 a = reinterpret_cast<const double4*>(acc)[p];
  if (cf) {
    const float4 q = reinterpret_cast<const float4*>(acc)[2 * p];
    const float2 r = reinterpret_cast<const float2*>(acc)[4 * p + 2];
    a.x = f2_value(F2{q.x, q.y});
    a.y = f2_value(F2{q.z, q.w});
    a.z = f2_value(F2{r.x, r.y});
  }
  y[p] = on ? a.x : 0.0;
  if (nc == 3) {
    y[npix + p] = on ? a.y : 0.0;
    y[2 * npix + p] = on ? a.z : 0.0;
  }
}

// ------------------------------------------------------------- single pass
// CSR = true: store the filtered, packed timestream to the pass buffer for the
// per-pixel reduce instead of scattering it.
// MIX: M is a mixed-radix length (2^a 3^b 5^c), transformed by lds_fft_mx.
template <typename T, typename S, int NC, int SRC, bool CSR, bool MIX>
__global__ void __launch_bounds__(kNT) k_single(PassArgs<T, S> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem);
  T* bufr = reinterpret_cast<T*>(smem);
  const int M = a.Mi;
  const int g = blockIdx.x;
  const int64_t base = int64_t(g) * a.n;
  const int nsamp = 2 * M;
  for (int e = threadIdx.x; e < nsamp; e += kNT) bufr[e] = source_sample<T, S, NC, SRC>(a, base + e);
  __syncthreads();
  FftShape sh{a.logM, 0, 1, M, false, a.logLmax};
  const MixShape mx{M, 1, 1, M, false, a.mix_code, 1};
  if constexpr (MIX)
    lds_fft_mx<T, kNT, kE, false>(buf, mx, a.tw);
  else
    lds_fft<T, kNT, kE, false>(buf, sh, a.tw);
  const float* iN = a.iN + int64_t(g) * (M + 1);
  for (int k = threadIdx.x; k <= M / 2; k += kNT) {
    const T sq = T(0.25) * a.scale;   // the filter's gains are iN/(4M)
    if (k == 0) {
      buf[0] = dc_filter(buf[0], sq * T(iN[0]), sq * T(iN[M]));
    } else {
      Cx<T> zk = buf[k], zm = buf[M - k];
      pair_filter(zk, zm, a.wn(k), sq * T(iN[k]), sq * T(iN[M - k]));
      buf[k] = zk;
      if (k != M - k) buf[M - k] = zm;
    }
  }
  __syncthreads();
  if constexpr (MIX)
    lds_fft_mx<T, kNT, kE, true>(buf, mx, a.tw);
  else
    lds_fft<T, kNT, kE, true>(buf, sh, a.tw);
  if constexpr (CSR) {
    auto* w = a.work + int64_t(g) * M;
    for (int j = threadIdx.x; j < M; j += kNT) Sto<T, S>::st(w + j, buf[j]);
    return;
  }
  // every lane of a wave takes the same number of trips (the scatter shuffles)
  for (int e0 = 0; e0 < nsamp; e0 += kNT) {
    const int e = e0 + threadIdx.x;
    const bool in = e < nsamp;
    scatter_sample<T, NC>(a, in ? base + e : int64_t(-1), in ? bufr[e] : T(0));
  }
}

// ------------------------------------------------------------- four-step
constexpr int kNT13 = 1024;  // threads per pass-1/3 block
#ifndef MM_UB
#define MM_UB 1
#endif
constexpr int UB = MM_UB;     // sample groups in flight per thread with boresight pointing
#ifndef MM_U0
#define MM_U0 2
#endif
constexpr int U0 = MM_U0;     // ... with stored pointing
// complex elements per thread: 8 (C * M1 <= 8192) or 16 (C * M1 <= 16384,
// float math only: 128 KB of LDS per block)
constexpr int kPad2 = 3;     // pass-2 LDS padding: one slot per 8 elements

#ifndef MM_NT
#define MM_NT 1
#endif
#ifndef MM_P3_BATCH
#define MM_P3_BATCH 1
#endif
#ifndef MM_P2_BATCH
#define MM_P2_BATCH 1
#endif
#ifndef MM_BORE_FAST
#define MM_BORE_FAST 1
#endif
constexpr bool kBoreFast = MM_BORE_FAST != 0;
#ifndef MM_P2_CHUNK
#define MM_P2_CHUNK 4
#endif
#ifndef MM_RED_XCD
#define MM_RED_XCD 1
#endif

// Streaming loads of the stored pointing (read once per launch), marked
// non-temporal so they do not push the map, which pass 1 gathers from, out of
// the caches (pass 1: 252 -> 243 us per 64-detector launch).  The gather's
// index and weights are not streamed: neighbouring pixels share their lines
// (non-temporal there: 266 -> 336 us).
__device__ __forceinline__ int4 ld_stream(const int4* p) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  if (MM_NT) {
    const v4i v = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(p));
    return make_int4(v.x, v.y, v.z, v.w);
  }
  return *p;
}
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  typedef float v4f __attribute__((ext_vector_type(4)));
  if (MM_NT) {
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
  }
  return *p;
}

// Four consecutive doubles (16-byte aligned) with two 16-byte loads.
__device__ __forceinline__ void ld4d(const double* p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0];
  const double2 b = reinterpret_cast<const double2*>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

// Four consecutive samples s..s+3 (s a multiple of 4) with 16-byte loads.
template <typename T, typename S, int NC, int SRC>
__device__ __forceinline__ void source4(const PassArgs<T, S>& a, int64_t s, T (&v)[4],
                                        const float2* tab = nullptr) {
  if constexpr (SRC == 1) {
    if constexpr (std::is_same<S, Bf16>::value) {
      const uint2 t = *reinterpret_cast<const uint2*>(a.tod + s);
      v[0] = __uint_as_float(t.x << 16);
      v[1] = __uint_as_float(t.x & 0xffff0000u);
      v[2] = __uint_as_float(t.y << 16);
      v[3] = __uint_as_float(t.y & 0xffff0000u);
    } else if constexpr (sizeof(T) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(a.tod + s);
      v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    } else {
      const double2 t0 = *reinterpret_cast<const double2*>(a.tod + s);
      const double2 t1 = *reinterpret_cast<const double2*>(a.tod + s + 2);
      v[0] = t0.x; v[1] = t0.y; v[2] = t1.x; v[3] = t1.y;
    }
  } else if constexpr (SRC == 2) {
    // pointing from the boresight model for samples t..t+3 of one detector
    const int d = a.det0 + int(s >> a.bo.logn);
    const int64_t n = int64_t(1) << a.bo.logn;
    const int64_t t = s & (n - 1);
    const double* b = a.bo.b + t;
    const double dy = a.bo.det[d], dx = a.bo.det[a.bo.ndet + d];
    double yb[4], xb[4], cp[4], sp[4];
    ld4d(b, yb);
    ld4d(b + n, xb);
    ld4d(b + 2 * n, cp);
    ld4d(b + 3 * n, sp);
    double cc[4] = {0.0, 0.0, 0.0, 0.0}, ss[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (NC == 3) {
      double c2f[4], s2f[4];
      ld4d(b + 4 * n, c2f);
      ld4d(b + 5 * n, s2f);
      const double c2p = a.bo.det[2 * a.bo.ndet + d], s2p = a.bo.det[3 * a.bo.ndet + d];
#pragma unroll
      for (int i = 0; i < 4; ++i) bore_weights(c2p, s2p, c2f[i], s2f[i], &cc[i], &ss[i]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int p = bore_pixel(yb[i], xb[i], cp[i], sp[i], dy, dx, a.bo.ny, a.bo.nx);
      const V4<T> m = a.gmap[p >= 0 ? p : a.npix];
      v[i] = (NC == 3) ? m.x + T(cc[i]) * m.y + T(ss[i]) * m.z : m.x;
    }
  } else if constexpr (SRC == 4) {
    // boresight model, float32 copies: 20 B per time sample shared by every
    // detector; the float64 definition where float32 cannot decide the pixel
    const int d = a.det0 + int(s >> a.bo.logn);
    const int64_t n = int64_t(1) << a.bo.logn;
    const int64_t t = s & (n - 1);
    const float2 df = a.det_f[d];
    const uint32_t ad = a.det_a[d];
    const int4 au = *reinterpret_cast<const int4*>(a.bore_a + t);
    const uint32_t aa[4] = {uint32_t(au.x), uint32_t(au.y), uint32_t(au.z), uint32_t(au.w)};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 b = a.bore_f[t + i];
      int p = bore_pixel_f32(b.x, b.y, b.z, b.w, df.x, df.y, a.bo.ny, a.bo.nx);
      if (p == -2) p = bore_pixel_slow(a.bo, d, t + i);
      const V4<T> m = a.gmap[p >= 0 ? p : a.npix];
      if constexpr (NC == 3) {
        float c, sn;
        angle_cs(ad + aa[i], tab, &c, &sn);
        v[i] = m.x + T(c) * m.y + T(sn) * m.z;
      } else {
        v[i] = m.x;
      }
    }
  } else if constexpr (SRC == 5) {
    // chunk-coded pixels and angles: 4 B a sample and the chunk's header
    const int4 h = a.ptc_h[s >> kPtcLog];
    const int4 w4 = ld_stream(reinterpret_cast<const int4*>(a.ptc + s));
    const uint32_t ww[4] = {uint32_t(w4.x), uint32_t(w4.y), uint32_t(w4.z), uint32_t(w4.w)};
    // the angle trend at the first of the four samples, then one step each
    const uint32_t t0 = uint32_t(h.y) + uint32_t(h.z) * uint32_t(s & (kPtcChunk - 1));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t dp = ww[i] & 0xFFFFu;
      float c, sn;
      angle_cs(t0 + uint32_t(h.z) * uint32_t(i) + (ww[i] >> 16), tab, &c, &sn);
      const V4<T> m = a.gmap[dp == 0xFFFFu ? a.npix : h.x + int(dp)];
      v[i] = m.x + T(c) * m.y + T(sn) * m.z;
    }
  } else if constexpr (SRC == 3) {
    // stored pixels and angle-coded weights: 8 B a sample instead of 12
    const int4 p4 = ld_stream(reinterpret_cast<const int4*>(a.pix + s));
    const int4 u4 = ld_stream(reinterpret_cast<const int4*>(a.ang_t + s));
    const int pp[4] = {p4.x, p4.y, p4.z, p4.w};
    const uint32_t uu[4] = {uint32_t(u4.x), uint32_t(u4.y), uint32_t(u4.z), uint32_t(u4.w)};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float c, sn;
      angle_cs(uu[i], tab, &c, &sn);
      const V4<T> m = a.gmap[unsigned(pp[i]) < unsigned(a.npix) ? pp[i] : a.npix];
      v[i] = m.x + T(c) * m.y + T(sn) * m.z;
    }
  } else {
    const int4 p4 = ld_stream(reinterpret_cast<const int4*>(a.pix + s));
    const int pp[4] = {p4.x, p4.y, p4.z, p4.w};
    float cc[4] = {0.f, 0.f, 0.f, 0.f}, ss[4] = {0.f, 0.f, 0.f, 0.f};
    if constexpr (NC == 3) {
      const float4 c4 = ld_stream(reinterpret_cast<const float4*>(a.c2 + s));
      const float4 s4 = ld_stream(reinterpret_cast<const float4*>(a.s2 + s));
      cc[0] = c4.x; cc[1] = c4.y; cc[2] = c4.z; cc[3] = c4.w;
      ss[0] = s4.x; ss[1] = s4.y; ss[2] = s4.z; ss[3] = s4.w;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const V4<T> m = a.gmap[unsigned(pp[i]) < unsigned(a.npix) ? pp[i] : a.npix];
      v[i] = (NC == 3) ? m.x + T(cc[i]) * m.y + T(ss[i]) * m.z : m.x;
    }
  }
}

// U groups of four samples (sample indices s[u], multiples of 4) from stored
// pointing with angle-coded weights (SRC 3, or SRC 5 chunk-coded), in three
// phases so that the memory round trips of the groups overlap: every group's
// pointing words, then every map gather, then the weights, decoded while the
// gathers are in flight, and the sums.
template <typename T, typename S, int SRC, int U>
__device__ __forceinline__ void stored_groups(const PassArgs<T, S>& a, const int64_t (&s)[U],
                                              const float2* tab, T (&v)[U][4]) {
  static_assert(SRC == 3 || SRC == 5, "stored pointing with angle-coded weights");
  uint32_t pw[U][4], aw[U][4];
  int4 h[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if constexpr (SRC == 5) {
      const int4 w4 = ld_stream(reinterpret_cast<const int4*>(a.ptc + s[u]));
      h[u] = a.ptc_h[s[u] >> kPtcLog];
      pw[u][0] = uint32_t(w4.x); pw[u][1] = uint32_t(w4.y);
      pw[u][2] = uint32_t(w4.z); pw[u][3] = uint32_t(w4.w);
    } else {
      const int4 p4 = ld_stream(reinterpret_cast<const int4*>(a.pix + s[u]));
      const int4 u4 = ld_stream(reinterpret_cast<const int4*>(a.ang_t + s[u]));
      pw[u][0] = uint32_t(p4.x); pw[u][1] = uint32_t(p4.y);
      pw[u][2] = uint32_t(p4.z); pw[u][3] = uint32_t(p4.w);
      aw[u][0] = uint32_t(u4.x); aw[u][1] = uint32_t(u4.y);
      aw[u][2] = uint32_t(u4.z); aw[u][3] = uint32_t(u4.w);
    }
  }
  V4<T> m[U][4];
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int p;
      if constexpr (SRC == 5) {
        const uint32_t dp = pw[u][i] & 0xFFFFu;
        p = dp == 0xFFFFu ? a.npix : h[u].x + int(dp);
      } else {
        p = pw[u][i] < uint32_t(a.npix) ? int(pw[u][i]) : a.npix;
      }
      m[u][i] = a.gmap[p];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t ua;
      if constexpr (SRC == 5) {   // the chunk's angle trend at this sample, plus the residual
        ua = uint32_t(h[u].y) + uint32_t(h[u].z) * uint32_t((s[u] & (kPtcChunk - 1)) + i) +
             (pw[u][i] >> 16);
      } else {
        ua = aw[u][i];
      }
      float c, sn;
      angle_cs(ua, tab, &c, &sn);
      v[u][i] = m[u][i].x + T(c) * m[u][i].y + T(sn) * m[u][i].z;
    }
  }
}

template <typename T>
__device__ __forceinline__ void store4(T* dst, const T (&v)[4]) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    reinterpret_cast<double2*>(dst)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2*>(dst)[1] = make_double2(v[2], v[3]);
  }
}

// Copies the length-L Stockham twiddles (W_L^m = W_Lmax^(m Lmax/L)) to LDS.
template <typename T, int NT>
__device__ __forceinline__ void stage_twiddles(Cx<T>* stw, const Cx<T>* tw, int logL, int logLmax) {
  for (int m = threadIdx.x; m < (1 << logL); m += NT) stw[m] = tw[m << (logLmax - logL)];
}

// Blocks are dealt to the 8 XCDs round-robin (block i runs on XCD i mod 8).
// For pass 1/3 the column blocks of a detector are renumbered so that XCD x
// handles the x-th eighth of them: its samples then sit in one eighth of each
// sweep, and the map pixels they touch stay in that XCD's L2.
//
// With boresight pointing (DET_FAST) the slots of an XCD take its column
// blocks one at a time for every detector of the group in turn: the blocks
// resident together then read the same boresight samples, which stay in
// that XCD's L2 instead of being streamed once per detector.
template <bool DET_FAST = false>
__device__ __forceinline__ void col_block(int logNB, int* g, int* cb) {
  const int bid = blockIdx.x;
  if (DET_FAST && logNB >= 3) {
    const int x = bid & 7, slot = bid >> 3;
    const int per = 1 << (logNB - 3);
    const int gd = int(gridDim.x) >> logNB;                // detectors in the group
    *g = slot % gd;
    *cb = x * per + slot / gd;
    return;
  }
  if (logNB >= 3) {
    const int x = bid & 7, slot = bid >> 3;              // XCD, slot on it
    const int per = 1 << (logNB - 3);                      // column blocks per XCD
    *g = slot >> (logNB - 3);
    *cb = x * per + (slot & (per - 1));
  } else {
    *g = bid >> logNB;
    *cb = bid & ((1 << logNB) - 1);
  }
}

// MIX: the column length M1 is mixed-radix (lds_fft_mx on the columns).
// Blocks of at most 8 elements a thread (C * M1 <= 8192, 68 KB of LDS) can
// run two to a CU when a thread holds at most 64 VGPRs (eight waves a SIMD):
// ask for that; the larger tiles fit one block a CU anyway.
template <typename T, int E13>
constexpr int pass1_waves() {
  return (E13 == 8 && sizeof(T) == 4) ? 8 : 1;
}

template <typename T, typename S, int NC, int SRC, int E13, bool MIX>
__global__ void __launch_bounds__(kNT13)
__attribute__((amdgpu_waves_per_eu(pass1_waves<T, E13>())))
k_pass1(PassArgs<T, S> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem);
  T* bufr = reinterpret_cast<T*>(smem);
  const int logNB = a.logM2 - a.logC;
  int g, cb;
  col_block<SRC == 2 || SRC == 4>(logNB, &g, &cb);
  const int C = 1 << a.logC;
  const int M1 = a.M1i, M2 = 1 << a.logM2;
  Cx<T>* stw = buf + C * M1;
  const int j20 = cb << a.logC;
  const int64_t base = int64_t(g) * a.n;
  if constexpr (MIX)
    for (int m = threadIdx.x; m < M1; m += kNT13) stw[m] = a.twm[m];
  else
    stage_twiddles<T, kNT13>(stw, a.tw, a.logM1, a.logLmax);
  __shared__ float2 angtab[SRC >= 3 ? 256 : 1];   // angle-coded weights' table
  if constexpr (SRC >= 3) {
    if (threadIdx.x < 256) angtab[threadIdx.x] = a.ang_tab[threadIdx.x];
    __syncthreads();
  }
  const int nq = (C * M1) >> 1;  // groups of 4 samples
  // U groups per thread per trip, every load of a trip issued before the
  // first use; a group past the end re-reads group e40 and is not stored.
  constexpr int U = (SRC == 2 || SRC == 4) ? UB : U0;
  int e40 = threadIdx.x;
  if constexpr (SRC == 3 || SRC == 5) {
    // trips whose U groups are all in range, without a branch between the
    // groups' loads
    for (; e40 + (U - 1) * kNT13 < nq; e40 += U * kNT13) {
      T v[U][4];
      int64_t si[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = (e40 + u * kNT13) << 2;
        const int j1 = e >> (a.logC + 1);
        const int q = e & (2 * C - 1);
        si[u] = base + 2 * (int64_t(j1) * M2 + j20) + q;
      }
      stored_groups<T, S, SRC, U>(a, si, angtab, v);
#pragma unroll
      for (int u = 0; u < U; ++u) store4(bufr + ((e40 + u * kNT13) << 2), v[u]);
    }
  }
  for (; e40 < nq; e40 += U * kNT13) {
    T v[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e4 = e40 + u * kNT13;
      const int e = (e4 < nq ? e4 : e40) << 2;
      const int j1 = e >> (a.logC + 1);
      const int q = e & (2 * C - 1);
      source4<T, S, NC, SRC>(a, base + 2 * (int64_t(j1) * M2 + j20) + q, v[u], angtab);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e4 = e40 + u * kNT13;
      if (e4 < nq) store4(bufr + (e4 << 2), v[u]);
    }
  }
  __syncthreads();
  FftShape sh{a.logM1, a.logC, C, 1, true, a.logM1};
  if constexpr (MIX)
    lds_fft_mx<T, kNT13, E13, false>(buf, MixShape{M1, C, C, 1, true, a.mix_code, 1}, stw);
  else
    lds_fft<T, kNT13, E13, false>(buf, sh, stw);
  auto* w = a.work + int64_t(g) * a.Mi;
  for (int e = threadIdx.x; e < C * M1; e += kNT13) {
    const int k1 = e >> a.logC;
    const int c = e & (C - 1);
    Sto<T, S>::st(w + int64_t(k1) * M2 + j20 + c, buf[e]);
  }
}

// Rows k1 = ra and rb = M1 - ra (or 0 and M1/2) of one detector.  The
// four-step twiddle W_M^(k1 j2) = A[j2 >> 6] * B[j2 & 63] comes from two
// small per-row LDS tables; W_n^k = W_n^k1 * W_2M2^k2; 1/N(f) is read from
// its copy in four-step order (row k1 contiguous).
template <typename T, typename S, int E>
__global__ void __launch_bounds__(kNT) k_pass2(PassArgs<T, S> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M1 = a.M1i, M2 = 1 << a.logM2;
  const int M = a.Mi;
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem);
  Cx<T>* stw = buf + lds_at<kPad2>(2 * M2);   // length-M2 Stockham twiddles
  const int logJL = a.logM2 < 6 ? a.logM2 : 6;
  const int JL = 1 << logJL, JH = M2 >> logJL;
  Cx<T>* tA = stw + M2;      // [2][JH]
  Cx<T>* tB = tA + 2 * JH;   // [2][JL]
  const int half = M1 >> 1;   // row pairs per detector
  const int g = blockIdx.x / half;
  const int pr = blockIdx.x % half;
  const int ra = pr;
  const int rb = (pr == 0) ? (M1 >> 1) : (M1 - pr);
  stage_twiddles<T, kNT>(stw, a.tw, a.logM2, a.logLmax);
  for (int t = threadIdx.x; t < 2 * JH; t += kNT) {
    const int r = t >= JH, jh = t - r * JH;
    tA[t] = a.wn(2 * int64_t(r ? rb : ra) * (int64_t(jh) << logJL));
  }
  for (int t = threadIdx.x; t < 2 * JL; t += kNT) {
    const int r = t >= JL, jl = t - r * JL;
    tB[t] = a.wn(2 * int64_t(r ? rb : ra) * jl);
  }
  __syncthreads();
  auto* w = a.work + int64_t(g) * M;
  for (int e = threadIdx.x; e < 2 * M2; e += kNT) {
    const int row = e >> a.logM2;
    const int j2 = e & (M2 - 1);
    const int k1 = row ? rb : ra;
    const Cx<T> v = Sto<T, S>::ld(w + int64_t(k1) * M2 + j2);
    buf[lds_at<kPad2>(e)] = v * (tA[row * JH + (j2 >> logJL)] * tB[row * JL + (j2 & (JL - 1))]);
  }
  __syncthreads();
  FftShape sh{a.logM2, 1, 1, M2, false, a.logM2};
  lds_fft<T, kNT, E, false, kPad2, true>(buf, sh, stw);
  const float* iN = a.iNt + int64_t(g) * (M + 1);  // [k1][k2] order, then iN[M]
  const T sc = T(0.25) * a.scale;   // the filter's gains are iN/(4M)
  if (pr != 0) {
    const Cx<T> wa = a.wn(ra);
    const float* ia = iN + int64_t(ra) * M2;
    const float* ib = iN + int64_t(rb) * M2;
    for (int k2 = threadIdx.x; k2 < M2; k2 += kNT) {
      const int im = M2 + (M2 - 1 - k2);
      Cx<T> zk = buf[lds_at<kPad2>(k2)], zm = buf[lds_at<kPad2>(im)];
      pair_filter(zk, zm, wa * a.tw2[k2], sc * T(ia[k2]), sc * T(ib[M2 - 1 - k2]));
      buf[lds_at<kPad2>(k2)] = zk;
      buf[lds_at<kPad2>(im)] = zm;
    }
  } else {
    const Cx<T> wh = a.wn(M1 >> 1);
    const float* ih = iN + int64_t(M1 >> 1) * M2;
    for (int t = threadIdx.x; t < M2; t += kNT) {
      if (t < M2 / 2) {
        // row 0: k = M1*k2, partner M1*(M2-k2)
        const int k2 = t;
        if (k2 == 0) {
          buf[lds_at<kPad2>(0)] = dc_filter(buf[lds_at<kPad2>(0)], sc * T(iN[0]), sc * T(iN[M]));
          // k = M/2 (k2 = M2/2) pairs with itself
          const int h = M2 / 2;
          Cx<T> zk = buf[lds_at<kPad2>(h)], zm = buf[lds_at<kPad2>(h)];
          pair_filter(zk, zm, a.tw2[h], sc * T(iN[h]), sc * T(iN[h]));
          buf[lds_at<kPad2>(h)] = zk;
        } else {
          Cx<T> zk = buf[lds_at<kPad2>(k2)], zm = buf[lds_at<kPad2>(M2 - k2)];
          pair_filter(zk, zm, a.tw2[k2], sc * T(iN[k2]), sc * T(iN[M2 - k2]));
          buf[lds_at<kPad2>(k2)] = zk;
          buf[lds_at<kPad2>(M2 - k2)] = zm;
        }
      } else {
        // row M1/2: k = M1/2 + M1*k2, partner at column M2-1-k2
        const int k2 = t - M2 / 2;
        const int i0 = M2 + k2, i1 = M2 + (M2 - 1 - k2);
        Cx<T> zk = buf[lds_at<kPad2>(i0)], zm = buf[lds_at<kPad2>(i1)];
        pair_filter(zk, zm, wh * a.tw2[k2], sc * T(ih[k2]), sc * T(ih[M2 - 1 - k2]));
        buf[lds_at<kPad2>(i0)] = zk;
        buf[lds_at<kPad2>(i1)] = zm;
      }
    }
  }
  __syncthreads();
  lds_fft<T, kNT, E, true, kPad2, true>(buf, sh, stw);
  for (int e = threadIdx.x; e < 2 * M2; e += kNT) {
    const int row = e >> a.logM2;
    const int j2 = e & (M2 - 1);
    const int k1 = row ? rb : ra;
    Sto<T, S>::st(w + int64_t(k1) * M2 + j2,
                  buf[lds_at<kPad2>(e)] *
                      conj(tA[row * JH + (j2 >> logJL)] * tB[row * JL + (j2 & (JL - 1))]));
  }
}

// Pass 2 with one wavefront per row, for rows of M2 = 64 E (E = 8, 16, 32).
// A block holds PB row pairs (2 PB waves).  Per row the length-M2 FFT is a
// radix-E stage in registers fed straight from global memory (lane l holds
// elements l + 64 r), then two radix-8 Stockham stages through this wave's
// padded LDS row; the spectrum ends in natural order.  Stage twiddles come
// from the global table (it stays in cache); keeping them out of LDS lets
// more blocks share a CU.  The pair filter runs on the two rows of a pair,
// the inverse FFT mirrors the forward one and its last stage stores straight
// to global memory.
#ifndef MM_PASS2W
#define MM_PASS2W 1
#endif

// LDS slot of element i of a row: one pad slot after every 32 elements.
// Every access of the kernel (radix-E writes at stride E, radix-8 reads and
// writes, the filter's forward and reversed walks) is then a per-lane base
// plus a constant, so the compiler folds it into the LDS instruction's
// offset; a bank model of those accesses (8-byte elements, 32 or 64 banks)
// costs 1.125 of the conflict-free cycles at 1024-bin rows, 1.0 at 2048 and
// at most 1.375 at 512.
constexpr int kP2PadLog = 5;
template <int LOGE>
__device__ __forceinline__ int pad_e(int i) {
  return i + (i >> kP2PadLog);
}

// MODE 0: forward FFT, 1/N(f) filter, inverse FFT.  MODE 1 (correlated
// noise): forward FFT and unpack to the real-input spectrum X, stored in
// place in natural order.  MODE 2: load the filtered spectrum Y, repack,
// inverse FFT.
template <typename T, typename S, int E, int PB, int MODE>
#ifndef MM_P2_REV
#define MM_P2_REV 1
#endif
#ifndef MM_P2W_WAVES
#define MM_P2W_WAVES 0
#endif
__global__ void __launch_bounds__(128 * PB)
#if MM_P2W_WAVES > 0
__attribute__((amdgpu_waves_per_eu(MM_P2W_WAVES)))
#endif
k_pass2w(PassArgs<T, S> a, CorrArgs c) {
  constexpr int LOGE = (E == 8) ? 3 : (E == 16) ? 4 : 5;
  constexpr int L = 64 * E;              // = M2
  constexpr int LOGL = LOGE + 6;
  constexpr int RS = L + (L >> kP2PadLog);   // padded LDS row
  constexpr int NB = E / 8;              // radix-8 butterflies per lane
  constexpr int NW = 2 * PB;             // waves (rows) per block
  constexpr int NT = 64 * NW;
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* rows = reinterpret_cast<Cx<T>*>(smem);   // [NW][RS]
  Cx<T>* tA = rows + NW * RS;                      // [NW][E]
  const int M1 = a.M1i;
  const int M = a.Mi;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int half = M1 >> 1;   // row pairs per detector
  // blocks run from the last detector of the group to the first: pass 1
  // wrote the last detectors last, so their rows are the likeliest to be
  // still in the memory-side cache
  const int bx = MM_P2_REV ? int(gridDim.x) - 1 - int(blockIdx.x) : int(blockIdx.x);
  auto row_of = [&](int w) {
    const int prw = (bx * PB + (w >> 1)) % half;
    return (w & 1) ? ((prw == 0) ? (M1 >> 1) : (M1 - prw)) : prw;
  };
  const int pair = bx * PB + (wave >> 1);
  const int g = pair / half;
  const int pr = pair % half;
  const int ra = pr;
  const int rb = (pr == 0) ? (M1 >> 1) : (M1 - pr);
  const int myrow = row_of(wave);
  auto* w = a.work + int64_t(g) * M + int64_t(myrow) * L;
  // the row's loads are issued before the twiddles are formed, so the two
  // latencies overlap.  The four-step twiddle of element j2 = l + 64 r of
  // the row is W_M^(row j2) = tA[r] * tb: tA[r] = W_M^(64 row r) from a
  // small per-row LDS table, tb = W_M^(row l) in a register (the last
  // inverse stage stores index j2 from lane j2 mod 64 too)
  Cx<T> v[E];
  if constexpr (MODE != 2) {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = Sto<T, S>::ld(w + lane + 64 * r);
  }
  for (int t = threadIdx.x; t < NW * E; t += NT)
    tA[t] = a.wn(2 * int64_t(row_of(t / E)) * (int64_t(t % E) << 6));
  const Cx<T> tb = a.wn(2 * int64_t(myrow) * lane);
  __syncthreads();
  const int tsh = a.logLmax - LOGL;
  auto twL = [&](int m) { return a.tw[m << tsh]; };   // W_L^m, from the cached table
  Cx<T>* R = rows + wave * RS;
  const ConstTw<T, (E < 16 ? 16 : E)> twE;   // W_E^m (unused at E = 8)
  // ---------------- forward: radix-E from global, then 2 x radix-8
  if constexpr (MODE != 2) {
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = v[r] * (tA[wave * E + r] * tb);
    dft_regs<T, E, false>(v, twE);
#pragma unroll
    for (int r = 0; r < E; ++r) R[pad_e<LOGE>(lane * E + r)] = v[r];
  } else {
    // Y = (1/M) (iN_d X - sum_j V_b[d][j] t_j) for this wave's row (detector g)
    const Cx<T>* t = static_cast<const Cx<T>*>(c.t);
    const float* iNr = a.iNt + int64_t(g) * (M + 1);
    const T sc = a.scale;
    // all loads of the row first (lane holds elements lane + 64 r), then the
    // rank terms, whose V rows depend on the loaded bins
    Cx<T> xs[E];
    T dn[E];
    int bs[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int slot = myrow * L + lane + 64 * r;
      xs[r] = Sto<T, S>::ld(w + lane + 64 * r);
      dn[r] = T(iNr[slot]);
      bs[r] = c.bin[slot];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = lane + 64 * r;
      const int slot = myrow * L + i;
      const Cx<T> x = xs[r];
      Cx<T> y;
      if (slot != 0) {
        const float* v = c.V + (int64_t(bs[r]) * c.ndet + g) * c.rank;
        T yr = dn[r] * x.x, yi = dn[r] * x.y;
        for (int j = 0; j < c.rank; ++j) {
          const Cx<T> tj = t[(int64_t(j) << a.logM) + slot];
          yr -= T(v[j]) * tj.x;
          yi -= T(v[j]) * tj.y;
        }
        y = cx(sc * yr, sc * yi);
      } else {   // X[0] and X[M], real, with their own bins and gains
        const float* v0 = c.V + (int64_t(c.bin[0]) * c.ndet + g) * c.rank;
        const float* vN = c.V + (int64_t(c.bin[M]) * c.ndet + g) * c.rank;
        T y0 = T(iNr[0]) * x.x, yM = T(iNr[M]) * x.y;
        for (int j = 0; j < c.rank; ++j) {
          const Cx<T> tj = t[int64_t(j) << a.logM];
          y0 -= T(v0[j]) * tj.x;
          yM -= T(vN[j]) * tj.y;
        }
        y = cx(sc * y0, sc * yM);
      }
      R[pad_e<LOGE>(i)] = y;
    }
  }
  __syncthreads();
  auto radix8 = [&](int logNs, bool inv, bool to_lds) {
    const int Ns = 1 << logNs;
    const int sh = LOGL - logNs - 3;     // W_{8 Ns}^(r k) = W_L^(r k << sh)
    // with Ns <= 64 every butterfly of a lane has k = lane mod Ns: one set
    constexpr int NQ = NB;
    const int nq = Ns <= 64 ? 1 : NQ;
    // W and W^4 of each butterfly, read before the stage's LDS reads and
    // barrier so their latency overlaps them
    Cx<T> q1[NQ], q4[NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      if (i < nq) {
        const int k = (lane + 64 * i) & (Ns - 1);
        q1[i] = twL(k << sh);
        q4[i] = twL((4 * k) << sh);
      }
    }
    Cx<T> u[NB][8];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = lane + 64 * i;
#pragma unroll
      for (int r = 0; r < 8; ++r) u[i][r] = R[pad_e<LOGE>(j + (L / 8) * r)];
    }
    __syncthreads();
    // the twiddles W_{8 Ns}^(r k), r = 1..7, of butterfly i's k from W and
    // W^4: the other powers by products
    auto twiddles = [&](int i, Cx<T> (&t)[8]) {
      Cx<T> t1 = q1[i], t4 = q4[i];
      if (inv) {
        t1.y = -t1.y;
        t4.y = -t4.y;
      }
      t[1] = t1;
      t[2] = t1 * t1;
      t[3] = t[2] * t1;
      t[4] = t4;
      t[5] = t4 * t1;
      t[6] = t4 * t[2];
      t[7] = t4 * t[3];
    };
    Cx<T> ts[8];
    if (Ns <= 64) twiddles(0, ts);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int j = lane + 64 * i;
      const int k = j & (Ns - 1);
      Cx<T> tt[8];
      if (Ns > 64) twiddles(i, tt);
#pragma unroll
      for (int r = 1; r < 8; ++r) u[i][r] = u[i][r] * (Ns <= 64 ? ts[r] : tt[r]);
      if (inv)
        dft_reg<T, 8, true>(u[i]);
      else
        dft_reg<T, 8, false>(u[i]);
      const int out = ((j - k) << 3) + k;
      if (to_lds) {
#pragma unroll
        for (int r = 0; r < 8; ++r) R[pad_e<LOGE>(out + r * Ns)] = u[i][r];
      } else {
        // last inverse stage: natural order out = j + r * L/8; conjugate twiddle, store
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int idx = out + r * Ns;
          Sto<T, S>::st(w + idx, u[i][r] * conj(tA[wave * E + (idx >> 6)] * tb));
        }
      }
    }
    if (to_lds) __syncthreads();
  };
  if constexpr (MODE != 2) {
    radix8(LOGE, false, true);
    radix8(LOGE + 3, false, true);
  }
  // the pair operation: the filter, or the unpack / repack of MODE 1 / 2
  auto pair_op = [&](Cx<T>& zk, Cx<T>& zm, Cx<T> W, T fa, T fb) {
    if constexpr (MODE == 0)
      pair_filter(zk, zm, W, fa, fb);
    else if constexpr (MODE == 1)
      pair_unpack(zk, zm, W);
    else
      pair_repack(zk, zm, W);
  };
  auto dc_op = [&](Cx<T> z, T f0, T fM) {
    if constexpr (MODE == 0)
      return dc_filter(z, f0, fM);
    else if constexpr (MODE == 1)
      return dc_unpack(z);
    else
      return dc_repack(z);
  };
  // ---------------- pair operation on rows ra (wave 2h) and rb (wave 2h+1)
  {
    const int h = wave >> 1;
    Cx<T>* Ra = rows + (2 * h) * RS;
    Cx<T>* Rb = Ra + RS;
    const int tp = threadIdx.x & 127;   // thread within the pair
    const float* iN = a.iNt + int64_t(g) * (M + 1);
    const T sc = T(0.25) * a.scale;
    // the filter's gains iN/(4M) (MODE 0 only reads 1/N(f))
    auto gain = [&](const float* p, int i) { return MODE == 0 ? sc * T(p[i]) : T(0); };
    if (pr != 0) {
      const Cx<T> wa = a.wn(ra);
      const float* ia = iN + int64_t(ra) * L;
      const float* ib = iN + int64_t(rb) * L;
#if MM_P2_BATCH
      // the pair loop's global loads in flight in chunks of NC2 before use
      constexpr int NP = L / 128;
      constexpr int NC2 = NP < MM_P2_CHUNK ? NP : MM_P2_CHUNK;
#pragma unroll
      for (int i0c = 0; i0c < NP; i0c += NC2) {
        T ga[NC2], gb[NC2];
        Cx<T> tw[NC2];
#pragma unroll
        for (int i = 0; i < NC2; ++i) {
          const int k2 = tp + 128 * (i0c + i);
          ga[i] = gain(ia, k2);
          gb[i] = gain(ib, L - 1 - k2);
          tw[i] = a.tw2[k2];
        }
#pragma unroll
        for (int i = 0; i < NC2; ++i) {
          const int k2 = tp + 128 * (i0c + i);
          const int i0 = pad_e<LOGE>(k2), i1 = pad_e<LOGE>(L - 1 - k2);
          Cx<T> zk = Ra[i0], zm = Rb[i1];
          pair_op(zk, zm, wa * tw[i], ga[i], gb[i]);
          Ra[i0] = zk;
          Rb[i1] = zm;
        }
      }
#else
      for (int k2 = tp; k2 < L; k2 += 128) {
        const int i0 = pad_e<LOGE>(k2), i1 = pad_e<LOGE>(L - 1 - k2);
        Cx<T> zk = Ra[i0], zm = Rb[i1];
        pair_op(zk, zm, wa * a.tw2[k2], gain(ia, k2), gain(ib, L - 1 - k2));
        Ra[i0] = zk;
        Rb[i1] = zm;
      }
#endif
    } else {
      const Cx<T> wh = a.wn(M1 >> 1);
      const float* ih = iN + int64_t(M1 >> 1) * L;
      for (int t = tp; t < L; t += 128) {
        if (t < L / 2) {
          const int k2 = t;
          if (k2 == 0) {
            Ra[0] = dc_op(Ra[0], gain(iN, 0), gain(iN, M));
            const int hh = pad_e<LOGE>(L / 2);
            Cx<T> zk = Ra[hh], zm = Ra[hh];
            pair_op(zk, zm, a.tw2[L / 2], gain(iN, L / 2), gain(iN, L / 2));
            Ra[hh] = zk;
          } else {
            const int i0 = pad_e<LOGE>(k2), i1 = pad_e<LOGE>(L - k2);
            Cx<T> zk = Ra[i0], zm = Ra[i1];
            pair_op(zk, zm, a.tw2[k2], gain(iN, k2), gain(iN, L - k2));
            Ra[i0] = zk;
            Ra[i1] = zm;
          }
        } else {
          const int k2 = t - L / 2;
          const int i0 = pad_e<LOGE>(k2), i1 = pad_e<LOGE>(L - 1 - k2);
          Cx<T> zk = Rb[i0], zm = Rb[i1];
          pair_op(zk, zm, wh * a.tw2[k2], gain(ih, k2), gain(ih, L - 1 - k2));
          Rb[i0] = zk;
          Rb[i1] = zm;
        }
      }
    }
  }
  __syncthreads();
  if constexpr (MODE == 1) {   // store the unpacked spectrum of this wave's row
    for (int i = lane; i < L; i += 64) Sto<T, S>::st(w + i, R[pad_e<LOGE>(i)]);
    return;
  }
  // ---------------- inverse: radix-E from LDS, then 2 x radix-8, store
  {
    Cx<T> v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = R[pad_e<LOGE>(lane + 64 * r)];
    __syncthreads();
    dft_regs<T, E, true>(v, twE);
#pragma unroll
    for (int r = 0; r < E; ++r) R[pad_e<LOGE>(lane * E + r)] = v[r];
  }
  __syncthreads();
  radix8(LOGE, true, true);
  radix8(LOGE + 3, true, false);
}

// Inter-detector correlated N^-1, first half: on the unpacked spectra of the
// one group that holds every detector (slot s = k1*M2 + k2 holds X_d[k] for
// k = k1 + M1*k2; slot 0 holds X_d[0] and X_d[M] as re and im), the low-rank
// projections t_j[s] = sum_d V_b[d][j] X_d[s] with b = bin[s] (slot 0: bins of
// k = 0 and k = M for the two real parts).  The second half,
// Y_d = (1/M) (iN_d X_d - sum_j V_b[d][j] t_j), is fused into the repack of
// pass 2 (MODE 2).  One thread per slot, detectors unrolled four deep.
template <typename T, typename S, int RMAX, int SPT>
__global__ void __launch_bounds__(256) k_corr_t(PassArgs<T, S> a, CorrArgs c) {
  // SPT consecutive slots per thread, so a wavefront reads 64 * SPT
  // contiguous entries of each detector's spectrum
  const int M = 1 << a.logM;
  const int s0 = (blockIdx.x * blockDim.x + threadIdx.x) * SPT;
  if (s0 >= M) return;
  int b[SPT];
#pragma unroll
  for (int q = 0; q < SPT; ++q) b[q] = c.bin[s0 + q];
  const int bN = c.bin[M];   // slot 0's imaginary part is the Nyquist bin
  T tr[SPT][RMAX], ti[SPT][RMAX];
#pragma unroll
  for (int q = 0; q < SPT; ++q)
#pragma unroll
    for (int j = 0; j < RMAX; ++j) tr[q][j] = ti[q][j] = T(0);
  const auto* w = a.work + s0;
  for (int d = 0; d < c.ndet; ++d) {
    Cx<T> x[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) x[q] = Sto<T, S>::ld(w + (int64_t(d) << a.logM) + q);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const float* vr = c.V + (int64_t(b[q]) * c.ndet + d) * c.rank;
      const float* vi = (s0 + q == 0) ? c.V + (int64_t(bN) * c.ndet + d) * c.rank : vr;
#pragma unroll
      for (int j = 0; j < RMAX; ++j)
        if (j < c.rank) {
          tr[q][j] += T(vr[j]) * x[q].x;
          ti[q][j] += T(vi[j]) * x[q].y;
        }
    }
  }
  Cx<T>* t = static_cast<Cx<T>*>(c.t);
#pragma unroll
  for (int q = 0; q < SPT; ++q)
#pragma unroll
    for (int j = 0; j < RMAX; ++j)
      if (j < c.rank) t[(int64_t(j) << a.logM) + s0 + q] = cx(tr[q][j], ti[q][j]);
}

template <typename T, typename S>
static void launch_corr_t(int M, hipStream_t st, const PassArgs<T, S>& a, const CorrArgs& c) {
  constexpr int SPT = sizeof(T) == 8 ? 2 : 1;   // measured best at 256 detectors
  const dim3 g((M / SPT + 255) / 256), b(256);
  if (c.rank <= 4)
    hipLaunchKernelGGL((k_corr_t<T, S, 4, SPT>), g, b, 0, st, a, c);
  else if (c.rank <= 8)
    hipLaunchKernelGGL((k_corr_t<T, S, 8, SPT>), g, b, 0, st, a, c);
  else
    hipLaunchKernelGGL((k_corr_t<T, S, kMaxCorrRank, 1>), dim3((M + 255) / 256), b, 0, st, a, c);
}

// CSR = true: store the filtered, packed timestream back in place (the block
// owns exactly the addresses it loaded); the per-pixel reduce applies P^T.
template <typename T, typename S, int NC, bool CSR, int E13, bool MIX>
__global__ void __launch_bounds__(kNT13) k_pass3(PassArgs<T, S> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* buf = reinterpret_cast<Cx<T>*>(smem);
  T* bufr = reinterpret_cast<T*>(smem);
  const int logNB = a.logM2 - a.logC;
  int g, cb;
  col_block(logNB, &g, &cb);
  const int C = 1 << a.logC;
  const int M1 = a.M1i, M2 = 1 << a.logM2;
  Cx<T>* stw = buf + C * M1;
  const int j20 = cb << a.logC;
  if constexpr (MIX)
    for (int m = threadIdx.x; m < M1; m += kNT13) stw[m] = a.twm[m];
  else
    stage_twiddles<T, kNT13>(stw, a.tw, a.logM1, a.logLmax);
  const auto* w = a.work + int64_t(g) * a.Mi;
  // all of a thread's (at most E13) loads in flight before the LDS writes
  const int ntile = C * M1;
#if MM_P3_BATCH
  for (int e0 = threadIdx.x; e0 < ntile; e0 += E13 * kNT13) {
    Cx<T> v[E13];
#pragma unroll
    for (int i = 0; i < E13; ++i) {
      const int e = e0 + i * kNT13;
      if (e < ntile) v[i] = Sto<T, S>::ld(w + int64_t(e >> a.logC) * M2 + j20 + (e & (C - 1)));
    }
#pragma unroll
    for (int i = 0; i < E13; ++i) {
      const int e = e0 + i * kNT13;
      if (e < ntile) buf[e] = v[i];
    }
  }
#else
  for (int e = threadIdx.x; e < ntile; e += kNT13) {
    const int k1 = e >> a.logC;
    const int c = e & (C - 1);
    buf[e] = Sto<T, S>::ld(w + int64_t(k1) * M2 + j20 + c);
  }
#endif
  __syncthreads();
  FftShape sh{a.logM1, a.logC, C, 1, true, a.logM1};
  if constexpr (MIX)
    lds_fft_mx<T, kNT13, E13, true>(buf, MixShape{M1, C, C, 1, true, a.mix_code, 1}, stw);
  else
    lds_fft<T, kNT13, E13, true>(buf, sh, stw);
  if constexpr (CSR) {
    auto* wo = a.work + int64_t(g) * a.Mi;
    for (int e = threadIdx.x; e < C * M1; e += kNT13) {
      const int k1 = e >> a.logC;
      const int c = e & (C - 1);
      Sto<T, S>::st(wo + int64_t(k1) * M2 + j20 + c, buf[e]);
    }
    return;
  }
  const int64_t base = int64_t(g) * a.n;
  const int nsamp = 2 * C * M1;
  for (int e = threadIdx.x; e < nsamp; e += kNT13) {
    const int j1 = e >> (a.logC + 1);
    const int q = e & (2 * C - 1);
    const int64_t s = base + 2 * (int64_t(j1) * M2 + j20) + q;
    scatter_sample<T, NC>(a, s, bufr[e]);
  }
}

// P^T for one detector group as a per-pixel gather: 16 lanes per pixel walk
// its CSR entries, each lane summing a fixed stride of them, then a fixed
// xor-tree; acc[p] += (sum u, sum c u, sum s u).  No atomics.
// Weights of gather entry ik (group-relative sample d_local * n + t).
// WM 0: stored with the index as float32 (cos 2psi, sin 2psi); WM 1: from the
// boresight model; WM 2: stored as the angle u = 2psi * 2^32 / 2pi (mod 2^32)
// when every sample's weights have unit norm, which halves the bytes: with
// k = u >> 24 and d = (u mod 2^24) 2pi / 2^32 < 2pi/256, (cos, sin)(2psi) is
// the table entry k turned by d, whose cos and sin are Taylor polynomials to
// d^4 and d^5 (truncation below 1e-12); a few float32 roundings in all.
__device__ __forceinline__ void angle_weights(uint32_t u, const float2* tab, double* c,
                                              double* sn) {
  float cf, sf;
  angle_cs(u, tab, &cf, &sf);
  *c = double(cf);
  *sn = double(sf);
}

template <typename T, typename S, int NC, int WM>
__device__ __forceinline__ void entry_weights(const PassArgs<T, S>& a, const float2* tab, int k,
                                              int ik, double* c, double* sn) {
  if constexpr (WM == 1) {
    const int d = a.det0 + (ik >> a.bo.logn);
    bore_weights_at(a.bo, d, ik & ((1 << a.bo.logn) - 1), c, sn);
  } else {
    const float2 cs = a.csr_w[k];
    *c = double(cs.x);
    *sn = double(cs.y);
  }
}

#ifndef MM_LPP
#define MM_LPP 16
#endif
#ifndef MM_RUNROLL
#define MM_RUNROLL 4
#endif
constexpr int kReduceLanes = MM_LPP;   // lanes per pixel in the gather

template <typename T, typename S, int NC, bool CF, int WM>
__global__ void __launch_bounds__(256) k_csr_reduce(PassArgs<T, S> a) {
  constexpr int LPP = kReduceLanes;
  const int sub = threadIdx.x / LPP;
  const int l = threadIdx.x % LPP;
  __shared__ float2 tab[WM == 2 ? 256 : 1];
  if constexpr (WM == 2) {
    tab[threadIdx.x] = a.ang_tab[threadIdx.x];   // blockDim.x == 256
    __syncthreads();
  }
  // chunks of 256/LPP pixels: each XCD (blocks i mod 8) takes a contiguous eighth of
  // them, so a line of the pass buffer shared by neighbouring pixels is
  // fetched into one L2 (266 -> 256 us per 64-detector launch)
  int chunk = blockIdx.x;
  if (MM_RED_XCD && (gridDim.x & 7) == 0)
    chunk = (blockIdx.x & 7) * int(gridDim.x >> 3) + (blockIdx.x >> 3);
  const int p = chunk * (256 / LPP) + sub;
  if (p >= a.npix) return;            // whole 16-lane groups leave together
  if (!a.mask[p]) {
    if (a.y_out && l == 0)
      for (int c = 0; c < NC; ++c) a.y_out[int64_t(c) * a.npix + p] = 0.0;
    return;
  }
  // the pass buffer read as packed reals: sample 2j is Re z[j], 2j+1 is Im z[j]
  const auto* u = reinterpret_cast<const typename Sto<T, S>::R*>(a.work);
  const int b = a.csr_off[p], e = a.csr_off[p + 1];
  if constexpr (!CF) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll MM_RUNROLL
    for (int k = b + l; k < e; k += LPP) {
      int ik;
      uint32_t ua = 0;
      if constexpr (WM == 2) {   // index and angle in one 8-byte load
        const int2 r = a.csr_ia[k];
        ik = r.x;
        ua = uint32_t(r.y);
      } else {
        ik = a.csr_idx[k];
      }
      const double uu = double(Sto<T, S>::ldr(u + ik));
      s0 += uu;
      if constexpr (NC == 3) {
        double c, sn;
        if constexpr (WM == 2)
          angle_weights(ua, tab, &c, &sn);
        else
          entry_weights<T, S, NC, WM>(a, tab, k, ik, &c, &sn);
        s1 += c * uu;
        s2 += sn * uu;
      }
    }
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, LPP);
      if constexpr (NC == 3) {
        s1 += __shfl_xor(s1, off, LPP);
        s2 += __shfl_xor(s2, off, LPP);
      }
    }
    if (l == 0) {
      double* d = a.acc + 4 * int64_t(p);
      if (a.y_out) {
        a.y_out[p] = d[0] + s0;
        if constexpr (NC == 3) {
          a.y_out[a.npix + int64_t(p)] = d[1] + s1;
          a.y_out[2 * int64_t(a.npix) + p] = d[2] + s2;
        }
      } else {
        d[0] += s0;
        if constexpr (NC == 3) {
          d[1] += s1;
          d[2] += s2;
        }
      }
    }
  } else {
    // compensated float32: products exact as (p, fma error), sums error-free
    F2 s0{0.f, 0.f}, s1{0.f, 0.f}, s2{0.f, 0.f};
#pragma unroll 4
    for (int k = b + l; k < e; k += LPP) {
      int ik;
      uint32_t ua = 0;
      if constexpr (WM == 2) {
        const int2 r = a.csr_ia[k];
        ik = r.x;
        ua = uint32_t(r.y);
      } else {
        ik = a.csr_idx[k];
      }
      const T ut = Sto<T, S>::ldr(u + ik);
      F2 uu;
      if constexpr (sizeof(T) == 8)
        uu = f2_split(ut);
      else
        uu = F2{float(ut), 0.f};
      f2_acc(s0, uu.hi, uu.lo);
      if constexpr (NC == 3) {
        double c, sn;
        if constexpr (WM == 2)
          angle_weights(ua, tab, &c, &sn);
        else
          entry_weights<T, S, NC, WM>(a, tab, k, ik, &c, &sn);
        f2_fma_acc(s1, float(c), uu);
        f2_fma_acc(s2, float(sn), uu);
      }
    }
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
      s0 = f2_add(s0, f2_shfl_xor(s0, off, LPP));
      if constexpr (NC == 3) {
        s1 = f2_add(s1, f2_shfl_xor(s1, off, LPP));
        s2 = f2_add(s2, f2_shfl_xor(s2, off, LPP));
      }
    }
    if (l == 0) {
      F2* d = reinterpret_cast<F2*>(a.acc + 4 * int64_t(p));
      d[0] = f2_add(d[0], s0);
      if constexpr (NC == 3) {
        d[1] = f2_add(d[1], s1);
        d[2] = f2_add(d[2], s2);
      }
    }
  }
}

// P^T through the run-length index: 16 lanes per pixel, each lane summing
// whole runs (runs l, l + 16, ... of the pixel), a run's timestream values
// and pixel-major angles read four samples at a time with one vector load
// each (a run is consecutive samples, and the angles are stored in the same
// order), so a run of up to four samples costs one timestream load and one
// angle load instead of one per sample.  The angles' pixel-major offset of a
// run comes from a prefix sum of the run lengths over the 16 lanes.  Then the
// same xor-tree and accumulator update as the per-sample gather.  Weights
// other than angles come from the time-major storage sample by sample (WM 0:
// the caller's float32 cos 2psi, sin 2psi; WM 1: the boresight model).
template <typename T, typename S, int NC, int WM>
__device__ __forceinline__ void sample_w(const PassArgs<T, S>& a, const float2* tab, int ik,
                                         double* c, double* sn) {
  if constexpr (WM == 2) {
    angle_weights(a.ang_t[ik], tab, c, sn);
  } else if constexpr (WM == 1) {
    bore_weights_at(a.bo, a.det0 + (ik >> a.bo.logn), ik & ((1 << a.bo.logn) - 1), c, sn);
  } else {
    *c = double(a.c2[ik]);
    *sn = double(a.s2[ik]);
  }
}

template <typename T, typename S, int NC, bool CF, int WM>
__global__ void __launch_bounds__(256) k_rle_reduce(PassArgs<T, S> a) {
  constexpr int LPP = kReduceLanes;
  constexpr int U = 4;   // samples per lane whose loads are issued together
  const int sub = threadIdx.x / LPP;
  const int l = threadIdx.x % LPP;
  __shared__ float2 tab[WM == 2 ? 256 : 1];
  if constexpr (WM == 2) {
    tab[threadIdx.x] = a.ang_tab[threadIdx.x];   // blockDim.x == 256
    __syncthreads();
  }
  int chunk = blockIdx.x;
  if (MM_RED_XCD && (gridDim.x & 7) == 0)
    chunk = (blockIdx.x & 7) * int(gridDim.x >> 3) + (blockIdx.x >> 3);
  const int p = chunk * (256 / LPP) + sub;
  if (p >= a.npix) return;            // whole 16-lane groups leave together
  if (!a.mask[p]) {
    if (a.y_out && l == 0)
      for (int c = 0; c < NC; ++c) a.y_out[int64_t(c) * a.npix + p] = 0.0;
    return;
  }
  const auto* u = reinterpret_cast<const typename Sto<T, S>::R*>(a.work);
  const int b = a.csr_off[p], e = a.csr_off[p + 1];
  // WM 2 with pixel-major angles: the pixel's samples in gather order
  const uint32_t* pa = nullptr;
  if constexpr (WM == 2) pa = a.rle_ang ? a.rle_ang + a.rle_soff[p] : nullptr;
  using Acc = typename std::conditional<CF, F2, double>::type;
  Acc s0{}, s1{}, s2{};
  auto add = [&](T ut, double c, double sn) {
    if constexpr (CF) {
      F2 uu;
      if constexpr (sizeof(T) == 8)
        uu = f2_split(ut);
      else
        uu = F2{float(ut), 0.f};
      f2_acc(s0, uu.hi, uu.lo);
      if constexpr (NC == 3) {
        f2_fma_acc(s1, float(c), uu);
        f2_fma_acc(s2, float(sn), uu);
      }
    } else {
      const double uu = double(ut);
      s0 += uu;
      if constexpr (NC == 3) {
        s1 += c * uu;
        s2 += sn * uu;
      }
    }
  };
  static_assert(LPP == 16, "the run scan works on DPP rows of 16 lanes");
  using R = typename Sto<T, S>::R;
  uint32_t hnext = b + l < e ? a.rle[b + l] : 0u;
  for (int kb = b; kb < e; kb += LPP) {
    // this lane's run of the batch (lanes past the pixel's end: empty), and
    // the next batch's entry loaded meanwhile
    const uint32_t h = hnext;
    hnext = kb + LPP + l < e ? a.rle[kb + LPP + l] : 0u;
    const int first = int(h >> 4), len = int(h & 15u);
    // offset of the run's first angle: prefix sum over the 16 lanes of a DPP
    // row (lanes shifted in from outside the row read 0)
    int incl = len;
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x111, 0xf, 0xf, true);   // row_shr:1
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x112, 0xf, 0xf, true);   // row_shr:2
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xf, true);   // row_shr:4
    incl += __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xf, true);   // row_shr:8
    const int excl = incl - len;
    const int total = __shfl(incl, LPP - 1, LPP);
    // runs are at most four samples (U): one pass, all lanes in step
    for (int j0 = 0; j0 < len; j0 += U) {
      // four samples from the run's j0-th on, loaded whole (the buffers have
      // 64 B of padding past their end, so reading beyond a run's last sample
      // stays inside); the samples past the run's end are replaced by zeros,
      // which leave the sums unchanged
      struct { R r[U]; } v;
      __builtin_memcpy(&v, u + first + j0, sizeof(v));
      uint32_t ua[U] = {};
      if constexpr (NC == 3 && WM == 2) {
        if (pa) {
          uint4 w4;
          __builtin_memcpy(&w4, pa + excl + j0, sizeof(w4));
          ua[0] = w4.x;
          ua[1] = w4.y;
          ua[2] = w4.z;
          ua[3] = w4.w;
        } else {
#pragma unroll
          for (int jj = 0; jj < U; ++jj) ua[jj] = a.ang_t[first + j0 + (j0 + jj < len ? jj : 0)];
        }
      }
#pragma unroll
      for (int jj = 0; jj < U; ++jj) {
        const bool on = j0 + jj < len;
        double c = 0.0, sn = 0.0;
        if constexpr (NC == 3) {
          if constexpr (WM == 2)
            angle_weights(ua[jj], tab, &c, &sn);
          else
            sample_w<T, S, NC, WM>(a, tab, first + j0 + (on ? jj : 0), &c, &sn);
        }
        const T x = Sto<T, S>::up_r(v.r[jj]);
        add(on ? x : T(0), c, sn);
      }
    }
    if (pa) pa += total;
  }
  if constexpr (!CF) {
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off, LPP);
      if constexpr (NC == 3) {
        s1 += __shfl_xor(s1, off, LPP);
        s2 += __shfl_xor(s2, off, LPP);
      }
    }
    if (l == 0) {
      double* d = a.acc + 4 * int64_t(p);
      if (a.y_out) {
        a.y_out[p] = d[0] + s0;
        if constexpr (NC == 3) {
          a.y_out[a.npix + int64_t(p)] = d[1] + s1;
          a.y_out[2 * int64_t(a.npix) + p] = d[2] + s2;
        }
      } else {
        d[0] += s0;
        if constexpr (NC == 3) {
          d[1] += s1;
          d[2] += s2;
        }
      }
    }
  } else {
#pragma unroll
    for (int off = LPP / 2; off > 0; off >>= 1) {
      s0 = f2_add(s0, f2_shfl_xor(s0, off, LPP));
      if constexpr (NC == 3) {
        s1 = f2_add(s1, f2_shfl_xor(s1, off, LPP));
        s2 = f2_add(s2, f2_shfl_xor(s2, off, LPP));
      }
    }
    if (l == 0) {
      F2* d = reinterpret_cast<F2*>(a.acc + 4 * int64_t(p));
      d[0] = f2_add(d[0], s0);
      if constexpr (NC == 3) {
        d[1] = f2_add(d[1], s1);
        d[2] = f2_add(d[2], s2);
      }
    }
  }
}

// ------------------------------------------------------------- host side
static int ilog2(int64_t v) {
  int l = 0;
  while ((int64_t(1) << l) < v) ++l;
  return l;
}

template <typename K>
static void raise_lds_limit(K kernel, size_t bytes) {
  if (bytes > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

// pass 2 with one wavefront per row (one row pair per block) in a given mode
template <typename T, typename S, int MODE>
static void launch_pass2w(int M2, dim3 g, size_t lds, hipStream_t st, const PassArgs<T, S>& a,
                          const CorrArgs& c) {
  const dim3 b(128);
  if (M2 == 512) {
    raise_lds_limit(k_pass2w<T, S, 8, 1, MODE>, lds);
    hipLaunchKernelGGL((k_pass2w<T, S, 8, 1, MODE>), g, b, lds, st, a, c);
  } else if (M2 == 1024) {
    raise_lds_limit(k_pass2w<T, S, 16, 1, MODE>, lds);
    hipLaunchKernelGGL((k_pass2w<T, S, 16, 1, MODE>), g, b, lds, st, a, c);
  } else {
    raise_lds_limit(k_pass2w<T, S, 32, 1, MODE>, lds);
    hipLaunchKernelGGL((k_pass2w<T, S, 32, 1, MODE>), g, b, lds, st, a, c);
  }
}

template <typename T, typename S, int NC>
static void launch_reduce(ScanImpl* s, const PassArgs<T, S>& a, hipStream_t st) {
  constexpr int PPB = 256 / kReduceLanes;   // pixels per 256-thread block
  const dim3 grid((s->npix + PPB - 1) / PPB);
  // weights: 1 from the boresight model, 2 as stored angles, 0 as stored floats
  // (the run-length gather with boresight pointing has no stored floats)
  const int wm = NC != 3                                           ? 0
                 : !s->plan.csr_w                                   ? 1
                 : s->csr_ang                                       ? 2
                 : (s->plan.rle && s->plan.otf)                     ? 1
                                                                    : 0;
  auto go = [&](auto cf, auto w) {
    constexpr bool CF_ = decltype(cf)::value;
    constexpr int WM_ = decltype(w)::value;
    if (s->plan.rle)
      hipLaunchKernelGGL((k_rle_reduce<T, S, NC, CF_, WM_>), grid, dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL((k_csr_reduce<T, S, NC, CF_, WM_>), grid, dim3(256), 0, st, a);
  };
  using W0 = std::integral_constant<int, 0>;
  using W1 = std::integral_constant<int, 1>;
  using W2 = std::integral_constant<int, 2>;
  auto by_w = [&](auto cf) {
    if (wm == 1)
      go(cf, W1{});
    else if (wm == 2)
      go(cf, W2{});
    else
      go(cf, W0{});
  };
  if (s->plan.acc32)
    by_w(std::true_type{});
  else
    by_w(std::false_type{});
}

template <typename T, typename S, int NC, int SRC>
static mm_status run_pipeline_t(ScanImpl* s, const void* tod, hipStream_t st) {
  using A = PassArgs<T, S>;
  const Plan& pl = s->plan;
  const int M = int(s->n / 2);
  A a;
  a.y_out = nullptr;
  a.Mi = M;
  a.M1i = pl.M1;
  a.mix_code = pl.mix_code;
  a.twm = pl.mix_code && !pl.single ? s->at<Cx<T>>(s->lay.tw_m1) : nullptr;
  a.gmap = s->at<V4<T>>(s->lay.gmap);
  a.acc = s->at<double>(s->lay.acc);
  a.work = s->at<typename A::W>(s->lay.tod);
  a.tw = s->at<Cx<T>>(s->lay.tw);
  a.wn.hi = s->at<Cx<T>>(s->lay.wn_hi);
  a.wn.lo = s->at<Cx<T>>(s->lay.wn_lo);
  a.wn.logS = pl.logS;
  a.n = s->n;
  a.npix = s->npix;
  a.logM = pl.logM;
  a.logM1 = pl.logM1;
  a.logM2 = pl.logM2;
  a.logC = pl.logC;
  a.logLmax = pl.logLmax;
  a.scale = T(1) / T(M);
  a.mask = s->at<int32_t>(s->lay.mask);
  a.tw2 = s->at<Cx<T>>(s->lay.tw2);
  a.bo = scan_bore(s);
  a.ang_tab = s->at<float2>(s->lay.ang_tab);
  if (s->bore_fast) {
    a.bore_f = s->at<float4>(s->lay.bore_f);
    a.bore_a = s->at<uint32_t>(s->lay.bore_a);
    a.det_f = s->at<float2>(s->lay.det_f);
    a.det_a = s->at<uint32_t>(s->lay.det_a);
  }
  const int G = pl.G;
  for (int d0 = 0; d0 < s->ndet; d0 += G) {
    const int gd = (s->ndet - d0 < G) ? (s->ndet - d0) : G;
    const int64_t off = int64_t(d0) * s->n;
    a.det0 = d0;
    a.ang_t = s->ang_t_ready ? s->at<uint32_t>(s->lay.ang_t) + off : nullptr;
    a.ptc = s->ptc_ready ? s->at<uint32_t>(s->lay.ptc) + off : nullptr;
    a.ptc_h = s->ptc_ready ? s->at<int4>(s->lay.ptc_h) + off / kPtcChunk : nullptr;
    a.pix = s->d.pix ? s->d.pix + off : nullptr;
    a.c2 = s->d.cos2psi ? s->d.cos2psi + off : nullptr;
    a.s2 = s->d.sin2psi ? s->d.sin2psi + off : nullptr;
    a.iN = s->d.inv_noise + int64_t(d0) * (M + 1);
    a.iNt = pl.single ? nullptr : s->at<float>(s->lay.int_) + int64_t(d0) * (M + 1);
    a.tod = tod ? static_cast<const typename A::R*>(tod) + off : nullptr;
    if (pl.csr) {
      const int gi = d0 / G;
      a.csr_off = s->at<int32_t>(s->lay.csr_off) + int64_t(gi) * (s->npix + 1);
      a.csr_idx = s->at<int32_t>(s->lay.csr_idx) + int64_t(gi) * G * s->n;
      a.csr_w = pl.csr_w && !s->csr_ang && !pl.rle
                    ? s->at<float2>(s->lay.csr_w) + int64_t(gi) * G * s->n
                    : nullptr;
      // stored angles live in the first half of the weights' region
      a.csr_ia = s->csr_ang && !pl.rle ? s->at<int2>(s->lay.csr_w) + int64_t(gi) * G * s->n
                                       : nullptr;
      a.rle = pl.rle ? s->at<uint32_t>(s->lay.csr_idx) + int64_t(gi) * G * s->n : nullptr;
      a.rle_ang = s->rle_pa ? s->at<uint32_t>(s->lay.csr_w) + int64_t(gi) * G * s->n : nullptr;
      a.rle_soff = s->rle_pa ? s->at<int32_t>(s->lay.csr_soff) + int64_t(gi) * (s->npix + 1)
                             : nullptr;
      // the last group's gather writes the result itself (float64 sums only)
      a.y_out = (d0 + G >= s->ndet && !pl.acc32) ? s->fuse_y : nullptr;
      if (a.y_out) s->fused_y = true;
    }
    const int64_t gs = int64_t(gd) * s->n;
    hipEvent_t tok;
    if (pl.single) {
      const size_t lds = size_t(M) * sizeof(Cx<T>);
      prof_begin(s, st, &tok, kProfSingle);
      auto single = [&](auto csr, auto mix) {
        constexpr bool C_ = decltype(csr)::value, X_ = decltype(mix)::value;
        raise_lds_limit(k_single<T, S, NC, SRC, C_, X_>, lds);
        hipLaunchKernelGGL((k_single<T, S, NC, SRC, C_, X_>), dim3(gd), dim3(kNT), lds, st, a);
      };
      using TT = std::true_type;
      using FF = std::false_type;
      if constexpr (SRC == 2 || SRC == 4) {   // boresight pointing: gather, powers of two
        single(TT{}, FF{});
      } else {
        if (pl.csr)
          pl.mix_code ? single(TT{}, TT{}) : single(TT{}, FF{});
        else
          pl.mix_code ? single(FF{}, TT{}) : single(FF{}, FF{});
      }
      prof_end(s, st, tok, kProfSingle, gs);
      if (pl.csr) {
        prof_begin(s, st, &tok, kProfReduce);
        launch_reduce<T, S, NC>(s, a, st);
        prof_end(s, st, tok, kProfReduce, gs);
      }
    } else {
      const int C = 1 << pl.logC;
      const int M1 = pl.M1, M2 = 1 << pl.logM2;
      const size_t lds13 = (size_t(C) * M1 + M1) * sizeof(Cx<T>);
      const int JL = M2 < 64 ? M2 : 64;
      const size_t lds2 =
          (size_t(2) * M2 + (size_t(2) * M2 >> kPad2) + M2 + 2 * (M2 / JL) + 2 * JL) * sizeof(Cx<T>);
      const bool e16 = size_t(C) * M1 > size_t(8) * kNT13;   // 16 elements per thread
      prof_begin(s, st, &tok, kProfPass1);
      using TT = std::true_type;
      using FF = std::false_type;
      auto pass1 = [&](auto e, auto mix) {
        constexpr int E_ = decltype(e)::value;
        constexpr bool X_ = decltype(mix)::value;
        raise_lds_limit(k_pass1<T, S, NC, SRC, E_, X_>, lds13);
        hipLaunchKernelGGL((k_pass1<T, S, NC, SRC, E_, X_>), dim3(gd * (M2 / C)), dim3(kNT13),
                           lds13, st, a);
      };
      using E8 = std::integral_constant<int, 8>;
      using E16 = std::integral_constant<int, 16>;
      const bool mix1 = pl.mix_code != 0;
      if constexpr (sizeof(T) == 4) {
        if (e16) {
          if constexpr (SRC == 2 || SRC == 4)
            pass1(E16{}, FF{});
          else
            mix1 ? pass1(E16{}, TT{}) : pass1(E16{}, FF{});
        }
      }
      if (!e16) {
        if constexpr (SRC == 2 || SRC == 4)
          pass1(E8{}, FF{});
        else
          mix1 ? pass1(E8{}, TT{}) : pass1(E8{}, FF{});
      }
      prof_end(s, st, tok, kProfPass1, gs);
      prof_begin(s, st, &tok, kProfPass2);
      const dim3 g2(gd * (M1 / 2));
      // one row pair per block: two waves
      constexpr int PB = 1;
      const size_t lds2w =
          size_t(2 * PB) * (M2 + (M2 >> kP2PadLog) + M2 / 64) * sizeof(Cx<T>);
      const bool wave_rows = MM_PASS2W && lds2w <= 80 * 1024 && ((int64_t(gd) * M1 / 2) % PB) == 0;
      const dim3 g2w(unsigned(int64_t(gd) * M1 / 2 / PB)), b2w(128 * PB);
      if (pl.corr_rank > 0) {
        // correlated noise: unpack every detector's spectrum, mix across
        // detectors, repack and invert (the plan keeps M2 in 512..2048)
        if (!wave_rows || M2 < 512 || M2 > 2048)
          return fail(MM_EINVAL, "correlated noise: unsupported pass-2 row length");
        CorrArgs c;
        c.V = s->d.corr_V;
        c.bin = s->at<int16_t>(s->lay.corr_bin);
        c.t = s->at<void>(s->lay.corr_t);
        c.rank = pl.corr_rank;
        c.ndet = gd;
        launch_pass2w<T, S, 1>(M2, g2w, lds2w, st, a, c);
        prof_end(s, st, tok, kProfPass2, gs);
        prof_begin(s, st, &tok, kProfCorr);
        launch_corr_t<T, S>(M, st, a, c);
        prof_end(s, st, tok, kProfCorr, gs);
        prof_begin(s, st, &tok, kProfPass2);
        launch_pass2w<T, S, 2>(M2, g2w, lds2w, st, a, c);
      } else if (wave_rows && M2 == 512) {
        raise_lds_limit(k_pass2w<T, S, 8, PB, 0>, lds2w);
        hipLaunchKernelGGL((k_pass2w<T, S, 8, PB, 0>), g2w, b2w, lds2w, st, a, CorrArgs{});
      } else if (wave_rows && M2 == 1024) {
        raise_lds_limit(k_pass2w<T, S, 16, PB, 0>, lds2w);
        hipLaunchKernelGGL((k_pass2w<T, S, 16, PB, 0>), g2w, b2w, lds2w, st, a, CorrArgs{});
      } else if (wave_rows && M2 == 2048) {
        raise_lds_limit(k_pass2w<T, S, 32, PB, 0>, lds2w);
        hipLaunchKernelGGL((k_pass2w<T, S, 32, PB, 0>), g2w, b2w, lds2w, st, a, CorrArgs{});
      } else if (M2 <= 1024) {
        raise_lds_limit(k_pass2<T, S, 8>, lds2);
        hipLaunchKernelGGL((k_pass2<T, S, 8>), g2, dim3(kNT), lds2, st, a);
      } else if (M2 <= 2048) {
        raise_lds_limit(k_pass2<T, S, 16>, lds2);
        hipLaunchKernelGGL((k_pass2<T, S, 16>), g2, dim3(kNT), lds2, st, a);
      } else {
        raise_lds_limit(k_pass2<T, S, 32>, lds2);
        hipLaunchKernelGGL((k_pass2<T, S, 32>), g2, dim3(kNT), lds2, st, a);
      }
      prof_end(s, st, tok, kProfPass2, gs);
      prof_begin(s, st, &tok, kProfPass3);
      const dim3 g13(gd * (M2 / C));
      auto pass3 = [&](auto csr, auto e, auto mix) {
        constexpr bool C_ = decltype(csr)::value, X_ = decltype(mix)::value;
        constexpr int E_ = decltype(e)::value;
        raise_lds_limit(k_pass3<T, S, NC, C_, E_, X_>, lds13);
        hipLaunchKernelGGL((k_pass3<T, S, NC, C_, E_, X_>), g13, dim3(kNT13), lds13, st, a);
      };
      auto pass3e = [&](auto e) {
        if (pl.csr)
          mix1 ? pass3(TT{}, e, TT{}) : pass3(TT{}, e, FF{});
        else
          mix1 ? pass3(FF{}, e, TT{}) : pass3(FF{}, e, FF{});
      };
      if constexpr (sizeof(T) == 4) {
        if (e16) pass3e(E16{});
      }
      if (!e16) pass3e(E8{});
      prof_end(s, st, tok, kProfPass3, gs);
      if (pl.csr) {
        prof_begin(s, st, &tok, kProfReduce);
        launch_reduce<T, S, NC>(s, a, st);
        prof_end(s, st, tok, kProfReduce, gs);
      }
    }
  }
  MM_HIP(hipGetLastError());
  return MM_OK;
}

// src 0: the map through stored pointing (SRC 0) or the boresight model
// (SRC 2); src 1: a timestream (SRC 1)
template <typename T, typename S>
static mm_status run_pipeline(ScanImpl* s, int src, const void* tod, hipStream_t st) {
  const bool otf = s->plan.otf;
  if (s->nc == 3)
    return src               ? run_pipeline_t<T, S, 3, 1>(s, tod, st)
           : otf             ? (s->bore_fast ? run_pipeline_t<T, S, 3, 4>(s, tod, st)
                                             : run_pipeline_t<T, S, 3, 2>(s, tod, st))
           : s->ptc_ready    ? run_pipeline_t<T, S, 3, 5>(s, tod, st)
           : s->ang_t_ready  ? run_pipeline_t<T, S, 3, 3>(s, tod, st)
                             : run_pipeline_t<T, S, 3, 0>(s, tod, st);
  return src   ? run_pipeline_t<T, S, 1, 1>(s, tod, st)
         : otf ? (s->bore_fast ? run_pipeline_t<T, S, 1, 4>(s, tod, st)
                               : run_pipeline_t<T, S, 1, 2>(s, tod, st))
               : run_pipeline_t<T, S, 1, 0>(s, tod, st);
}

mm_status filter_pipeline(ScanImpl* s, int src, const void* tod, const double* x, double* y,
                          hipStream_t st) {
  const int npix = s->npix;
  const dim3 blk(256), grd((npix + 255) / 256);
  const int32_t* mask = s->at<int32_t>(s->lay.mask);
  double* acc = s->at<double>(s->lay.acc);
  hipEvent_t tok;
  prof_begin(s, st, &tok, kProfApplyA);
  if (src == 0) {
    const dim3 grd1((npix + 1 + 255) / 256);   // npix + 1: the zero entry too
    if (s->plan.f64)
      hipLaunchKernelGGL(k_prologue<double>, grd1, blk, 0, st, x, mask,
                         s->at<V4<double>>(s->lay.gmap), acc, npix, s->nc);
    else
      hipLaunchKernelGGL(k_prologue<float>, grd1, blk, 0, st, x, mask,
                         s->at<V4<float>>(s->lay.gmap), acc, npix, s->nc);
  } else {
    hipLaunchKernelGGL(k_zero_acc, grd, blk, 0, st, acc, npix);
  }
  MM_HIP(hipGetLastError());
  s->fuse_y = y;
  s->fused_y = false;
  mm_status r = s->plan.f64    ? run_pipeline<double, double>(s, src, tod, st)
                : s->plan.bf16 ? run_pipeline<float, Bf16>(s, src, tod, st)
                               : run_pipeline<float, float>(s, src, tod, st);
  s->fuse_y = nullptr;
  if (r != MM_OK) return r;
  if (!s->fused_y)   // otherwise the last group's gather wrote y
    hipLaunchKernelGGL(k_epilogue, grd, blk, 0, st, acc, mask, y, npix, s->nc,
                       s->plan.acc32 ? 1 : 0);
  MM_HIP(hipGetLastError());
  prof_end(s, st, tok, kProfApplyA, int64_t(s->ndet) * s->n);
  return MM_OK;
}

// 1/N(f) of every detector in four-step order: out[k1*M2 + k2] = iN[k1 + M1*k2]
// for k < M, out[M] = iN[M].
__global__ void k_permute_iN(const float* __restrict__ iN, float* __restrict__ out, int M1,
                             int M2) {
  const int d = blockIdx.y;
  const int64_t M = int64_t(M1) * M2;
  const float* src = iN + d * (M + 1);
  float* dst = out + d * (M + 1);
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k <= M;
       k += int64_t(gridDim.x) * blockDim.x) {
    if (k == M) {
      dst[M] = src[M];
    } else {
      const int64_t k1 = k % M1, k2 = k / M1;
      dst[k1 * M2 + k2] = src[k];
    }
  }
}

// bin[s] of four-step slot s = k1*M2 + k2 (frequency k1 + M1*k2), bin[M] of k = M
__global__ void k_corr_bins(const int32_t* __restrict__ edges, int nbins, int logM1, int logM2,
                            int16_t* __restrict__ bin) {
  const int M = 1 << (logM1 + logM2);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > M) return;
  const int k = (s == M) ? M : (s >> logM2) + ((s & ((1 << logM2) - 1)) << logM1);
  int lo = 0, hi = nbins - 1;   // largest b with edges[b] <= k
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (edges[mid] <= k) lo = mid; else hi = mid - 1;
  }
  bin[s] = int16_t(lo);
}

mm_status permute_inverse_spectrum(ScanImpl* s, hipStream_t st) {
  if (s->plan.single) return MM_OK;
  if (s->plan.corr_rank > 0) {
    const int M = 1 << s->plan.logM;
    hipLaunchKernelGGL(k_corr_bins, dim3((M + 1 + 255) / 256), dim3(256), 0, st,
                       s->at<int32_t>(s->lay.corr_edges), s->plan.corr_nbins, s->plan.logM1,
                       s->plan.logM2, s->at<int16_t>(s->lay.corr_bin));
    MM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_permute_iN, dim3(64, s->ndet), dim3(256), 0, st, s->d.inv_noise,
                     s->at<float>(s->lay.int_), s->plan.M1, 1 << s->plan.logM2);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

// --------------------------------------------------------- plan / tables
mm_status plan_and_layout(const mm_scan_desc* d, Plan* pl, Layout* L) {
  const int64_t n = d->nsamp;
  pl->f64 = d->tod_dtype == MM_F64;
  pl->bf16 = d->tod_dtype == MM_BF16;
  pl->logn = ilog2(n);                         // ceil(log2 n) for mixed-radix n
  pl->logM = pl->logn - 1;
  const int M = int(n / 2);
  // n = 2^a 3^b 5^c that is not a power of two: mixed-radix LDS transforms
  // (the whole of M on the one-kernel path, the columns M1 of the four-step)
  const bool mixed = (n & (n - 1)) != 0;
  pl->mix_code = 0;
  if (mixed) {
    int64_t r = M;
    for (int f : {2, 3, 5})
      while (r % f == 0) r /= f;
    if (r != 1) return fail(MM_EINVAL, "nsamp must be 2^a 3^b 5^c");
    if (d->corr_rank > 0)
      return fail(MM_EINVAL, "correlated noise needs nsamp a power of two");
    if (d->pointing == MM_POINT_BORESIGHT)
      return fail(MM_EINVAL, "MM_POINT_BORESIGHT needs nsamp a power of two");
  }
  const size_t cxb = pl->f64 ? 16 : 8;          // one complex in the math type
  const size_t wxb = pl->bf16 ? 4 : cxb;         // ... in the pass buffer
  pl->acc32 = d->acc == MM_ACC_F32X2;
  pl->corr_rank = d->corr_rank;
  pl->corr_nbins = d->corr_rank > 0 ? d->corr_nbins : 0;
  // correlated noise needs every detector's spectrum at once: the four-step
  // pipeline with wavefront rows of 512-2048 bins
  pl->single = (M <= kE * kNT) && pl->corr_rank == 0;
  // the compensated accumulation exists only in the per-pixel gather
  pl->otf = d->pointing == MM_POINT_BORESIGHT;
  // boresight pointing stores no per-sample pixels: P^T is always the gather
  pl->csr = d->scatter != MM_SCATTER_ATOMIC && (!pl->single || pl->acc32 || pl->otf);
  pl->M1 = 1;
  if (pl->single) {
    pl->logM1 = 0;
    pl->logM2 = pl->logM;
    pl->logC = 0;
    if (mixed && (pl->mix_code = mixed_radix_code(M)) == 0)
      return fail(MM_EINVAL, "nsamp/2 needs more than 10 FFT stages");
    int G = d->ndet;
    if (pl->csr && d->det_group > 0 && d->det_group < G) G = d->det_group;
    while (G > 1 && int64_t(G) * n > (int64_t(1) << 31) - 1) --G;
    pl->G = G;
    pl->logLmax = pl->logM;
  } else {
    int l1;
    int64_t odd = M;
    int e2 = 0;
    while ((odd & 1) == 0) {
      odd >>= 1;
      ++e2;
    }
    if (mixed) {
      // rows M2 = 2^l2 stay a power of two (2048 at most, 32 at least); the
      // columns M1 = M / M2 carry every factor 3 and 5 and at least one 2
      int l2 = e2 - 1 < 10 ? e2 - 1 : 10;
      const int64_t cap1 = pl->f64 ? int64_t(4) * kNT13 : int64_t(8) * kNT13;   // C >= 2
      while (l2 < 12 && l2 < e2 - 1 && (M >> l2) > cap1) ++l2;
      if (l2 < 5 || (M >> l2) > cap1 || (M >> l2) % 2 != 0)
        return fail(MM_EINVAL, "nsamp gives no four-step split (odd part of nsamp/2 too large)");
      l1 = pl->logM - l2;   // ceil(log2 M1)
      pl->logM1 = l1;
      pl->logM2 = l2;
      pl->M1 = int(M >> l2);
      pl->mix_code = mixed_radix_code(pl->M1);
    } else if (pl->corr_rank > 0) {
      l1 = pl->logM - 9;                   // rows of 512 bins
      if (l1 > 9) l1 = 9;                  // up to 2048 at M = 2^20
      if (l1 < 3 || pl->logM - l1 > 11)
        return fail(MM_EINVAL, "correlated noise needs nsamp in [2^13, 2^21]");
    } else if (d->fft_m1 > 0) {
      l1 = ilog2(d->fft_m1);
    } else {
      // columns of at most 512 (two pass-1/3 blocks a CU), unless that leaves
      // rows longer than 2048 bins, which the one-wavefront pass 2 cannot
      // take: then columns of 1024 (n = 2^22: 0.72 ms against 1.16 ms an
      // A-apply at 16 detectors)
      l1 = pl->logM / 2;
      if (l1 > 9) l1 = 9;
      if (pl->logM - l1 > 11) l1 = pl->logM - 11 < 10 ? pl->logM - 11 : 10;
      if (pl->logM - l1 > 12) l1 = pl->logM - 12;
    }
    if (!mixed) {
      pl->logM1 = l1;
      pl->logM2 = pl->logM - l1;
      pl->M1 = 1 << l1;
      if (pl->logM1 < 2 || pl->logM2 < 5 || pl->logM2 > 12 || pl->logM1 > 10)
        return fail(MM_EINVAL, "fft_m1 gives an unsupported four-step split");
    }
    int lc = d->fft_cols > 0 ? ilog2(d->fft_cols) : 4;
    // pass-1/3 tile: C * M1 complex in LDS, at most 16 per thread (float
    // math) or 8 (double), and within 160 KB with the twiddles
    const int64_t cap = pl->f64 ? int64_t(8) * kNT13 : int64_t(16) * kNT13;
    while (lc > 0 && ((int64_t(1) << lc) * pl->M1 > cap ||
                      ((int64_t(1) << lc) + 1) * pl->M1 * int64_t(cxb) > 160 * 1024))
      --lc;
    if (lc > pl->logM2) lc = pl->logM2;
    if (lc < 1) return fail(MM_EINVAL, "fft_cols leaves fewer than two columns per block");
    pl->logC = lc;
    if (!mixed && ((2 << (lc + pl->logM1)) % kNT != 0 || (2 << pl->logM2) % kNT != 0))
      return fail(MM_EINVAL, "four-step blocks too small for the thread count");
    int G = pl->corr_rank > 0 ? d->ndet : d->det_group;
    if (G <= 0) {
      // about 512 MiB of timestream scratch per group: fewer, larger launches
      // (iqu_256det: 128 detectors a group, A-apply 3.14 -> 3.01 ms against 64)
      const int64_t per = int64_t(M) * int64_t(wxb);
      G = int((int64_t(512) << 20) / per);
      if (G < 1) G = 1;
    }
    if (G > d->ndet) G = d->ndet;
    while (G > 1 && int64_t(G) * n > (int64_t(1) << 31) - 1) --G;
    if (pl->corr_rank > 0 && G != d->ndet)
      return fail(MM_EINVAL, "correlated noise needs ndet * nsamp < 2^31");
    pl->G = G;
    pl->logLmax = mixed ? pl->logM2 : (pl->logM1 > pl->logM2 ? pl->logM1 : pl->logM2);
  }
  pl->logS = (pl->logn + 1) / 2;
  const int maxside = d->ny > d->nx ? d->ny : d->nx;
  pl->logMapL = ilog2(maxside);
  // layout
  const int64_t npix = int64_t(d->ny) * d->nx;
  const int nc = d->ncomp;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  // (+64 B: the run-length gather reads four samples at a time from a run's
  // first sample, so its last loads may reach up to three samples past the end)
  L->tod = take(pl->single && !pl->csr ? 0 : size_t(pl->G) * size_t(M) * wxb + 64);
  L->tw = take((pl->mix_code && pl->single ? size_t(M) : (size_t(1) << pl->logLmax)) * cxb);
  L->tw2 = take(pl->single ? 0 : (size_t(1) << pl->logM2) * cxb);
  L->tw_m1 = take(pl->mix_code && !pl->single ? size_t(pl->M1) * cxb : 0);
  L->int_ = take(pl->single ? 0 : size_t(d->ndet) * size_t(M + 1) * 4);
  L->wn_hi = take(size_t((n + (int64_t(1) << pl->logS) - 1) >> pl->logS) * cxb);
  L->wn_lo = take((size_t(1) << pl->logS) * cxb);
  L->gmap = take(size_t(npix + 1) * 4 * (pl->f64 ? 8 : 4));
  L->acc = take(size_t(npix) * 4 * 8);
  L->detw = take(size_t(d->ndet) * 8);
  L->hits = take(size_t(npix) * 8);
  L->bb = take(size_t(npix) * 6 * 8);
  L->bj = take(size_t(npix) * 6 * 8);
  L->binv_b = take(size_t(npix) * 6 * 8);
  L->binv_j = take(size_t(npix) * 6 * 8);
  L->siginv = take(size_t(npix) * 6 * 8);
  L->sigma = take(size_t(npix) * 6 * 8);
  L->mask = take(size_t(npix) * 4);
  L->kinv = take(size_t(npix) * nc * nc * 16);
  L->planes = take(size_t(npix) * nc * nc * 16);
  L->probe = take(size_t(npix) * nc * nc * 8);
  L->tw_map = take((size_t(1) << pl->logMapL) * 16);
  L->vec = take(size_t(npix) * nc * 8 * 5);
  L->partials = take(size_t(kMaxPartials) * 4 * 8);
  L->pcg = take(sizeof(PcgDev));
  L->hist = take(size_t(3) * (kHistCap + 1) * 8);
  L->misc = take(256);
  L->spec = take(size_t(kSpecBlocks + 1) * kSpecMaxBins * 4 * 8);
  L->corr_edges = take(pl->corr_rank > 0 ? size_t(pl->corr_nbins + 1) * 4 : 0);
  L->corr_bin = take(pl->corr_rank > 0 ? size_t(M + 1) * 2 : 0);
  L->corr_t = take(pl->corr_rank > 0 ? size_t(pl->corr_rank) * M * cxb : 0);
  const int ngroups = (d->ndet + pl->G - 1) / pl->G;
  const size_t csr_n = pl->csr ? size_t(ngroups) * pl->G * size_t(n) : 0;
  L->csr_cnt = take(pl->csr ? size_t(ngroups) * npix * 4 : 0);
  L->csr_off = take(pl->csr ? size_t(ngroups) * (npix + 1) * 4 : 0);
  L->csr_idx = take(csr_n * 4);
  // the run-length index keeps the angle-coded weights pixel-major (4 B a
  // sample, in the gather's sample order) when the weights can be angles
  // (weights of unit norm on the float paths, checked at creation: stored
  // ones, or the boresight model's)
  const bool rle_pa = pl->csr && !pl->f64 && nc == 3 && d->scatter != MM_SCATTER_SAMPLES &&
                      int64_t(pl->G) * n <= (int64_t(1) << 28);
  L->csr_soff = take(rle_pa ? size_t(ngroups) * (npix + 1) * 4 : 0);
  // stored weights beside the index, except for boresight pointing on the
  // float64 path, whose gather computes float64 weights from the model; the
  // run-length index (groups of at most 2^28 samples) stores none beside it:
  // its gather reads the pixel-major angles, the time-major weights or the
  // boresight model
  pl->csr_w = nc == 3 && !(pl->otf && pl->f64);
  pl->rle = pl->csr && d->scatter != MM_SCATTER_SAMPLES &&
            int64_t(pl->G) * n <= (int64_t(1) << 28);
  L->csr_w = take(pl->csr_w && !pl->rle ? csr_n * 8 : rle_pa ? csr_n * 4 + 64 : 0);
  L->ang_tab = take(256 * 8);
  // float32 copies of the boresight model for pass 1 (float paths)
  const bool bfast = pl->otf && !pl->f64;
  L->bore_f = take(bfast ? size_t(n) * 16 : 0);
  L->bore_a = take(bfast ? size_t(n) * 4 : 0);
  L->det_f = take(bfast ? size_t(d->ndet) * 8 : 0);
  L->det_a = take(bfast ? size_t(d->ndet) * 4 : 0);
  // time-major angle-coded weights for pass 1 (stored pointing, float paths)
  L->ang_t = take(nc == 3 && pl->csr && !pl->f64 && !pl->otf ? size_t(d->ndet) * size_t(n) * 4 : 0);
  // chunk-coded pointing for pass 1 (4 B a sample and 16 B per 64 samples;
  // built from the time-major angles at creation when every chunk fits)
  pl->ptc = nc == 3 && pl->csr && !pl->f64 && !pl->otf && !pl->single && n % kPtcChunk == 0 &&
            d->pointing_code == MM_PTC_AUTO;
  L->ptc_h = take(pl->ptc ? size_t(d->ndet) * size_t(n / kPtcChunk) * 16 : 0);
  L->ptc = take(pl->ptc ? size_t(d->ndet) * size_t(n) * 4 : 0);
  L->total = off;
  return MM_OK;
}

template <typename T>
static void table(std::vector<Cx<T>>& v, int64_t count, int64_t step, int64_t n) {
  v.resize(count);
  for (int64_t m = 0; m < count; ++m) {
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L *
                            (long double)((m * step) % n) / (long double)n;
    v[m].x = T(std::cos(double(ang)));
    v[m].y = T(std::sin(double(ang)));
  }
}

template <typename T>
static mm_status upload_t(ScanImpl* s, hipStream_t st) {
  const Plan& pl = s->plan;
  std::vector<Cx<T>> tw, hi, lo;
  const int64_t Lmax = int64_t(1) << pl.logLmax;
  if (pl.mix_code && pl.single)
    table(tw, s->n / 2, 1, s->n / 2);   // W_M^m for the mixed-radix stages
  else
    table(tw, Lmax, 1, Lmax);
  if (pl.mix_code && !pl.single) {     // W_M1^m for the mixed-radix columns
    std::vector<Cx<T>> tm1;
    table(tm1, pl.M1, 1, pl.M1);
    MM_HIP(hipMemcpyAsync(s->ws + s->lay.tw_m1, tm1.data(), tm1.size() * sizeof(Cx<T>),
                          hipMemcpyHostToDevice, st));
    MM_HIP(hipStreamSynchronize(st));   // tm1 leaves scope
  }
  const int64_t n = s->n;
  const int64_t S = int64_t(1) << pl.logS;
  table(hi, (n + S - 1) / S, S, n);
  table(lo, S, 1, n);
  MM_HIP(hipMemcpyAsync(s->ws + s->lay.tw, tw.data(), tw.size() * sizeof(Cx<T>),
                        hipMemcpyHostToDevice, st));
  std::vector<Cx<T>> t2;
  if (!pl.single) {
    const int64_t M2 = int64_t(1) << pl.logM2;
    table(t2, M2, 1, 2 * M2);
    MM_HIP(hipMemcpyAsync(s->ws + s->lay.tw2, t2.data(), t2.size() * sizeof(Cx<T>),
                          hipMemcpyHostToDevice, st));
  }
  MM_HIP(hipMemcpyAsync(s->ws + s->lay.wn_hi, hi.data(), hi.size() * sizeof(Cx<T>),
                        hipMemcpyHostToDevice, st));
  std::vector<float> at(512);   // (cos, sin)(2 pi k / 256), for angle-coded weights
  for (int k = 0; k < 256; ++k) {
    const long double ang = 2.0L * 3.14159265358979323846264338327950288L * k / 256.0L;
    at[2 * k] = float(std::cos(double(ang)));
    at[2 * k + 1] = float(std::sin(double(ang)));
  }
  MM_HIP(hipMemcpyAsync(s->ws + s->lay.ang_tab, at.data(), at.size() * 4, hipMemcpyHostToDevice,
                        st));
  MM_HIP(hipMemcpyAsync(s->ws + s->lay.wn_lo, lo.data(), lo.size() * sizeof(Cx<T>),
                        hipMemcpyHostToDevice, st));
  std::vector<Cx<double>> tm;
  const int64_t Lm = int64_t(1) << pl.logMapL;
  table(tm, Lm, 1, Lm);
  MM_HIP(hipMemcpyAsync(s->ws + s->lay.tw_map, tm.data(), tm.size() * sizeof(Cx<double>),
                        hipMemcpyHostToDevice, st));
  if (pl.corr_rank > 0)
    MM_HIP(hipMemcpyAsync(s->ws + s->lay.corr_edges, s->d.corr_edges,
                          size_t(pl.corr_nbins + 1) * 4, hipMemcpyHostToDevice, st));
  MM_HIP(hipStreamSynchronize(st));
  return MM_OK;
}

// Float32 copies of the boresight model and the angles of its weights; counts
// |cos phi| or |sin phi| above 1 (the float32 pixel's error bound needs them
// at most 1).
__global__ void k_bore_prep(const double* __restrict__ b, const double* __restrict__ det,
                            int64_t n, int ndet, int ny, int nx, float4* __restrict__ bf,
                            uint32_t* __restrict__ ba, float2* __restrict__ df,
                            uint32_t* __restrict__ da, int* __restrict__ bad) {
  const double cy = 0.5 * double(ny - 1), cx = 0.5 * double(nx - 1);
  int cnt = 0;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += stride) {
    const double c = b[2 * n + t], sn = b[3 * n + t];
    bf[t] = make_float4(float(b[t] - cy), float(b[n + t] - cx), float(c), float(sn));
    ba[t] = weight_angle(b[4 * n + t], b[5 * n + t]);
    cnt += (fabs(c) <= 1.0 && fabs(sn) <= 1.0) ? 0 : 1;
    if (t < ndet) {
      df[t] = make_float2(float(det[t]), float(det[ndet + t]));
      da[t] = weight_angle(det[2 * ndet + t], det[3 * ndet + t]);
    }
  }
  if (cnt) atomicAdd(bad, cnt);
}

mm_status bore_setup(ScanImpl* s, hipStream_t st) {
  s->bore_fast = false;
  if (!s->plan.otf || s->plan.f64 || s->ndet > s->n) return MM_OK;
  const Layout& L = s->lay;
  int* bad = s->at<int>(L.misc);
  mm_status r;
  if ((r = fill_zero(bad, 4, st)) != MM_OK) return r;
  hipLaunchKernelGGL(k_bore_prep, dim3(1024), dim3(256), 0, st, s->d.bore, s->d.det_off, s->n,
                     s->ndet, s->ny, s->nx, s->at<float4>(L.bore_f), s->at<uint32_t>(L.bore_a),
                     s->at<float2>(L.det_f), s->at<uint32_t>(L.det_a), bad);
  MM_HIP(hipGetLastError());
  int h = 0;
  MM_HIP(hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, st));
  MM_HIP(hipStreamSynchronize(st));
  s->bore_fast = (h == 0) && kBoreFast;
  return MM_OK;
}

mm_status upload_tables(ScanImpl* s, hipStream_t st) {
  return s->plan.f64 ? upload_t<double>(s, st) : upload_t<float>(s, st);
}

}  // namespace mm
