// Device-side helpers shared by the map-making kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mm {

constexpr int kWave = 64;

template <typename T>
struct Cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ Cx<T> cx(T a, T b) {
  Cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return cx(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return cx(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ Cx<T> operator*(Cx<T> a, Cx<T> b) {
  return cx(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ Cx<T> operator*(T s, Cx<T> a) { return cx(s * a.x, s * a.y); }
template <typename T>
__device__ __forceinline__ Cx<T> conj(Cx<T> a) { return cx(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <typename T>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) { return cx(a.y, -a.x); }
template <typename T>
__device__ __forceinline__ Cx<T> mul_pi(Cx<T> a) { return cx(-a.y, a.x); }

// Two-level table of W_n^m = exp(-2 pi i m / n), m < n:
// W_n^m = hi[m >> logS] * lo[m & (S-1)].
template <typename T>
struct TwoLevel {
  const Cx<T>* hi;
  const Cx<T>* lo;
  int logS;
  __device__ __forceinline__ Cx<T> operator()(int64_t m) const {
    return hi[m >> logS] * lo[m & ((int64_t(1) << logS) - 1)];
  }
};

// ---------------------------------------------------------------------------
// Wave-level segmented sum over runs of equal keys in consecutive lanes.
// After the call, the lane that heads each run (first lane of the run, or
// every kSpan-th lane of a longer run) holds the sum of up to kSpan values
// of its run starting at itself, and `issue` is true for those lanes.
// kSpan = 2^STEPS.  Keys < 0 never issue.
template <int STEPS, int NV>
__device__ __forceinline__ bool wave_segmented_sum(int key, double (&v)[NV]) {
  const int lane = threadIdx.x & (kWave - 1);
  const int prev = __shfl_up(key, 1);
  const bool head = (lane == 0) || (prev != key);
  const uint64_t hm = __ballot(head);
#pragma unroll
  for (int s = 0; s < STEPS; ++s) {
    const int off = 1 << s;
    bool ok = false;
    if (lane + off < kWave) {
      const uint64_t range = ((uint64_t(1) << off) - 1) << (lane + 1);
      ok = (hm & range) == 0;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double t = __shfl_down(v[i], off);
      if (ok) v[i] += t;
    }
  }
  // position of this lane inside its run
  const uint64_t below = hm & ((lane == 63) ? ~uint64_t(0) : ((uint64_t(2) << lane) - 1));
  const int head_lane = 63 - __clzll(below);
  const int pos = lane - head_lane;
  return key >= 0 && (pos & ((1 << STEPS) - 1)) == 0;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }

// Block-wide sum of NV doubles (blockDim.x a multiple of 64, <= 1024).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sm /* >= 16*NV */) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] += __shfl_xor(v[i], off);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sm[w * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += sm[k * NV + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Compensated float32 ("float-float") accumulation: a value is the unevaluated
// sum hi + lo of two floats with |lo| <= ulp(hi) / 2, about 48 significant
// bits.  two_sum is Knuth's error-free transformation of a sum; a product's
// rounding error comes from one fma.  Contraction is off inside these
// helpers: fusing a product into a following two_sum would count its
// rounding error twice.
struct F2 {
  float hi, lo;
};

__device__ __forceinline__ F2 two_sum(float a, float b) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  const float e = (a - (s - bb)) + (b - bb);
  return F2{s, e};
}

// s += x + xe, where xe is the (small) rounding error carried with x
__device__ __forceinline__ void f2_acc(F2& s, float x, float xe) {
#pragma clang fp contract(off)
  F2 t = two_sum(s.hi, x);
  t.lo += s.lo + xe;
  s = two_sum(t.hi, t.lo);  // renormalise (robust to cancellation in t.hi)
}

__device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
#pragma clang fp contract(off)
  F2 t = two_sum(a.hi, b.hi);
  t.lo += a.lo + b.lo;
  return two_sum(t.hi, t.lo);
}

// a double as hi + lo (exact to about 48 bits)
__device__ __forceinline__ F2 f2_split(double x) {
#pragma clang fp contract(off)
  const float h = float(x);
  return F2{h, float(x - double(h))};
}

// s += a * b for float-float a and b
__device__ __forceinline__ void f2_fma_acc(F2& s, F2 a, F2 b) {
#pragma clang fp contract(off)
  const float p = a.hi * b.hi;
  float e = fmaf(a.hi, b.hi, -p);
  e = fmaf(a.hi, b.lo, e);
  e = fmaf(a.lo, b.hi, e);
  f2_acc(s, p, e);
}

// s += a * b for a float a and a float-float b
__device__ __forceinline__ void f2_fma_acc(F2& s, float a, F2 b) {
#pragma clang fp contract(off)
  const float p = a * b.hi;
  float e = fmaf(a, b.hi, -p);
  e = fmaf(a, b.lo, e);
  f2_acc(s, p, e);
}

__device__ __forceinline__ double f2_value(F2 a) { return double(a.hi) + double(a.lo); }

__device__ __forceinline__ F2 f2_shfl_xor(F2 a, int off, int width = 64) {
  return F2{__shfl_xor(a.hi, off, width), __shfl_xor(a.lo, off, width)};
}

// block-wide float-float sums in a fixed order; sm holds >= 16 * NV entries
template <int NV>
__device__ __forceinline__ void block_sum_f2(F2 (&v)[NV], F2* sm) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = f2_add(v[i], f2_shfl_xor(v[i], off));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sm[w * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 0; i < NV; ++i) {
      F2 s{0.f, 0.f};
      for (int k = 0; k < nw; ++k) s = f2_add(s, sm[k * NV + i]);
      v[i] = s;
    }
  }
  __syncthreads();
}

}  // namespace mm
