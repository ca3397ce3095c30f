// Mixed-radix (2, 3, 4, 5, 8) complex FFTs on data resident in LDS, for
// lengths L = 2^a 3^b 5^c that are not powers of two.
//
// Same Stockham autosort scheme as the power-of-two transforms: a stage of
// radix R (after stages whose radices multiply to Ns) reads R points L/R
// apart, multiplies point r by W_{Ns R}^{r k} (k = j mod Ns), does a length-R
// DFT in registers and writes the results Ns apart into the autosorted
// position; loads go to registers before a barrier, stores follow it, so the
// stage works in place.  The stage radices are a host-built code of 3-bit
// digits (1: 2, 2: 4, 3: 8, 4: 3, 5: 5), lowest digit first.
//
// Twiddles: tw[m] = W_Lt^m, m < Lt = L * tstride, from float64 on the host;
// every power W_{Ns R}^{r k} is one table read (index r k (L / (Ns R))
// tstride < Lt), so no products of rounded twiddles.
#pragma once
#include "fft_lds.h"

namespace mm {

// radix-3 DFT, forward W = exp(-2 pi i / 3)
template <typename T, bool INV>
__device__ __forceinline__ void dft_r3(Cx<T> (&v)[3]) {
  const T s = T(0.86602540378443864676372317075294);
  const Cx<T> t1 = v[1] + v[2];
  const Cx<T> t2 = cx(v[0].x - T(0.5) * t1.x, v[0].y - T(0.5) * t1.y);
  const Cx<T> d = v[1] - v[2];
  // t3 = -i s d (forward), +i s d (inverse)
  const Cx<T> t3 = INV ? cx(-s * d.y, s * d.x) : cx(s * d.y, -s * d.x);
  v[0] = v[0] + t1;
  v[1] = t2 + t3;
  v[2] = t2 - t3;
}

// radix-5 DFT: with a_1 = v1 + v4, a_2 = v2 + v3, b_1 = v1 - v4, b_2 = v2 - v3,
// X1,4 = (v0 + c1 a1 + c2 a2) -/+ i (s1 b1 + s2 b2),
// X2,3 = (v0 + c2 a1 + c1 a2) -/+ i (s2 b1 - s1 b2)  (forward; inverse flips i)
template <typename T, bool INV>
__device__ __forceinline__ void dft_r5(Cx<T> (&v)[5]) {
  const T c1 = T(0.30901699437494742410229341718282);    // cos 2pi/5
  const T c2 = T(-0.80901699437494742410229341718282);   // cos 4pi/5
  const T s1 = T(0.95105651629515357211643933337938);    // sin 2pi/5
  const T s2 = T(0.58778525229247312916870595463907);    // sin 4pi/5
  const Cx<T> a1 = v[1] + v[4], a2 = v[2] + v[3];
  const Cx<T> b1 = v[1] - v[4], b2 = v[2] - v[3];
  const Cx<T> t1 = cx(v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y);
  const Cx<T> t2 = cx(v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y);
  const Cx<T> u1 = cx(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
  const Cx<T> u2 = cx(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
  // -i u = (u.y, -u.x)
  const Cx<T> mu1 = INV ? cx(-u1.y, u1.x) : cx(u1.y, -u1.x);
  const Cx<T> mu2 = INV ? cx(-u2.y, u2.x) : cx(u2.y, -u2.x);
  v[0] = v[0] + a1 + a2;
  v[1] = t1 + mu1;
  v[4] = t1 - mu1;
  v[2] = t2 + mu2;
  v[3] = t2 - mu2;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_any(Cx<T> (&v)[R]) {
  if constexpr (R == 3) {
    dft_r3<T, INV>(v);
  } else if constexpr (R == 5) {
    dft_r5<T, INV>(v);
  } else {
    dft_reg<T, R, INV>(v);
  }
}

// Division of n < 2^16 by d < 2^16 as a multiply-high: q = (n * ceil(2^32 / d))
// >> 32 is exact when n d < 2^32 (the rounding error of the reciprocal, at
// most d / 2^32 per unit of n, stays below 1 / d).
struct FastDiv {
  uint32_t d, m;
  __device__ __forceinline__ explicit FastDiv(uint32_t dd)
      : d(dd), m(dd == 1 ? 0u : uint32_t((uint64_t(1) << 32) / dd + 1)) {}
  __device__ __forceinline__ uint32_t div(uint32_t n) const {
    return d == 1 ? n : __umulhi(n, m);
  }
};

struct MixShape {
  int L;          // transform length
  int B;          // batch count
  int es, bs;     // element / batch strides (complex elements)
  bool batch_fast;
  uint32_t code;  // stage radices, 3-bit digits, lowest first
  int tstride;    // table stride: tw has L * tstride entries
};

template <typename T, int R, int NT, int E, bool INV>
__device__ __forceinline__ void stockham_stage_mx(Cx<T>* __restrict__ buf, const MixShape& s,
                                                  int Ns, const Cx<T>* __restrict__ tw) {
  constexpr int NB = (E + R - 1) / R;
  const int LR = s.L / R;
  const int nbf = s.B * LR;
  const int step = (LR / Ns) * s.tstride;   // W_{Ns R} = W_Lt^step
  const FastDiv dB{uint32_t(s.B)}, dLR{uint32_t(LR)}, dNs{uint32_t(Ns)};
  // butterfly w -> transform b, index j
  auto split = [&](int w, int* b, int* j) {
    if (s.batch_fast) {
      *j = int(dB.div(uint32_t(w)));
      *b = w - *j * s.B;
    } else {
      *b = int(dLR.div(uint32_t(w)));
      *j = w - *b * LR;
    }
  };
  Cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int w = threadIdx.x + i * NT;
    if (w < nbf) {
      int b, j;
      split(w, &b, &j);
      const int base = b * s.bs + j * s.es;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[base + (r * LR) * s.es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int w = threadIdx.x + i * NT;
    if (w < nbf) {
      int b, j;
      split(w, &b, &j);
      const int k = j - int(dNs.div(uint32_t(j))) * Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> t = tw[r * k * step];
          if (INV) t.y = -t.y;
          v[i][r] = v[i][r] * t;
        }
      }
      dft_any<T, R, INV>(v[i]);
      const int out = (j - k) * R + k;
      const int base = b * s.bs + out * s.es;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + (r * Ns) * s.es] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform; must be called by all NT threads of the block.
template <typename T, int NT, int E, bool INV>
__device__ __forceinline__ void lds_fft_mx(Cx<T>* __restrict__ buf, const MixShape& s,
                                           const Cx<T>* __restrict__ tw) {
  int Ns = 1;
  for (uint32_t c = s.code; c != 0; c >>= 3) {
    switch (c & 7u) {
      case 1: stockham_stage_mx<T, 2, NT, E, INV>(buf, s, Ns, tw); Ns *= 2; break;
      case 2: stockham_stage_mx<T, 4, NT, E, INV>(buf, s, Ns, tw); Ns *= 4; break;
      case 3: stockham_stage_mx<T, 8, NT, E, INV>(buf, s, Ns, tw); Ns *= 8; break;
      case 4: stockham_stage_mx<T, 3, NT, E, INV>(buf, s, Ns, tw); Ns *= 3; break;
      default: stockham_stage_mx<T, 5, NT, E, INV>(buf, s, Ns, tw); Ns *= 5; break;
    }
  }
}

// Host: the stage code of L = 2^a 3^b 5^c (radix 8 first, then 4 or 2, then
// 3s and 5s); 0 if L has another prime factor or needs more than 10 stages.
inline uint32_t mixed_radix_code(int64_t L) {
  uint32_t code = 0;
  int shift = 0;
  auto push = [&](uint32_t d) {
    if (shift > 27) return false;
    code |= d << shift;
    shift += 3;
    return true;
  };
  int a = 0;
  while (L % 2 == 0) { L /= 2; ++a; }
  while (a >= 3) { if (!push(3)) return 0; a -= 3; }
  if (a == 2 && !push(2)) return 0;
  if (a == 1 && !push(1)) return 0;
  while (L % 3 == 0) { L /= 3; if (!push(4)) return 0; }
  while (L % 5 == 0) { L /= 5; if (!push(5)) return 0; }
  return L == 1 ? code : 0;
}

}  // namespace mm
