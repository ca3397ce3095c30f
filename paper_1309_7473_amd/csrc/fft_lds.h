// Batched power-of-two complex FFTs on data resident in LDS.
//
// Radix-8/4/2 Stockham autosort: every stage reads R points spaced L/R apart,
// applies the twiddles W_{Ns R}^{r k}, k = j mod Ns, does a length-R DFT in
// registers and writes the R results Ns apart into the autosorted position.
// The stage works in place in LDS: all loads of a stage go to registers
// before a barrier, the stores follow it.  Output is in natural order.
//
// Layout: transform b (0 <= b < B) has its element j at buf[b*bs + j*es].
// Work items (one butterfly each) are spread over the NT threads of the
// block, at most E/R per thread (so B*L <= E*NT).  With batch_fast the batch
// index varies fastest across threads (contiguous columns: es = B, bs = 1);
// otherwise the element index does (contiguous rows: es = 1).
//
// Twiddles come from a table tw[m] = W_Lmax^m, m < Lmax, computed in float64
// on the host and rounded once; a length-L transform reads it with stride
// Lmax/L.  A radix-8 butterfly reads W and W^4 and forms the other powers by
// complex products (at most three roundings more than the table).  Forward
// uses W = exp(-2 pi i / L); inverse uses conj and is unnormalised.
#pragma once
#include "mm_device.h"

namespace mm {

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_reg(Cx<T> (&v)[R]) {
  if constexpr (R == 2) {
    Cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    Cx<T> a0 = v[0] + v[2], a1 = v[0] - v[2];
    Cx<T> b0 = v[1] + v[3], b1 = v[1] - v[3];
    b1 = INV ? mul_pi(b1) : mul_mi(b1);
    v[0] = a0 + b0;
    v[2] = a0 - b0;
    v[1] = a1 + b1;
    v[3] = a1 - b1;
  } else if constexpr (R == 8) {
    const T h = T(0.70710678118654752440084436210485);
    Cx<T> a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = v[r] + v[r + 4];
      b[r] = v[r] - v[r + 4];
    }
    // b[r] *= W8^r (forward) or conj (inverse)
    if constexpr (!INV) {
      b[1] = cx(h * (b[1].x + b[1].y), h * (b[1].y - b[1].x));
      b[2] = mul_mi(b[2]);
      b[3] = cx(h * (b[3].y - b[3].x), -h * (b[3].x + b[3].y));
    } else {
      b[1] = cx(h * (b[1].x - b[1].y), h * (b[1].y + b[1].x));
      b[2] = mul_pi(b[2]);
      b[3] = cx(-h * (b[3].x + b[3].y), h * (b[3].x - b[3].y));
    }
    dft_reg<T, 4, INV>(a);
    dft_reg<T, 4, INV>(b);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      v[2 * m] = a[m];
      v[2 * m + 1] = b[m];
    }
  }
}

// Length-(A*B) DFT of values held in registers, natural order in and out:
// with n = B n1 + n2 and k = k1 + A k2,
//   X[k] = sum_n2 W_B^(n2 k2) W_AB^(n2 k1) sum_n1 W_A^(n1 k1) x[B n1 + n2].
// tw(m) returns W_AB^m (forward sign); the inverse uses conjugates.
template <typename T, int A, int B, bool INV, typename TW>
__device__ __forceinline__ void dft_2level(Cx<T> (&v)[A * B], TW tw) {
  Cx<T> y[B][A];
#pragma unroll
  for (int n2 = 0; n2 < B; ++n2) {
    Cx<T> t[A];
#pragma unroll
    for (int n1 = 0; n1 < A; ++n1) t[n1] = v[B * n1 + n2];
    dft_reg<T, A, INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      if (n2 * k1 == 0) {
        y[n2][k1] = t[k1];
      } else {
        Cx<T> w = tw(n2 * k1);
        if (INV) w.y = -w.y;
        y[n2][k1] = t[k1] * w;
      }
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < A; ++k1) {
    Cx<T> s[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) s[n2] = y[n2][k1];
    dft_reg<T, B, INV>(s);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) v[k1 + A * k2] = s[k2];
  }
}

// W_N^m = exp(-2 pi i m / N) for N dividing 32, from literal constants
// (cos(pi j / 16), j = 0..8, rounded by the compiler to T), so a DFT in
// registers needs no table loads and its powers fold into the arithmetic.
template <typename T, int N>
struct ConstTw {
  static_assert(N == 8 || N == 16 || N == 32, "N must divide 32");
  __device__ __forceinline__ static constexpr double cospi16(int j) {
    constexpr double c[9] = {1.0,
                             0.98078528040323044912618223613424,
                             0.92387953251128675612818318939679,
                             0.83146961230254523707878837761791,
                             0.70710678118654752440084436210485,
                             0.55557023301960222474283081394853,
                             0.38268343236508977172845998403040,
                             0.19509032201612826784828486847702,
                             0.0};
    j &= 31;
    if (j > 16) j = 32 - j;            // cos(2 pi - x) = cos(x)
    return j <= 8 ? c[j] : -c[16 - j];   // cos(pi - x) = -cos(x)
  }
  __device__ __forceinline__ Cx<T> operator()(int m) const {
    const int j = m * (32 / N);        // W_N^m = exp(-i pi j / 16)
    return cx(T(cospi16(j)), T(-cospi16(8 - j)));
  }
};

// In-register DFT of length E in {8, 16, 32}; tw(m) = W_E^m.
template <typename T, int E, bool INV, typename TW>
__device__ __forceinline__ void dft_regs(Cx<T> (&v)[E], TW tw) {
  if constexpr (E == 8) {
    dft_reg<T, 8, INV>(v);
  } else if constexpr (E == 16) {
    dft_2level<T, 4, 4, INV>(v, tw);
  } else {
    static_assert(E == 32, "E must be 8, 16 or 32");
    dft_2level<T, 4, 8, INV>(v, tw);
  }
}

struct FftShape {
  int logL;      // transform length L = 2^logL
  int logB;      // batch count B = 2^logB
  int es, bs;    // element / batch strides (in complex elements)
  bool batch_fast;
  int logLmax;   // table length
};

// Padded LDS addressing: element i lives at i + (i >> PAD) (PAD = 0: none).
// One pad slot per 2^PAD elements spreads the stride-R stores of the early
// stages of contiguous transforms over the LDS banks.
template <int PAD>
__device__ __forceinline__ int lds_at(int i) {
  if constexpr (PAD == 0) {
    return i;
  } else {
    return i + (i >> PAD);
  }
}

template <typename T, int R, int NT, int E, bool INV, int PAD>
__device__ __forceinline__ void stockham_stage(Cx<T>* __restrict__ buf, const FftShape& s,
                                               int logNs, const Cx<T>* __restrict__ tw) {
  constexpr int NB = E / R;
  constexpr int logR = (R == 8) ? 3 : (R == 4) ? 2 : 1;
  const int logLR = s.logL - logR;
  const int LR = 1 << logLR;
  const int nbf = 1 << (s.logB + logLR);
  const int Ns = 1 << logNs;
  // twiddle index step: r * k * (L / (Ns R)) in units of the L-table, times Lmax/L
  const int tshift = (s.logL - logNs - logR) + (s.logLmax - s.logL);
  Cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int w = threadIdx.x + i * NT;
    if (w < nbf) {
      int b, j;
      if (s.batch_fast) {
        b = w & ((1 << s.logB) - 1);
        j = w >> s.logB;
      } else {
        j = w & (LR - 1);
        b = w >> logLR;
      }
      const int base = b * s.bs + j * s.es;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = buf[lds_at<PAD>(base + (r * LR) * s.es)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int w = threadIdx.x + i * NT;
    if (w < nbf) {
      int b, j;
      if (s.batch_fast) {
        b = w & ((1 << s.logB) - 1);
        j = w >> s.logB;
      } else {
        j = w & (LR - 1);
        b = w >> logLR;
      }
      const int k = j & (Ns - 1);
      if (logNs > 0) {
        // W^r for r < R from two table reads (W and W^4) and products
        Cx<T> w[R];
        w[1] = tw[k << tshift];
        if (INV) w[1].y = -w[1].y;
        if constexpr (R >= 4) w[2] = w[1] * w[1];
        if constexpr (R >= 4) w[3] = w[2] * w[1];
        if constexpr (R == 8) {
          w[4] = tw[(4 * k) << tshift];
          if (INV) w[4].y = -w[4].y;
          w[5] = w[4] * w[1];
          w[6] = w[4] * w[2];
          w[7] = w[4] * w[3];
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = v[i][r] * w[r];
      }
      dft_reg<T, R, INV>(v[i]);
      const int out = ((j - k) << logR) + k;
      const int base = b * s.bs + out * s.es;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[lds_at<PAD>(base + (r * Ns) * s.es)] = v[i][r];
    }
  }
  __syncthreads();
}

// Full transform; must be called by all NT threads of the block.  The
// radix-2/4 stage (if log2 L is not a multiple of 3) runs first, or last with
// SMALL_LAST: for contiguous transforms (es = 1) the stride of the stores of
// the stages that follow the first one is then R * Ns >= 64 elements apart
// only in whole 64-element runs.
template <typename T, int NT, int E, bool INV, int PAD = 0, bool SMALL_LAST = false>
__device__ __forceinline__ void lds_fft(Cx<T>* __restrict__ buf, const FftShape& s,
                                        const Cx<T>* __restrict__ tw) {
  int logNs = 0;
  int rem = s.logL;
  const int small = rem % 3;
  auto small_stage = [&]() {
    if (small == 1) {
      stockham_stage<T, 2, NT, E, INV, PAD>(buf, s, logNs, tw);
    } else if (small == 2) {
      stockham_stage<T, 4, NT, E, INV, PAD>(buf, s, logNs, tw);
    }
    logNs += small;
  };
  if (!SMALL_LAST && small) small_stage();
  rem -= small;
  while (rem >= 3) {
    stockham_stage<T, 8, NT, E, INV, PAD>(buf, s, logNs, tw);
    logNs += 3;
    rem -= 3;
  }
  if (SMALL_LAST && small) small_stage();
}

}  // namespace mm
