// Small dense symmetric eigen-solvers in float64 (per pixel / per wavenumber).
#pragma once
#include <hip/hip_runtime.h>

namespace mm {

// Cyclic Jacobi eigen-decomposition of a real symmetric N x N matrix A
// (overwritten).  On return lam[i] = A[i][i] are the eigenvalues and the
// columns of V the eigenvectors.
template <int N>
__device__ __forceinline__ void jacobi_eig(double (&A)[N][N], double (&V)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    double off = 0.0, diag = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      diag += A[i][i] * A[i][i];
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[i][j] * A[i][j];
    }
    if (off <= 1e-32 * diag || off == 0.0) break;
#pragma unroll
    for (int p = 0; p < N; ++p) {
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0);
        const double s = t * c;
        // A <- J^T A J with J the rotation in the (p, q) plane
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        A[p][q] = A[q][p] = 0.0;
#pragma unroll
        for (int k = 0; k < N; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
    }
  }
}

// Packed symmetric 3x3 <-> full.  Order: xx, xy, xz, yy, yz, zz.
__device__ __forceinline__ void unpack_sym3(const double* a, double (&A)[3][3]) {
  A[0][0] = a[0]; A[0][1] = a[1]; A[0][2] = a[2];
  A[1][0] = a[1]; A[1][1] = a[3]; A[1][2] = a[4];
  A[2][0] = a[2]; A[2][1] = a[4]; A[2][2] = a[5];
}

__device__ __forceinline__ void pack_sym3(const double (&A)[3][3], double* a) {
  a[0] = A[0][0]; a[1] = A[0][1]; a[2] = A[0][2];
  a[3] = A[1][1]; a[4] = A[1][2]; a[5] = A[2][2];
}

// f(A) = V diag(f(lam)) V^T for a symmetric 3x3 from its decomposition.
template <typename F>
__device__ __forceinline__ void sym3_func(const double (&V)[3][3], const double (&lam)[3], F f,
                                          double (&out)[3][3]) {
  double fl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) fl[i] = f(lam[i]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) s += V[i][k] * fl[k] * V[j][k];
      out[i][j] = s;
    }
}

}  // namespace mm
