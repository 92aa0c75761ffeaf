// Small fixed-size matrix helpers for the SRTM kernels (gfx950).
//
// Every matrix lives in registers as a T[R][C] array with compile-time shape; loops
// are fully unrolled so no array is ever indexed dynamically (which would force it
// into scratch memory).
#pragma once

#include <hip/hip_runtime.h>

#define SRTM_DEV __device__ __forceinline__

namespace srtm {

template <typename T> SRTM_DEV T my_fma(T a, T b, T c) { return fma(a, b, c); }

template <typename T, int R, int C>
SRTM_DEV void load(T (&a)[R][C], const T* __restrict__ p) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) a[r][c] = p[r * C + c];
}

template <typename T, int R>
SRTM_DEV void loadv(T (&a)[R], const T* __restrict__ p) {
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = p[r];
}

// Loads from device (global) memory through a global-address-space pointer, for arrays whose
// pointers were read from memory (generic) but always live in device memory. Never for LDS.
template <typename T>
SRTM_DEV T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Loads from LDS through a local-address-space pointer (p must point into LDS).
template <typename T>
SRTM_DEV T sld(const T* p) {
  return *(const __attribute__((address_space(3))) T*)p;
}

template <typename T, int R, int C>
SRTM_DEV void gload(T (&a)[R][C], const T* __restrict__ p) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) a[r][c] = gld(p + r * C + c);
}

template <typename T, int R>
SRTM_DEV void gloadv(T (&a)[R], const T* __restrict__ p) {
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = gld(p + r);
}

// C = A B
template <typename T, int M, int K, int N>
SRTM_DEV void mm(const T (&A)[M][K], const T (&B)[K][N], T (&C)[M][N]) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T s = A[i][0] * B[0][j];
#pragma unroll
      for (int k = 1; k < K; ++k) s = my_fma(A[i][k], B[k][j], s);
      C[i][j] = s;
    }
}

// C = A B^T   (A: M x K, B: N x K)
template <typename T, int M, int K, int N>
SRTM_DEV void mm_nt(const T (&A)[M][K], const T (&B)[N][K], T (&C)[M][N]) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T s = A[i][0] * B[j][0];
#pragma unroll
      for (int k = 1; k < K; ++k) s = my_fma(A[i][k], B[j][k], s);
      C[i][j] = s;
    }
}

// C = A^T B   (A: K x M, B: K x N)
template <typename T, int M, int K, int N>
SRTM_DEV void mm_tn(const T (&A)[K][M], const T (&B)[K][N], T (&C)[M][N]) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T s = A[0][i] * B[0][j];
#pragma unroll
      for (int k = 1; k < K; ++k) s = my_fma(A[k][i], B[k][j], s);
      C[i][j] = s;
    }
}

// S = A B A^T + D for symmetric B and D (upper triangle computed, then mirrored).
template <typename T, int M, int K>
SRTM_DEV void sandwich(const T (&A)[M][K], const T (&B)[K][K], const T (&D)[M][M], T (&S)[M][M]) {
  T AB[M][K];
  mm(A, B, AB);
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = i; j < M; ++j) {
      T s = D[i][j];
#pragma unroll
      for (int k = 0; k < K; ++k) s = my_fma(AB[i][k], A[j][k], s);
      S[i][j] = s;
      S[j][i] = s;
    }
}

// y = A x (+ b)
template <typename T, int M, int K>
SRTM_DEV void mv(const T (&A)[M][K], const T (&x)[K], T (&y)[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = A[i][0] * x[0];
#pragma unroll
    for (int k = 1; k < K; ++k) s = my_fma(A[i][k], x[k], s);
    y[i] = s;
  }
}

template <typename T, int M, int K>
SRTM_DEV void mv_acc(const T (&A)[M][K], const T (&x)[K], T (&y)[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int k = 0; k < K; ++k) y[i] = my_fma(A[i][k], x[k], y[i]);
}

// y = A^T x
template <typename T, int K, int M>
SRTM_DEV void mtv(const T (&A)[K][M], const T (&x)[K], T (&y)[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = A[0][i] * x[0];
#pragma unroll
    for (int k = 1; k < K; ++k) s = my_fma(A[k][i], x[k], s);
    y[i] = s;
  }
}

template <typename T, int R, int C>
SRTM_DEV void symmetrize(T (&A)[R][C]) {
#pragma unroll
  for (int i = 0; i < R; ++i)
#pragma unroll
    for (int j = i + 1; j < C; ++j) {
      T s = T(0.5) * (A[i][j] + A[j][i]);
      A[i][j] = s;
      A[j][i] = s;
    }
}

// Solves A X = B for X (returned in B) by Gaussian elimination with partial pivoting.
// A is destroyed. For each column the row with the strictly largest magnitude is
// brought up by conditional swaps (ties keep the upper row). Returns false when a
// pivot is zero or not finite.
template <typename T, int N, int M>
SRTM_DEV bool solve_pp(T (&A)[N][N], T (&B)[N][M]) {
  bool ok = true;
  T ipiv[N];
#pragma unroll
  for (int c = 0; c < N; ++c) {
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      const bool sw = fabs(A[r][c]) > fabs(A[c][c]);
#pragma unroll
      for (int j = c; j < N; ++j) {
        const T a = A[c][j], b = A[r][j];
        A[c][j] = sw ? b : a;
        A[r][j] = sw ? a : b;
      }
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const T a = B[c][j], b = B[r][j];
        B[c][j] = sw ? b : a;
        B[r][j] = sw ? a : b;
      }
    }
    const T piv = A[c][c];
    ok = ok && (piv != T(0)) && isfinite(piv);
    ipiv[c] = T(1) / piv;
#pragma unroll
    for (int r = c + 1; r < N; ++r) {
      const T f = A[r][c] * ipiv[c];
#pragma unroll
      for (int j = c + 1; j < N; ++j) A[r][j] = my_fma(-f, A[c][j], A[r][j]);
#pragma unroll
      for (int j = 0; j < M; ++j) B[r][j] = my_fma(-f, B[c][j], B[r][j]);
    }
  }
#pragma unroll
  for (int c = N - 1; c >= 0; --c)
#pragma unroll
    for (int j = 0; j < M; ++j) {
      T s = B[c][j];
#pragma unroll
      for (int k = c + 1; k < N; ++k) s = my_fma(-A[c][k], B[k][j], s);
      B[c][j] = s * ipiv[c];
    }
  return ok;
}

// 1/sqrt(s) for s > 0: hardware estimate refined by Newton steps y <- y (3 - s y^2) / 2
// (two steps for double, one for float).
SRTM_DEV double rsqrt_nr(double s) {
  double y = __builtin_amdgcn_rsq(s);
  const double h = 0.5 * s;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
SRTM_DEV float rsqrt_nr(float s) {
  float y = __builtin_amdgcn_rsqf(s);
  const float h = 0.5f * s;
  y = y * fmaf(-h * y, y, 1.5f);
  return y;
}

// 1/x: hardware estimate refined by Newton steps y <- y (2 - x y).
SRTM_DEV double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}
SRTM_DEV float rcp_nr(float x) {
  float y = __builtin_amdgcn_rcpf(x);
  y = y * fmaf(-x, y, 2.0f);
  return y;
}

// Explicit inverse through the adjugate (cofactors over the determinant) for N <= 4: a short
// dependency chain with wide instruction-level parallelism, for the small, well-conditioned
// matrices of the scan combines. Returns false when the determinant is zero or not finite.
template <typename T, int N>
SRTM_DEV bool inv_adj(const T (&a)[N][N], T (&b)[N][N]) {
  static_assert(N >= 1 && N <= 4, "inv_adj: N <= 4");
  T det;
  if constexpr (N == 1) {
    det = a[0][0];
    b[0][0] = T(1);
  } else if constexpr (N == 2) {
    det = a[0][0] * a[1][1] - a[0][1] * a[1][0];
    b[0][0] = a[1][1];
    b[0][1] = -a[0][1];
    b[1][0] = -a[1][0];
    b[1][1] = a[0][0];
  } else if constexpr (N == 3) {
    const T c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
    const T c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
    const T c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
    det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
    b[0][0] = c00;
    b[0][1] = a[0][2] * a[2][1] - a[0][1] * a[2][2];
    b[0][2] = a[0][1] * a[1][2] - a[0][2] * a[1][1];
    b[1][0] = c01;
    b[1][1] = a[0][0] * a[2][2] - a[0][2] * a[2][0];
    b[1][2] = a[0][2] * a[1][0] - a[0][0] * a[1][2];
    b[2][0] = c02;
    b[2][1] = a[0][1] * a[2][0] - a[0][0] * a[2][1];
    b[2][2] = a[0][0] * a[1][1] - a[0][1] * a[1][0];
  } else {
    // 2x2 minors of rows {0,1} (s) and rows {2,3} (c)
    const T s0 = a[0][0] * a[1][1] - a[1][0] * a[0][1], s1 = a[0][0] * a[1][2] - a[1][0] * a[0][2];
    const T s2 = a[0][0] * a[1][3] - a[1][0] * a[0][3], s3 = a[0][1] * a[1][2] - a[1][1] * a[0][2];
    const T s4 = a[0][1] * a[1][3] - a[1][1] * a[0][3], s5 = a[0][2] * a[1][3] - a[1][2] * a[0][3];
    const T c5 = a[2][2] * a[3][3] - a[3][2] * a[2][3], c4 = a[2][1] * a[3][3] - a[3][1] * a[2][3];
    const T c3 = a[2][1] * a[3][2] - a[3][1] * a[2][2], c2 = a[2][0] * a[3][3] - a[3][0] * a[2][3];
    const T c1 = a[2][0] * a[3][2] - a[3][0] * a[2][2], c0 = a[2][0] * a[3][1] - a[3][0] * a[2][1];
    det = s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
    b[0][0] = a[1][1] * c5 - a[1][2] * c4 + a[1][3] * c3;
    b[0][1] = -a[0][1] * c5 + a[0][2] * c4 - a[0][3] * c3;
    b[0][2] = a[3][1] * s5 - a[3][2] * s4 + a[3][3] * s3;
    b[0][3] = -a[2][1] * s5 + a[2][2] * s4 - a[2][3] * s3;
    b[1][0] = -a[1][0] * c5 + a[1][2] * c2 - a[1][3] * c1;
    b[1][1] = a[0][0] * c5 - a[0][2] * c2 + a[0][3] * c1;
    b[1][2] = -a[3][0] * s5 + a[3][2] * s2 - a[3][3] * s1;
    b[1][3] = a[2][0] * s5 - a[2][2] * s2 + a[2][3] * s1;
    b[2][0] = a[1][0] * c4 - a[1][1] * c2 + a[1][3] * c0;
    b[2][1] = -a[0][0] * c4 + a[0][1] * c2 - a[0][3] * c0;
    b[2][2] = a[3][0] * s4 - a[3][1] * s2 + a[3][3] * s0;
    b[2][3] = -a[2][0] * s4 + a[2][1] * s2 - a[2][3] * s0;
    b[3][0] = -a[1][0] * c3 + a[1][1] * c1 - a[1][2] * c0;
    b[3][1] = a[0][0] * c3 - a[0][1] * c1 + a[0][2] * c0;
    b[3][2] = -a[3][0] * s3 + a[3][1] * s1 - a[3][2] * s0;
    b[3][3] = a[2][0] * s3 - a[2][1] * s1 + a[2][2] * s0;
  }
  const T id = rcp_nr(det);
#pragma unroll
  for (int r = 0; r < N; ++r)
#pragma unroll
    for (int c = 0; c < N; ++c) b[r][c] *= id;
  return det != T(0) && isfinite(id);
}

// Inverse of a small general matrix: adjugate for N <= 4, Gaussian elimination with partial
// pivoting against the identity otherwise. Returns false when the matrix is singular.
template <typename T, int N>
SRTM_DEV bool inv_small(const T (&a)[N][N], T (&b)[N][N]) {
  if constexpr (N <= 4) {
    return inv_adj(a, b);
  } else {
    T A[N][N];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        A[r][c] = a[r][c];
        b[r][c] = (r == c) ? T(1) : T(0);
      }
    return solve_pp(A, b);
  }
}

// Inverse of a symmetric positive-definite matrix (N <= 4: adjugate, exactly symmetrised;
// larger N: Cholesky). Returns false when the matrix is not numerically positive definite.
template <typename T, int N>
SRTM_DEV bool spd_inv(const T (&A)[N][N], T (&Ai)[N][N]);

// Lower-triangular L with L L^T = A for a symmetric positive semi-definite A, and the
// reciprocal diagonal idg. A pivot that is not positive gives a zero column (idg = 0).
// Returns false if a pivot was dropped.
template <typename T, int N>
SRTM_DEV bool chol_lower(const T (&A)[N][N], T (&Lf)[N][N], T (&idg)[N]) {
  bool pd = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s = my_fma(-Lf[j][k], Lf[j][k], s);
    const bool pos = s > T(0);
    pd = pd && pos;
    const T d = pos ? rsqrt_nr(s) : T(0);
    idg[j] = d;
    Lf[j][j] = s * d;
#pragma unroll
    for (int i = 0; i < j; ++i) Lf[i][j] = T(0);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = my_fma(-Lf[i][k], Lf[j][k], t);
      Lf[i][j] = t * d;
    }
  }
  return pd;
}

// X = B N^{-T} for lower-triangular N with reciprocal diagonal idg (row-wise forward substitution).
template <typename T, int M, int N>
SRTM_DEV void right_solve_lt(const T (&B)[M][N], const T (&Nf)[N][N], const T (&idg)[N], T (&X)[M][N]) {
#pragma unroll
  for (int r = 0; r < M; ++r)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T t = B[r][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = my_fma(-X[r][k], Nf[j][k], t);
      X[r][j] = t * idg[j];
    }
}

// x = N^{-1} b for lower-triangular N (forward substitution).
template <typename T, int N>
SRTM_DEV void left_solve_l(const T (&Nf)[N][N], const T (&idg)[N], const T (&b)[N], T (&x)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T t = b[j];
#pragma unroll
    for (int k = 0; k < j; ++k) t = my_fma(-Nf[j][k], x[k], t);
    x[j] = t * idg[j];
  }
}

// Inverse of a symmetric positive-definite matrix through its Cholesky factor.
// Returns false when a diagonal pivot is not positive (the result is then garbage).
template <typename T, int N>
SRTM_DEV bool chol_inv(const T (&A)[N][N], T (&Ai)[N][N]) {
  T Lf[N][N];
  T id[N];
  bool ok = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    T s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s = my_fma(-Lf[j][k], Lf[j][k], s);
    ok = ok && (s > T(0));
    id[j] = rsqrt_nr(s);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = my_fma(-Lf[i][k], Lf[j][k], t);
      Lf[i][j] = t * id[j];
    }
  }
  // Li = L^{-1} (lower triangular)
  T Li[N][N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    Li[j][j] = id[j];
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      T s = T(0);
#pragma unroll
      for (int k = j; k < i; ++k) s = my_fma(Lf[i][k], Li[k][j], s);
      Li[i][j] = -s * id[i];
    }
  }
  // A^{-1} = Li^T Li
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      T s = T(0);
#pragma unroll
      for (int k = j; k < N; ++k) s = my_fma(Li[k][i], Li[k][j], s);
      Ai[i][j] = s;
      Ai[j][i] = s;
    }
  return ok;
}

template <typename T> SRTM_DEV bool all_finite(T x) { return isfinite(x); }

// Wave-level barrier with LDS visibility between the lanes of one wavefront.
SRTM_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace srtm

namespace srtm {
template <typename T, int N>
SRTM_DEV bool spd_inv(const T (&A)[N][N], T (&Ai)[N][N]) {
  if constexpr (N <= 4) {
    bool ok = inv_adj(A, Ai);
    symmetrize(Ai);
#pragma unroll
    for (int j = 0; j < N; ++j) ok = ok && (A[j][j] > T(0)) && (Ai[j][j] > T(0));
    return ok;
  } else {
    return chol_inv(A, Ai);
  }
}
}  // namespace srtm
