// Workgroup-level dense linear algebra for one graph per workgroup:
// blocked left-looking Cholesky on FP64 MFMA tiles and the two triangular
// solves that reuse the factor.
//
// Storage: the matrix is row-major with leading dimension npad (a multiple
// of 16); only its lower triangle is read.  After chol_dense it holds the
// factor L (lower) and `linv` holds, for every 16x16 diagonal tile j, the
// inverse of L_jj (row-major, 256 doubles per tile).
//
// MFMA f64 16x16x4 operand layouts (lane l, lq = l / 16, lm = l % 16):
//   A (16 x 4): lane supplies A[lm][k]   with k = lq
//   B (4 x 16): lane supplies B[k][lm]   with k = lq
//   C (16 x 16): lane holds   C[lq + 4 r][lm], r = 0..3
// A reduction index k may be permuted freely as long as A and B agree; the
// kernels below give lane l the four consecutive k = 4 lq + s (s = 0..3) so
// that each lane fetches one 32-byte vector per four MFMAs.
#pragma once

#include <hip/hip_runtime.h>

namespace dnls {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kNT = 256;            // threads per workgroup
constexpr int kNW = kNT / 64;       // waves per workgroup
constexpr int kRB = 4;              // row tiles per wave and pass
constexpr int kTS = 17;             // LDS row stride of a 16x16 tile (bank spread)

struct DenseLds {
  double diag[16 * kTS];
  double inv[16 * kTS];
  double red[16 * kTS];
  int flag;
};

__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Factor the 16x16 SPD tile held in lds.diag (lower part used) on one wave:
// lane i (i < 16) owns row i.  Writes L_jj to lds.diag (full tile, upper
// zero), L_jj^-1 to lds.inv, and returns false if a pivot is not positive.
__device__ inline bool chol16_wave(DenseLds& s) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15;
  double a[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = s.diag[i * kTS + q];
  bool ok = true;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const double piv = __shfl(a[p], p);
    ok = ok && (piv > 0.0);
    const double d = ::sqrt(piv);
    const double lip = (i == p) ? d : (i > p ? a[p] / d : 0.0);
    a[p] = lip;
#pragma unroll
    for (int q = p + 1; q < 16; ++q) {
      const double lqp = __shfl(lip, q);
      if (i >= q) a[q] -= lip * lqp;
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = (q > i) ? 0.0 : a[q];
  // X = L^-1 by forward substitution over rows; lane i owns row i of X
  double x[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) x[c] = (c == i) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double lkk = __shfl(a[k], k);
    if (i == k) {
#pragma unroll
      for (int c = 0; c < 16; ++c) x[c] = x[c] / lkk;
    }
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const double xkc = __shfl(x[c], k);
      if (i > k) x[c] -= a[k] * xkc;
    }
  }
  if (lane < 16) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      s.diag[i * kTS + q] = a[q];
      s.inv[i * kTS + q] = x[q];
    }
  }
  return ok;
}

// In-place blocked left-looking Cholesky of the npad x npad row-major
// matrix A.  All threads of the workgroup must call it.  Returns false
// (uniformly) if the matrix is not numerically positive definite.
__device__ inline bool chol_dense(double* __restrict__ A, int npad, double* __restrict__ linv, DenseLds& s) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lq = lane >> 4;
  const int T = npad >> 4;
  for (int j = 0; j < T; ++j) {
    // Phase A: tiles (i, j), i >= j:  A_ij -= sum_{k<j} L_ik L_jk^T
    for (int i0 = j + wave * kRB; i0 < T; i0 += kNW * kRB) {
      d4v acc[kRB];
#pragma unroll
      for (int t = 0; t < kRB; ++t) {
        const int i = i0 + t;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[t][r] = (i < T) ? A[(size_t)(16 * i + lq + 4 * r) * npad + 16 * j + lm] : 0.0;
      }
      const double* brow = A + (size_t)(16 * j + lm) * npad + 4 * lq;
      for (int k = 0; k < j; ++k) {
        const d4v bv = *reinterpret_cast<const d4v*>(brow + 16 * k);
#pragma unroll
        for (int t = 0; t < kRB; ++t) {
          const int i = i0 + t;
          if (i < T) {
            const d4v av = *reinterpret_cast<const d4v*>(A + (size_t)(16 * i + lm) * npad + 16 * k + 4 * lq);
            acc[t] = mfma16(-av[0], bv[0], acc[t]);
            acc[t] = mfma16(-av[1], bv[1], acc[t]);
            acc[t] = mfma16(-av[2], bv[2], acc[t]);
            acc[t] = mfma16(-av[3], bv[3], acc[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < kRB; ++t) {
        const int i = i0 + t;
        if (i == j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) s.diag[(lq + 4 * r) * kTS + lm] = acc[t][r];
        } else if (i < T) {
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(size_t)(16 * i + lq + 4 * r) * npad + 16 * j + lm] = acc[t][r];
        }
      }
    }
    __syncthreads();
    // Phase B: factor and invert the diagonal tile
    if (wave == 0) {
      const bool ok = chol16_wave(s);
      if (lane == 0) s.flag = ok ? 0 : 1;
      if (lane < 16) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          A[(size_t)(16 * j + lane) * npad + 16 * j + q] = s.diag[lane * kTS + q];
          linv[j * 256 + lane * 16 + q] = s.inv[lane * kTS + q];
        }
      }
    }
    __syncthreads();
    if (s.flag) return false;
    // Phase C: L_ij = A_ij L_jj^-T for i > j
    for (int i0 = j + 1 + wave * kRB; i0 < T; i0 += kNW * kRB) {
      d4v acc[kRB];
      double bk[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) bk[q] = s.inv[lm * kTS + 4 * lq + q];
#pragma unroll
      for (int t = 0; t < kRB; ++t) {
        acc[t] = d4v{0.0, 0.0, 0.0, 0.0};
        const int i = i0 + t;
        if (i < T) {
          const d4v av = *reinterpret_cast<const d4v*>(A + (size_t)(16 * i + lm) * npad + 16 * j + 4 * lq);
          acc[t] = mfma16(av[0], bk[0], acc[t]);
          acc[t] = mfma16(av[1], bk[1], acc[t]);
          acc[t] = mfma16(av[2], bk[2], acc[t]);
          acc[t] = mfma16(av[3], bk[3], acc[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < kRB; ++t) {
        const int i = i0 + t;
        if (i < T) {
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(size_t)(16 * i + lq + 4 * r) * npad + 16 * j + lm] = acc[t][r];
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// x <- L^-1 x  (x in LDS, length npad); all threads call.
__device__ inline void trsv_lower(const double* __restrict__ L, int npad, const double* __restrict__ linv,
                                  double* x, DenseLds& s) {
  const int T = npad >> 4;
  const int r = threadIdx.x >> 4, q = threadIdx.x & 15;
  for (int j = 0; j < T; ++j) {
    double acc = 0.0;
    const double* row = L + (size_t)(16 * j + r) * npad;
    for (int c = q; c < 16 * j; c += 16) acc += row[c] * x[c];
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (q == 0) s.red[r] = x[16 * j + r] - acc;
    __syncthreads();
    if (threadIdx.x < 16) {
      const double* li = linv + j * 256 + threadIdx.x * 16;
      double y = 0.0;
      for (int c = 0; c <= (int)threadIdx.x; ++c) y += li[c] * s.red[c];
      x[16 * j + threadIdx.x] = y;
    }
    __syncthreads();
  }
}

// x <- L^-T x  (x in LDS, length npad); all threads call.
__device__ inline void trsv_upper_t(const double* __restrict__ L, int npad, const double* __restrict__ linv,
                                    double* x, DenseLds& s) {
  const int T = npad >> 4;
  const int c = threadIdx.x & 15, q = threadIdx.x >> 4;
  for (int j = T - 1; j >= 0; --j) {
    double acc = 0.0;
    for (int r = 16 * (j + 1) + q; r < npad; r += 16) acc += L[(size_t)r * npad + 16 * j + c] * x[r];
    s.red[q * kTS + c] = acc;
    __syncthreads();
    if (threadIdx.x < 16) {
      double z = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) z += s.red[k * kTS + threadIdx.x];
      s.diag[threadIdx.x] = x[16 * j + threadIdx.x] - z;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
      // x_j[c] = sum_r Linv[r][c] z[r], Linv lower: r >= c
      const double* li = linv + j * 256;
      double y = 0.0;
      for (int rr = threadIdx.x; rr < 16; ++rr) y += li[rr * 16 + threadIdx.x] * s.diag[rr];
      x[16 * j + threadIdx.x] = y;
    }
    __syncthreads();
  }
}

}  // namespace dnls
