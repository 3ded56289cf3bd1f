// Workgroup-level dense linear algebra, one graph per workgroup (256 threads):
// blocked left-looking Cholesky on FP64 MFMA tiles and the triangular solves
// that reuse the factor.
//
// Storage: row-major, leading dimension npad (a multiple of 64), only the
// lower triangle is read.  The buffer has 16 extra rows: row npad holds the
// right-hand side b^T, and the factorisation writes y = L^-1 b into row npad
// of the factor (the forward substitution rides along: the diagonal group of
// each panel forms b_J - sum_k L_Jk y_k from the panel rows it stages
// anyway, and y_J = L_JJ^-1 of that); rows npad + 1 .. npad + 15 are padding.
// After chol_dense the lower triangle holds L, and winv[J] (64 x 64 row-major
// per panel) holds L_JJ^-1 of every diagonal 64 x 64 block.
//
// MFMA f64 16x16x4 operand layouts (lane l, lq = l / 16, lm = l % 16):
//   A (16 x 4): lane supplies A[lm][k]     B (4 x 16): lane supplies B[k][lm]
//   C (16 x 16): lane holds C[lq + 4 r][lm], r = 0..3
// Within one 16-wide k tile, MFMA number s gives lane l the index
// k = 4 lq + s for A and B alike (a permutation of k, so the sum is
// unchanged) and each lane fetches one 32-byte vector for four MFMAs.
//
// The panel update computes the transposed tile D^T = A_iJ^T - L_J L_i^T:
// its C layout puts row lm of D in lane lm with columns lq + 4 r in the four
// registers, which is exactly the A-operand layout needed by the triangular
// solve D L_JJ^-T that follows -- no transpose through LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace dnls {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kNT = 256;             // threads per workgroup
constexpr int kNW = kNT / 64;        // waves per workgroup
constexpr int kNB = 64;              // panel width
constexpr int kSP = 68;              // LDS row stride (doubles) of a 64-wide panel
constexpr int kMaxDenseN = 2048;     // npad limit of the one-workgroup dense path

struct DenseLds {
  double stage[2][kNB * kSP];        // double-buffered panel chunk L_J[0:64][k0:k0+64]
  double W[kNB * kSP];               // L_JJ^-1 of the current panel
  double vec[kNB];                   // broadcast vector of the solves
  double red[kNW];
  int flag;
};

__device__ __forceinline__ d4v mfma16(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// acc += A (16x16 at a, row stride lda) * M^T (M 16x16 at m, row stride ldm)
__device__ __forceinline__ void mma_abt(d4v& acc, const double* a, int lda, const double* m, int ldm, double sign) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  const d4v av = *reinterpret_cast<const d4v*>(a + lm * lda + 4 * lq);
  const d4v bv = *reinterpret_cast<const d4v*>(m + lm * ldm + 4 * lq);
  acc = mfma16(sign * av[0], bv[0], acc);
  acc = mfma16(sign * av[1], bv[1], acc);
  acc = mfma16(sign * av[2], bv[2], acc);
  acc = mfma16(sign * av[3], bv[3], acc);
}

// acc += A (16x16 at a, stride lda) * M (16x16 at m, stride ldm)
__device__ __forceinline__ void mma_ab(d4v& acc, const double* a, int lda, const double* m, int ldm, double sign) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  const d4v av = *reinterpret_cast<const d4v*>(a + lm * lda + 4 * lq);
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = mfma16(sign * av[s], m[(4 * lq + s) * ldm + lm], acc);
}

// C-layout accumulator -> 16x16 tile at t (stride ldt)
__device__ __forceinline__ void store_tile(double* t, int ldt, const d4v& acc) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[(lq + 4 * r) * ldt + lm] = acc[r];
}
__device__ __forceinline__ d4v load_tile(const double* t, int ldt) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  d4v acc;
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = t[(lq + 4 * r) * ldt + lm];
  return acc;
}

// Broadcast of lane q of each 16-lane row to the whole row: one 64-bit DPP
// move with row_newbcast (every source lane is valid, so no previous value
// is needed).
__device__ __forceinline__ double bcast16(double v, int q) {
  switch (q) {
    case 0: return __builtin_amdgcn_mov_dpp(v, 0x150, 0xf, 0xf, true);
    case 1: return __builtin_amdgcn_mov_dpp(v, 0x151, 0xf, 0xf, true);
    case 2: return __builtin_amdgcn_mov_dpp(v, 0x152, 0xf, 0xf, true);
    case 3: return __builtin_amdgcn_mov_dpp(v, 0x153, 0xf, 0xf, true);
    case 4: return __builtin_amdgcn_mov_dpp(v, 0x154, 0xf, 0xf, true);
    case 5: return __builtin_amdgcn_mov_dpp(v, 0x155, 0xf, 0xf, true);
    case 6: return __builtin_amdgcn_mov_dpp(v, 0x156, 0xf, 0xf, true);
    case 7: return __builtin_amdgcn_mov_dpp(v, 0x157, 0xf, 0xf, true);
    case 8: return __builtin_amdgcn_mov_dpp(v, 0x158, 0xf, 0xf, true);
    case 9: return __builtin_amdgcn_mov_dpp(v, 0x159, 0xf, 0xf, true);
    case 10: return __builtin_amdgcn_mov_dpp(v, 0x15a, 0xf, 0xf, true);
    case 11: return __builtin_amdgcn_mov_dpp(v, 0x15b, 0xf, 0xf, true);
    case 12: return __builtin_amdgcn_mov_dpp(v, 0x15c, 0xf, 0xf, true);
    case 13: return __builtin_amdgcn_mov_dpp(v, 0x15d, 0xf, 0xf, true);
    case 14: return __builtin_amdgcn_mov_dpp(v, 0x15e, 0xf, 0xf, true);
    default: return __builtin_amdgcn_mov_dpp(v, 0x15f, 0xf, 0xf, true);
  }
}

// Cholesky factor and inverse of the 16x16 SPD tile at t (stride ldt, lower
// part read) on one wave: lane i (i = lane % 16) of each 16-lane row owns
// row i; the column values each step needs are broadcast within the 16-lane
// row by DPP.  The factorisation runs in all four rows alike; entries above
// the diagonal are carried along unmasked (they never feed the lower part)
// and cleared at the end.  The inverse is formed from unscaled rows
// y_i = e_i - sum_{k<i} (L_ik / L_kk) y_k, then L^-1 row i = y_i / L_ii,
// reusing 1/L_kk from the factorisation; its columns are dealt to the four
// rows (row g takes the columns 4 m + g; entries right of the diagonal of
// every y_k are zero, so all four columns take every step).  Writes L (upper
// part zero) back to t and L^-1 to w.  Returns false if a pivot is not
// positive (NaN included).
__device__ __forceinline__ bool chol16_wave(double* t, int ldt, double* w, int ldw) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  double a[16], rdv[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) a[q] = t[i * ldt + q];
  bool ok = true;
  double myrd = 0.0;
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const double piv = bcast16(a[p], p);
    ok = ok && (piv > 0.0);
    const double rd = rsqrt(piv);            // 1 / L_pp
    rdv[p] = rd;
    myrd = (i == p) ? rd : myrd;
    const double lip = a[p] * rd;            // L_ip for i >= p (L_pp = piv / sqrt(piv))
    a[p] = lip;
#pragma unroll
    for (int q = p + 1; q < 16; ++q) a[q] = __builtin_fma(-lip, bcast16(lip, q), a[q]);
  }
  double y[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) y[m] = (4 * m + g == i) ? 1.0 : 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double coef = (k < i) ? a[k] * rdv[k] : 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) y[m] = __builtin_fma(-coef, bcast16(y[m], k), y[m]);
  }
  if (lane < 16) {
#pragma unroll
    for (int q = 0; q < 16; ++q) t[i * ldt + q] = (q > i) ? 0.0 : a[q];
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) w[i * ldw + 4 * m + g] = y[m] * myrd;
  return ok;
}

// Factor the (16 NBLK)^2 diagonal block D (LDS, stride kSP, lower part read)
// in place into L_JJ, and its inverse into W (stride kSP, lower blocks).  All
// threads of a workgroup of at least four waves call (NBLK <= 4).  Per block
// column b: the waves form L_rb = D_rb W_bb^T (r > b) and, on the waves left
// over, the inverse blocks of row b, W_bc = -W_bb sum_{k=c}^{b-1} L_bk W_kc
// (c < b); then wave 0 updates D_{b+1,b+1} and factors it while the other
// waves update the rest of the trailing blocks, D_rc -= L_rb L_cb^T.  Two
// barriers per block column.
template <int NBLK>
__device__ __forceinline__ bool chol_block(double* D, double* W, DenseLds& s, int nlive = NBLK) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  const int nw = blockDim.x >> 6;
  auto dblk = [&](int r, int c) { return D + 16 * r * kSP + 16 * c; };
  auto wblk = [&](int r, int c) { return W + 16 * r * kSP + 16 * c; };
  bool ok = true;
  if (wave == 0) {
    const bool okb = chol16_wave(dblk(0, 0), kSP, wblk(0, 0), kSP);
    if (lane == 0) s.flag = okb ? 0 : 1;
  }
  __syncthreads();
  for (int b = 0; b < nlive; ++b) {
    if (s.flag) ok = false;
    const int ntr = nlive - 1 - b;  // blocks below the diagonal in column b
    if (wave < ntr) {
      const int r = b + 1 + wave;
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      mma_abt(acc, dblk(r, b), kSP, wblk(b, b), kSP, 1.0);
      store_tile(dblk(r, b), kSP, acc);
    } else if (wave - ntr < b) {
      const int c = wave - ntr;
      d4v tt = {0.0, 0.0, 0.0, 0.0};
      for (int k = c; k < b; ++k) mma_ab(tt, dblk(b, k), kSP, wblk(k, c), kSP, 1.0);
      // -W_bb T with T in the accumulator layout as the B operand: lane
      // (lm, lq) holds T[lq + 4 r][lm], so MFMA number r takes k = lq + 4 r
      const double* wbb = wblk(b, b) + lm * kSP + lq;
      d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = mfma16(-wbb[4 * r], tt[r], acc);
      store_tile(wblk(b, c), kSP, acc);
    }
    __syncthreads();
    if (b + 1 < nlive) {
      if (wave == 0) {
        d4v acc = load_tile(dblk(b + 1, b + 1), kSP);
        mma_abt(acc, dblk(b + 1, b), kSP, dblk(b + 1, b), kSP, -1.0);
        store_tile(dblk(b + 1, b + 1), kSP, acc);
        const bool okb = chol16_wave(dblk(b + 1, b + 1), kSP, wblk(b + 1, b + 1), kSP);
        if (lane == 0) s.flag = okb ? 0 : 1;
      } else {
        int idx = 0;
        for (int r = b + 1; r < nlive; ++r)
          for (int c = b + 1; c <= r; ++c) {
            if (r == b + 1 && c == b + 1) continue;
            if (idx++ % (nw - 1) + 1 == wave) {
              d4v acc = load_tile(dblk(r, c), kSP);
              mma_abt(acc, dblk(r, b), kSP, dblk(c, b), kSP, -1.0);
              store_tile(dblk(r, c), kSP, acc);
            }
          }
      }
      __syncthreads();
    }
  }
  // blocks past the live ones hold unit diagonal padding (their coupling to
  // the live unknowns is zero): L = I there already, and its inverse is I
  if (nlive < NBLK) {
    for (int e = threadIdx.x; e < (NBLK - nlive) * 16 * 16 * NBLK; e += blockDim.x) {
      const int r = 16 * nlive + e / (16 * NBLK), c = e % (16 * NBLK);
      W[r * kSP + c] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
  }
  return ok;
}

// Forward substitution of the diagonal group, three pieces.  The thread
// (srow, scol) of the chunk staging holds L_J[srow][k + scol .. + 15] of the
// chunk at column k in st; y[0 : 64 J] sits flat in LDS at y.
__device__ __forceinline__ double ydot16(const d4v st[4], const double* y) {
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const d4v w = *reinterpret_cast<const d4v*>(y + 4 * q);
    v = __builtin_fma(st[q][0], w[0], v);
    v = __builtin_fma(st[q][1], w[1], v);
    v = __builtin_fma(st[q][2], w[2], v);
    v = __builtin_fma(st[q][3], w[3], v);
  }
  return v;
}

// sum of v over the four threads of a staging row (lanes 4 r .. 4 r + 3)
__device__ __forceinline__ double row4_sum(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  return v;
}

// y_J = L_JJ^-1 t (W = L_JJ^-1 at stride kSP, lower part; t = s.vec) written
// to y[col0 ..]: thread (srow, scol) takes 16 columns, four threads a row.
__device__ __forceinline__ void ypanel(const double* W, const double* t, double* y, int col0) {
  const int srow = threadIdx.x >> 2, scol = (threadIdx.x & 3) * 16;
  double v = 0.0;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int c = scol + e;
    v += (c <= srow) ? W[srow * kSP + c] * t[c] : 0.0;
  }
  v = row4_sum(v);
  if ((threadIdx.x & 3) == 0) y[col0 + srow] = v;
}

// 16-row blocks of the 64-wide diagonal block at column col0 that hold
// unknowns (n < 0: all four); the rest is the unit-diagonal padding
__device__ __forceinline__ int live_blocks(int n, int col0) {
  if (n < 0 || n >= col0 + kNB) return 4;
  return max(1, (n - col0 + 15) >> 4);
}

// dst (64x64, global, row stride ld; kNB for store_inv) <- the lower
// triangle of W (LDS, stride kSP), zeros above it; and the way back.  Four
// values per thread and access.  All threads call.
__device__ __forceinline__ void store_lower(double* __restrict__ dst, int ld, const double* W) {
  for (int e = threadIdx.x; e < kNB * kNB / 4; e += kNT) {
    const int rr = e >> 4, c = (e & 15) * 4;
    d4v v = *reinterpret_cast<const d4v*>(W + rr * kSP + c);
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (c + k <= rr) ? v[k] : 0.0;
    *reinterpret_cast<d4v*>(dst + (size_t)rr * ld + c) = v;
  }
}
__device__ __forceinline__ void store_inv(double* __restrict__ dst, const double* W) { store_lower(dst, kNB, W); }
__device__ __forceinline__ void load_inv(double* W, const double* __restrict__ src) {
  for (int e = threadIdx.x; e < kNB * kNB / 4; e += kNT) {
    const int rr = e >> 4, c = (e & 15) * 4;
    *reinterpret_cast<d4v*>(W + rr * kSP + c) = *reinterpret_cast<const d4v*>(src + rr * kNB + c);
  }
}

// Chunk loop of a panel's diagonal tile (J, J): its own rows are the staged
// panel rows, so each chunk is loaded once (no separate own-row operand),
// two chunks ahead; adds -sum_k L_Jk L_Jk^T to acc (wave w: rows 16 w ..
// 16 w + 15, transposed accumulator layout) and this thread's part of
// sum_k L_Jk y_k to ypart.  y of the panels before col0 must be in yrow;
// s.W is used for it.  All threads call, nchunk > 0.
__device__ __forceinline__ void diag_chunks(const double* A, int npad, int col0, int nchunk, const double* yrow,
                                            DenseLds& s, d4v (&acc)[4], double& ypart) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lq = lane >> 4;
  const int srow = threadIdx.x >> 2, scol = (threadIdx.x & 3) * 16;
  const double* Brow = A + (size_t)(col0 + srow) * npad + scol;
  d4v st1[4], st2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) st1[q] = *reinterpret_cast<const d4v*>(Brow + 4 * q);
  for (int u = threadIdx.x; u < col0; u += kNT) s.W[u] = yrow[u];
#pragma unroll
  for (int q = 0; q < 4; ++q) *reinterpret_cast<d4v*>(&s.stage[0][srow * kSP + scol + 4 * q]) = st1[q];
  if (nchunk > 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) st1[q] = *reinterpret_cast<const d4v*>(Brow + kNB + 4 * q);
  }
  if (nchunk > 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) st2[q] = *reinterpret_cast<const d4v*>(Brow + 2 * kNB + 4 * q);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* buf = s.stage[ch & 1];
    {
      d4v sv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) sv[q] = *reinterpret_cast<const d4v*>(buf + srow * kSP + scol + 4 * q);
      ypart += ydot16(sv, s.W + kNB * ch + scol);
    }
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
      d4v aop[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) aop[c] = *reinterpret_cast<const d4v*>(buf + (16 * c + lm) * kSP + 16 * kt + 4 * lq);
      const d4v bv = *reinterpret_cast<const d4v*>(buf + (16 * wave + lm) * kSP + 16 * kt + 4 * lq);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = mfma16(-aop[c][q], bv[q], acc[c]);
    }
    if (ch + 1 < nchunk) {
#pragma unroll
      for (int q = 0; q < 4; ++q) *reinterpret_cast<d4v*>(&s.stage[(ch + 1) & 1][srow * kSP + scol + 4 * q]) = st1[q];
      if (ch + 2 < nchunk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) st1[q] = st2[q];
      }
      if (ch + 3 < nchunk) {
#pragma unroll
        for (int q = 0; q < 4; ++q) st2[q] = *reinterpret_cast<const d4v*>(Brow + kNB * (ch + 3) + 4 * q);
      }
    }
    __syncthreads();
  }
}

// Blocked left-looking Cholesky of the (npad + 16) x npad row-major matrix H
// (row npad = right-hand side; lower part read) into L (same layout; L may
// be H itself): on return L holds the factor and y = L^-1 b in row npad,
// winv holds the inverses of the diagonal blocks.  H is only read, so a
// caller can keep its structural zeros across factorisations.  All threads
// call; returns false (uniformly) if the matrix is not positive definite.
__device__ __forceinline__ bool chol_dense(double* A, const double* H, int npad, double* __restrict__ winv, DenseLds& s,
                                           int n = -1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lq = lane >> 4;
  const int T16 = npad >> 4;          // row tiles of the matrix
  const int P = npad / kNB;
  const int srow = threadIdx.x >> 2, scol = (threadIdx.x & 3) * 16;
  const double* hb = H + (size_t)npad * npad;   // b
  double* yrow = A + (size_t)npad * npad;       // y = L^-1 b
  bool ok = true;
  // the next group's H tile (transposed accumulator layout) and chunk 0 of
  // its own rows, loaded while the current group finishes (its triangular
  // solve, or for the diagonal group the write-back of L_JJ)
  d4v acc_n[4], bop_n[4];
  auto prefetch = [&](int J, int i0n) {
    const int in = i0n + wave, col0 = kNB * J;
    const double* Hr = H + (size_t)(16 * in + lm) * npad;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc_n[c][r] = Hr[col0 + 16 * c + lq + 4 * r];
    if (J > 0) {
      const double* Ar = A + (size_t)(16 * in + lm) * npad;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) bop_n[kt] = *reinterpret_cast<const d4v*>(Ar + 16 * kt + 4 * lq);
    }
  };
  prefetch(0, 0);
  for (int J = 0; J < P; ++J) {
    const int col0 = kNB * J;
    const int nchunk = J;             // k chunks of 64 columns
    for (int i0 = 4 * J; i0 < T16; i0 += kNW) {
      const int i = i0 + wave;
      const double* Arow = A + (size_t)(16 * i + lm) * npad;
      const bool diag = i0 == 4 * J;
      const bool last_group = i0 + kNW >= T16;
      // transposed accumulators: acc[c][r] = D[lm][16 c + lq + 4 r] for tile (i, J)
      d4v acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = acc_n[c];
      // diagonal group: sum_k L_Jk y_k (this thread's row srow, 16 columns of each chunk)
      double ypart = 0.0;
      if (nchunk > 0 && diag) {
        diag_chunks(A, npad, col0, nchunk, yrow, s, acc, ypart);
      } else if (nchunk > 0) {
        d4v st[4], bop[4], bnx[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) st[q] = *reinterpret_cast<const d4v*>(A + (size_t)(col0 + srow) * npad + scol + 4 * q);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) bop[kt] = bop_n[kt];
        // y of the panels before J, flat in W (L_{J-1,J-1}^-1 is no longer needed)
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<d4v*>(&s.stage[0][srow * kSP + scol + 4 * q]) = st[q];
        __syncthreads();
        for (int ch = 0; ch < nchunk; ++ch) {
          const bool more = ch + 1 < nchunk;
          const int k1 = kNB * (ch + 1);
          // st still holds this thread's part of chunk ch
          if (more) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              st[q] = *reinterpret_cast<const d4v*>(A + (size_t)(col0 + srow) * npad + k1 + scol + 4 * q);
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) bnx[kt] = *reinterpret_cast<const d4v*>(Arow + k1 + 16 * kt + 4 * lq);
          }
          const double* buf = s.stage[ch & 1];
#pragma unroll
          for (int kt = 0; kt < 4; ++kt) {
            d4v aop[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) aop[c] = *reinterpret_cast<const d4v*>(buf + (16 * c + lm) * kSP + 16 * kt + 4 * lq);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int c = 0; c < 4; ++c) acc[c] = mfma16(-aop[c][q], bop[kt][q], acc[c]);
          }
          if (more) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              *reinterpret_cast<d4v*>(&s.stage[(ch + 1) & 1][srow * kSP + scol + 4 * q]) = st[q];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) bop[kt] = bnx[kt];
          }
          __syncthreads();
        }
      }
      if (diag) {
        // t = b_J - sum_k L_Jk y_k for the forward substitution
        ypart = row4_sum(ypart);
        if ((threadIdx.x & 3) == 0) s.vec[srow] = hb[col0 + srow] - ypart;
        // the diagonal block: factor in LDS
        double* D = s.stage[0];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) D[(16 * wave + lm) * kSP + 16 * c + lq + 4 * r] = acc[c][r];
        __syncthreads();
        if (!chol_block<4>(D, s.W, s, live_blocks(n, col0))) ok = false;
        if (!last_group) prefetch(J, i0 + kNW);
        // write L_JJ (zero above the diagonal), its inverse and y_J = L_JJ^-1 t
        store_inv(winv + (size_t)J * kNB * kNB, s.W);
        store_lower(A + (size_t)col0 * npad + col0, npad, D);
        ypanel(s.W, s.vec, yrow, col0);
        __syncthreads();
      } else {
        // the next group's loads (H, and L of panels before J) overlap this
        // group's triangular solve, which writes panel J only
        if (!last_group) prefetch(J, i0 + kNW);
        // L_iJ = D L_JJ^-T:  out[m][n] = sum_k D[m][k] W[n][k]
#pragma unroll
        for (int cn = 0; cn < 4; ++cn) {
          d4v out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kt = 0; kt <= cn; ++kt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) out = mfma16(acc[kt][q], s.W[(16 * cn + lm) * kSP + 16 * kt + lq + 4 * q], out);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(size_t)(16 * i + lq + 4 * r) * npad + col0 + 16 * cn + lm] = out[r];
        }
      }
    }
    __syncthreads();
    // the diagonal group of the next panel reads L of panel 0 (its chunk 0),
    // which for J = 0 is written by this panel: load after the barrier
    if (J + 1 < P) prefetch(J + 1, 4 * (J + 1));
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Several workgroups per graph (a pair for the pose-graph solve, four for the
// bundle-adjustment camera system) share one factorisation, each taking every
// nway-th group of row tiles of a panel (the leader, role 0, starts with the
// diagonal group), with three kinds of events posted through monotone
// 64-bit counters in device memory (agent-scope release / acquire): the
// leader's diagonal block of panel J written (the follower then reads
// L_JJ^-1 from the factor cache), and each role's end of panel J (both wait
// for the other before the next panel, whose updates read every row's L).
// Waits are bounded: after `spin` polls the wait fails and the caller gives
// up the graph instead of hanging.  The pair must be co-resident, which the
// cooperative launch of the caller guarantees.
// ---------------------------------------------------------------------------
struct PairSync {
  unsigned long long* lead_h;     // leader: the system of factorisation f is assembled (base + f + 1)
  unsigned long long* lead_stop;  // leader: left its loop (base + 1)
  unsigned long long* lead_diag;  // leader: diagonal block J of factorisation f written (base + f P + J + 1)
  unsigned long long* panel;      // [nway] role r: panel J of factorisation f finished (base + f P + J + 1)
  unsigned long long base;        // this launch's origin of the counters
  int role;                       // 0 = leader
  int nway;                       // workgroups sharing the factorisation (2 for the pair)
  int spin;                       // poll limit of a wait
};

// all threads call: every wave waits until its stores have completed
// (vmcnt 0), then after the barrier one thread makes them visible at agent
// scope (one release fence, i.e. one L2 write-back, per event) and
// publishes v
__device__ __forceinline__ void pair_post(unsigned long long* ctr, unsigned long long v) {
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0), expcnt and lgkmcnt left at their maxima
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(ctr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// all threads call: thread 0 polls (relaxed loads, no cache invalidation per
// poll) until *ctr >= target (or *stop >= stop_at when stop is given), then
// one acquire fence makes the partner's data visible; returns false on
// timeout or stop, uniformly
__device__ __forceinline__ bool pair_wait(const unsigned long long* ctr, unsigned long long target,
                                          const unsigned long long* stop, int spin, DenseLds& s,
                                          unsigned long long stop_at = 0) {
  if (threadIdx.x == 0) {
    int ok = 0;
    for (int n = 0; n < spin; ++n) {
      if (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      if (stop && __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= stop_at) break;
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s.flag = ok;
  }
  __syncthreads();
  const bool ok = s.flag != 0;
  __syncthreads();
  return ok;
}

// Blocked left-looking Cholesky as chol_dense, shared by the pair of
// workgroups described above; f numbers the factorisation within the launch.
// Returns the leader's positive-definiteness verdict (the follower's value is
// meaningless); sets bail (and returns false) if a wait timed out.
__device__ __forceinline__ bool chol_dense_pair(double* A, const double* H, int npad, double* __restrict__ winv,
                                                DenseLds& s, const PairSync& ps, int f, bool& bail) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lq = lane >> 4;
  const int T16 = npad >> 4;          // row tiles of the matrix
  const int P = npad / kNB;
  const int srow = threadIdx.x >> 2, scol = (threadIdx.x & 3) * 16;
  const double* hb = H + (size_t)npad * npad;   // b
  double* yrow = A + (size_t)npad * npad;       // y = L^-1 b (the leader's)
  bool ok = true;
  // the next group's H tile (transposed accumulator layout) and chunk 0 of
  // its own rows, loaded while the current group finishes (its triangular
  // solve, or for the diagonal group the write-back of L_JJ)
  d4v acc_n[4], bop_n[4];
  auto prefetch = [&](int J, int i0n) {
    const int in = i0n + wave, col0 = kNB * J;
    const double* Hr = H + (size_t)(16 * in + lm) * npad;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc_n[c][r] = Hr[col0 + 16 * c + lq + 4 * r];
    if (J > 0) {
      const double* Ar = A + (size_t)(16 * in + lm) * npad;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) bop_n[kt] = *reinterpret_cast<const d4v*>(Ar + 16 * kt + 4 * lq);
    }
  };
  // this role's row groups of a panel: every nway-th group of 4 row tiles,
  // the leader's starting with the diagonal group
  const int first = ps.role * kNW, stride = ps.nway * kNW;
  const unsigned long long fbase = ps.base + (unsigned long long)f * P;
  if (first < T16) prefetch(0, first);
  for (int J = 0; J < P; ++J) {
    const int col0 = kNB * J;
    const int nchunk = J;             // k chunks of 64 columns
    bool have_w = ps.role == 0;       // the leader factors the diagonal block itself
    for (int i0 = 4 * J + first; i0 < T16; i0 += stride) {
      const int i = i0 + wave;
      const double* Arow = A + (size_t)(16 * i + lm) * npad;
      const bool diag = i0 == 4 * J;
      const bool last_group = i0 + stride >= T16;
      // transposed accumulators: acc[c][r] = D[lm][16 c + lq + 4 r] for tile (i, J)
      d4v acc[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] = acc_n[c];
      // diagonal group: sum_k L_Jk y_k (this thread's row srow, 16 columns of each chunk)
      double ypart = 0.0;
      if (nchunk > 0 && diag) {
        diag_chunks(A, npad, col0, nchunk, yrow, s, acc, ypart);
      } else if (nchunk > 0) {
        d4v st[4], bop[4], bnx[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) st[q] = *reinterpret_cast<const d4v*>(A + (size_t)(col0 + srow) * npad + scol + 4 * q);
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) bop[kt] = bop_n[kt];
        // y of the panels before J, flat in W (L_{J-1,J-1}^-1 is no longer needed)
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<d4v*>(&s.stage[0][srow * kSP + scol + 4 * q]) = st[q];
        __syncthreads();
        for (int ch = 0; ch < nchunk; ++ch) {
          const bool more = ch + 1 < nchunk;
          const int k1 = kNB * (ch + 1);
          // st still holds this thread's part of chunk ch
          if (more) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              st[q] = *reinterpret_cast<const d4v*>(A + (size_t)(col0 + srow) * npad + k1 + scol + 4 * q);
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) bnx[kt] = *reinterpret_cast<const d4v*>(Arow + k1 + 16 * kt + 4 * lq);
          }
          const double* buf = s.stage[ch & 1];
#pragma unroll
          for (int kt = 0; kt < 4; ++kt) {
            d4v aop[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) aop[c] = *reinterpret_cast<const d4v*>(buf + (16 * c + lm) * kSP + 16 * kt + 4 * lq);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int c = 0; c < 4; ++c) acc[c] = mfma16(-aop[c][q], bop[kt][q], acc[c]);
          }
          if (more) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              *reinterpret_cast<d4v*>(&s.stage[(ch + 1) & 1][srow * kSP + scol + 4 * q]) = st[q];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) bop[kt] = bnx[kt];
          }
          __syncthreads();
        }
      }
      if (diag) {
        // t = b_J - sum_k L_Jk y_k for the forward substitution
        ypart = row4_sum(ypart);
        if ((threadIdx.x & 3) == 0) s.vec[srow] = hb[col0 + srow] - ypart;
        // the diagonal block: factor in LDS
        double* D = s.stage[0];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) D[(16 * wave + lm) * kSP + 16 * c + lq + 4 * r] = acc[c][r];
        __syncthreads();
        if (!chol_block<4>(D, s.W, s)) ok = false;
        if (!last_group) prefetch(J, i0 + stride);
        // write L_JJ (zero above the diagonal), its inverse and y_J = L_JJ^-1 t
        store_inv(winv + (size_t)J * kNB * kNB, s.W);
        store_lower(A + (size_t)col0 * npad + col0, npad, D);
        ypanel(s.W, s.vec, yrow, col0);
        __syncthreads();
        pair_post(ps.lead_diag, fbase + J + 1);
      } else {
        if (!have_w) {
          // the follower takes L_JJ^-1 from the leader's write-back
          if (!pair_wait(ps.lead_diag, fbase + J + 1, nullptr, ps.spin, s)) {
            bail = true;
            return false;
          }
          load_inv(s.W, winv + (size_t)J * kNB * kNB);
          __syncthreads();
          have_w = true;
        }
        // the next group's loads (H, and L of panels before J) overlap this
        // group's triangular solve, which writes panel J only
        if (!last_group) prefetch(J, i0 + stride);
        // L_iJ = D L_JJ^-T:  out[m][n] = sum_k D[m][k] W[n][k]
#pragma unroll
        for (int cn = 0; cn < 4; ++cn) {
          d4v out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int kt = 0; kt <= cn; ++kt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) out = mfma16(acc[kt][q], s.W[(16 * cn + lm) * kSP + 16 * kt + lq + 4 * q], out);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(size_t)(16 * i + lq + 4 * r) * npad + col0 + 16 * cn + lm] = out[r];
        }
      }
    }
    __syncthreads();
    // every role has written its tiles of panel J
    pair_post(ps.panel + ps.role, fbase + J + 1);
    for (int r = 0; r < ps.nway; ++r)
      if (r != ps.role && !pair_wait(ps.panel + r, fbase + J + 1, nullptr, ps.spin, s)) {
        bail = true;
        return false;
      }
    if (J + 1 < P && 4 * (J + 1) + first < T16) prefetch(J + 1, 4 * (J + 1) + first);
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Pair factorisation with row ownership and look-ahead (the pose-graph solve
// with DNLS_FLAG_PAIR).  Row group r (rows 64 r .. 64 r + 63) belongs to the
// workgroup of role r mod 2, which computes every tile (r, J), J <= r, of it
// in panel order, so its own rows never need a wait.  Role w runs
//   [w = 1: the tile (1, 0)]
//   for J = w, w + 2, ...:  the diagonal tile (J, J);
//                           its rows' tiles of panel J - 1 (r >= J + 2);
//                           its rows' tiles of panel J (r >= J + 2);
//                           the look-ahead tile (J + 2, J + 1)
// and the look-ahead tile is what the next diagonal tile waits for, so the
// chain diagonal block -> look-ahead tile -> next diagonal block no longer
// waits for the rest of a panel.  Events (monotone counters, this
// factorisation's origin fbase = base + f P): diag = fbase + J + 1 when
// L_JJ, L_JJ^-1 and y_J are written (posted by the owner of J, in J order),
// la = fbase + r + 1 when row group r is complete up to panel r - 1 (tile
// (r, r - 1) written).  A tile of another role's panel J reads that role's
// rows J (after la >= fbase + J + 1) and L_JJ^-1 (after diag >= fbase + J +
// 1).  Role 1 ends with done = base + f + 1 (and fail = the same value if
// one of its diagonal blocks was not positive definite); role 0 waits for
// it, so on return the whole factor, y and the inverses are written.
// ---------------------------------------------------------------------------
struct PairLa {
  unsigned long long* diag;
  unsigned long long* la;
  unsigned long long* done;
  unsigned long long* fail;
  unsigned long long base;
  int role;
  int spin;
};

__device__ __forceinline__ bool chol_dense_pair_la(double* A, const double* H, int npad, double* __restrict__ winv,
                                                   DenseLds& s, const PairLa& ps, int f, bool& bail, int n = -1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lm = lane & 15, lq = lane >> 4;
  const int P = npad / kNB;
  const int srow = threadIdx.x >> 2, scol = (threadIdx.x & 3) * 16;
  const double* hb = H + (size_t)npad * npad;   // b
  double* yrow = A + (size_t)npad * npad;       // y = L^-1 b
  const int w = ps.role;
  const unsigned long long fbase = ps.base + (unsigned long long)f * P;
  enum { kEnd = 0, kDiag = 1, kTile = 2, kAhead = 3 };
  bool ok = true;
  int wcur = -1;                      // panel whose L_JJ^-1 is in s.W
  // the task after (kind, r, J) in this role's sequence
  auto next_task = [&](int& kind, int& r, int& J) {
    if (kind == kAhead) {             // (J + 1, J) -> diagonal J + 1
      kind = kDiag; r = J + 1; J = J + 1;
    } else if (kind == kDiag) {       // diagonal Jd -> tiles (Jd + 2.., Jd - 1) or (Jd + 2.., Jd)
      const int Jd = J;
      if (Jd + 2 >= P) { kind = kEnd; return; }
      kind = kTile; r = Jd + 2; J = Jd >= 1 ? Jd - 1 : Jd;
    } else if (kind == kTile) {
      const int Jd = ((J & 1) == w) ? J : J + 1;   // this iteration's diagonal panel
      if (r + 2 < P) { r += 2; return; }
      if (J + 1 == Jd) { r = Jd + 2; J = Jd; return; }       // from panel Jd - 1 to panel Jd
      kind = kAhead; r = Jd + 2; J = Jd + 1;                 // Jd + 2 < P here
    }
  };
  d4v acc_n[4], bop_n[4];
  auto prefetch = [&](int r, int J, bool own_chunk0) {
    const int in = 4 * r + wave, col0 = kNB * J;
    const double* Hr = H + (size_t)(16 * in + lm) * npad;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc_n[c][q] = Hr[col0 + 16 * c + lq + 4 * q];
    if (J > 0 && own_chunk0) {
      const double* Ar = A + (size_t)(16 * in + lm) * npad;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) bop_n[kt] = *reinterpret_cast<const d4v*>(Ar + 16 * kt + 4 * lq);
    }
  };
  int kind, r, J;
  if (w == 1) {
    kind = P > 1 ? kAhead : kEnd; r = 1; J = 0;
  } else {
    kind = kDiag; r = 0; J = 0;
  }
  bool have_b = true;                 // bop_n holds chunk 0 of the task's own rows
  if (kind != kEnd) prefetch(r, J, true);
  while (kind != kEnd) {
    int kn = kind, rn = r, Jn = J;
    next_task(kn, rn, Jn);
    // the next task's chunk 0 is this task's tile when both are row group r
    // and this is panel 0: load it after this task's writes
    const bool pre_b = !(rn == r && J == 0);
    const int i = 4 * r + wave, col0 = kNB * J, nchunk = J;
    const double* Arow = A + (size_t)(16 * i + lm) * npad;
    const bool diag = kind == kDiag;
    if (kind == kAhead && J > 0) {
      // row group J (the other role's) complete up to panel J - 1
      if (!pair_wait(ps.la, fbase + J + 1, nullptr, ps.spin, s)) {
        bail = true;
        return false;
      }
    }
    if (!have_b && nchunk > 0 && !diag) {
      __syncthreads();
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) bop_n[kt] = *reinterpret_cast<const d4v*>(Arow + 16 * kt + 4 * lq);
    }
    d4v acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = acc_n[c];
    double ypart = 0.0;
    if (nchunk > 0 && diag) {
      diag_chunks(A, npad, col0, nchunk, yrow, s, acc, ypart);
      wcur = -1;
    } else if (nchunk > 0) {
      d4v st[4], bop[4], bnx[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) st[q] = *reinterpret_cast<const d4v*>(A + (size_t)(col0 + srow) * npad + scol + 4 * q);
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) bop[kt] = bop_n[kt];
#pragma unroll
      for (int q = 0; q < 4; ++q) *reinterpret_cast<d4v*>(&s.stage[0][srow * kSP + scol + 4 * q]) = st[q];
      __syncthreads();
      for (int ch = 0; ch < nchunk; ++ch) {
        const bool more = ch + 1 < nchunk;
        const int k1 = kNB * (ch + 1);
        if (more) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            st[q] = *reinterpret_cast<const d4v*>(A + (size_t)(col0 + srow) * npad + k1 + scol + 4 * q);
#pragma unroll
          for (int kt = 0; kt < 4; ++kt) bnx[kt] = *reinterpret_cast<const d4v*>(Arow + k1 + 16 * kt + 4 * lq);
        }
        const double* buf = s.stage[ch & 1];
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
          d4v aop[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) aop[c] = *reinterpret_cast<const d4v*>(buf + (16 * c + lm) * kSP + 16 * kt + 4 * lq);
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = mfma16(-aop[c][q], bop[kt][q], acc[c]);
        }
        if (more) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *reinterpret_cast<d4v*>(&s.stage[(ch + 1) & 1][srow * kSP + scol + 4 * q]) = st[q];
#pragma unroll
          for (int kt = 0; kt < 4; ++kt) bop[kt] = bnx[kt];
        }
        __syncthreads();
      }
    }
    if (diag) {
      // t = b_J - sum_k L_Jk y_k for the forward substitution
      ypart = row4_sum(ypart);
      if ((threadIdx.x & 3) == 0) s.vec[srow] = hb[col0 + srow] - ypart;
      double* D = s.stage[0];
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) D[(16 * wave + lm) * kSP + 16 * c + lq + 4 * q] = acc[c][q];
      __syncthreads();
      if (!chol_block<4>(D, s.W, s, live_blocks(n, col0))) ok = false;
      wcur = J;
      if (kn != kEnd) prefetch(rn, Jn, pre_b && kn != kDiag);
      // L_JJ^-1 and y_J = L_JJ^-1 t are what the other role waits for; L_JJ
      // itself is read only by the solves (after the done event), so its
      // stores go out after the post
      store_inv(winv + (size_t)J * kNB * kNB, s.W);
      ypanel(s.W, s.vec, yrow, col0);
      pair_post(ps.diag, fbase + J + 1);
      for (int e = threadIdx.x; e < kNB * kNB; e += kNT) {
        const int rr = e >> 6, c = e & 63;
        A[(size_t)(col0 + rr) * npad + col0 + c] = (c <= rr) ? D[rr * kSP + c] : 0.0;
      }
      __syncthreads();   // D (stage 0) is read before the next task stages into it
    } else {
      if (kind == kAhead && !pair_wait(ps.diag, fbase + J + 1, nullptr, ps.spin, s)) {
        bail = true;
        return false;
      }
      if (wcur != J) {
        load_inv(s.W, winv + (size_t)J * kNB * kNB);
        __syncthreads();
        wcur = J;
      }
      if (kn != kEnd) prefetch(rn, Jn, pre_b && kn != kDiag);
      // L_iJ = D L_JJ^-T:  out[m][n] = sum_k D[m][k] W[n][k]
#pragma unroll
      for (int cn = 0; cn < 4; ++cn) {
        d4v out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kt = 0; kt <= cn; ++kt) {
#pragma unroll
          for (int q = 0; q < 4; ++q) out = mfma16(acc[kt][q], s.W[(16 * cn + lm) * kSP + 16 * kt + lq + 4 * q], out);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) A[(size_t)(16 * i + lq + 4 * q) * npad + col0 + 16 * cn + lm] = out[q];
      }
      if (kind == kAhead) pair_post(ps.la, fbase + r + 1);
    }
    have_b = pre_b;
    kind = kn; r = rn; J = Jn;
  }
  if (w == 1) {
    if (!ok) {
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_store(ps.fail, ps.base + f + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    pair_post(ps.done, ps.base + f + 1);
    return ok;
  }
  if (!pair_wait(ps.done, ps.base + f + 1, nullptr, ps.spin, s)) {
    bail = true;
    return false;
  }
  if (__hip_atomic_load(ps.fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= ps.base + f + 1) ok = false;
  return ok;
}

// v[0:64] <- W v (lower = true) or W^T v (lower = false) for the 64x64
// lower-triangular panel inverse W (global, row-major); all threads call,
// 4 partial sums per output reduced through LDS.
__device__ __forceinline__ void panel_inv_matvec(const double* __restrict__ W, const double* v, double* out,
                                                 bool lower, DenseLds& s) {
  const int c = threadIdx.x & 63, part = threadIdx.x >> 6;
  double acc = 0.0;
  if (lower) {
    // out[c] = sum_{k <= c} W[c][k] v[k], k in this part's 16 columns
    const d4v* row = reinterpret_cast<const d4v*>(W + c * kNB + 16 * part);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const d4v w = row[q];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = 16 * part + 4 * q + e;
        acc += (k <= c) ? w[e] * v[k] : 0.0;
      }
    }
  } else {
    // out[c] = sum_{r >= c} W[r][c] v[r], r in this part's 16 rows
    double w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = W[(16 * part + q) * kNB + c];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int r = 16 * part + q;
      acc += (r >= c) ? w[q] * v[r] : 0.0;
    }
  }
  s.W[part * kNB + c] = acc;
  __syncthreads();
  if (threadIdx.x < kNB) out[c] = s.W[c] + s.W[kNB + c] + s.W[2 * kNB + c] + s.W[3 * kNB + c];
  __syncthreads();
}

// x <- L^-T x (x in LDS, length npad).  Per panel J (descending):
// x_J = W_J^T x_J, then x[0:r0] -= L[r0:r0+64][0:r0]^T x_J.  A pass takes 64
// columns: wave w the columns 16 w .. 16 w + 15 of it, the four 16-lane
// rows of a wave the four quarters of the panel's 64 rows (each load
// instruction reads 128 contiguous bytes per quarter), the quarters' sums
// joined by shuffles; so every panel keeps all 256 threads busy.  The L
// loads of the first four passes do not depend on x and are issued before
// the W_J product.
__device__ __forceinline__ void trsv_upper_t(const double* __restrict__ L, int npad, const double* __restrict__ winv,
                                             double* x, DenseLds& s) {
  const int P = npad / kNB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = 16 * wave + (lane & 15), k = lane >> 4;
  auto col_dot = [&](const double (&l)[16]) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc += l[i] * s.vec[16 * k + i];
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    return acc;
  };
  for (int J = P - 1; J >= 0; --J) {
    const int r0 = kNB * J;
    // this thread's column of the first pass in its quarter's 16 rows; pass
    // ps is 64 ps columns on (the passes below J are uniform)
    const double* Lc = L + (size_t)(r0 + 16 * k) * npad + cl;
    double l[4][16];
#pragma unroll
    for (int ps = 0; ps < 4; ++ps) {
      if (ps < J) {
#pragma unroll
        for (int i = 0; i < 16; ++i) l[ps][i] = Lc[i * npad + kNB * ps];
      }
    }
    panel_inv_matvec(winv + (size_t)J * kNB * kNB, x + r0, s.vec, false, s);
    if (threadIdx.x < kNB) x[r0 + threadIdx.x] = s.vec[threadIdx.x];
#pragma unroll
    for (int ps = 0; ps < 4; ++ps) {
      if (ps < J) {
        const double acc = col_dot(l[ps]);
        if (k == 0) x[kNB * ps + cl] -= acc;
      }
    }
    for (int ps = 4; ps < J; ++ps) {
      double u[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) u[i] = Lc[i * npad + kNB * ps];
      const double acc = col_dot(u);
      if (k == 0) x[kNB * ps + cl] -= acc;
    }
    __syncthreads();
  }
}

// x <- L^-T x (x in LDS, length npad) as trsv_upper_t, each thread owning
// whole columns of the update (no reductions, fewer live registers: the form
// the fused solve kernel takes).  Per panel J (descending):
// x_J = W_J^T x_J, then x[0:r0] -= L[r0:r0+64][0:r0]^T x_J.  The L loads of
// the update do not depend on x, so they are issued before the W_J product
// and their latency overlaps it.
__device__ __forceinline__ void trsv_upper_t_cols(const double* __restrict__ L, int npad, const double* __restrict__ winv,
                                             double* x, DenseLds& s) {
  const int P = npad / kNB;
  for (int J = P - 1; J >= 0; --J) {
    const int r0 = kNB * J;
    const int c = threadIdx.x;
    double l[kNB];
    if (c < r0) {
#pragma unroll
      for (int r = 0; r < kNB; ++r) l[r] = L[(size_t)(r0 + r) * npad + c];
    }
    panel_inv_matvec(winv + (size_t)J * kNB * kNB, x + r0, s.vec, false, s);
    if (threadIdx.x < kNB) x[r0 + threadIdx.x] = s.vec[threadIdx.x];
    if (c < r0) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < kNB; ++r) acc += l[r] * s.vec[r];
      x[c] -= acc;
    }
    for (int c2 = c + kNT; c2 < r0; c2 += kNT) {
#pragma unroll
      for (int r = 0; r < kNB; ++r) l[r] = L[(size_t)(r0 + r) * npad + c2];
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < kNB; ++r) acc += l[r] * s.vec[r];
      x[c2] -= acc;
    }
    __syncthreads();
  }
}

// x <- L^-1 x (x in LDS).  Per panel J (ascending): x_J = W_J x_J, then
// x[r] -= L[r][r0:r0+64] x_J for the rows below, four threads a row (thread
// j of a row reads the doubles 16 q + 4 j .. + 3, so each load instruction
// takes whole cache lines; the partial sums meet by shuffles).  The loads
// of the first 256 rows are issued before the W_J product.
__device__ __forceinline__ void trsv_lower(const double* __restrict__ L, int npad, const double* __restrict__ winv,
                                           double* x, DenseLds& s) {
  const int P = npad / kNB;
  const int rq = threadIdx.x >> 2, j = threadIdx.x & 3;
  auto row_dot = [&](const d4v (&v)[4]) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const d4v w = *reinterpret_cast<const d4v*>(s.vec + 16 * q + 4 * j);
      acc += v[q][0] * w[0] + v[q][1] * w[1] + v[q][2] * w[2] + v[q][3] * w[3];
    }
    return row4_sum(acc);
  };
  for (int J = 0; J < P; ++J) {
    const int r0 = kNB * J, rb = r0 + kNB;
    d4v v[4][4];
#pragma unroll
    for (int ps = 0; ps < 4; ++ps) {
      const int r = rb + kNB * ps + rq;
      if (r < npad) {
        const d4v* row = reinterpret_cast<const d4v*>(L + (size_t)r * npad + r0 + 4 * j);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[ps][q] = row[4 * q];
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[ps][q] = d4v{0.0, 0.0, 0.0, 0.0};
      }
    }
    panel_inv_matvec(winv + (size_t)J * kNB * kNB, x + r0, s.vec, true, s);
    if (threadIdx.x < kNB) x[r0 + threadIdx.x] = s.vec[threadIdx.x];
#pragma unroll
    for (int ps = 0; ps < 4; ++ps) {
      const int r = rb + kNB * ps + rq;
      const double acc = row_dot(v[ps]);
      if (r < npad && j == 0) x[r] -= acc;
    }
    for (int r = rb + kNT + rq; r < npad; r += kNB) {
      const d4v* row = reinterpret_cast<const d4v*>(L + (size_t)r * npad + r0 + 4 * j);
      d4v u[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) u[q] = row[4 * q];
      const double acc = row_dot(u);
      if (j == 0) x[r] -= acc;
    }
    __syncthreads();
  }
}

}  // namespace dnls
