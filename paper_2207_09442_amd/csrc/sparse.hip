// Block-sparse pose graphs (solver SPARSE): tile-supernodal right-looking
// Cholesky on FP64 MFMA, for large graphs such as the 16^3 lattice.
//
// Symbolic analysis (once, host, symbolic.hpp): minimum-degree order of the
// pose graph, postorder of its elimination tree, and the non-zero 48 x 48
// tiles of the factor (48 = 8 poses = 3 MFMA tiles, so tiles never split a
// pose).  Numeric factorisation, per tile column J (host loop, batched over
// graphs in grid y):
//   1. factor the diagonal tile:        L_JJ L_JJ^T = A_JJ, W = L_JJ^-1
//   2. triangular solve down the column: L_IJ = A_IJ W^T
//   3. right-looking update of every pair of tiles of the column:
//        A_IK -= L_IJ L_KJ^T   (I >= K, both non-zero in column J)
// Each target tile of step 3 is written by exactly one workgroup, so no
// atomics are needed.  Linearisation, assembly and the triangular solves use
// the same per-cost code as the dense path; the step is retracted in the
// original pose order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "costs.hpp"
#include "dense.hpp"
#include "plan.hpp"
#include "pose_costs.hpp"
#include "reproj.hpp"
#include "symbolic.hpp"

namespace dnls {
namespace {

constexpr int kTS = 48;            // tile size
constexpr int kTT = kTS * kTS;     // doubles per tile
constexpr int kBT = 256;           // threads of the grid kernels
constexpr int kTW = 192;           // threads of the tile kernels (3 waves x 16 rows)
constexpr int kWG = 512;           // threads of the one-workgroup-per-graph kernels (2 waves per SIMD)
constexpr int kWGW = kWG / 64;
constexpr int kPT = 256;           // threads of the persistent whole-solve kernel (one wave per SIMD)

struct SpArgs {
  const SpDesc* sd;
  const int* edge_ij;
  const int* prior_var;
  const int* pos;          // position of every pose in its graph's elimination order
  const int* inc_off;
  const int* inc_slot;
  const int4* od_blk;
  const int* od_slot;
  const int* tix;          // tile ids: [tix_off + I * P + J], -1 if zero
  const int* colptr;       // [col_off + J] .. [col_off + J + 1] -> rowidx
  const int* rowidx;       // tile rows of each column, diagonal first
  const int2* sn;          // [col_off + J]: first and last tile column of J's supernode
  const int* rowptr;       // [row_off + I] .. [row_off + I + 1] -> rowcol
  const int* rowcol;       // tile columns J < I of each tile row
  double* poses;
  const double* edge_meas;
  const double* edge_logw;
  const double* edge_tau;
  const double* prior_meas;
  const double* prior_logw;
  const double* edge_logc; // Welsch log-radii or null
  double* objective;
  int* status;
  double* factor;          // tile pools and panel inverses
  double* ws64;
  float* ws32;
  double* ycost;
  double* vec;             // per graph: [4][nvec]: step, right-hand side, work, forward result
  double* partial;
  int* failed;
  double* lastobj;
  const double* seed;
  double* uout;            // backward: adjoint in original pose order [V][d]
  double* g_logw_e;
  double* g_tau;
  double* g_logw_p;
  double* g_logc;
  double* hvp;             // exact backward: [cost][2][d] second-order terms
  double* lam_g;           // adaptive damping: lambda per graph
  double* pose_bak;        // adaptive damping: theta_t while the trial step is evaluated
  double* s_t;             // adaptive damping: float64 objective at theta_t per graph
  int* rej;                // adaptive damping / dogleg: the graph's trial step was rejected
  double* dl;              // dogleg per graph: radius, predicted decrease, |delta|, on the boundary
  double* traj;            // persistent schedule with DNLS_FLAG_KEEP_ITERATES: theta_t, [K][V][sz]
  const int* lvlptr;       // BLOCK: columns of each elimination-tree level, [lvl_off + L] .. [+1] into lvlcol
  const int* lvlcol;
  const int* lvlbptr;      // BLOCK: factor blocks of each level's columns, into lvlblk
  const int4* lvlblk;      //   (tile id, first and end contribution in cpair, 2 J + diagonal)
  const int2* cpair;       // BLOCK: the (L_IK, L_JK) tile-id pairs that update each level block
  const int* rowid;        // BLOCK: tile id of every (I, rowcol) entry
  int ts;                  // tile size: kTS (48) or the pose dimension d (BLOCK)
  // bundle adjustment (points eliminated first inside the tile factorisation)
  double* pts;             // [Vp][3]
  const double* obs_uv;
  const double* obs_w;
  const double* delta_b;   // per-problem Huber radius, or NULL for huber
  const int* obs_cam;
  const int* obs_pt;
  const int* soff_cam;     // scalar offset of every camera / point in its problem's elimination order
  const int* soff_pt;
  const int* cam_obs_off;  // observations of every camera
  const int* cam_obs;
  const int* pt_obs_off;   // observations of every point
  const int* pt_obs;
  const int4* cp_blk;      // (camera, point, first, count) per camera-point block
  const int* cp_obs;
  void* orec;              // [obs][20] J~cam (2x6), J~pt (2x3), r~ (2) in the linearisation's precision
  double* gob;             // mixed: float64 gradient parts [obs][9] (camera 6, point 3)
  const double* seed_pt;   // backward: point seed [Vp][3] or NULL
  double* g_w;             // backward: observation weights, per-observation radii, per-problem radii
  double* g_delta;
  double* g_huber;
  double fx, fy, cx, cy, huber;
  int E, V, K, it, nx, refine;
  double lambda, radius0;
};

__device__ __forceinline__ PoseCostData cost_data(const SpArgs& a) {
  return PoseCostData{a.edge_ij, a.prior_var, a.poses, a.edge_meas, a.edge_logw,
                      a.edge_tau, a.prior_meas, a.prior_logw, a.E, a.edge_logc};
}

__device__ __forceinline__ double* tile_ptr(const SpArgs& a, const SpDesc& g, int I, int J) {
  const int id = a.tix[g.tix_off + I * g.P + J];
  return a.factor + g.pool_off + (size_t)id * (a.ts * a.ts);
}

__device__ double block_sum_sp(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  __syncthreads();
  return t;
}

// linearisation of the costs of graph blockIdx.y (grid x over its costs)
template <int G, class S>
__global__ void __launch_bounds__(kBT) k_sp_lin(SpArgs a, S* rec) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  __shared__ double red[kBT / 64];
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  double s = 0.0;
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (!a.failed[b] && k < g.nedge + g.nprior) {
    const int rk = (k < g.nedge) ? g.edge0 + k : a.E + g.prior0 + (k - g.nedge);
    s = linearize_cost<G, S>(cost_data(a), rk, rec + (size_t)rk * RN);
  }
  s = block_sum_sp(s, red);
  if (threadIdx.x == 0) a.partial[b * a.nx + blockIdx.x] = s;
}

// objective of the step and the non-finite check (thread per graph)
__global__ void k_sp_objective(SpArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double* obj = a.objective + (size_t)b * (a.K + 1);
  if (a.failed[b]) {
    obj[a.it] = a.lastobj[b];
    return;
  }
  double S = 0.0;
  for (int k = 0; k < a.nx; ++k) S += a.partial[b * a.nx + k];
  obj[a.it] = S;
  a.lastobj[b] = S;
  if (a.s_t) a.s_t[b] = S;
  if (!isfinite(S)) {
    a.failed[b] = DNLS_GRAPH_NONFINITE;
    a.status[b] = DNLS_GRAPH_NONFINITE;
  }
}

// zero every tile of the graph's pool
__global__ void __launch_bounds__(kBT) k_sp_zero(SpArgs a) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  double* pool = a.factor + g.pool_off;
  const size_t n = (size_t)g.ntile * (a.ts * a.ts);
  for (size_t u = (size_t)blockIdx.x * kBT + threadIdx.x; u < n; u += (size_t)gridDim.x * kBT) pool[u] = 0.0;
}

__device__ __forceinline__ void put(const SpArgs& a, const SpDesc& g, int row, int col, double v) {
  const int ts = a.ts;
  double* t = tile_ptr(a, g, row / ts, col / ts);
  t[(row % ts) * ts + col % ts] = v;
}

// Hessian blocks into the tiles (permuted, lower triangle), g into vec[1].
// Item u < npose + nod: one diagonal or off-diagonal block (and, for u <
// npose with rhs_from_rec, that pose's segment of g).
template <int G, class S>
__device__ __forceinline__ void sp_assemble_item(const SpArgs& a, const SpDesc& g, int u, const S* rec,
                                                 double lambda, int rhs_from_rec) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  S h[d * d];
#pragma unroll
  for (int q = 0; q < d * d; ++q) h[q] = S(0);
  int pa, pb;
  if (u < g.npose) {
    pa = pb = u;
    const int gp = g.pose0 + u;
    for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
      const int slot = a.inc_slot[s];
      const S* J = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
#pragma unroll
      for (int k = 0; k < d; ++k)
#pragma unroll
        for (int r = 0; r < d; ++r)
#pragma unroll
          for (int c = 0; c < d; ++c) h[r * d + c] += J[k * d + r] * J[k * d + c];
    }
  } else {
    const int4 blk = a.od_blk[g.od0 + (u - g.npose)];
    pa = blk.x;
    pb = blk.y;
    for (int s = blk.z; s < blk.z + blk.w; ++s) {
      const int slot = a.od_slot[s];
      const S* Jr = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
      const S* Jc = rec + (size_t)(slot >> 1) * RN + ((slot & 1) ^ 1) * d * d;
#pragma unroll
      for (int k = 0; k < d; ++k)
#pragma unroll
        for (int r = 0; r < d; ++r)
#pragma unroll
          for (int c = 0; c < d; ++c) h[r * d + c] += Jr[k * d + r] * Jc[k * d + c];
    }
  }
  const int ra = a.pos[g.pose0 + pa], rb = a.pos[g.pose0 + pb];
#pragma unroll
  for (int r = 0; r < d; ++r)
#pragma unroll
    for (int c = 0; c < d; ++c) {
      double v = double(h[r * d + c]);
      if (pa == pb) {
        if (c > r) continue;
        if (c == r) v += lambda;
        put(a, g, ra * d + r, ra * d + c, v);
      } else if (ra > rb) {
        put(a, g, ra * d + r, rb * d + c, v);
      } else {
        put(a, g, rb * d + c, ra * d + r, v);
      }
    }
  if (rhs_from_rec && u < g.npose) {
    double* rhs = a.vec + g.vec_off + g.nvec;
    const int gp = g.pose0 + u;
    S acc[d];
#pragma unroll
    for (int r = 0; r < d; ++r) acc[r] = S(0);
    for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
      const int slot = a.inc_slot[s];
      const S* J = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
      const S* res = rec + (size_t)(slot >> 1) * RN + 2 * d * d;
#pragma unroll
      for (int k = 0; k < d; ++k)
#pragma unroll
        for (int r = 0; r < d; ++r) acc[r] += J[k * d + r] * res[k];
    }
#pragma unroll
    for (int r = 0; r < d; ++r) rhs[ra * d + r] = double(acc[r]);
  }
}

// padding of the last tile (unit diagonal) and of the right-hand side
// (zero), threads t = t0, t0 + stride, ...
__device__ __forceinline__ void sp_assemble_pad(const SpArgs& a, const SpDesc& g, int t0, int stride) {
  for (int r = g.n + t0; r < g.P * a.ts; r += stride) put(a, g, r, r, 1.0);
  double* rhs = a.vec + g.vec_off + g.nvec;
  for (int r = g.n + t0; r < g.nvec; r += stride) rhs[r] = 0.0;
}

template <int G, class S>
__global__ void __launch_bounds__(kBT) k_sp_assemble(SpArgs a, const S* rec, double lambda, int rhs_from_rec,
                                                     int lam_per_graph) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  if (lam_per_graph) lambda = a.lam_g[b];
  const int u = blockIdx.x * kBT + threadIdx.x;
  if (u < g.npose + g.nod) sp_assemble_item<G, S>(a, g, u, rec, lambda, rhs_from_rec);
  if (blockIdx.x == 0) sp_assemble_pad(a, g, threadIdx.x, kBT);
}

// float64 right-hand side into vec[1] (mixed path with refinement)
template <int G>
__device__ __forceinline__ void sp_rhs64_item(const SpArgs& a, const SpDesc& g, int u) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const int gp = g.pose0 + u, ra = a.pos[gp];
  double acc[d];
#pragma unroll
  for (int r = 0; r < d; ++r) acc[r] = 0.0;
  for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
    const int slot = a.inc_slot[s];
    const double* J = a.ws64 + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
    const double* res = a.ws64 + (size_t)(slot >> 1) * RN + 2 * d * d;
#pragma unroll
    for (int k = 0; k < d; ++k)
#pragma unroll
      for (int r = 0; r < d; ++r) acc[r] += J[k * d + r] * res[k];
  }
  double* rhs = a.vec + g.vec_off + g.nvec;
#pragma unroll
  for (int r = 0; r < d; ++r) rhs[ra * d + r] = acc[r];
}

template <int G>
__global__ void __launch_bounds__(kBT) k_sp_rhs64(SpArgs a) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int u = blockIdx.x * kBT + threadIdx.x;
  if (u < g.npose) sp_rhs64_item<G>(a, g, u);
}

// 1. diagonal tile of column J
__global__ void __launch_bounds__(kNT) k_sp_diag(SpArgs a, int J) {
  __shared__ DenseLds s;
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b] || J >= g.P) return;
  double* T = tile_ptr(a, g, J, J);
  double* D = s.stage[0];
  // four values per thread and access (a tile row is 12 of them)
  for (int e = threadIdx.x; e < kTT / 4; e += kNT) {
    const int r = e / (kTS / 4), c = (e % (kTS / 4)) * 4;
    *reinterpret_cast<d4v*>(D + r * kSP + c) = *reinterpret_cast<const d4v*>(T + 4 * e);
  }
  __syncthreads();
  const bool ok = chol_block<3>(D, s.W, s);
  double* winv = a.factor + g.winv_off + (size_t)J * kTT;
  for (int e = threadIdx.x; e < kTT / 4; e += kNT) {
    const int r = e / (kTS / 4), c = (e % (kTS / 4)) * 4;
    d4v l = *reinterpret_cast<const d4v*>(D + r * kSP + c);
    d4v w = *reinterpret_cast<const d4v*>(s.W + r * kSP + c);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      l[k] = (c + k <= r) ? l[k] : 0.0;
      w[k] = (c + k <= r) ? w[k] : 0.0;
    }
    *reinterpret_cast<d4v*>(T + 4 * e) = l;
    *reinterpret_cast<d4v*>(winv + 4 * e) = w;
  }
  if (!ok && threadIdx.x == 0) {
    a.failed[b] = DNLS_GRAPH_NOT_PD;
    a.status[b] = DNLS_GRAPH_NOT_PD;
  }
}

// 2. L_IJ = A_IJ W^T for the tiles below the diagonal of column J
__global__ void __launch_bounds__(kTW) k_sp_trsm(SpArgs a, int J) {
  __shared__ double W[kTS * (kTS + 4)];
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b] || J >= g.P) return;
  const int c0 = a.colptr[g.col_off + J], c1 = a.colptr[g.col_off + J + 1];
  const int t = blockIdx.x;
  if (t >= c1 - c0 - 1) return;
  const int I = a.rowidx[c0 + 1 + t];
  const double* winv = a.factor + g.winv_off + (size_t)J * kTT;
  constexpr int LW = kTS + 4;
  for (int e = threadIdx.x; e < kTT / 4; e += kTW) {
    const int r = e / (kTS / 4), c = (e % (kTS / 4)) * 4;
    *reinterpret_cast<d4v*>(&W[r * LW + c]) = *reinterpret_cast<const d4v*>(winv + 4 * e);
  }
  __syncthreads();
  double* T = tile_ptr(a, g, I, J);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  // rows 16 wave .. +16 of the tile; out[m][n] = sum_k A[m][k] W[n][k]
  d4v acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = d4v{0.0, 0.0, 0.0, 0.0};
  const double* arow = T + (16 * wave + lm) * kTS;
#pragma unroll
  for (int kt = 0; kt < 3; ++kt) {
    const d4v av = *reinterpret_cast<const d4v*>(arow + 16 * kt + 4 * lq);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (kt > c) continue;   // W lower triangular
      const d4v wv = *reinterpret_cast<const d4v*>(&W[(16 * c + lm) * LW + 16 * kt + 4 * lq]);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[c] = mfma16(av[q], wv[q], acc[c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * wave + lq + 4 * r) * kTS + 16 * c + lm] = acc[c][r];
}

// 3. A_IK -= L_IJ L_KJ^T for every pair I >= K of tiles below the diagonal of
// J.  Inside a supernode [s, e] (the runs of tile_supernodes) a column J < e
// updates only the targets with K <= e, which the next columns of the run
// need; its last column e applies A_IK -= sum_{J'=s}^{e} L_IJ' L_KJ'^T to the
// targets right of the run, each target read and written once.
__global__ void __launch_bounds__(kTW) k_sp_update(SpArgs a, int J) {
  __shared__ double LK[kTS * (kTS + 4)];
  constexpr int LW = kTS + 4;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b] || J >= g.P) return;
  const int c0 = a.colptr[g.col_off + J], c1 = a.colptr[g.col_off + J + 1];
  const int m = c1 - c0 - 1;
  const long long t = blockIdx.x;
  if (t >= (long long)m * (m + 1) / 2) return;
  // triangular index t -> (p, q), p >= q
  int p = (int)((::sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((long long)(p + 1) * (p + 2) / 2 <= t) ++p;
  while ((long long)p * (p + 1) / 2 > t) --p;
  const int q = (int)(t - (long long)p * (p + 1) / 2);
  const int2 sn = a.sn[g.col_off + J];
  // rows J + 1 .. sn.y come first below the diagonal of a column of the run
  if (J < sn.y && q >= sn.y - J) return;
  const int jfirst = J == sn.y ? sn.x : J;
  const int I = a.rowidx[c0 + 1 + p], Kt = a.rowidx[c0 + 1 + q];
  double* T = tile_ptr(a, g, I, Kt);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  d4v acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[c][r] = T[(16 * wave + lq + 4 * r) * kTS + 16 * c + lm];
  for (int Jp = jfirst; Jp <= J; ++Jp) {
    const double* LI = tile_ptr(a, g, I, Jp);
    const double* LKg = tile_ptr(a, g, Kt, Jp);
    if (Jp > jfirst) __syncthreads();   // the previous column's LK is read
    for (int e = threadIdx.x; e < kTT / 4; e += kTW) {
      const int r = (4 * e) / kTS, c = (4 * e) % kTS;
      *reinterpret_cast<d4v*>(&LK[r * LW + c]) = *reinterpret_cast<const d4v*>(LKg + 4 * e);
    }
    d4v av[3];
#pragma unroll
    for (int kt = 0; kt < 3; ++kt) av[kt] = *reinterpret_cast<const d4v*>(LI + (16 * wave + lm) * kTS + 16 * kt + 4 * lq);
    __syncthreads();
#pragma unroll
    for (int kt = 0; kt < 3; ++kt)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const d4v bv = *reinterpret_cast<const d4v*>(&LK[(16 * c + lm) * LW + 16 * kt + 4 * lq]);
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) acc[c] = mfma16(-av[kt][qq], bv[qq], acc[c]);
      }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * wave + lq + 4 * r) * kTS + 16 * c + lm] = acc[c][r];
}

// Whole numeric factorisation with one workgroup per graph (small graphs):
// per tile column the diagonal tile is factored in LDS, then the waves take
// 16-row slabs of the column's tiles (L_IJ = A_IJ W^T) and then of the lower
// pairs of them (A_IK -= L_IJ L_KJ^T), with no launches between the steps.
// Same arithmetic per tile as the per-column kernels.
// One 16-row slab of a 48x48 tile operation per wave; every operand of the
// slab is loaded before its first product (one memory round trip).
// Slab sr of T <- T W^T, W lower triangular in LDS (stride kSP).
__device__ __forceinline__ void wave_slab_trsm(double* T, const double* W, int sr) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  d4v av[3], acc[3];
#pragma unroll
  for (int kt = 0; kt < 3; ++kt) av[kt] = *reinterpret_cast<const d4v*>(T + (16 * sr + lm) * kTS + 16 * kt + 4 * lq);
#pragma unroll
  for (int c = 0; c < 3; ++c) acc[c] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kt = 0; kt < 3; ++kt)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (kt > c) continue;
      const d4v wv = *reinterpret_cast<const d4v*>(&W[(16 * c + lm) * kSP + 16 * kt + 4 * lq]);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[c] = mfma16(av[kt][q], wv[q], acc[c]);
    }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * sr + lq + 4 * r) * kTS + 16 * c + lm] = acc[c][r];
}

// slab sr of T -= LI LK^T (48x48 tiles in global memory)
__device__ __forceinline__ void wave_slab_update(double* T, const double* LI, const double* LK, int sr) {
  const int lane = threadIdx.x & 63, lm = lane & 15, lq = lane >> 4;
  d4v acc[3], av[3], bv[3][3];
#pragma unroll
  for (int kt = 0; kt < 3; ++kt)
#pragma unroll
    for (int c = 0; c < 3; ++c) bv[kt][c] = *reinterpret_cast<const d4v*>(LK + (16 * c + lm) * kTS + 16 * kt + 4 * lq);
#pragma unroll
  for (int kt = 0; kt < 3; ++kt) av[kt] = *reinterpret_cast<const d4v*>(LI + (16 * sr + lm) * kTS + 16 * kt + 4 * lq);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[c][r] = T[(16 * sr + lq + 4 * r) * kTS + 16 * c + lm];
#pragma unroll
  for (int kt = 0; kt < 3; ++kt)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[c] = mfma16(-av[kt][q], bv[kt][c][q], acc[c]);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) T[(16 * sr + lq + 4 * r) * kTS + 16 * c + lm] = acc[c][r];
}

// (NT threads, a multiple of 64) returns false if the graph is not positive definite
template <int NT>
__device__ bool sp_factor_wg_body(const SpArgs& a, int b, const SpDesc& g, DenseLds& s) {
  const int wave = threadIdx.x >> 6;
  for (int J = 0; J < g.P; ++J) {
    // 1. diagonal tile
    double* TJ = tile_ptr(a, g, J, J);
    double* D = s.stage[0];
    for (int e = threadIdx.x; e < kTT / 4; e += NT) {
      const int r = e / (kTS / 4), c = (e % (kTS / 4)) * 4;
      *reinterpret_cast<d4v*>(D + r * kSP + c) = *reinterpret_cast<const d4v*>(TJ + 4 * e);
    }
    __syncthreads();
    const bool ok = chol_block<3>(D, s.W, s);
    double* winv = a.factor + g.winv_off + (size_t)J * kTT;
    for (int e = threadIdx.x; e < kTT / 4; e += NT) {
      const int r = e / (kTS / 4), c = (e % (kTS / 4)) * 4;
      d4v l = *reinterpret_cast<const d4v*>(D + r * kSP + c);
      d4v w = *reinterpret_cast<const d4v*>(s.W + r * kSP + c);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        l[k] = (c + k <= r) ? l[k] : 0.0;
        w[k] = (c + k <= r) ? w[k] : 0.0;
      }
      *reinterpret_cast<d4v*>(TJ + 4 * e) = l;
      *reinterpret_cast<d4v*>(winv + 4 * e) = w;
    }
    if (!ok) {
      if (threadIdx.x == 0) {
        a.failed[b] = DNLS_GRAPH_NOT_PD;
        a.status[b] = DNLS_GRAPH_NOT_PD;
      }
      return false;
    }
    const int c0 = a.colptr[g.col_off + J], m = a.colptr[g.col_off + J + 1] - c0 - 1;
    // 2. L_IJ = A_IJ W^T for the tiles below the diagonal (W stays in LDS)
#pragma unroll 1
    for (int u = wave; u < 3 * m; u += (NT / 64)) wave_slab_trsm(tile_ptr(a, g, a.rowidx[c0 + 1 + u / 3], J), s.W, u % 3);
    __syncthreads();
    // 3. A_IK -= L_IJ L_KJ^T for every lower pair of them
    const int npair = m * (m + 1) / 2;
#pragma unroll 1
    for (int u = wave; u < 3 * npair; u += (NT / 64)) {
      const int t = u / 3;
      int p = (int)((::sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
      while ((p + 1) * (p + 2) / 2 <= t) ++p;
      while (p * (p + 1) / 2 > t) --p;
      const int q = t - p * (p + 1) / 2;
      const int I = a.rowidx[c0 + 1 + p], K = a.rowidx[c0 + 1 + q];
      wave_slab_update(tile_ptr(a, g, I, K), tile_ptr(a, g, I, J), tile_ptr(a, g, K, J), u % 3);
    }
    __syncthreads();
  }
  return true;
}

__global__ void __launch_bounds__(kWG) k_sp_factor_wg(SpArgs a) {
  __shared__ DenseLds s;
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  sp_factor_wg_body<kWG>(a, b, g, s);
}

// ---------------------------------------------------------------------------
// Triangular solves L L^T x = b as sweeps of one launch per tile column
// (forward) and per tile row (backward); every tile of the column / row is
// handled by its own workgroup, so each launch touches distinct targets.
// Vector slots per graph (nvec doubles each): 0 step x, 1 right-hand side,
// 2 work vector b, 3 forward result y.
// ---------------------------------------------------------------------------
constexpr int kSW = kTS + 1;       // LDS row stride of the solve kernels

__device__ __forceinline__ double* slot(const SpArgs& a, const SpDesc& g, int k) {
  return a.vec + g.vec_off + (long long)k * g.nvec;
}

// stage a 48 x 48 tile (row-major, global) into LDS with stride kSW
__device__ __forceinline__ void stage_tile(double* dst, const double* src) {
  for (int e = threadIdx.x; e < kTT / 4; e += blockDim.x) {
    const d4v v = *reinterpret_cast<const d4v*>(src + 4 * e);
    const int r = e / (kTS / 4), c = (e % (kTS / 4)) * 4;
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[r * kSW + c + k] = v[k];
  }
}

// forward step of column J: x_J = W_J b_J; b_I -= L_IJ x_J for the tiles I of the column
__global__ void __launch_bounds__(kTW) k_sp_fwd(SpArgs a, int J, int src, int dst) {
  __shared__ double Wl[kTS * kSW];
  __shared__ double T[kTS * kSW];
  __shared__ double bv[kTS], yv[kTS];
  __shared__ double part[kTW / kTS][kTS];
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b] || J >= g.P) return;
  const int c0 = a.colptr[g.col_off + J], c1 = a.colptr[g.col_off + J + 1];
  const int t = blockIdx.x;
  if (t > c1 - c0 - 1) return;
  double* bvec = slot(a, g, src);
  stage_tile(Wl, a.factor + g.winv_off + (size_t)J * kTT);
  int I = -1;
  if (t > 0) {
    I = a.rowidx[c0 + t];
    stage_tile(T, tile_ptr(a, g, I, J));
  }
  if (threadIdx.x < kTS) bv[threadIdx.x] = bvec[J * kTS + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < kTS) {
    const int c = threadIdx.x;
    double acc = 0.0;
    for (int k = 0; k <= c; ++k) acc += Wl[c * kSW + k] * bv[k];
    yv[c] = acc;
  }
  __syncthreads();
  if (t == 0) {
    if (threadIdx.x < kTS) slot(a, g, dst)[J * kTS + threadIdx.x] = yv[threadIdx.x];
    return;
  }
  // rows r = tid % 48, k range quarter q = tid / 48
  constexpr int NQ = kTW / kTS, KQ = kTS / NQ;
  const int r = threadIdx.x % kTS, q = threadIdx.x / kTS;
  double acc = 0.0;
#pragma unroll
  for (int k = q * KQ; k < q * KQ + KQ; ++k) acc += T[r * kSW + k] * yv[k];
  part[q][r] = acc;
  __syncthreads();
  if (threadIdx.x < kTS) {
    double s = 0.0;
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) s += part[qq][threadIdx.x];
    bvec[I * kTS + threadIdx.x] -= s;
  }
}

// backward step of row I: x_I = W_I^T z_I; z_J -= L_IJ^T x_I for the tiles J of the row
__global__ void __launch_bounds__(kTW) k_sp_bwd(SpArgs a, int I, int zs, int dst) {
  __shared__ double Wl[kTS * kSW];
  __shared__ double T[kTS * kSW];
  __shared__ double zv[kTS], yv[kTS];
  __shared__ double part[kTW / kTS][kTS];
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b] || I >= g.P) return;
  const int r0 = a.rowptr[g.row_off + I], r1 = a.rowptr[g.row_off + I + 1];
  const int t = blockIdx.x;
  if (t > r1 - r0) return;
  double* z = slot(a, g, zs);
  stage_tile(Wl, a.factor + g.winv_off + (size_t)I * kTT);
  int J = -1;
  if (t > 0) {
    J = a.rowcol[r0 + t - 1];
    stage_tile(T, tile_ptr(a, g, I, J));
  }
  if (threadIdx.x < kTS) zv[threadIdx.x] = z[I * kTS + threadIdx.x];
  __syncthreads();
  if (threadIdx.x < kTS) {
    const int c = threadIdx.x;
    double acc = 0.0;
    for (int r = c; r < kTS; ++r) acc += Wl[r * kSW + c] * zv[r];
    yv[c] = acc;
  }
  __syncthreads();
  if (t == 0) {
    if (threadIdx.x < kTS) slot(a, g, dst)[I * kTS + threadIdx.x] = yv[threadIdx.x];
    return;
  }
  constexpr int NQ = kTW / kTS, RQ = kTS / NQ;
  const int c = threadIdx.x % kTS, q = threadIdx.x / kTS;
  double acc = 0.0;
#pragma unroll
  for (int r = q * RQ; r < q * RQ + RQ; ++r) acc += T[r * kSW + c] * yv[r];
  part[q][c] = acc;
  __syncthreads();
  if (threadIdx.x < kTS) {
    double s = 0.0;
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) s += part[qq][threadIdx.x];
    z[J * kTS + threadIdx.x] -= s;
  }
}

// Whole solve x (slot dst) = (L L^T)^-1 b (slot src) with one workgroup per
// graph and the vector in LDS, for plans whose graphs have at most
// kSolveLds unknowns (padded): per tile column a 48x48 product with W_J and
// the rows of the column's tiles; then per tile row (descending) W_I^T and
// the transposed tiles of the row.  Two barriers per tile step and no
// launches, where the sweeps need two launches per tile column.
constexpr int kSolveLds = 6144;
constexpr int kFactorWgMaxP = 16;  // AUTO: one-workgroup factorisation up to 16 tile columns
// (NT >= 192 threads, a multiple of 64) v: nvec doubles, Wl: kTS x kSW, y: kTS, all in LDS
template <int NT>
__device__ void sp_solve_wg_body(const SpArgs& a, const SpDesc& g, int src, int dst, double* v, double* Wl,
                                 double* y) {
  const double* bsrc = slot(a, g, src);
  for (int u = threadIdx.x; u < g.nvec; u += NT) v[u] = bsrc[u];
  // the 48 products with W are split over 4 adjacent lanes each (12 terms)
  const int wr = threadIdx.x >> 2, wp = threadIdx.x & 3;
  for (int J = 0; J < g.P; ++J) {
    stage_tile(Wl, a.factor + g.winv_off + (size_t)J * kTT);   // coalesced
    __syncthreads();
    if (threadIdx.x < 4 * kTS) {
      double acc = 0.0;
#pragma unroll
      for (int k = 12 * wp; k < 12 * wp + 12; ++k) acc += (k <= wr) ? Wl[wr * kSW + k] * v[J * kTS + k] : 0.0;
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      if (wp == 0) y[wr] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kTS) v[J * kTS + threadIdx.x] = y[threadIdx.x];
    const int c0 = a.colptr[g.col_off + J], m = a.colptr[g.col_off + J + 1] - c0 - 1;
    for (int e = threadIdx.x; e < m * kTS; e += NT) {
      const int I = a.rowidx[c0 + 1 + e / kTS], r = e % kTS;
      const d4v* row = reinterpret_cast<const d4v*>(tile_ptr(a, g, I, J) + r * kTS);
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < kTS / 4; ++q) {
        const d4v t = row[q];
        acc += t[0] * y[4 * q] + t[1] * y[4 * q + 1] + t[2] * y[4 * q + 2] + t[3] * y[4 * q + 3];
      }
      v[I * kTS + r] -= acc;
    }
    __syncthreads();
  }
  for (int I = g.P - 1; I >= 0; --I) {
    stage_tile(Wl, a.factor + g.winv_off + (size_t)I * kTT);
    __syncthreads();
    if (threadIdx.x < 4 * kTS) {
      double acc = 0.0;
#pragma unroll
      for (int r = 12 * wp; r < 12 * wp + 12; ++r) acc += (r >= wr) ? Wl[r * kSW + wr] * v[I * kTS + r] : 0.0;
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      if (wp == 0) y[wr] = acc;
    }
    __syncthreads();
    if (threadIdx.x < kTS) v[I * kTS + threadIdx.x] = y[threadIdx.x];
    const int r0 = a.rowptr[g.row_off + I], nr = a.rowptr[g.row_off + I + 1] - r0;
    for (int e = threadIdx.x; e < nr * kTS; e += NT) {
      const int J = a.rowcol[r0 + e / kTS], c = e % kTS;
      const double* T = tile_ptr(a, g, I, J);
      double acc = 0.0;
#pragma unroll 16
      for (int r = 0; r < kTS; ++r) acc += T[r * kTS + c] * y[r];
      v[J * kTS + c] -= acc;
    }
    __syncthreads();
  }
  double* xdst = slot(a, g, dst);
  for (int u = threadIdx.x; u < g.nvec; u += NT) xdst[u] = v[u];
}

__global__ void __launch_bounds__(kWG) k_sp_solve_wg(SpArgs a, int src, int dst) {
  __shared__ double v[kSolveLds];
  __shared__ double Wl[kTS * kSW];
  __shared__ double y[kTS];
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  sp_solve_wg_body<kWG>(a, g, src, dst, v, Wl, y);
}

// slot[to] = slot[from] (grid x over the vector, y over graphs)
__global__ void __launch_bounds__(kBT) k_sp_copy(SpArgs a, int from, int to) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* x = slot(a, g, from);
  double* y = slot(a, g, to);
  for (int u = blockIdx.x * kBT + threadIdx.x; u < g.nvec; u += gridDim.x * kBT) y[u] = x[u];
}

// X <- X Exp(-x) per pose, x read in permuted order
template <int G>
__device__ __forceinline__ void sp_retract_item(const SpArgs& a, const SpDesc& g, int p, int xs) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  retract_minus<G>(a.poses + (size_t)(g.pose0 + p) * sz, slot(a, g, xs) + a.pos[g.pose0 + p] * d);
}

template <int G>
__global__ void __launch_bounds__(kBT) k_sp_retract(SpArgs a, int xs) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p < g.npose) sp_retract_item<G>(a, g, p, xs);
}

// refinement residual b = g64 - (H64 + lambda) x (matrix-free, float64
// records and J x per cost in ycost), padding zero
template <int G>
__device__ __forceinline__ void sp_residual_item(const SpArgs& a, const SpDesc& g, int p, double lambda) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const double* x = slot(a, g, 0);
  const double* rhs = slot(a, g, 1);
  double* res = slot(a, g, 2);
  const int gp = g.pose0 + p, ra = a.pos[gp];
  double hv[d];
#pragma unroll
  for (int r = 0; r < d; ++r) hv[r] = lambda * x[ra * d + r];
  for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
    const int sl = a.inc_slot[s];
    const double* J = a.ws64 + (size_t)(sl >> 1) * RN + (sl & 1) * d * d;
    const double* yc = a.ycost + (size_t)(sl >> 1) * d;
#pragma unroll
    for (int k = 0; k < d; ++k)
#pragma unroll
      for (int r = 0; r < d; ++r) hv[r] += J[k * d + r] * yc[k];
  }
#pragma unroll
  for (int r = 0; r < d; ++r) res[ra * d + r] = rhs[ra * d + r] - hv[r];
}

template <int G>
__global__ void __launch_bounds__(kBT) k_sp_residual(SpArgs a, double lambda, int lam_per_graph) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  if (lam_per_graph) lambda = a.lam_g[b];
  if (blockIdx.x == 0) {
    double* res = slot(a, g, 2);
    for (int u = g.n + threadIdx.x; u < g.nvec; u += kBT) res[u] = 0.0;
  }
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p < g.npose) sp_residual_item<G>(a, g, p, lambda);
}

// refinement: J delta per cost (float64 records), delta read in permuted order
template <int G>
__device__ __forceinline__ void sp_jx_item(const SpArgs& a, const SpDesc& g, int k, int xs) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const double* x = slot(a, g, xs);
  int rk, pi = -1, pj;
  if (k < g.nedge) {
    rk = g.edge0 + k;
    pi = a.pos[a.edge_ij[2 * rk]];
    pj = a.pos[a.edge_ij[2 * rk + 1]];
  } else {
    rk = a.E + g.prior0 + (k - g.nedge);
    pj = a.pos[a.prior_var[g.prior0 + (k - g.nedge)]];
  }
  const double* J = a.ws64 + (size_t)rk * RN;
#pragma unroll
  for (int r = 0; r < d; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      if (pi >= 0) acc += J[r * d + q] * x[pi * d + q];
      acc += J[d * d + r * d + q] * x[pj * d + q];
    }
    a.ycost[(size_t)rk * d + r] = acc;
  }
}

template <int G>
__global__ void __launch_bounds__(kBT) k_sp_jx(SpArgs a, int xs) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (k < g.nedge + g.nprior) sp_jx_item<G>(a, g, k, xs);
}

// y = (H64 + lambda I) x per pose from J x per cost (ycost), x and y slots
// in permuted order, padding zero
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_hx(SpArgs a, int xs, int ys, double lambda) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* x = slot(a, g, xs);
  double* y = slot(a, g, ys);
  if (blockIdx.x == 0)
    for (int u = g.n + threadIdx.x; u < g.nvec; u += kBT) y[u] = 0.0;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const int gp = g.pose0 + p, ra = a.pos[gp];
  double hv[d];
#pragma unroll
  for (int r = 0; r < d; ++r) hv[r] = lambda * x[ra * d + r];
  for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
    const int sl = a.inc_slot[s];
    const double* J = a.ws64 + (size_t)(sl >> 1) * RN + (sl & 1) * d * d;
    const double* yc = a.ycost + (size_t)(sl >> 1) * d;
#pragma unroll
    for (int k = 0; k < d; ++k)
#pragma unroll
      for (int r = 0; r < d; ++r) hv[r] += J[k * d + r] * yc[k];
  }
#pragma unroll
  for (int r = 0; r < d; ++r) y[ra * d + r] = hv[r];
}

// Powell's dogleg in ||delta|| <= radius for the model
// S - g^T delta + 1/2 delta^T (H + lambda I) delta, one workgroup per graph:
// Gauss-Newton step in slot 0, g in slot 1, (H + lambda I) g in slot 2;
// the chosen step replaces slot 0
__global__ void __launch_bounds__(kBT) k_sp_dogleg(SpArgs a) {
  __shared__ double red[kBT / 64];
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  double* x = slot(a, g, 0);
  const double* gv = slot(a, g, 1);
  const double* hg = slot(a, g, 2);
  const double radius = a.dl[4 * b];
  double p0 = 0.0;
  for (int u = threadIdx.x; u < g.n; u += kBT) p0 += x[u] * x[u];
  const double n_gn = ::sqrt(block_sum_sp(p0, red));
  int boundary = 0;
  if (!(n_gn <= radius)) {
    boundary = 1;
    double p1 = 0.0, p2 = 0.0;
    for (int u = threadIdx.x; u < g.n; u += kBT) {
      p1 += gv[u] * gv[u];
      p2 += gv[u] * hg[u];
    }
    const double gg = block_sum_sp(p1, red);
    const double gHg = block_sum_sp(p2, red);
    const double alpha = gg / gHg;
    if (alpha * ::sqrt(gg) >= radius) {
      // the Cauchy point is outside: gradient direction cut at the boundary
      const double sc = radius / ::sqrt(gg);
      for (int u = threadIdx.x; u < g.n; u += kBT) x[u] = sc * gv[u];
    } else {
      // between the Cauchy point alpha g and the Gauss-Newton point
      double q1 = 0.0, q2 = 0.0;
      for (int u = threadIdx.x; u < g.n; u += kBT) {
        const double sd = alpha * gv[u], dd = x[u] - sd;
        q1 += dd * dd;
        q2 += sd * dd;
      }
      const double qa = block_sum_sp(q1, red);
      const double qb = 2.0 * block_sum_sp(q2, red);
      const double qc = alpha * alpha * gg - radius * radius;
      const double beta = (-qb + ::sqrt(qb * qb - 4.0 * qa * qc)) / (2.0 * qa);
      for (int u = threadIdx.x; u < g.n; u += kBT) {
        const double sd = alpha * gv[u];
        x[u] = sd + beta * (x[u] - sd);
      }
    }
  }
  if (threadIdx.x == 0) a.dl[4 * b + 3] = boundary;
}

// dogleg: predicted decrease g^T delta - 1/2 delta^T (H + lambda I) delta and
// |delta| (delta in slot 0, g in slot 1, (H + lambda I) delta in slot 2)
__global__ void __launch_bounds__(kBT) k_sp_dl_pred(SpArgs a) {
  __shared__ double red[kBT / 64];
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* x = slot(a, g, 0);
  const double* gv = slot(a, g, 1);
  const double* hx = slot(a, g, 2);
  double r1 = 0.0, r2 = 0.0, r3 = 0.0;
  for (int u = threadIdx.x; u < g.n; u += kBT) {
    r1 += gv[u] * x[u];
    r2 += x[u] * hx[u];
    r3 += x[u] * x[u];
  }
  const double s1 = block_sum_sp(r1, red);
  const double s2 = block_sum_sp(r2, red);
  const double s3 = block_sum_sp(r3, red);
  if (threadIdx.x == 0) {
    a.dl[4 * b + 1] = s1 - 0.5 * s2;
    a.dl[4 * b + 2] = ::sqrt(s3);
  }
}

// x += correction (slot 2) per pose, then retract on the last sweep
template <int G>
__device__ __forceinline__ void sp_accumulate_item(const SpArgs& a, const SpDesc& g, int p, int retract) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  double* x = slot(a, g, 0) + a.pos[g.pose0 + p] * d;
  const double* dx = slot(a, g, 2) + a.pos[g.pose0 + p] * d;
#pragma unroll
  for (int r = 0; r < d; ++r) x[r] += dx[r];
  if (retract) retract_minus<G>(a.poses + (size_t)(g.pose0 + p) * sz, x);
}

template <int G>
__global__ void __launch_bounds__(kBT) k_sp_accumulate(SpArgs a, int retract) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p < g.npose) sp_accumulate_item<G>(a, g, p, retract);
}

// exact-Hessian backward, per cost: J u (ycost) and the second-order terms
// w^2 (dC/ds)^T c of both sides along u (hvp), u in slot 0 (permuted order)
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_hvp_cost(SpArgs a) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (k >= g.nedge + g.nprior) return;
  const double* x = slot(a, g, 0);
  int rk, pi = -1, pj;
  if (k < g.nedge) {
    rk = g.edge0 + k;
    pi = a.pos[a.edge_ij[2 * rk]];
    pj = a.pos[a.edge_ij[2 * rk + 1]];
  } else {
    rk = a.E + g.prior0 + (k - g.nedge);
    pj = a.pos[a.prior_var[g.prior0 + (k - g.nedge)]];
  }
  const double* J = a.ws64 + (size_t)rk * RN;
#pragma unroll
  for (int r = 0; r < d; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      if (pi >= 0) acc += J[r * d + q] * x[pi * d + q];
      acc += J[d * d + r * d + q] * x[pj * d + q];
    }
    a.ycost[(size_t)rk * d + r] = acc;
  }
  double* o = a.hvp + (size_t)rk * 2 * d;
  cost_hvp_residual<G>(cost_data(a), rk, J, pi >= 0 ? x + pi * d : nullptr, x + pj * d, o, o + d);
}

// exact-Hessian backward, per pose: residual v - Hx u of the refinement into
// slot 2 (permuted order, padding zero), Hx u = sum J^T J u + the cost terms
// - 1/2 ad(u_p)^T g_p with g_p = sum J^T r at theta_K
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_hvp_res(SpArgs a) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* x = slot(a, g, 0);
  double* res = slot(a, g, 2);
  if (blockIdx.x == 0)
    for (int u = g.n + threadIdx.x; u < g.nvec; u += kBT) res[u] = 0.0;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const int gp = g.pose0 + p, ra = a.pos[gp];
  double hv[d], gv[d];
#pragma unroll
  for (int r = 0; r < d; ++r) hv[r] = gv[r] = 0.0;
  for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
    const int sl = a.inc_slot[s];
    const double* J = a.ws64 + (size_t)(sl >> 1) * RN + (sl & 1) * d * d;
    const double* rr = a.ws64 + (size_t)(sl >> 1) * RN + 2 * d * d;
    const double* yc = a.ycost + (size_t)(sl >> 1) * d;
    const double* hc = a.hvp + (size_t)(sl >> 1) * 2 * d + (sl & 1) * d;
#pragma unroll
    for (int k = 0; k < d; ++k)
#pragma unroll
      for (int r = 0; r < d; ++r) {
        hv[r] += J[k * d + r] * yc[k];
        gv[r] += J[k * d + r] * rr[k];
      }
#pragma unroll
    for (int r = 0; r < d; ++r) hv[r] += hc[r];
  }
  double t[d];
  ad_transpose_mul<G>(x + ra * d, gv, t);
#pragma unroll
  for (int r = 0; r < d; ++r) res[ra * d + r] = a.seed[(size_t)gp * d + r] - (hv[r] - 0.5 * t[r]);
}

// DLM backward, per cost: dS/dphi at the poses `x`, times `scale`, stored
// or added; graphs marked failed get zero gradients
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_param_grads(SpArgs a, const double* x, double scale, int accumulate) {
  constexpr int d = GroupTraits<G>::d;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (k >= g.nedge + g.nprior) return;
  const bool zero = a.failed[b] != 0;
  PoseCostData cd = cost_data(a);
  cd.poses = x;
  double dl = 0.0, dt[d], dlc = 0.0;
#pragma unroll
  for (int q = 0; q < d; ++q) dt[q] = 0.0;
  if (k < g.nedge) {
    const int e = g.edge0 + k;
    if (!zero) cost_param_grad<G>(cd, e, &dl, dt, &dlc);
    if (a.g_logw_e) a.g_logw_e[e] = zero ? 0.0 : (accumulate ? a.g_logw_e[e] : 0.0) + scale * dl;
    if (a.g_logc) a.g_logc[e] = zero ? 0.0 : (accumulate ? a.g_logc[e] : 0.0) + scale * dlc;
    if (a.g_tau)
#pragma unroll
      for (int q = 0; q < d; ++q) {
        double& o = a.g_tau[(size_t)e * d + q];
        o = zero ? 0.0 : (accumulate ? o : 0.0) + scale * dt[q];
      }
  } else {
    const int pq = g.prior0 + (k - g.nedge);
    if (!zero) cost_param_grad<G>(cd, a.E + pq, &dl, dt, nullptr);
    if (a.g_logw_p) a.g_logw_p[pq] = zero ? 0.0 : (accumulate ? a.g_logw_p[pq] : 0.0) + scale * dl;
  }
}

// DLM backward: right-hand side g* - eps v in slot 2 (permuted order, padding
// zero), so that the solve gives -delta of (H* + 2 eps^2 I) delta = -g* + eps v
__global__ void __launch_bounds__(kBT) k_sp_dlm_rhs(SpArgs a, int d, double eps) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* rhs = slot(a, g, 1);
  double* x = slot(a, g, 2);
  if (blockIdx.x == 0)
    for (int u = g.n + threadIdx.x; u < g.nvec; u += kBT) x[u] = 0.0;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const int ra = a.pos[g.pose0 + p];
  for (int r = 0; r < d; ++r) x[ra * d + r] = rhs[ra * d + r] - eps * a.seed[(size_t)(g.pose0 + p) * d + r];
}

// unrolled backward (truncated to the last T steps), a reverse sweep through
// theta_{t+1} = theta_t Exp(-delta_t), delta_t = (H_t + lambda I)^-1 g_t, the
// iterates read from the factor cache.  Per step, with abar (uout, original
// order) the cotangent at theta_{t+1}:
//   dbar_p = -Jr(-delta_p)^T abar_p,  abar_p <- Ad(Exp(delta_p))^T abar_p,
//   y = (H_t + lambda I)^-1 dbar, then the gradient of
//   s = y^T g_t - y^T (H_t + lambda I) delta_t (y, delta_t fixed) is added to
//   abar and to the parameter gradients.

// abar = seed (init = 1) or, for graphs marked failed, zero (init = 0: only those)
__global__ void __launch_bounds__(kBT) k_sp_unroll_adj(SpArgs a, int d, int init) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const bool failed = a.failed[b] != 0;
  if (!init && !failed) return;
  for (int r = 0; r < d; ++r) {
    const size_t u = (size_t)(g.pose0 + p) * d + r;
    a.uout[u] = failed ? 0.0 : a.seed[u];
  }
}

// parameter gradients zero (all graphs, or only = 1: the graphs marked failed)
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_grads_zero(SpArgs a, int only) {
  constexpr int d = GroupTraits<G>::d;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (only && !a.failed[b]) return;
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (k >= g.nedge + g.nprior) return;
  if (k < g.nedge) {
    const int e = g.edge0 + k;
    if (a.g_logw_e) a.g_logw_e[e] = 0.0;
    if (a.g_tau)
      for (int q = 0; q < d; ++q) a.g_tau[(size_t)e * d + q] = 0.0;
  } else if (a.g_logw_p) {
    a.g_logw_p[g.prior0 + (k - g.nedge)] = 0.0;
  }
}

// through the retraction: dbar into slot 2 (permuted order, padding zero),
// delta_t in slot 0
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_unroll_retr(SpArgs a) {
  constexpr int d = GroupTraits<G>::d;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* vd = slot(a, g, 0);
  double* vw = slot(a, g, 2);
  if (blockIdx.x == 0)
    for (int u = g.n + threadIdx.x; u < g.nvec; u += kBT) vw[u] = 0.0;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const int gp = g.pose0 + p, ra = a.pos[gp];
  double dl[d], md[d], Jr[d * d], Ad[d * d], ab[d];
  for (int q = 0; q < d; ++q) {
    dl[q] = vd[ra * d + q];
    md[q] = -dl[q];
    ab[q] = a.uout[(size_t)gp * d + q];
  }
  if constexpr (G == 3) {
    double E[12], R[9], tv[3];
    se3_jr(md, Jr);
    se3_exp(dl, E);
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) R[r * 3 + q] = E[r * 4 + q];
      tv[r] = E[r * 4 + 3];
    }
    se3_adjoint(R, tv, Ad);
  } else {
    double E[4];
    se2_jr(md, Jr);
    se2_exp(dl, E);
    se2_adjoint(E[0], E[1], E[2], E[3], Ad);
  }
  for (int m = 0; m < d; ++m) {
    double s1 = 0.0, s2 = 0.0;
    for (int q = 0; q < d; ++q) {
      s1 += Jr[q * d + m] * ab[q];
      s2 += Ad[q * d + m] * ab[q];
    }
    vw[ra * d + m] = -s1;
    a.uout[(size_t)gp * d + m] = s2;
  }
}

// per cost: the gradient of s at the poses (hvp buffer, both sides) and at
// the parameters (accumulated); y in slot 2, delta_t in slot 0
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_unroll_cost(SpArgs a) {
  constexpr int d = GroupTraits<G>::d;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (k >= g.nedge + g.nprior) return;
  const double* vd = slot(a, g, 0);
  const double* vw = slot(a, g, 2);
  int rk, pi = -1, pj;
  if (k < g.nedge) {
    rk = g.edge0 + k;
    pi = a.pos[a.edge_ij[2 * rk]];
    pj = a.pos[a.edge_ij[2 * rk + 1]];
  } else {
    rk = a.E + g.prior0 + (k - g.nedge);
    pj = a.pos[a.prior_var[g.prior0 + (k - g.nedge)]];
  }
  double* o = a.hvp + (size_t)rk * 2 * d;
  double dlw, dt[d];
  cost_unroll_vjp<G>(cost_data(a), rk, pi >= 0 ? vw + pi * d : nullptr, vw + pj * d,
                     pi >= 0 ? vd + pi * d : nullptr, vd + pj * d, o, o + d, &dlw, k < g.nedge ? dt : nullptr);
  if (pi < 0)
    for (int q = 0; q < d; ++q) o[q] = 0.0;
  if (k < g.nedge) {
    if (a.g_logw_e) a.g_logw_e[rk] += dlw;
    if (a.g_tau)
      for (int q = 0; q < d; ++q) a.g_tau[(size_t)rk * d + q] += dt[q];
  } else if (a.g_logw_p) {
    a.g_logw_p[rk - a.E] += dlw;
  }
}

// abar += the pose terms of the step's costs (incidence lists)
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_unroll_gather(SpArgs a) {
  constexpr int d = GroupTraits<G>::d;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const int gp = g.pose0 + p;
  double v[d];
  for (int r = 0; r < d; ++r) v[r] = 0.0;
  for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
    const int sl = a.inc_slot[s];
    const double* o = a.hvp + (size_t)(sl >> 1) * 2 * d + (sl & 1) * d;
    for (int r = 0; r < d; ++r) v[r] += o[r];
  }
  for (int r = 0; r < d; ++r) a.uout[(size_t)gp * d + r] += v[r];
}

// backward: b = seed in permuted order (padding zero)
__global__ void __launch_bounds__(kBT) k_sp_seed(SpArgs a, int d) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  double* x = slot(a, g, 2);
  if (blockIdx.x == 0)
    for (int u = g.n + threadIdx.x; u < g.nvec; u += kBT) x[u] = 0.0;
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  for (int r = 0; r < d; ++r) x[a.pos[g.pose0 + p] * d + r] = a.seed[(size_t)(g.pose0 + p) * d + r];
}

// backward: adjoint in the original pose order (zero for graphs not OK)
__global__ void __launch_bounds__(kBT) k_sp_uout(SpArgs a, int d) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  const int p = blockIdx.x * kBT + threadIdx.x;
  if (p >= g.npose) return;
  const bool ok = a.status[b] == DNLS_GRAPH_OK;
  const double* x = slot(a, g, 0);
  for (int r = 0; r < d; ++r)
    a.uout[(size_t)(g.pose0 + p) * d + r] = ok ? x[a.pos[g.pose0 + p] * d + r] : 0.0;
}

template <int G>
__global__ void __launch_bounds__(kBT) k_sp_vjp(SpArgs a) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (k >= g.nedge + g.nprior) return;
  const bool ok = a.status[b] == DNLS_GRAPH_OK;
  int rk;
  const double *ui = nullptr, *uj;
  if (k < g.nedge) {
    rk = g.edge0 + k;
    ui = a.uout + (size_t)a.edge_ij[2 * rk] * d;
    uj = a.uout + (size_t)a.edge_ij[2 * rk + 1] * d;
  } else {
    rk = a.E + g.prior0 + (k - g.nedge);
    uj = a.uout + (size_t)a.prior_var[rk - a.E] * d;
  }
  if (!ok) {
    if (k < g.nedge) {
      if (a.g_logw_e) a.g_logw_e[rk] = 0.0;
      if (a.g_logc) a.g_logc[rk] = 0.0;
      if (a.g_tau)
        for (int q = 0; q < d; ++q) a.g_tau[(size_t)rk * d + q] = 0.0;
    } else if (a.g_logw_p) {
      a.g_logw_p[rk - a.E] = 0.0;
    }
    return;
  }
  cost_vjp<G>(cost_data(a), rk, a.ws64 + (size_t)rk * RN, ui, uj, a.g_logw_e, a.g_tau, a.g_logw_p, a.g_logc);
}

// ---------------------------------------------------------------------------
// BLOCK schedule: the factor in d x d pose blocks (tile size d), factored
// left-looking by levels of the elimination tree.  A column's level is one
// more than the highest level of the columns it depends on (its children in
// the tree), so all columns of a level are computed at once from lower
// levels only:
//   A. L_IJ = A_IJ - sum_{K < J} L_IK L_JK^T for every block (I, J) of the
//      level's columns (K runs over row J's structure; the diagonal block's
//      lower triangle only);
//   B. L_JJ = chol(L_JJ) and W_J = L_JJ^-1, one thread per column;
//   C. L_IJ <- L_IJ W_J^T below the diagonal, one thread per block row.
// The triangular solves run by the same levels (forward: ascending,
// backward: descending), the vector in LDS.  d <= 6.
// ---------------------------------------------------------------------------
template <int NT, int D>
__device__ bool sb_factor_body(const SpArgs& a, int b, const SpDesc& g, int* flag) {
  constexpr int ts = D, tt = D * D;
  for (int L = 0; L < g.nlvl; ++L) {
    // A. left-looking gather of the level's blocks
    const int b0 = a.lvlbptr[g.lvl_off + L], b1 = a.lvlbptr[g.lvl_off + L + 1];
    double* pool = a.factor + g.pool_off;
    for (int u = threadIdx.x; u < (b1 - b0) * tt; u += NT) {
      const int4 t = a.lvlblk[b0 + u / tt];
      const int e = u % tt, r = e / ts, c = e % ts;
      if ((t.w & 1) && c > r) continue;
      double* T = pool + (size_t)t.x * tt;
      double acc = T[e];
#pragma unroll 4
      for (int k = t.y; k < t.z; ++k) {
        const int2 pr = a.cpair[k];
        const double* LI = pool + (size_t)pr.x * tt + r * ts;
        const double* LJ = pool + (size_t)pr.y * tt + c * ts;
#pragma unroll
        for (int q = 0; q < ts; ++q) acc -= LI[q] * LJ[q];
      }
      T[e] = acc;
    }
    __syncthreads();
    // B. diagonal blocks: Cholesky and inverse, one thread per column
    const int c0 = a.lvlptr[g.lvl_off + L], c1 = a.lvlptr[g.lvl_off + L + 1];
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    for (int u = c0 + (int)threadIdx.x; u < c1; u += NT) {
      const int J = a.lvlcol[u];
      double* T = pool + (size_t)(a.colptr[g.col_off + J] - a.colptr[g.col_off]) * tt;
      double l[D][D], w[D][D];
      bool ok = true;
#pragma unroll
      for (int i = 0; i < ts; ++i)
#pragma unroll
        for (int j = 0; j < ts; ++j) l[i][j] = (j <= i) ? T[i * ts + j] : 0.0;
#pragma unroll
      for (int j = 0; j < ts; ++j) {
        double dj = l[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) dj -= l[j][k] * l[j][k];
        ok = ok && dj > 0.0;
        const double ljj = ::sqrt(dj > 0.0 ? dj : 1.0);
        l[j][j] = ljj;
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < ts; ++i) {
          double v = l[i][j];
#pragma unroll
          for (int k = 0; k < j; ++k) v -= l[i][k] * l[j][k];
          l[i][j] = v * inv;
        }
      }
      // W = L^-1 (lower), column by column of the identity
#pragma unroll
      for (int j = 0; j < ts; ++j)
#pragma unroll
        for (int i = 0; i < ts; ++i) {
          if (i < j) {
            w[i][j] = 0.0;
            continue;
          }
          double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
          for (int k = j; k < i; ++k) v -= l[i][k] * w[k][j];
          w[i][j] = v / l[i][i];
        }
      double* W = a.factor + g.winv_off + (size_t)J * tt;
#pragma unroll
      for (int i = 0; i < ts; ++i)
#pragma unroll
        for (int j = 0; j < ts; ++j) {
          T[i * ts + j] = (j <= i) ? l[i][j] : 0.0;
          W[i * ts + j] = w[i][j];
        }
      if (!ok) *flag = 1;
    }
    __syncthreads();
    if (*flag) {
      if (threadIdx.x == 0) {
        a.failed[b] = DNLS_GRAPH_NOT_PD;
        a.status[b] = DNLS_GRAPH_NOT_PD;
      }
      return false;
    }
    // C. L_IJ <- L_IJ W_J^T below the diagonal, one thread per block row
    for (int u = threadIdx.x; u < (b1 - b0) * ts; u += NT) {
      const int4 t = a.lvlblk[b0 + u / ts];
      if (t.w & 1) continue;
      const int r = u % ts;
      double* row = pool + (size_t)t.x * tt + r * ts;
      const double* W = a.factor + g.winv_off + (size_t)(t.w >> 1) * tt;
      double x[D], y[D];
#pragma unroll
      for (int q = 0; q < ts; ++q) x[q] = row[q];
#pragma unroll
      for (int c = 0; c < ts; ++c) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q <= c; ++q) v += x[q] * W[c * ts + q];
        y[c] = v;
      }
#pragma unroll
      for (int c = 0; c < ts; ++c) row[c] = y[c];
    }
    __syncthreads();
  }
  return true;
}

// x (slot dst) = (L L^T)^-1 b (slot src), v: nvec doubles of LDS
template <int NT, int D>
__device__ void sb_solve_body(const SpArgs& a, const SpDesc& g, int src, int dst, double* v) {
  constexpr int ts = D, tt = D * D;
  const double* pool = a.factor + g.pool_off;
  const double* bsrc = slot(a, g, src);
  for (int u = threadIdx.x; u < g.nvec; u += NT) v[u] = bsrc[u];
  __syncthreads();
  // forward: v_J <- W_J (v_J - sum_{K < J} L_JK v_K), levels ascending
  for (int L = 0; L < g.nlvl; ++L) {
    const int c0 = a.lvlptr[g.lvl_off + L], c1 = a.lvlptr[g.lvl_off + L + 1];
    for (int u = threadIdx.x; u < (c1 - c0) * ts; u += NT) {
      const int J = a.lvlcol[c0 + u / ts], r = u % ts;
      double acc = v[J * ts + r];
#pragma unroll 4
      for (int k = a.rowptr[g.row_off + J]; k < a.rowptr[g.row_off + J + 1]; ++k) {
        const int K = a.rowcol[k];
        const double* row = pool + (size_t)a.rowid[k] * tt + r * ts;
#pragma unroll
        for (int q = 0; q < ts; ++q) acc -= row[q] * v[K * ts + q];
      }
      v[J * ts + r] = acc;
    }
    __syncthreads();
    for (int u = c0 + (int)threadIdx.x; u < c1; u += NT) {
      const int J = a.lvlcol[u];
      const double* W = a.factor + g.winv_off + (size_t)J * tt;
      double x[D];
#pragma unroll
      for (int q = 0; q < ts; ++q) x[q] = v[J * ts + q];
#pragma unroll
      for (int r = 0; r < ts; ++r) {
        double y = 0.0;
#pragma unroll
        for (int q = 0; q <= r; ++q) y += W[r * ts + q] * x[q];
        v[J * ts + r] = y;
      }
    }
    __syncthreads();
  }
  // backward: v_J <- W_J^T (v_J - sum_{I > J} L_IJ^T v_I), levels descending
  for (int L = g.nlvl - 1; L >= 0; --L) {
    const int c0 = a.lvlptr[g.lvl_off + L], c1 = a.lvlptr[g.lvl_off + L + 1];
    for (int u = threadIdx.x; u < (c1 - c0) * ts; u += NT) {
      const int J = a.lvlcol[c0 + u / ts], r = u % ts;
      double acc = v[J * ts + r];
#pragma unroll 4
      for (int k = a.colptr[g.col_off + J] + 1; k < a.colptr[g.col_off + J + 1]; ++k) {
        const int I = a.rowidx[k];
        const double* T = pool + (size_t)(k - a.colptr[g.col_off]) * tt;
#pragma unroll
        for (int q = 0; q < ts; ++q) acc -= T[q * ts + r] * v[I * ts + q];
      }
      v[J * ts + r] = acc;
    }
    __syncthreads();
    for (int u = c0 + (int)threadIdx.x; u < c1; u += NT) {
      const int J = a.lvlcol[u];
      const double* W = a.factor + g.winv_off + (size_t)J * tt;
      double x[D];
#pragma unroll
      for (int q = 0; q < ts; ++q) x[q] = v[J * ts + q];
#pragma unroll
      for (int r = 0; r < ts; ++r) {
        double y = 0.0;
#pragma unroll
        for (int q = r; q < ts; ++q) y += W[q * ts + r] * x[q];
        v[J * ts + r] = y;
      }
    }
    __syncthreads();
  }
  double* xdst = slot(a, g, dst);
  for (int u = threadIdx.x; u < g.nvec; u += NT) xdst[u] = v[u];
  __syncthreads();
}

template <int D>
__global__ void __launch_bounds__(kPT) k_sb_factor(SpArgs a) {
  __shared__ int flag;
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  sb_factor_body<kPT, D>(a, b, g, &flag);
}

template <int D>
__global__ void __launch_bounds__(kPT) k_sb_solve(SpArgs a, int src, int dst) {
  __shared__ double v[kSolveLds];
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  sb_solve_body<kPT, D>(a, g, src, dst, v);
}

// ---------------------------------------------------------------------------
// Persistent whole-solve kernel (schedule PERSISTENT): one launch runs every
// step of every graph.  A grid of at most one workgroup per resident slot
// takes graphs from a device-memory queue (largest first, the plan's launch
// order), and each workgroup then runs the graph's K steps and its final
// linearisation with no launch in between: linearisation, assembly into the
// tile pool, the one-workgroup tile factorisation, the one-workgroup
// triangular solves in LDS, the float64 refinement sweeps of the mixed path
// and the retraction, separated by workgroup barriers.  The same per-item
// code as the per-phase kernels, so the arithmetic is the same.
// queue[0]: next graph slot; queue[1]: workgroups done (the last one resets
// both, so every launch, or every replay of a captured graph, starts at 0).
// ---------------------------------------------------------------------------
union FusedLds {
  DenseLds f;
  struct {
    double v[kSolveLds];
    double Wl[kTS * kSW];
    double y[kTS];
  } s;
};
struct BlockLds {          // BLOCK: only the solve's vector
  struct {
    double v[kSolveLds];
  } s;
};

template <int G, bool MIXED, bool BLOCK>
__global__ void __launch_bounds__(kPT) k_sp_persistent(SpArgs a, const int* order, unsigned* queue, int B,
                                                       int refine_from, int refine_until) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n, sz = GroupTraits<G>::sz;
  __shared__ std::conditional_t<BLOCK, BlockLds, FusedLds> L;
  __shared__ double red[kPT / 64];
  __shared__ int q_slot, stop;
  const PoseCostData cd = cost_data(a);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) q_slot = (int)atomicAdd(&queue[0], 1u);
    __syncthreads();
    if (q_slot >= B) break;
    const int b = order[q_slot];
    const SpDesc g = a.sd[b];
    double* obj = a.objective + (size_t)b * (a.K + 1);
    if (threadIdx.x == 0) {
      a.failed[b] = 0;
      a.status[b] = DNLS_GRAPH_OK;
    }
    const int ncost = g.nedge + g.nprior;
    double last = 0.0;
    int it = 0;
    for (; it <= a.K; ++it) {
      const bool final_lin = it == a.K;
      const double lam = final_lin ? 0.0 : a.lambda;
      if (a.traj && !final_lin) {
        // DNLS_FLAG_KEEP_ITERATES: theta_t into the factor cache
        double* dst = a.traj + ((size_t)it * a.V + g.pose0) * sz;
        for (int u = threadIdx.x; u < g.npose * sz; u += kPT) dst[u] = a.poses[(size_t)g.pose0 * sz + u];
      }
      const bool lin32 = MIXED && !final_lin;
      const bool refine_now = lin32 && a.refine > 0 && it >= refine_from && it < refine_until;
      const bool lin64 = !MIXED || refine_now || final_lin;
      // 1. linearisation (float64 last, so that S is the float64 objective
      // whenever float64 records are made)
      double s32 = 0.0, s64 = 0.0;
      for (int k = threadIdx.x; k < ncost; k += kPT) {
        const int rk = (k < g.nedge) ? g.edge0 + k : a.E + g.prior0 + (k - g.nedge);
        if (lin32) s32 += linearize_cost<G, float>(cd, rk, a.ws32 + (size_t)rk * RN);
        if (lin64) s64 += linearize_cost<G, double>(cd, rk, a.ws64 + (size_t)rk * RN);
      }
      const double S = block_sum_sp(lin64 ? s64 : s32, red);
      last = S;
      if (threadIdx.x == 0) obj[it] = S;
      if (!isfinite(S)) {
        if (threadIdx.x == 0) {
          a.failed[b] = DNLS_GRAPH_NONFINITE;
          a.status[b] = DNLS_GRAPH_NONFINITE;
        }
        break;
      }
      // 2. zero the tile pool, then assemble H (+ lambda I) and g
      {
        double* pool = a.factor + g.pool_off;
        const size_t n = (size_t)g.ntile * (a.ts * a.ts);
        for (size_t u = threadIdx.x; u < n; u += kPT) pool[u] = 0.0;
      }
      __syncthreads();
      const int nblk = g.npose + g.nod;
      if (lin32) {
        for (int u = threadIdx.x; u < nblk; u += kPT)
          sp_assemble_item<G, float>(a, g, u, a.ws32, lam, refine_now ? 0 : 1);
        if (refine_now)
          for (int u = threadIdx.x; u < g.npose; u += kPT) sp_rhs64_item<G>(a, g, u);
      } else {
        for (int u = threadIdx.x; u < nblk; u += kPT) sp_assemble_item<G, double>(a, g, u, a.ws64, lam, 1);
      }
      sp_assemble_pad(a, g, threadIdx.x, kPT);
      __syncthreads();
      // 3. factorisation
      if constexpr (BLOCK) {
        if (!sb_factor_body<kPT, d>(a, b, g, &stop)) break;
      } else {
        if (!sp_factor_wg_body<kPT>(a, b, g, reinterpret_cast<FusedLds&>(L).f)) break;
      }
      if (final_lin) break;
      // 4. step: slot 2 = g, slot 0 = (L L^T)^-1 g
      {
        double* x = slot(a, g, 2);
        const double* rhs = slot(a, g, 1);
        for (int u = threadIdx.x; u < g.nvec; u += kPT) x[u] = rhs[u];
      }
      __syncthreads();
      if constexpr (BLOCK) sb_solve_body<kPT, d>(a, g, 2, 0, L.s.v);
      else sp_solve_wg_body<kPT>(a, g, 2, 0, L.s.v, reinterpret_cast<FusedLds&>(L).s.Wl,
                                 reinterpret_cast<FusedLds&>(L).s.y);
      __syncthreads();
      if (!refine_now) {
        for (int p = threadIdx.x; p < g.npose; p += kPT) sp_retract_item<G>(a, g, p, 0);
      } else {
        for (int sw = 0; sw < a.refine; ++sw) {
          // slot 2 = g64 - (H64 + lambda I) x;  x += (L L^T)^-1 slot 2
          for (int k = threadIdx.x; k < ncost; k += kPT) sp_jx_item<G>(a, g, k, 0);
          __syncthreads();
          {
            double* res = slot(a, g, 2);
            for (int u = g.n + threadIdx.x; u < g.nvec; u += kPT) res[u] = 0.0;
          }
          for (int p = threadIdx.x; p < g.npose; p += kPT) sp_residual_item<G>(a, g, p, lam);
          __syncthreads();
          if constexpr (BLOCK) sb_solve_body<kPT, d>(a, g, 2, 2, L.s.v);
          else sp_solve_wg_body<kPT>(a, g, 2, 2, L.s.v, reinterpret_cast<FusedLds&>(L).s.Wl,
                                     reinterpret_cast<FusedLds&>(L).s.y);
          __syncthreads();
          for (int p = threadIdx.x; p < g.npose; p += kPT) sp_accumulate_item<G>(a, g, p, sw + 1 == a.refine);
          __syncthreads();
        }
      }
      __syncthreads();
    }
    // a failed graph keeps its poses and repeats its last objective
    if (it < a.K && threadIdx.x == 0)
      for (int t = it + 1; t <= a.K; ++t) obj[t] = last;
  }
  // the last workgroup to finish resets the queue for the next launch
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&queue[1], 1u) == gridDim.x - 1) {
      atomicExch(&queue[0], 0u);
      atomicExch(&queue[1], 0u);
    }
  }
}

// ---------------------------------------------------------------------------
// Bundle adjustment on the block-sparse solver: cameras (6) and points (3)
// in one system, the points ordered first so that the tile factorisation
// eliminates them before the cameras (the point columns are block diagonal
// and their updates of the camera tiles form the Schur complement), the
// cameras after them in minimum-degree order of their co-observation graph.
// The same tile kernels factor and solve the system as for pose graphs.
// ---------------------------------------------------------------------------
constexpr int kObsRecSp = 20;

__device__ __forceinline__ double spba_radius(const SpArgs& a, int b) { return a.delta_b ? a.delta_b[b] : a.huber; }

// observation and prior records of problem blockIdx.y (grid x over its
// observations, then its priors) and the objective partials
template <class S>
__global__ void __launch_bounds__(kBT) k_spba_lin(SpArgs a) {
  constexpr int RN = CostRec<6>::n;
  __shared__ double red[kBT / 64];
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  double s = 0.0;
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (!a.failed[b]) {
    if (t < g.nobs) {
      const int o = g.obs0 + t;
      double c[2], Jc[12], Jp[6];
      reproj<double>(a.poses + (size_t)a.obs_cam[o] * 12, a.pts + (size_t)a.obs_pt[o] * 3, a.obs_uv + (size_t)o * 2,
                     a, c, Jc, Jp);
      const double w = a.obs_w[o];
      double rho, drho;
      huber(w * w * (c[0] * c[0] + c[1] * c[1]), spba_radius(a, b), rho, drho);
      const double sw = ::sqrt(drho) * w;
      S* rec = reinterpret_cast<S*>(a.orec) + (size_t)o * kObsRecSp;
#pragma unroll
      for (int k = 0; k < 12; ++k) rec[k] = S(sw * Jc[k]);
#pragma unroll
      for (int k = 0; k < 6; ++k) rec[12 + k] = S(sw * Jp[k]);
      rec[18] = S(sw * c[0]);
      rec[19] = S(sw * c[1]);
      if constexpr (!std::is_same<S, double>::value) {
        const double s2 = sw * sw;
        double* go = a.gob + (size_t)o * 9;
#pragma unroll
        for (int k = 0; k < 6; ++k) go[k] = s2 * (Jc[k] * c[0] + Jc[6 + k] * c[1]);
#pragma unroll
        for (int k = 0; k < 3; ++k) go[6 + k] = s2 * (Jp[k] * c[0] + Jp[3 + k] * c[1]);
      }
      s = 0.5 * rho;
    } else if (t < g.nobs + g.nprior) {
      const int rk = a.E + g.prior0 + (t - g.nobs);
      s = linearize_cost<3, double>(cost_data(a), rk, a.ws64 + (size_t)rk * RN);
    }
  }
  s = block_sum_sp(s, red);
  if (threadIdx.x == 0) a.partial[b * a.nx + blockIdx.x] = s;
}

// Hessian blocks into the tiles and g into slot 1: item u < ncam a camera's
// diagonal block (observations and priors), then the points' diagonal
// blocks, then the camera-point blocks (cameras follow the points, so these
// lie below the diagonal); the padding scalars get a unit diagonal
template <class S>
__global__ void __launch_bounds__(kBT) k_spba_assemble(SpArgs a, double lambda) {
  constexpr int RN = CostRec<6>::n;
  constexpr bool MIX = !std::is_same<S, double>::value;
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const S* rec = reinterpret_cast<const S*>(a.orec);
  double* rhs = slot(a, g, 1);
  const int u = blockIdx.x * kBT + threadIdx.x;
  if (u < g.npose) {
    const int cam = g.pose0 + u, r0 = a.soff_cam[cam];
    S h[36];
    double gr[6], hp[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) {
      h[k] = S(0);
      hp[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) gr[k] = 0.0;
    for (int s = a.cam_obs_off[cam]; s < a.cam_obs_off[cam + 1]; ++s) {
      const int o = a.cam_obs[s];
      const S* r = rec + (size_t)o * kObsRecSp;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) h[i * 6 + j] += r[i] * r[j] + r[6 + i] * r[6 + j];
        if constexpr (MIX) gr[i] += a.gob[(size_t)o * 9 + i];
        else gr[i] += r[i] * r[18] + r[6 + i] * r[19];
      }
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      if (a.prior_var[q] != cam) continue;
      const double* J = a.ws64 + (size_t)(a.E + q) * RN + 36;
      const double* res = a.ws64 + (size_t)(a.E + q) * RN + 72;
      for (int i = 0; i < 6; ++i) {
        for (int j = 0; j <= i; ++j) {
          double v = 0.0;
          for (int k = 0; k < 6; ++k) v += J[k * 6 + i] * J[k * 6 + j];
          hp[i * 6 + j] += v;
        }
        double v = 0.0;
        for (int k = 0; k < 6; ++k) v += J[k * 6 + i] * res[k];
        gr[i] += v;
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
      for (int j = 0; j <= i; ++j) put(a, g, r0 + i, r0 + j, double(h[i * 6 + j]) + hp[i * 6 + j] + (i == j ? lambda : 0.0));
      rhs[r0 + i] = gr[i];
    }
  } else if (u < g.npose + g.npt) {
    const int pt = g.pt0 + (u - g.npose), r0 = a.soff_pt[pt];
    S h[9];
    double gr[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 9; ++k) h[k] = S(0);
    for (int s = a.pt_obs_off[pt]; s < a.pt_obs_off[pt + 1]; ++s) {
      const int o = a.pt_obs[s];
      const S* r = rec + (size_t)o * kObsRecSp;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) h[i * 3 + j] += r[12 + i] * r[12 + j] + r[15 + i] * r[15 + j];
        if constexpr (MIX) gr[i] += a.gob[(size_t)o * 9 + 6 + i];
        else gr[i] += r[12 + i] * r[18] + r[15 + i] * r[19];
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j <= i; ++j) put(a, g, r0 + i, r0 + j, double(h[i * 3 + j]) + (i == j ? lambda : 0.0));
      rhs[r0 + i] = gr[i];
    }
  } else if (u < g.npose + g.npt + g.ncp) {
    const int4 blk = a.cp_blk[g.cp0 + (u - g.npose - g.npt)];
    const int rc = a.soff_cam[blk.x], rp = a.soff_pt[blk.y];
    S h[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) h[k] = S(0);
    for (int s = blk.z; s < blk.z + blk.w; ++s) {
      const S* r = rec + (size_t)a.cp_obs[s] * kObsRecSp;
#pragma unroll
      for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) h[i * 3 + j] += r[i] * r[12 + j] + r[6 + i] * r[15 + j];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) put(a, g, rc + i, rp + j, double(h[i * 3 + j]));
  }
  if (blockIdx.x == 0) {
    for (int r = g.pad0 + threadIdx.x; r < g.pad1; r += kBT) {
      put(a, g, r, r, 1.0);
      rhs[r] = 0.0;
    }
    sp_assemble_pad(a, g, threadIdx.x, kBT);
  }
}

// cameras X <- X Exp(-x_c), points q <- q - x_q (x in slot xs, elimination order)
__global__ void __launch_bounds__(kBT) k_spba_update(SpArgs a, int xs) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  const double* x = slot(a, g, xs);
  const int u = blockIdx.x * kBT + threadIdx.x;
  if (u < g.npose) {
    const int cam = g.pose0 + u;
    retract_minus<3>(a.poses + (size_t)cam * 12, x + a.soff_cam[cam]);
  } else if (u < g.npose + g.npt) {
    const int pt = g.pt0 + (u - g.npose);
    const double* xp = x + a.soff_pt[pt];
#pragma unroll
    for (int k = 0; k < 3; ++k) a.pts[(size_t)pt * 3 + k] -= xp[k];
  }
}

// backward: the seed (cameras, points) into slot 2 in elimination order, padding zero
__global__ void __launch_bounds__(kBT) k_spba_seed(SpArgs a) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  double* x = slot(a, g, 2);
  if (blockIdx.x == 0) {
    for (int r = g.pad0 + threadIdx.x; r < g.pad1; r += kBT) x[r] = 0.0;
    for (int r = g.n + threadIdx.x; r < g.nvec; r += kBT) x[r] = 0.0;
  }
  const int u = blockIdx.x * kBT + threadIdx.x;
  if (u < g.npose) {
    const int cam = g.pose0 + u;
#pragma unroll
    for (int k = 0; k < 6; ++k) x[a.soff_cam[cam] + k] = a.seed[(size_t)cam * 6 + k];
  } else if (u < g.npose + g.npt) {
    const int pt = g.pt0 + (u - g.npose);
#pragma unroll
    for (int k = 0; k < 3; ++k) x[a.soff_pt[pt] + k] = a.seed_pt ? a.seed_pt[(size_t)pt * 3 + k] : 0.0;
  }
}

// backward, per observation and prior (Proposition 1): with u = H*^-1 v in
// slot 0, dL/dphi = -d/dphi [u^T g(theta_K; phi)] for the observation
// weights, each observation's Huber radius and the prior log-weights; the
// camera adjoint into uout.  Zero for problems whose solve failed.
__global__ void __launch_bounds__(kBT) k_spba_vjp(SpArgs a) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  const bool ok = a.status[b] == DNLS_GRAPH_OK;
  const double* u = slot(a, g, 0);
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (t < g.nobs) {
    const int o = g.obs0 + t;
    double gw = 0.0, gd = 0.0;
    if (ok) {
      double c[2], Jc[12], Jp[6];
      reproj<double>(a.poses + (size_t)a.obs_cam[o] * 12, a.pts + (size_t)a.obs_pt[o] * 3, a.obs_uv + (size_t)o * 2,
                     a, c, Jc, Jp);
      const double* uc = u + a.soff_cam[a.obs_cam[o]];
      const double* up = u + a.soff_pt[a.obs_pt[o]];
      double y[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += Jc[r * 6 + k] * uc[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += Jp[r * 3 + k] * up[k];
        y[r] = acc;
      }
      const double w = a.obs_w[o];
      const double yc = y[0] * c[0] + y[1] * c[1];
      const double cn2 = c[0] * c[0] + c[1] * c[1];
      const double hd = spba_radius(a, b);
      // g_o = rho'(s) w^2 C^T c, rho' = 1 inside and delta / sqrt(s) outside
      if (w * w * cn2 <= hd * hd) {
        gw = -2.0 * w * yc;
      } else {
        gw = -hd * yc / ::sqrt(cn2);
        gd = -w * yc / ::sqrt(cn2);
      }
    }
    if (a.g_w) a.g_w[o] = gw;
    if (a.g_delta) a.g_delta[o] = gd;
  } else if (t < g.nobs + g.nprior) {
    const int q = g.prior0 + (t - g.nobs);
    double gl = 0.0;
    if (ok) {
      double c[6], C[36];
      prior_cost<3, double>(a.poses + (size_t)a.prior_var[q] * 12, a.prior_meas + (size_t)q * 12, c, C);
      const double w = exp(a.prior_logw[q]);
      const double* uq = u + a.soff_cam[a.prior_var[q]];
      double yr = 0.0;
      for (int r = 0; r < 6; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 6; ++k) acc += C[r * 6 + k] * uq[k];
        yr += w * acc * w * c[r];
      }
      gl = -2.0 * yr;
    }
    if (a.g_logw_p) a.g_logw_p[q] = gl;
  }
  if (t < g.npose && a.uout) {
    const int cam = g.pose0 + t;
#pragma unroll
    for (int k = 0; k < 6; ++k) a.uout[(size_t)cam * 6 + k] = ok ? u[a.soff_cam[cam] + k] : 0.0;
  }
}

// per-problem Huber radius gradient: the sum of its observations' per-radius
// gradients, one workgroup per problem (strided partial sums, then a fixed
// tree in LDS: the same order on every call)
__global__ void __launch_bounds__(kBT) k_spba_delta_sum(SpArgs a) {
  __shared__ double red[kBT];
  const int b = blockIdx.x;
  const SpDesc g = a.sd[b];
  double s = 0.0;
  for (int t = threadIdx.x; t < g.nobs; t += kBT) s += a.g_delta[g.obs0 + t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.g_huber[b] = red[0];
}

__global__ void k_sp_reset(int* failed, int* status, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    failed[b] = 0;
    status[b] = DNLS_GRAPH_OK;
  }
}

// ---------------------------------------------------------------------------
// adaptive damping: keep a step iff the float64 objective strictly decreases
// (lambda / 10), else restore theta_t (lambda x 10), lambda in [1e-7, 1e7]
// ---------------------------------------------------------------------------
constexpr double kLambdaMin = 1e-7, kLambdaMax = 1e7;
constexpr double kRadiusMax = 1e4;   // dogleg: largest trust radius

__global__ void k_sp_lam_init(SpArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) a.lam_g[b] = a.lambda;
}

// float64 objective partial sums of the graph's costs at the current poses
template <int G>
__global__ void __launch_bounds__(kBT) k_sp_obj(SpArgs a) {
  __shared__ double red[kBT / 64];
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  double s = 0.0;
  const int k = blockIdx.x * kBT + threadIdx.x;
  if (!a.failed[b] && k < g.nedge + g.nprior) {
    const int rk = (k < g.nedge) ? g.edge0 + k : a.E + g.prior0 + (k - g.nedge);
    s = cost_objective<G>(cost_data(a), rk);
  }
  s = block_sum_sp(s, red);
  if (threadIdx.x == 0) a.partial[b * a.nx + blockIdx.x] = s;
}

// s_t[b] = sum of the partials (thread per graph)
__global__ void k_sp_obj_store(SpArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || a.failed[b]) return;
  double S = 0.0;
  for (int k = 0; k < a.nx; ++k) S += a.partial[b * a.nx + k];
  a.s_t[b] = S;
}

__global__ void __launch_bounds__(kBT) k_sp_backup(SpArgs a, int sz) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b]) return;
  for (int u = blockIdx.x * kBT + threadIdx.x; u < g.npose * sz; u += gridDim.x * kBT)
    a.pose_bak[(size_t)g.pose0 * sz + u] = a.poses[(size_t)g.pose0 * sz + u];
}

// decision from the trial objective's partials and s_t (thread per graph)
__global__ void k_sp_dl_init(SpArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) a.dl[4 * b] = a.radius0;
}

// dogleg: keep the trial step iff the float64 objective strictly decreases;
// with rho = actual / predicted decrease the radius becomes |delta| / 4 if
// rho < 1/4 (or undefined) and min(2 radius, kRadiusMax) if rho > 3/4 on the
// boundary (thread per graph)
__global__ void k_sp_dl_decide(SpArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  a.rej[b] = 0;
  if (a.failed[b]) return;
  double S = 0.0;
  for (int k = 0; k < a.nx; ++k) S += a.partial[b * a.nx + k];
  const double s_t = a.s_t[b];
  const double rho = (s_t - S) / a.dl[4 * b + 1];
  if (!(S < s_t)) a.rej[b] = 1;
  if (!(rho >= 0.25)) a.dl[4 * b] = 0.25 * a.dl[4 * b + 2];
  else if (rho > 0.75 && a.dl[4 * b + 3] != 0.0) a.dl[4 * b] = fmin(2.0 * a.dl[4 * b], kRadiusMax);
}

__global__ void k_sp_decide(SpArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  a.rej[b] = 0;
  if (a.failed[b]) return;
  double S = 0.0;
  for (int k = 0; k < a.nx; ++k) S += a.partial[b * a.nx + k];
  if (S < a.s_t[b]) {
    a.lam_g[b] = fmax(a.lam_g[b] / 10.0, kLambdaMin);
  } else {
    a.lam_g[b] = fmin(a.lam_g[b] * 10.0, kLambdaMax);
    a.rej[b] = 1;
  }
}

__global__ void __launch_bounds__(kBT) k_sp_restore(SpArgs a, int sz) {
  const int b = blockIdx.y;
  const SpDesc g = a.sd[b];
  if (a.failed[b] || !a.rej[b]) return;
  for (int u = blockIdx.x * kBT + threadIdx.x; u < g.npose * sz; u += gridDim.x * kBT)
    a.poses[(size_t)g.pose0 * sz + u] = a.pose_bak[(size_t)g.pose0 * sz + u];
}

__global__ void k_sp_failed_from_status(int* failed, const int* status, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) failed[b] = status[b] != DNLS_GRAPH_OK;
}

int max_desc(const std::vector<SpDesc>& v, int SpDesc::*f) {
  int m = 1;
  for (const auto& x : v) m = std::max(m, x.*f);
  return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// Supernodes of the tile factor, per graph: consecutive tile columns J, J + 1
// whose structures below the diagonal are {J + 1} and then the same rows
// (column J's rows are J + 1 followed by column J + 1's), at most
// kSnMax columns.  The per-column update launches apply the updates of such
// a run to the tiles right of it once, at its last column, summed over its
// columns (one read and write of each target tile instead of one per
// column); sn[col_off + J] = (first, last) column of J's run.
constexpr int kSnMax = 32;
static std::vector<int2> tile_supernodes(const std::vector<dnls::SpDesc>& sd, const std::vector<int>& colptr,
                                         const std::vector<int>& rowidx) {
  std::vector<int2> sn(colptr.size(), int2{0, 0});
  auto same_tail = [&](int col_off, int J) {   // column J = {J + 1} + column J + 1
    const int a0 = colptr[col_off + J] + 1, a1 = colptr[col_off + J + 1];
    const int b0 = colptr[col_off + J + 1] + 1, b1 = colptr[col_off + J + 2];
    if (a1 - a0 != b1 - b0 + 1 || a1 == a0 || rowidx[a0] != J + 1) return false;
    for (int k = 0; k < b1 - b0; ++k)
      if (rowidx[a0 + 1 + k] != rowidx[b0 + k]) return false;
    return true;
  };
  for (const dnls::SpDesc& g : sd) {
    for (int J = 0; J < g.P;) {
      int e = J;
      while (e + 1 < g.P && e - J + 1 < kSnMax && same_tail(g.col_off, e)) ++e;
      for (int j = J; j <= e; ++j) sn[g.col_off + j] = int2{J, e};
      J = e + 1;
    }
  }
  return sn;
}

dnls_status sp_plan_create(dnls_plan p, const dnls_problem* pr) {
  const int B = pr->batch, d = p->d;
  std::vector<int> edge_ij(2 * (size_t)p->E), prior_var(p->P), pos(p->V);
  std::vector<std::vector<int>> inc(p->V);
  std::vector<int4> od_blk;
  std::vector<int> od_slot, tix, colptr, rowidx, rowptr, rowcol;
  p->sd.resize(B);
  long long fac = 0, vecoff = 0;
  int maxP = 0;
  // tile size: 48 (three 16-wide MFMA tiles) or, for BLOCK, the pose blocks
  // themselves.  AUTO takes BLOCK for float64 fixed-damping plans whose
  // graphs fit one workgroup's solve but exceed 16 tile columns (measured on
  // the 256-walk batch: 27 ms per step against 30 ms for HYBRID; with mixed
  // precision the refinement sweeps' level-by-level solves make it slower)
  int maxP48 = 0;
  for (int b = 0; b < B; ++b) maxP48 = std::max(maxP48, ((pr->pose_off[b + 1] - pr->pose_off[b]) * d + kTS - 1) / kTS);
  const bool auto_block = p->opt.sparse_solve == DNLS_SPSOLVE_AUTO && maxP48 * kTS <= kSolveLds &&
                          maxP48 > kFactorWgMaxP && p->opt.precision == DNLS_PREC_FP64 &&
                          !(p->opt.flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG));
  if (auto_block) p->opt.sparse_solve = DNLS_SPSOLVE_BLOCK;
  const int tsz = p->opt.sparse_solve == DNLS_SPSOLVE_BLOCK ? d : kTS;
  const long long tt = (long long)tsz * tsz;
  p->sp_ts = tsz;
  for (int b = 0; b < B; ++b) {
    SpDesc& g = p->sd[b];
    g.pose0 = pr->pose_off[b];
    g.npose = pr->pose_off[b + 1] - g.pose0;
    g.edge0 = pr->edge_off[b];
    g.nedge = pr->edge_off[b + 1] - g.edge0;
    g.prior0 = pr->prior_off[b];
    g.nprior = pr->prior_off[b + 1] - g.prior0;
    g.n = g.npose * d;
    std::vector<std::vector<int>> adj(g.npose);
    std::map<std::pair<int, int>, std::vector<int>> blocks;
    for (int e = g.edge0; e < g.edge0 + g.nedge; ++e) {
      const int i = pr->edge_ij[2 * (size_t)e], j = pr->edge_ij[2 * (size_t)e + 1];
      if (i < g.pose0 || i >= g.pose0 + g.npose || j < g.pose0 || j >= g.pose0 + g.npose || i == j)
        return fail(DNLS_ERR_INVALID_ARG, "edge " + std::to_string(e) + " has an index outside its graph or i == j");
      edge_ij[2 * (size_t)e] = i;
      edge_ij[2 * (size_t)e + 1] = j;
      inc[i].push_back(2 * e + 0);
      inc[j].push_back(2 * e + 1);
      const int li = i - g.pose0, lj = j - g.pose0;
      adj[li].push_back(lj);
      adj[lj].push_back(li);
      if (li > lj) blocks[{li, lj}].push_back(2 * e + 0);
      else blocks[{lj, li}].push_back(2 * e + 1);
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      const int v = pr->prior_var[q];
      if (v < g.pose0 || v >= g.pose0 + g.npose)
        return fail(DNLS_ERR_INVALID_ARG, "prior " + std::to_string(q) + " refers to a pose outside its graph");
      prior_var[q] = v;
      inc[v].push_back(2 * (p->E + q) + 1);
    }
    // ordering: minimum degree, then an elimination-tree postorder
    const std::vector<int> order = sym::min_degree_order(g.npose, adj);
    std::vector<int> lpos(g.npose);
    for (int k = 0; k < g.npose; ++k) lpos[order[k]] = k;
    lpos = sym::postorder_positions(g.npose, adj, lpos);
    for (int v = 0; v < g.npose; ++v) pos[g.pose0 + v] = lpos[v];
    std::vector<std::pair<int, int>> bl;
    for (auto& kv : blocks) bl.push_back(kv.first);
    const sym::TileStructure ts = sym::tile_symbolic(g.npose, d, tsz, lpos, bl);
    p->flops_alg += sym::block_flops(sym::block_column_counts(g.npose, adj, lpos), d);
    p->flops_exec += sym::tile_flops(ts, tsz);
    g.P = ts.P;
    maxP = std::max(maxP, g.P);
    g.ntile = (int)ts.row_idx.size();
    g.tix_off = (int)tix.size();
    tix.resize(tix.size() + (size_t)g.P * g.P, -1);
    g.col_off = (int)colptr.size();
    const int rbase = (int)rowidx.size();
    for (int J = 0; J <= g.P; ++J) colptr.push_back(rbase + ts.col_ptr[J]);
    for (int J = 0; J < g.P; ++J)
      for (int k = ts.col_ptr[J]; k < ts.col_ptr[J + 1]; ++k) {
        const int I = ts.row_idx[k];
        tix[g.tix_off + (size_t)I * g.P + J] = k;
        rowidx.push_back(I);
      }
    // transposed structure: the off-diagonal tiles of every tile row
    {
      std::vector<std::vector<int>> rows(g.P);
      for (int J = 0; J < g.P; ++J)
        for (int k = ts.col_ptr[J] + 1; k < ts.col_ptr[J + 1]; ++k) rows[ts.row_idx[k]].push_back(J);
      g.row_off = (int)rowptr.size();
      for (int I = 0; I < g.P; ++I) {
        rowptr.push_back((int)rowcol.size());
        for (int J : rows[I]) rowcol.push_back(J);
      }
      rowptr.push_back((int)rowcol.size());
    }
    g.pool_off = fac;
    fac += (long long)g.ntile * tt;
    g.winv_off = fac;
    fac += (long long)g.P * tt;
    fac = (fac + 31) / 32 * 32;
    g.nvec = g.P * tsz;
    g.lvl_off = 0;
    g.nlvl = 0;
    g.vec_off = vecoff;
    vecoff += 4LL * g.nvec;
    g.od0 = (int)od_blk.size();
    for (auto& kv : blocks) {
      od_blk.push_back(int4{kv.first.first, kv.first.second, (int)od_slot.size(), (int)kv.second.size()});
      for (int s : kv.second) od_slot.push_back(s);
    }
    g.nod = (int)od_blk.size() - g.od0;
  }
  std::vector<int> inc_off(p->V + 1, 0), inc_slot;
  for (int v = 0; v < p->V; ++v) {
    inc_off[v + 1] = inc_off[v] + (int)inc[v].size();
    for (int s : inc[v]) inc_slot.push_back(s);
  }
  // BLOCK: elimination-tree levels of every graph (a column's parent is its
  // first off-diagonal row; level = 1 + the highest level of its children)
  std::vector<int> lvlptr, lvlcol, lvlbptr, rowid;
  std::vector<int4> lvlblk;
  std::vector<int2> cpair;
  if (tsz != kTS) {
    for (int b = 0; b < B; ++b) {
      SpDesc& g = p->sd[b];
      std::vector<int> lev(g.P, 0);
      int nl = 0;
      for (int J = 0; J < g.P; ++J) {
        const int k0 = colptr[g.col_off + J], k1 = colptr[g.col_off + J + 1];
        if (k1 - k0 > 1) {
          const int par = rowidx[k0 + 1];
          lev[par] = std::max(lev[par], lev[J] + 1);
        }
        nl = std::max(nl, lev[J] + 1);
      }
      g.lvl_off = (int)lvlptr.size();
      g.nlvl = nl;
      std::vector<std::vector<int>> cols(nl);
      for (int J = 0; J < g.P; ++J) cols[lev[J]].push_back(J);
      // every block (I, J) of a level's columns with the tile-id pairs
      // (L_IK, L_JK), K < J, of its left-looking update
      const int base = colptr[g.col_off];
      auto tid = [&](int I, int J) { return tix[g.tix_off + (size_t)I * g.P + J]; };
      for (int L = 0; L < nl; ++L) {
        lvlptr.push_back((int)lvlcol.size());
        lvlbptr.push_back((int)lvlblk.size());
        for (int J : cols[L]) {
          lvlcol.push_back(J);
          for (int k = colptr[g.col_off + J]; k < colptr[g.col_off + J + 1]; ++k) {
            const int I = rowidx[k];
            const int c0 = (int)cpair.size();
            for (int q = rowptr[g.row_off + J]; q < rowptr[g.row_off + J + 1]; ++q) {
              const int K = rowcol[q], ik = tid(I, K);
              if (ik >= 0) cpair.push_back(int2{ik, tid(J, K)});
            }
            lvlblk.push_back(int4{k - base, c0, (int)cpair.size(), 2 * J + (I == J ? 1 : 0)});
          }
        }
      }
      lvlptr.push_back((int)lvlcol.size());
      lvlbptr.push_back((int)lvlblk.size());
    }
    // tile id of every row-structure entry (I, rowcol) for the forward solve
    rowid.resize(rowcol.size());
    for (int b = 0; b < B; ++b) {
      const SpDesc& g = p->sd[b];
      for (int I = 0; I < g.P; ++I)
        for (int q = rowptr[g.row_off + I]; q < rowptr[g.row_off + I + 1]; ++q)
          rowid[q] = tix[g.tix_off + (size_t)I * g.P + rowcol[q]];
    }
  }
  // per tile column: the widest column and pair count over the batch
  p->sp_ntrsm.assign(maxP, 0);
  p->sp_npair.assign(maxP, 0);
  p->sp_nrow.assign(maxP, 0);
  for (int b = 0; b < B; ++b) {
    const SpDesc& g = p->sd[b];
    for (int J = 0; J < g.P; ++J) {
      const int m = colptr[g.col_off + J + 1] - colptr[g.col_off + J] - 1;
      p->sp_ntrsm[J] = std::max(p->sp_ntrsm[J], m);
      p->sp_npair[J] = std::max(p->sp_npair[J], (long long)m * (m + 1) / 2);
      p->sp_nrow[J] = std::max(p->sp_nrow[J], rowptr[g.row_off + J + 1] - rowptr[g.row_off + J]);
    }
  }
  p->sp_maxP = maxP;
  const bool fits = max_desc(p->sd, &SpDesc::nvec) <= kSolveLds;
  const int mode = p->opt.sparse_solve;
  const bool fixed_damping = !(p->opt.flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG));
  const bool persistent_mode = mode == DNLS_SPSOLVE_PERSISTENT || mode == DNLS_SPSOLVE_BLOCK;
  if ((mode == DNLS_SPSOLVE_WORKGROUP || mode == DNLS_SPSOLVE_HYBRID || persistent_mode) && !fits)
    return fail(DNLS_ERR_UNSUPPORTED, "the workgroup solve holds at most " + std::to_string(kSolveLds) +
                                          " unknowns per graph");
  if (persistent_mode && !fixed_damping)
    return fail(DNLS_ERR_UNSUPPORTED, "the persistent schedules run fixed-damping steps only");
  // AUTO: for graphs of a few tile columns everything in one workgroup per
  // graph (the whole solve in one persistent launch with fixed damping); the
  // per-column launches spread larger graphs over the chip (one workgroup's
  // factorisation of a 32-column graph takes longer than the batch's
  // per-column launches)
  const bool small = fits && maxP <= kFactorWgMaxP;
  p->sp_persistent = persistent_mode || (mode == DNLS_SPSOLVE_AUTO && small && fixed_damping);
  p->sp_solve_wg = mode == DNLS_SPSOLVE_WORKGROUP || mode == DNLS_SPSOLVE_HYBRID || p->sp_persistent ||
                   (mode == DNLS_SPSOLVE_AUTO && fits);
  p->sp_factor_wg = mode == DNLS_SPSOLVE_WORKGROUP || p->sp_persistent || (mode == DNLS_SPSOLVE_AUTO && small);
  if (p->sp_persistent) {
    // queue order: decreasing factor work (tile-level flops), ties by index
    std::vector<double> work(B);
    for (int b = 0; b < B; ++b) {
      const SpDesc& g = p->sd[b];
      double w = 0.0;
      for (int J = 0; J < g.P; ++J) {
        const double m = colptr[g.col_off + J + 1] - colptr[g.col_off + J] - 1;
        w += 1.0 + m + m * (m + 1) / 2.0;
      }
      work[b] = w;
    }
    std::vector<int> order(B);
    for (int b = 0; b < B; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, tsz != kTS ? reinterpret_cast<const void*>(&k_sp_persistent<3, true, true>)
                            : reinterpret_cast<const void*>(&k_sp_persistent<3, true, false>), kPT, 0));
    p->sp_grid = std::max(1, std::min(B, std::max(1, per_cu) * std::max(1, cus)));
    dnls_status ust = upload(p, &p->d_sp_order, order);
    if (ust != DNLS_OK) return ust;
    HIP_TRY(hipMalloc(reinterpret_cast<void**>(&p->d_sp_queue), 2 * sizeof(unsigned)));
    p->allocs.push_back(p->d_sp_queue);
    HIP_TRY(hipMemset(p->d_sp_queue, 0, 2 * sizeof(unsigned)));
  }
  dnls_status st;
  if ((st = upload(p, &p->d_sd, p->sd)) != DNLS_OK || (st = upload(p, &p->d_edge_ij, edge_ij)) != DNLS_OK ||
      (st = upload(p, &p->d_prior_var, prior_var)) != DNLS_OK || (st = upload(p, &p->d_pos, pos)) != DNLS_OK ||
      (st = upload(p, &p->d_inc_off, inc_off)) != DNLS_OK || (st = upload(p, &p->d_inc_slot, inc_slot)) != DNLS_OK ||
      (st = upload(p, &p->d_od_blk, od_blk)) != DNLS_OK || (st = upload(p, &p->d_od_slot, od_slot)) != DNLS_OK ||
      (st = upload(p, &p->d_tix, tix)) != DNLS_OK || (st = upload(p, &p->d_colptr, colptr)) != DNLS_OK ||
      (st = upload(p, &p->d_rowidx, rowidx)) != DNLS_OK || (st = upload(p, &p->d_rowptr, rowptr)) != DNLS_OK ||
      (st = upload(p, &p->d_rowcol, rowcol)) != DNLS_OK ||
      (st = upload(p, &p->d_sn, tile_supernodes(p->sd, colptr, rowidx))) != DNLS_OK)
    return st;
  if (tsz != kTS &&
      ((st = upload(p, &p->d_lvlptr, lvlptr)) != DNLS_OK || (st = upload(p, &p->d_lvlcol, lvlcol)) != DNLS_OK ||
       (st = upload(p, &p->d_lvlbptr, lvlbptr)) != DNLS_OK || (st = upload(p, &p->d_lvlblk, lvlblk)) != DNLS_OK ||
       (st = upload(p, &p->d_cpair, cpair.empty() ? std::vector<int2>{int2{0, 0}} : cpair)) != DNLS_OK ||
       (st = upload(p, &p->d_rowid, rowid.empty() ? std::vector<int>{0} : rowid)) != DNLS_OK))
    return st;
  const size_t ncost = (size_t)p->E + p->P;
  const size_t rn = 2 * (size_t)d * d + d;
  const int nx = (max_desc(p->sd, &SpDesc::nedge) + max_desc(p->sd, &SpDesc::nprior) + kBT - 1) / kBT;
  p->nlin_blocks = nx;
  size_t off = 0;
  p->sp_off[0] = off; off += align256(ncost * rn * sizeof(double));                 // ws64
  p->sp_off[1] = off; off += align256(ncost * rn * sizeof(float));                  // ws32
  p->sp_off[2] = off; off += align256(ncost * d * sizeof(double));                  // ycost
  p->sp_off[3] = off; off += align256((size_t)vecoff * sizeof(double));             // vectors
  p->sp_off[4] = off; off += align256((size_t)B * nx * sizeof(double));             // partials
  p->sp_off[5] = off; off += align256((size_t)B * sizeof(int));                     // failed
  p->sp_off[6] = off; off += align256((size_t)B * sizeof(double));                  // last objective
  p->sp_off[7] = off; off += align256((size_t)p->V * d * sizeof(double));           // adjoint
  if (p->opt.flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG)) {
    p->sp_off[8] = off; off += align256((size_t)B * sizeof(double));                // lambda per graph
    p->sp_off[9] = off; off += align256((size_t)p->V * p->sz * sizeof(double));     // pose backup
    p->sp_off[10] = off; off += align256((size_t)B * sizeof(double));               // s_t
    p->sp_off[11] = off; off += align256((size_t)B * sizeof(int));                  // rejected
  }
  p->sp_off[12] = off; off += align256(ncost * 2 * d * sizeof(double));             // exact backward: per-cost terms
  p->sp_off[13] = off; off += align256((size_t)p->V * p->sz * sizeof(double));       // DLM backward: theta_direct
  p->sp_off[14] = off; off += align256((size_t)B * sizeof(int));                    // DLM backward: factor status
  p->sp_off[15] = off; off += align256((size_t)B * 4 * sizeof(double));             // dogleg state per graph
  p->ws_bytes = off;
  p->bwd_bytes = off;
  p->traj_off = (long long)fac;   // doubles: kept iterates theta_0 .. theta_{K-1}
  if (p->opt.flags & DNLS_FLAG_KEEP_ITERATES) fac += (size_t)p->opt.iterations * p->V * p->sz;
  p->fac_bytes = (size_t)fac * sizeof(double);
  return DNLS_OK;
}

// Bundle adjustment on the block-sparse solver (solver SPARSE given a
// problem with points).  Per problem: points first, ordered by their first
// observing camera and index, at scalar offsets 3 k; then, from the next
// multiple of the tile size, the cameras in minimum-degree order of their
// co-observation graph (an elimination-tree postorder of it), 6 scalars
// each; unit diagonal on the padding scalars.  The tile structure of the
// factor and the numeric tile kernels are the pose-graph path's.
dnls_status sp_plan_create_ba(dnls_plan p, const dnls_problem* pr) {
  const int B = pr->batch;
  int Vc = 0, Vp = 0, O = 0, P = 0;
  auto offs = [&](const int32_t* off, int* tot) {
    if (!off || off[0] != 0) return false;
    for (int b = 0; b < B; ++b)
      if (off[b + 1] < off[b]) return false;
    *tot = off[B];
    return true;
  };
  if (!offs(pr->pose_off, &Vc) || !offs(pr->point_off, &Vp) || !offs(pr->obs_off, &O) || !offs(pr->prior_off, &P))
    return fail(DNLS_ERR_INVALID_ARG, "bundle adjustment needs pose/point/obs/prior offsets starting at 0, non-decreasing");
  if (pr->group != DNLS_SE3) return fail(DNLS_ERR_UNSUPPORTED, "bundle adjustment uses SE3 cameras");
  if (O > 0 && (!pr->obs_cam || !pr->obs_pt)) return fail(DNLS_ERR_INVALID_ARG, "obs_cam / obs_pt are NULL");
  if (P > 0 && !pr->prior_var) return fail(DNLS_ERR_INVALID_ARG, "prior_var is NULL");
  if (!(pr->huber_delta > 0.0)) return fail(DNLS_ERR_INVALID_ARG, "huber_delta must be > 0");
  if (pr->edge_off && pr->edge_off[B] != 0)
    return fail(DNLS_ERR_UNSUPPORTED, "relative-pose costs and points in one problem are not supported");
  if (p->opt.flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG | DNLS_FLAG_KEEP_ITERATES))
    return fail(DNLS_ERR_UNSUPPORTED, "bundle adjustment on the block-sparse solver runs fixed-damping steps "
                                      "(adaptive damping, the dogleg and kept iterates are on the Schur solver)");
  const int mode = p->opt.sparse_solve;
  if (mode == DNLS_SPSOLVE_PERSISTENT || mode == DNLS_SPSOLVE_BLOCK || mode == DNLS_SPSOLVE_WORKGROUP)
    return fail(DNLS_ERR_UNSUPPORTED, "bundle adjustment on the block-sparse solver takes the HYBRID or SWEEPS schedule");
  p->sp_ba = true;
  p->V = Vc;
  p->Vp = Vp;
  p->O = O;
  p->P = P;
  p->E = 0;
  p->intr[0] = pr->fx;
  p->intr[1] = pr->fy;
  p->intr[2] = pr->cx;
  p->intr[3] = pr->cy;
  p->huber = pr->huber_delta;
  p->sp_ts = kTS;
  std::vector<int> obs_cam(O), obs_pt(O), prior_var(P), soff_cam(Vc), soff_pt(Vp);
  std::vector<std::vector<int>> cam_obs(Vc), pt_obs(Vp);
  std::vector<int4> cp_blk;
  std::vector<int> cp_obs, tix, colptr, rowidx, rowptr, rowcol;
  p->sd.resize(B);
  long long fac = 0, vecoff = 0;
  int maxP = 0, maxn = 0;
  for (int b = 0; b < B; ++b) {
    SpDesc& g = p->sd[b];
    g = SpDesc{};
    g.pose0 = pr->pose_off[b];
    g.npose = pr->pose_off[b + 1] - g.pose0;
    g.pt0 = pr->point_off[b];
    g.npt = pr->point_off[b + 1] - g.pt0;
    g.obs0 = pr->obs_off[b];
    g.nobs = pr->obs_off[b + 1] - g.obs0;
    g.prior0 = pr->prior_off[b];
    g.nprior = pr->prior_off[b + 1] - g.prior0;
    g.edge0 = 0;
    g.nedge = 0;
    std::map<std::pair<int, int>, std::vector<int>> blocks;   // (camera, point) -> observations
    std::vector<int> first_cam(g.npt, INT32_MAX);
    std::vector<std::vector<int>> cam_pts(g.npose);
    for (int o = g.obs0; o < g.obs0 + g.nobs; ++o) {
      const int c = pr->obs_cam[o], q = pr->obs_pt[o];
      if (c < g.pose0 || c >= g.pose0 + g.npose || q < g.pt0 || q >= g.pt0 + g.npt)
        return fail(DNLS_ERR_INVALID_ARG, "observation " + std::to_string(o) + " refers to a camera or point "
                                          "outside its problem");
      obs_cam[o] = c;
      obs_pt[o] = q;
      cam_obs[c].push_back(o);
      pt_obs[q].push_back(o);
      blocks[{c, q}].push_back(o);
      first_cam[q - g.pt0] = std::min(first_cam[q - g.pt0], c - g.pose0);
      cam_pts[c - g.pose0].push_back(q - g.pt0);
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      const int v = pr->prior_var[q];
      if (v < g.pose0 || v >= g.pose0 + g.npose)
        return fail(DNLS_ERR_INVALID_ARG, "prior " + std::to_string(q) + " refers to a camera outside its problem");
      prior_var[q] = v;
    }
    // points first, by first observing camera then index
    std::vector<int> porder(g.npt);
    for (int k = 0; k < g.npt; ++k) porder[k] = k;
    std::stable_sort(porder.begin(), porder.end(), [&](int x, int y) { return first_cam[x] < first_cam[y]; });
    for (int r = 0; r < g.npt; ++r) soff_pt[g.pt0 + porder[r]] = 3 * r;
    // cameras: minimum degree on the co-observation graph, then a postorder
    std::vector<std::vector<int>> cadj(g.npose);
    {
      std::vector<std::vector<int>> pt_cams(g.npt);
      for (int c = 0; c < g.npose; ++c)
        for (int q : cam_pts[c]) pt_cams[q].push_back(c);
      for (int q = 0; q < g.npt; ++q)
        for (size_t i = 0; i < pt_cams[q].size(); ++i)
          for (size_t j = i + 1; j < pt_cams[q].size(); ++j) {
            cadj[pt_cams[q][i]].push_back(pt_cams[q][j]);
            cadj[pt_cams[q][j]].push_back(pt_cams[q][i]);
          }
      for (auto& l : cadj) {
        std::sort(l.begin(), l.end());
        l.erase(std::unique(l.begin(), l.end()), l.end());
      }
    }
    const std::vector<int> corder = sym::min_degree_order(g.npose, cadj);
    std::vector<int> cpos(g.npose);
    for (int k = 0; k < g.npose; ++k) cpos[corder[k]] = k;
    cpos = sym::postorder_positions(g.npose, cadj, cpos);
    g.pad0 = 3 * g.npt;
    g.pad1 = (g.pad0 + kTS - 1) / kTS * kTS;
    for (int c = 0; c < g.npose; ++c) soff_cam[g.pose0 + c] = g.pad1 + 6 * cpos[c];
    g.n = g.pad1 + 6 * g.npose;
    maxn = std::max(maxn, g.n);
    // tile structure: variables are the points, the padding scalars (one
    // unit block each) and the cameras
    std::vector<int> start, size;
    for (int q = 0; q < g.npt; ++q) {
      start.push_back(soff_pt[g.pt0 + q]);
      size.push_back(3);
    }
    for (int r = g.pad0; r < g.pad1; ++r) {
      start.push_back(r);
      size.push_back(1);
    }
    const int cam_var0 = (int)start.size();
    for (int c = 0; c < g.npose; ++c) {
      start.push_back(soff_cam[g.pose0 + c]);
      size.push_back(6);
    }
    std::vector<std::pair<int, int>> bl;
    for (auto& kv : blocks) bl.push_back({cam_var0 + kv.first.first - g.pose0, kv.first.second - g.pt0});
    const sym::TileStructure ts = sym::tile_symbolic_vars(g.n, kTS, start, size, bl);
    p->flops_exec += sym::tile_flops(ts, kTS);
    // block flops of the points' elimination and the camera system (the
    // Schur complement's pairs and the dense-ish camera factor)
    {
      double f = 0.0;
      for (int q = 0; q < g.npt; ++q) {
        const double k = (double)pt_obs[g.pt0 + q].size();
        f += 9.0 + k * 27.0 * 2.0 + k * (k + 1) / 2.0 * 2.0 * 6 * 6 * 3;
      }
      const double nc = 6.0 * g.npose;
      f += nc * nc * nc / 3.0;
      p->flops_alg += f;
    }
    g.P = ts.P;
    maxP = std::max(maxP, g.P);
    g.ntile = (int)ts.row_idx.size();
    g.tix_off = (int)tix.size();
    tix.resize(tix.size() + (size_t)g.P * g.P, -1);
    g.col_off = (int)colptr.size();
    const int rbase = (int)rowidx.size();
    for (int J = 0; J <= g.P; ++J) colptr.push_back(rbase + ts.col_ptr[J]);
    for (int J = 0; J < g.P; ++J)
      for (int k = ts.col_ptr[J]; k < ts.col_ptr[J + 1]; ++k) {
        tix[g.tix_off + (size_t)ts.row_idx[k] * g.P + J] = k;
        rowidx.push_back(ts.row_idx[k]);
      }
    {
      std::vector<std::vector<int>> rows(g.P);
      for (int J = 0; J < g.P; ++J)
        for (int k = ts.col_ptr[J] + 1; k < ts.col_ptr[J + 1]; ++k) rows[ts.row_idx[k]].push_back(J);
      g.row_off = (int)rowptr.size();
      for (int I = 0; I < g.P; ++I) {
        rowptr.push_back((int)rowcol.size());
        for (int J : rows[I]) rowcol.push_back(J);
      }
      rowptr.push_back((int)rowcol.size());
    }
    g.pool_off = fac;
    fac += (long long)g.ntile * kTT;
    g.winv_off = fac;
    fac += (long long)g.P * kTT;
    fac = (fac + 31) / 32 * 32;
    g.nvec = g.P * kTS;
    g.vec_off = vecoff;
    vecoff += 4LL * g.nvec;
    g.cp0 = (int)cp_blk.size();
    for (auto& kv : blocks) {
      cp_blk.push_back(int4{kv.first.first, kv.first.second, (int)cp_obs.size(), (int)kv.second.size()});
      for (int o : kv.second) cp_obs.push_back(o);
    }
    g.ncp = (int)cp_blk.size() - g.cp0;
    g.od0 = 0;
    g.nod = 0;
    g.lvl_off = 0;
    g.nlvl = 0;
  }
  std::vector<int> cam_off(Vc + 1, 0), cam_list, pt_off(Vp + 1, 0), pt_list;
  for (int c = 0; c < Vc; ++c) {
    cam_off[c + 1] = cam_off[c] + (int)cam_obs[c].size();
    for (int o : cam_obs[c]) cam_list.push_back(o);
  }
  for (int q = 0; q < Vp; ++q) {
    pt_off[q + 1] = pt_off[q] + (int)pt_obs[q].size();
    for (int o : pt_obs[q]) pt_list.push_back(o);
  }
  p->sp_ntrsm.assign(maxP, 0);
  p->sp_npair.assign(maxP, 0);
  p->sp_nrow.assign(maxP, 0);
  for (int b = 0; b < B; ++b) {
    const SpDesc& g = p->sd[b];
    for (int J = 0; J < g.P; ++J) {
      const int m = colptr[g.col_off + J + 1] - colptr[g.col_off + J] - 1;
      p->sp_ntrsm[J] = std::max(p->sp_ntrsm[J], m);
      p->sp_npair[J] = std::max(p->sp_npair[J], (long long)m * (m + 1) / 2);
      p->sp_nrow[J] = std::max(p->sp_nrow[J], rowptr[g.row_off + J + 1] - rowptr[g.row_off + J]);
    }
  }
  p->sp_maxP = maxP;
  const bool fits = max_desc(p->sd, &SpDesc::nvec) <= kSolveLds;
  if (mode == DNLS_SPSOLVE_HYBRID && !fits)
    return fail(DNLS_ERR_UNSUPPORTED, "the workgroup solve holds at most " + std::to_string(kSolveLds) +
                                          " unknowns per problem");
  p->sp_solve_wg = mode == DNLS_SPSOLVE_HYBRID || (mode == DNLS_SPSOLVE_AUTO && fits);
  p->sp_factor_wg = false;
  p->sp_persistent = false;
  dnls_status st;
  if ((st = upload(p, &p->d_sd, p->sd)) != DNLS_OK || (st = upload(p, &p->d_prior_var, prior_var)) != DNLS_OK ||
      (st = upload(p, &p->d_obs_cam, obs_cam)) != DNLS_OK || (st = upload(p, &p->d_obs_pt, obs_pt)) != DNLS_OK ||
      (st = upload(p, &p->d_soff_cam, soff_cam)) != DNLS_OK || (st = upload(p, &p->d_soff_pt, soff_pt)) != DNLS_OK ||
      (st = upload(p, &p->d_cam_obs_off, cam_off)) != DNLS_OK || (st = upload(p, &p->d_cam_obs, cam_list)) != DNLS_OK ||
      (st = upload(p, &p->d_pt_obs_off, pt_off)) != DNLS_OK || (st = upload(p, &p->d_pt_obs, pt_list)) != DNLS_OK ||
      (st = upload(p, &p->d_cp_blk, cp_blk)) != DNLS_OK || (st = upload(p, &p->d_cp_obs, cp_obs)) != DNLS_OK ||
      (st = upload(p, &p->d_tix, tix)) != DNLS_OK || (st = upload(p, &p->d_colptr, colptr)) != DNLS_OK ||
      (st = upload(p, &p->d_rowidx, rowidx)) != DNLS_OK || (st = upload(p, &p->d_rowptr, rowptr)) != DNLS_OK ||
      (st = upload(p, &p->d_rowcol, rowcol)) != DNLS_OK ||
      (st = upload(p, &p->d_sn, tile_supernodes(p->sd, colptr, rowidx))) != DNLS_OK)
    return st;
  const size_t rn = CostRec<6>::n;
  const int maxc = std::max(max_desc(p->sd, &SpDesc::nobs) + max_desc(p->sd, &SpDesc::nprior), 1);
  p->nlin_blocks = (maxc + kBT - 1) / kBT;
  size_t off = 0;
  p->sp_off[0] = off; off += align256((size_t)std::max(P, 1) * rn * sizeof(double));   // prior records
  p->sp_off[3] = off; off += align256((size_t)vecoff * sizeof(double));                 // vectors
  p->sp_off[4] = off; off += align256((size_t)B * p->nlin_blocks * sizeof(double));     // partials
  p->sp_off[5] = off; off += align256((size_t)B * sizeof(int));                         // failed
  p->sp_off[6] = off; off += align256((size_t)B * sizeof(double));                      // last objective
  p->sp_off[7] = off; off += align256((size_t)Vc * 6 * sizeof(double));                // camera adjoint
  // observation records: float64, or (mixed) float records then the float64 gradient parts
  p->sp_off[16] = off;
  off += align256(std::max((size_t)O * kObsRecSp * sizeof(double),
                           align256((size_t)O * kObsRecSp * sizeof(float)) + (size_t)O * 9 * sizeof(double)));
  p->sp_off[17] = off; off += align256((size_t)std::max(O, 1) * sizeof(double));        // per-observation radius gradients
  p->ws_bytes = off;
  p->bwd_bytes = off;
  p->traj_off = (long long)fac;
  p->fac_bytes = (size_t)fac * sizeof(double);
  (void)maxn;
  return DNLS_OK;
}

static SpArgs sp_args(dnls_plan p, void* ws, void* factor) {
  SpArgs a{};
  a.sd = p->d_sd;
  a.edge_ij = p->d_edge_ij;
  a.prior_var = p->d_prior_var;
  a.pos = p->d_pos;
  a.inc_off = p->d_inc_off;
  a.inc_slot = p->d_inc_slot;
  a.od_blk = p->d_od_blk;
  a.od_slot = p->d_od_slot;
  a.tix = p->d_tix;
  a.colptr = p->d_colptr;
  a.rowidx = p->d_rowidx;
  a.sn = p->d_sn;
  a.rowptr = p->d_rowptr;
  a.rowcol = p->d_rowcol;
  char* w = static_cast<char*>(ws);
  a.ws64 = reinterpret_cast<double*>(w + p->sp_off[0]);
  a.ws32 = reinterpret_cast<float*>(w + p->sp_off[1]);
  a.ycost = reinterpret_cast<double*>(w + p->sp_off[2]);
  a.vec = reinterpret_cast<double*>(w + p->sp_off[3]);
  a.partial = reinterpret_cast<double*>(w + p->sp_off[4]);
  a.failed = reinterpret_cast<int*>(w + p->sp_off[5]);
  a.lastobj = reinterpret_cast<double*>(w + p->sp_off[6]);
  a.uout = reinterpret_cast<double*>(w + p->sp_off[7]);
  a.hvp = reinterpret_cast<double*>(w + p->sp_off[12]);
  a.dl = reinterpret_cast<double*>(w + p->sp_off[15]);
  a.radius0 = p->opt.trust_radius;
  if (p->opt.flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG)) {
    a.lam_g = reinterpret_cast<double*>(w + p->sp_off[8]);
    a.pose_bak = reinterpret_cast<double*>(w + p->sp_off[9]);
    a.s_t = reinterpret_cast<double*>(w + p->sp_off[10]);
    a.rej = reinterpret_cast<int*>(w + p->sp_off[11]);
  }
  a.factor = static_cast<double*>(factor);
  a.ts = p->sp_ts;
  if (p->sp_ba) {
    a.orec = w + p->sp_off[16];
    a.gob = reinterpret_cast<double*>(w + p->sp_off[16] + align256((size_t)p->O * kObsRecSp * sizeof(float)));
    a.g_delta = reinterpret_cast<double*>(w + p->sp_off[17]);
    a.obs_cam = p->d_obs_cam;
    a.obs_pt = p->d_obs_pt;
    a.soff_cam = p->d_soff_cam;
    a.soff_pt = p->d_soff_pt;
    a.cam_obs_off = p->d_cam_obs_off;
    a.cam_obs = p->d_cam_obs;
    a.pt_obs_off = p->d_pt_obs_off;
    a.pt_obs = p->d_pt_obs;
    a.cp_blk = p->d_cp_blk;
    a.cp_obs = p->d_cp_obs;
    a.fx = p->intr[0];
    a.fy = p->intr[1];
    a.cx = p->intr[2];
    a.cy = p->intr[3];
    a.huber = p->huber;
  }
  a.lvlptr = p->d_lvlptr;
  a.lvlcol = p->d_lvlcol;
  a.lvlbptr = p->d_lvlbptr;
  a.lvlblk = p->d_lvlblk;
  a.cpair = p->d_cpair;
  a.rowid = p->d_rowid;
  a.E = p->E;
  a.K = p->opt.iterations;
  a.nx = p->nlin_blocks;
  a.refine = p->opt.precision == DNLS_PREC_MIXED ? p->opt.refine : 0;
  a.lambda = p->opt.lambda;
  return a;
}

template <int G>
static void sp_factor(dnls_plan p, const SpArgs& a, hipStream_t st) {
  const int B = p->B;
  if (p->sp_ts != kTS) {
    if (p->d == 6) hipLaunchKernelGGL(k_sb_factor<6>, dim3(B), dim3(kPT), 0, st, a);
    else hipLaunchKernelGGL(k_sb_factor<3>, dim3(B), dim3(kPT), 0, st, a);
    return;
  }
  if (p->sp_factor_wg) {
    hipLaunchKernelGGL(k_sp_factor_wg, dim3(B), dim3(kWG), 0, st, a);
    return;
  }
  for (int J = 0; J < p->sp_maxP; ++J) {
    hipLaunchKernelGGL(k_sp_diag, dim3(B), dim3(kNT), 0, st, a, J);
    if (p->sp_ntrsm[J] > 0) {
      hipLaunchKernelGGL(k_sp_trsm, dim3(p->sp_ntrsm[J], B), dim3(kTW), 0, st, a, J);
      hipLaunchKernelGGL(k_sp_update, dim3((unsigned)p->sp_npair[J], B), dim3(kTW), 0, st, a, J);
    }
  }
}

// x (slot dst) = (L L^T)^-1 b (slot 2, destroyed); slot 3 holds the forward result
static void sp_sweeps(dnls_plan p, const SpArgs& a, int dst, hipStream_t st) {
  const int B = p->B;
  if (p->sp_ts != kTS) {
    if (p->d == 6) hipLaunchKernelGGL(k_sb_solve<6>, dim3(B), dim3(kPT), 0, st, a, 2, dst);
    else hipLaunchKernelGGL(k_sb_solve<3>, dim3(B), dim3(kPT), 0, st, a, 2, dst);
    return;
  }
  if (p->sp_solve_wg) {
    hipLaunchKernelGGL(k_sp_solve_wg, dim3(B), dim3(kWG), 0, st, a, 2, dst);
    return;
  }
  for (int J = 0; J < p->sp_maxP; ++J)
    hipLaunchKernelGGL(k_sp_fwd, dim3(p->sp_ntrsm[J] + 1, B), dim3(kTW), 0, st, a, J, 2, 3);
  for (int I = p->sp_maxP - 1; I >= 0; --I)
    hipLaunchKernelGGL(k_sp_bwd, dim3(p->sp_nrow[I] + 1, B), dim3(kTW), 0, st, a, I, 3, dst);
}

template <int G>
static dnls_status sp_solve_impl(dnls_plan p, const dnls_solve_args* s, hipStream_t st) {
  constexpr int d = GroupTraits<G>::d;
  SpArgs a = sp_args(p, s->workspace, s->factor);
  a.poses = s->poses;
  a.edge_meas = s->edge_meas;
  a.edge_logw = s->edge_logw;
  a.edge_tau = s->edge_tau;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.edge_logc = s->edge_logc;
  a.objective = s->objective;
  a.status = s->status;
  const int B = p->B;
  const bool mixed = p->opt.precision == DNLS_PREC_MIXED;
  const dim3 g_cost(p->nlin_blocks, B);
  const dim3 g_blk((max_desc(p->sd, &SpDesc::npose) + max_desc(p->sd, &SpDesc::nod) + kBT - 1) / kBT, B);
  const dim3 g_zero(256, B);
  const dim3 g_pose((max_desc(p->sd, &SpDesc::npose) + kBT - 1) / kBT, B);
  const dim3 g_vec(std::min(64, (max_desc(p->sd, &SpDesc::nvec) + kBT - 1) / kBT), B);
  const bool adaptive = (p->opt.flags & DNLS_FLAG_ADAPTIVE_LM) != 0;
  const bool dogleg = (p->opt.flags & DNLS_FLAG_DOGLEG) != 0;
  const bool keep = (p->opt.flags & DNLS_FLAG_KEEP_ITERATES) != 0;
  const int sz = GroupTraits<G>::sz;
  // mixed: steps refine_from <= it < refine_until run the refinement sweeps
  // (the last refine_last steps, or the first -refine_last, or all)
  const int K = p->opt.iterations, rl = p->opt.refine_last;
  const int refine_from = rl > 0 ? K - rl : 0, refine_until = rl < 0 ? -rl : K;
  if (p->sp_persistent) {
    a.traj = keep ? a.factor + p->traj_off : nullptr;
    a.V = p->V;
    const bool blk = p->sp_ts != kTS;
    if (mixed && blk)
      hipLaunchKernelGGL((k_sp_persistent<G, true, true>), dim3(p->sp_grid), dim3(kPT), 0, st, a, p->d_sp_order,
                         p->d_sp_queue, B, refine_from, refine_until);
    else if (mixed)
      hipLaunchKernelGGL((k_sp_persistent<G, true, false>), dim3(p->sp_grid), dim3(kPT), 0, st, a, p->d_sp_order,
                         p->d_sp_queue, B, refine_from, refine_until);
    else if (blk)
      hipLaunchKernelGGL((k_sp_persistent<G, false, true>), dim3(p->sp_grid), dim3(kPT), 0, st, a, p->d_sp_order,
                         p->d_sp_queue, B, refine_from, refine_until);
    else
      hipLaunchKernelGGL((k_sp_persistent<G, false, false>), dim3(p->sp_grid), dim3(kPT), 0, st, a, p->d_sp_order,
                         p->d_sp_queue, B, refine_from, refine_until);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  hipLaunchKernelGGL(k_sp_reset, dim3((B + 255) / 256), dim3(256), 0, st, a.failed, a.status, B);
  if (adaptive) hipLaunchKernelGGL(k_sp_lam_init, dim3((B + 255) / 256), dim3(256), 0, st, a, B);
  if (dogleg) hipLaunchKernelGGL(k_sp_dl_init, dim3((B + 255) / 256), dim3(256), 0, st, a, B);
  for (int it = 0; it <= p->opt.iterations; ++it) {
    const bool final_lin = it == p->opt.iterations;
    const double lam = final_lin ? 0.0 : p->opt.lambda;
    const int lam_g = (adaptive && !final_lin) ? 1 : 0;
    a.it = it;
    if (keep && !final_lin) {
      SpArgs ak = a;
      ak.pose_bak = a.factor + p->traj_off + (size_t)it * p->V * sz;
      hipLaunchKernelGGL(k_sp_backup, g_pose, dim3(kBT), 0, st, ak, sz);
    }
    const bool lin32 = mixed && !final_lin;
    const bool refine_now = lin32 && a.refine > 0 && it >= refine_from && it < refine_until;
    // the dogleg's model and decision use the float64 gradient and objective
    const bool lin64 = !mixed || refine_now || final_lin || dogleg;
    if (lin32) hipLaunchKernelGGL((k_sp_lin<G, float>), g_cost, dim3(kBT), 0, st, a, a.ws32);
    if (lin64) hipLaunchKernelGGL((k_sp_lin<G, double>), g_cost, dim3(kBT), 0, st, a, a.ws64);
    hipLaunchKernelGGL(k_sp_objective, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
    if (lam_g && !lin64) {
      // the decision compares float64 objectives: S at theta_t in float64
      hipLaunchKernelGGL(k_sp_obj<G>, g_cost, dim3(kBT), 0, st, a);
      hipLaunchKernelGGL(k_sp_obj_store, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
    }
    hipLaunchKernelGGL(k_sp_zero, g_zero, dim3(kBT), 0, st, a);
    if (lin32) {
      hipLaunchKernelGGL((k_sp_assemble<G, float>), g_blk, dim3(kBT), 0, st, a, (const float*)a.ws32, lam,
                         (refine_now || dogleg) ? 0 : 1, lam_g);
      if (refine_now || dogleg) hipLaunchKernelGGL(k_sp_rhs64<G>, g_blk, dim3(kBT), 0, st, a);
    } else {
      hipLaunchKernelGGL((k_sp_assemble<G, double>), g_blk, dim3(kBT), 0, st, a, (const double*)a.ws64, lam, 1,
                         lam_g);
    }
    sp_factor<G>(p, a, st);
    if (final_lin) break;
    if (lam_g) hipLaunchKernelGGL(k_sp_backup, g_pose, dim3(kBT), 0, st, a, sz);
    const bool refine = refine_now;
    hipLaunchKernelGGL(k_sp_copy, g_vec, dim3(kBT), 0, st, a, 1, 2);
    sp_sweeps(p, a, 0, st);
    if (!refine && !dogleg) hipLaunchKernelGGL(k_sp_retract<G>, g_pose, dim3(kBT), 0, st, a, 0);
    if (refine)
      for (int sw = 0; sw < a.refine; ++sw) {
        hipLaunchKernelGGL(k_sp_jx<G>, g_cost, dim3(kBT), 0, st, a, 0);
        hipLaunchKernelGGL(k_sp_residual<G>, g_pose, dim3(kBT), 0, st, a, lam, lam_g);
        sp_sweeps(p, a, 2, st);
        hipLaunchKernelGGL(k_sp_accumulate<G>, g_pose, dim3(kBT), 0, st, a,
                           (sw + 1 == a.refine && !dogleg) ? 1 : 0);
      }
    if (dogleg) {
      // (H + lambda I) g, the dogleg step, its predicted decrease, then the
      // trial retraction from a backup of theta_t
      hipLaunchKernelGGL(k_sp_jx<G>, g_cost, dim3(kBT), 0, st, a, 1);
      hipLaunchKernelGGL(k_sp_hx<G>, g_pose, dim3(kBT), 0, st, a, 1, 2, lam);
      hipLaunchKernelGGL(k_sp_dogleg, dim3(B), dim3(kBT), 0, st, a);
      hipLaunchKernelGGL(k_sp_jx<G>, g_cost, dim3(kBT), 0, st, a, 0);
      hipLaunchKernelGGL(k_sp_hx<G>, g_pose, dim3(kBT), 0, st, a, 0, 2, lam);
      hipLaunchKernelGGL(k_sp_dl_pred, dim3(B), dim3(kBT), 0, st, a);
      hipLaunchKernelGGL(k_sp_backup, g_pose, dim3(kBT), 0, st, a, sz);
      hipLaunchKernelGGL(k_sp_retract<G>, g_pose, dim3(kBT), 0, st, a, 0);
      hipLaunchKernelGGL(k_sp_obj<G>, g_cost, dim3(kBT), 0, st, a);
      hipLaunchKernelGGL(k_sp_dl_decide, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
      hipLaunchKernelGGL(k_sp_restore, g_pose, dim3(kBT), 0, st, a, sz);
    }
    if (lam_g) {
      hipLaunchKernelGGL(k_sp_obj<G>, g_cost, dim3(kBT), 0, st, a);
      hipLaunchKernelGGL(k_sp_decide, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
      hipLaunchKernelGGL(k_sp_restore, g_pose, dim3(kBT), 0, st, a, sz);
    }
  }
  HIP_TRY(hipGetLastError());
  (void)d;
  return DNLS_OK;
}

template <int G>
static dnls_status sp_backward_impl(dnls_plan p, const dnls_backward_args* s, hipStream_t st) {
  SpArgs a = sp_args(p, s->workspace, const_cast<void*>(s->factor));
  a.poses = const_cast<double*>(s->poses);
  a.edge_meas = s->edge_meas;
  a.edge_logw = s->edge_logw;
  a.edge_tau = s->edge_tau;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.status = const_cast<int*>(s->status);
  a.seed = s->seed_pose;
  a.g_logw_e = s->grad_edge_logw;
  a.g_tau = s->grad_edge_tau;
  a.g_logw_p = s->grad_prior_logw;
  a.edge_logc = s->edge_logc;
  a.g_logc = s->grad_edge_logc;
  const int B = p->B;
  const dim3 g_cost(p->nlin_blocks, B);
  const dim3 g_pose((max_desc(p->sd, &SpDesc::npose) + kBT - 1) / kBT, B);
  // float64 records at theta_K for the graphs whose solve succeeded
  hipLaunchKernelGGL(k_sp_failed_from_status, dim3((B + 255) / 256), dim3(256), 0, st, a.failed, a.status, B);
  if (s->mode == DNLS_BACKWARD_DLM) {
    const double eps = s->dlm_eps;
    const dim3 g_blk((max_desc(p->sd, &SpDesc::npose) + max_desc(p->sd, &SpDesc::nod) + kBT - 1) / kBT, B);
    const dim3 g_zero(256, B);
    char* w = static_cast<char*>(s->workspace);
    double* xd = reinterpret_cast<double*>(w + p->sp_off[13]);
    // dS/dphi at theta_K / eps; then (H* + 2 eps^2 I) assembled in float64
    // and factored into the factor cache (a failure there marks the graph in
    // a status copy of the workspace, not in the caller's status)
    hipLaunchKernelGGL(k_sp_param_grads<G>, g_cost, dim3(kBT), 0, st, a, (const double*)a.poses, 1.0 / eps, 0);
    hipLaunchKernelGGL((k_sp_lin<G, double>), g_cost, dim3(kBT), 0, st, a, a.ws64);
    hipLaunchKernelGGL(k_sp_zero, g_zero, dim3(kBT), 0, st, a);
    hipLaunchKernelGGL((k_sp_assemble<G, double>), g_blk, dim3(kBT), 0, st, a, (const double*)a.ws64,
                       2.0 * eps * eps, 1, 0);
    SpArgs ad = a;
    ad.status = reinterpret_cast<int*>(w + p->sp_off[14]);
    sp_factor<G>(p, ad, st);
    hipLaunchKernelGGL(k_sp_dlm_rhs, g_pose, dim3(kBT), 0, st, ad, GroupTraits<G>::d, eps);
    sp_sweeps(p, ad, 0, st);
    // theta_direct = theta_K Exp(delta) in the workspace, minus dS/dphi there / eps
    ad.pose_bak = xd;
    hipLaunchKernelGGL(k_sp_backup, g_pose, dim3(kBT), 0, st, ad, GroupTraits<G>::sz);
    ad.poses = xd;
    hipLaunchKernelGGL(k_sp_retract<G>, g_pose, dim3(kBT), 0, st, ad, 0);
    hipLaunchKernelGGL(k_sp_param_grads<G>, g_cost, dim3(kBT), 0, st, ad, (const double*)xd, -1.0 / eps, 1);
    // the factor cache again holds the factor of H* (same kernels and inputs
    // as the final linearisation of the solve)
    hipLaunchKernelGGL(k_sp_failed_from_status, dim3((B + 255) / 256), dim3(256), 0, st, a.failed, a.status, B);
    hipLaunchKernelGGL(k_sp_zero, g_zero, dim3(kBT), 0, st, a);
    hipLaunchKernelGGL((k_sp_assemble<G, double>), g_blk, dim3(kBT), 0, st, a, (const double*)a.ws64, 0.0, 1, 0);
    sp_factor<G>(p, a, st);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  if (s->mode == DNLS_BACKWARD_UNROLL) {
    constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
    const dim3 g_blk((max_desc(p->sd, &SpDesc::npose) + max_desc(p->sd, &SpDesc::nod) + kBT - 1) / kBT, B);
    const dim3 g_zero(256, B);
    const dim3 g_vec(std::min(64, (max_desc(p->sd, &SpDesc::nvec) + kBT - 1) / kBT), B);
    char* w = static_cast<char*>(s->workspace);
    int* fstat = reinterpret_cast<int*>(w + p->sp_off[14]);
    hipLaunchKernelGGL(k_sp_grads_zero<G>, g_cost, dim3(kBT), 0, st, a, 0);
    hipLaunchKernelGGL(k_sp_unroll_adj, g_pose, dim3(kBT), 0, st, a, d, 1);
    for (int t = p->opt.iterations - 1; t >= p->opt.iterations - s->steps; --t) {
      // the step's system at theta_t, factored in the factor cache (a failure
      // marks the graph in a status copy of the workspace)
      SpArgs at = a;
      at.poses = a.factor + p->traj_off + (size_t)t * p->V * sz;
      at.status = fstat;
      hipLaunchKernelGGL((k_sp_lin<G, double>), g_cost, dim3(kBT), 0, st, at, at.ws64);
      hipLaunchKernelGGL(k_sp_zero, g_zero, dim3(kBT), 0, st, at);
      hipLaunchKernelGGL((k_sp_assemble<G, double>), g_blk, dim3(kBT), 0, st, at, (const double*)at.ws64,
                         p->opt.lambda, 1, 0);
      sp_factor<G>(p, at, st);
      hipLaunchKernelGGL(k_sp_copy, g_vec, dim3(kBT), 0, st, at, 1, 2);
      sp_sweeps(p, at, 0, st);
      hipLaunchKernelGGL(k_sp_unroll_retr<G>, g_pose, dim3(kBT), 0, st, at);
      sp_sweeps(p, at, 2, st);
      hipLaunchKernelGGL(k_sp_unroll_cost<G>, g_cost, dim3(kBT), 0, st, at);
      hipLaunchKernelGGL(k_sp_unroll_gather<G>, g_pose, dim3(kBT), 0, st, at);
    }
    hipLaunchKernelGGL(k_sp_grads_zero<G>, g_cost, dim3(kBT), 0, st, a, 1);
    hipLaunchKernelGGL(k_sp_unroll_adj, g_pose, dim3(kBT), 0, st, a, d, 0);
    if (s->adjoint)
      HIP_TRY(hipMemcpyAsync(s->adjoint, a.uout, (size_t)p->V * d * sizeof(double), hipMemcpyDeviceToDevice, st));
    // the factor cache again holds the factor of H* at theta_K
    hipLaunchKernelGGL(k_sp_failed_from_status, dim3((B + 255) / 256), dim3(256), 0, st, a.failed, a.status, B);
    hipLaunchKernelGGL((k_sp_lin<G, double>), g_cost, dim3(kBT), 0, st, a, a.ws64);
    hipLaunchKernelGGL(k_sp_zero, g_zero, dim3(kBT), 0, st, a);
    hipLaunchKernelGGL((k_sp_assemble<G, double>), g_blk, dim3(kBT), 0, st, a, (const double*)a.ws64, 0.0, 1, 0);
    sp_factor<G>(p, a, st);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  hipLaunchKernelGGL((k_sp_lin<G, double>), g_cost, dim3(kBT), 0, st, a, a.ws64);
  hipLaunchKernelGGL(k_sp_seed, g_pose, dim3(kBT), 0, st, a, GroupTraits<G>::d);
  // u = H*^-1 v (slot 0; v kept in slot 1), then one step of float64
  // iterative refinement u <- u + H*^-1 (v - H* u), H* matrix-free from the
  // float64 records at theta_K: u then carries the rounding of that product
  // rather than the factorisation's rounding amplified by cond(H*)
  const dim3 g_vec(std::min(64, (max_desc(p->sd, &SpDesc::nvec) + kBT - 1) / kBT), B);
  hipLaunchKernelGGL(k_sp_copy, g_vec, dim3(kBT), 0, st, a, 2, 1);
  sp_sweeps(p, a, 0, st);
  hipLaunchKernelGGL(k_sp_jx<G>, g_cost, dim3(kBT), 0, st, a, 0);
  hipLaunchKernelGGL(k_sp_residual<G>, g_pose, dim3(kBT), 0, st, a, 0.0, 0);
  sp_sweeps(p, a, 2, st);
  hipLaunchKernelGGL(k_sp_accumulate<G>, g_pose, dim3(kBT), 0, st, a, 0);
  if (s->mode == DNLS_BACKWARD_EXACT)
    // u <- u + H*^-1 (v - Hx u), preconditioned by the cached factor
    for (int sw = 0; sw < s->sweeps; ++sw) {
      hipLaunchKernelGGL(k_sp_hvp_cost<G>, g_cost, dim3(kBT), 0, st, a);
      hipLaunchKernelGGL(k_sp_hvp_res<G>, g_pose, dim3(kBT), 0, st, a);
      sp_sweeps(p, a, 2, st);
      hipLaunchKernelGGL(k_sp_accumulate<G>, g_pose, dim3(kBT), 0, st, a, 0);
    }
  hipLaunchKernelGGL(k_sp_uout, g_pose, dim3(kBT), 0, st, a, GroupTraits<G>::d);
  hipLaunchKernelGGL(k_sp_vjp<G>, g_cost, dim3(kBT), 0, st, a);
  HIP_TRY(hipGetLastError());
  if (s->adjoint)
    HIP_TRY(hipMemcpyAsync(s->adjoint, a.uout, (size_t)p->V * p->d * sizeof(double), hipMemcpyDeviceToDevice, st));
  return DNLS_OK;
}

// Bundle adjustment on the block-sparse solver: K fixed-damping steps and
// the final linearisation, all through the tile factorisation and solves
static dnls_status sp_solve_ba(dnls_plan p, const dnls_solve_args* s, hipStream_t st) {
  if (!s->points || (p->O > 0 && (!s->obs_uv || !s->obs_w)) || (p->P > 0 && (!s->prior_meas || !s->prior_logw)))
    return fail(DNLS_ERR_INVALID_ARG, "points, obs_uv, obs_w and prior data are required");
  SpArgs a = sp_args(p, s->workspace, s->factor);
  a.poses = s->poses;
  a.pts = s->points;
  a.obs_uv = s->obs_uv;
  a.obs_w = s->obs_w;
  a.delta_b = s->huber_delta;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.objective = s->objective;
  a.status = s->status;
  const int B = p->B;
  const bool mixed = p->opt.precision == DNLS_PREC_MIXED;
  const dim3 g_lin(p->nlin_blocks, B);
  const int nvar = max_desc(p->sd, &SpDesc::npose) + max_desc(p->sd, &SpDesc::npt);
  const dim3 g_asm((nvar + max_desc(p->sd, &SpDesc::ncp) + kBT - 1) / kBT, B);
  const dim3 g_upd((nvar + kBT - 1) / kBT, B);
  const dim3 g_zero(256, B);
  const dim3 g_vec(std::min(64, (max_desc(p->sd, &SpDesc::nvec) + kBT - 1) / kBT), B);
  hipLaunchKernelGGL(k_sp_reset, dim3((B + 255) / 256), dim3(256), 0, st, a.failed, a.status, B);
  for (int it = 0; it <= p->opt.iterations; ++it) {
    const bool final_lin = it == p->opt.iterations;
    const double lam = final_lin ? 0.0 : p->opt.lambda;
    a.it = it;
    // float J^T J blocks inside the loop on the mixed path (float64 gradient
    // parts); the final, cached linearisation is float64
    const bool lin32 = mixed && !final_lin;
    if (lin32) hipLaunchKernelGGL(k_spba_lin<float>, g_lin, dim3(kBT), 0, st, a);
    else hipLaunchKernelGGL(k_spba_lin<double>, g_lin, dim3(kBT), 0, st, a);
    hipLaunchKernelGGL(k_sp_objective, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
    hipLaunchKernelGGL(k_sp_zero, g_zero, dim3(kBT), 0, st, a);
    if (lin32) hipLaunchKernelGGL(k_spba_assemble<float>, g_asm, dim3(kBT), 0, st, a, lam);
    else hipLaunchKernelGGL(k_spba_assemble<double>, g_asm, dim3(kBT), 0, st, a, lam);
    sp_factor<3>(p, a, st);
    if (final_lin) break;
    hipLaunchKernelGGL(k_sp_copy, g_vec, dim3(kBT), 0, st, a, 1, 2);
    sp_sweeps(p, a, 0, st);
    hipLaunchKernelGGL(k_spba_update, g_upd, dim3(kBT), 0, st, a, 0);
  }
  HIP_TRY(hipGetLastError());
  return DNLS_OK;
}

// implicit backward of bundle adjustment on the block-sparse solver
static dnls_status sp_backward_ba(dnls_plan p, const dnls_backward_args* s, hipStream_t st) {
  if (s->mode != DNLS_BACKWARD_IMPLICIT)
    return fail(DNLS_ERR_UNSUPPORTED, "bundle adjustment on the block-sparse solver has the implicit backward only");
  if (!s->points || (p->O > 0 && (!s->obs_uv || !s->obs_w)) || (p->P > 0 && (!s->prior_meas || !s->prior_logw)))
    return fail(DNLS_ERR_INVALID_ARG, "points, obs_uv, obs_w and prior data are required");
  SpArgs a = sp_args(p, s->workspace, const_cast<void*>(s->factor));
  a.poses = const_cast<double*>(s->poses);
  a.pts = const_cast<double*>(s->points);
  a.obs_uv = s->obs_uv;
  a.obs_w = s->obs_w;
  a.delta_b = s->huber_delta;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.status = const_cast<int*>(s->status);
  a.seed = s->seed_pose;
  a.seed_pt = s->seed_point;
  a.g_w = s->grad_obs_w;
  a.g_logw_p = s->grad_prior_logw;
  if (s->grad_obs_delta) a.g_delta = s->grad_obs_delta;
  a.g_huber = s->grad_huber_delta;
  const int B = p->B;
  const dim3 g_lin(p->nlin_blocks, B);
  const int nvar = max_desc(p->sd, &SpDesc::npose) + max_desc(p->sd, &SpDesc::npt);
  const dim3 g_upd((nvar + kBT - 1) / kBT, B);
  hipLaunchKernelGGL(k_sp_failed_from_status, dim3((B + 255) / 256), dim3(256), 0, st, a.failed, a.status, B);
  hipLaunchKernelGGL(k_spba_seed, g_upd, dim3(kBT), 0, st, a);
  sp_sweeps(p, a, 0, st);
  const int nv = std::max(max_desc(p->sd, &SpDesc::nobs) + max_desc(p->sd, &SpDesc::nprior),
                          max_desc(p->sd, &SpDesc::npose));
  hipLaunchKernelGGL(k_spba_vjp, dim3((nv + kBT - 1) / kBT, B), dim3(kBT), 0, st, a);
  if (a.g_huber) hipLaunchKernelGGL(k_spba_delta_sum, dim3(B), dim3(kBT), 0, st, a);
  HIP_TRY(hipGetLastError());
  if (s->adjoint)
    HIP_TRY(hipMemcpyAsync(s->adjoint, a.uout, (size_t)p->V * 6 * sizeof(double), hipMemcpyDeviceToDevice, st));
  return DNLS_OK;
}

dnls_status sp_solve(dnls_plan p, const dnls_solve_args* s, hipStream_t st) {
  if (p->sp_ba) return sp_solve_ba(p, s, st);
  if (p->group == DNLS_SE3) return sp_solve_impl<3>(p, s, st);
  return sp_solve_impl<2>(p, s, st);
}

dnls_status sp_backward(dnls_plan p, const dnls_backward_args* s, hipStream_t st) {
  if (p->sp_ba) return sp_backward_ba(p, s, st);
  if (p->group == DNLS_SE3) return sp_backward_impl<3>(p, s, st);
  return sp_backward_impl<2>(p, s, st);
}

}  // namespace dnls
