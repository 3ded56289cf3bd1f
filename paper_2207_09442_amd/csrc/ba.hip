// Bundle adjustment with the Schur complement (solver SCHUR).
//
// Variables: world-to-camera poses T (SE(3)) and world points q (R^3).  Cost
// per observation: pinhole reprojection c = pi(R q + t) - uv with a scalar
// weight w and a Huber loss on s = ||w c||^2 (Section 3 cost library: the
// reprojection error and robust losses; Appendix E.3).  The Gauss-Newton step
// uses the first-order reweighting rho'(s): J~ = sqrt(rho') w C, r~ =
// sqrt(rho') w c.  Camera priors c = Log(P^-1 T) fix the gauge.
//
// The point blocks are eliminated (Section 4.2: the Schur complement trick
// that sparse solvers for bundle adjustment rely on): with B the camera
// block, E the camera-point blocks and C the block-diagonal point block,
//   S = B - E C^-1 E^T,  g_s = g_c - E C^-1 g_p,
//   S delta_c = g_s (dense MFMA Cholesky),  delta_p = C^-1 (g_p - E^T delta_c).
// Levenberg-Marquardt damping adds lambda to the diagonals of B and C.
// The backward (Proposition 1) solves H* u = v with the same elimination and
// the cached factor of S*, then forms dL/dw_o = -d/dw_o [rho'(s) w^2 (C u)^T c].
//
// Kernels per step (grid y = problem): linearise observations, point blocks
// and E C^-1, Schur complement by gathering per camera pair (plan-built
// contribution lists: no atomics), dense factor + solve (one workgroup per
// problem), point back-substitution and retraction.
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
#include "reproj.hpp"

namespace dnls {
namespace {

constexpr int kBT = 256;
constexpr int kBaNway = 6;          // DNLS_FLAG_PAIR: workgroups per problem sharing the camera factorisation
constexpr int kBaCtr = 16;          // event counters per problem: diagonal block, then one per workgroup
static_assert(3 + kBaNway <= kBaCtr, "BA pair counters");
constexpr int kObsRec = 20;   // J~cam (2x6), J~pt (2x3), r~ (2)
constexpr int kPriorRec = 42; // w C (6x6), w c (6)

struct BAArgs {
  const BADesc* bd;
  const int* obs_cam;
  const int* obs_pt;
  const int* cam_obs_off;
  const int* cam_obs;
  const int* pt_obs_off;
  const int* pt_obs;
  const int4* sblk;
  const int2* spair;
  const int* prior_var;
  double* cams;
  double* pts;
  const double* obs_uv;
  const double* obs_w;
  const double* prior_meas;
  const double* prior_logw;
  double fx, fy, cx, cy, delta;
  const double* delta_b;   // per-problem Huber radius, or NULL for delta
  void* orec;
  double* gob;      // mixed: per-observation float64 gradient parts [obs][9] (camera 6, point 3)
  double* prec;
  double* E;
  double* F;
  double* Cinv;
  double* gp;
  double* partial;
  double* dc;
  int* frozen;
  double* lastobj;
  double* objective;
  int* status;
  double* factor;
  int K, it, npad_max, nx_lin;
  double lambda;
  // DNLS_FLAG_ADAPTIVE_LM: lambda per problem (read by the point and Schur
  // kernels when set), theta_t backup, trial step rejected
  double* lam_g;
  double* bak_c;
  double* bak_p;
  int* rej;
  // DLM backward: the right-hand side becomes g - dlm_eps v (v: seed_c, seed_p)
  double dlm_eps;
  // DNLS_FLAG_DOGLEG (float64 records): point step, camera gradient, J x per
  // observation, (H + lambda I) x, per-problem state (radius, predicted
  // decrease, |delta|, on the boundary)
  double* dp;
  double* gc;
  double* yo;
  double* hc;
  double* hp;
  double* dl;
  double radius0;
  // DNLS_FLAG_PAIR: nway co-resident workgroups per problem share the factorisation
  unsigned long long* pair_ctr;
  unsigned long long pair_base;
  int pair_spin, nway;
  // backward
  const double* seed_c;
  const double* seed_p;
  double* uc;
  double* up;
  double* g_w;
  double* g_logw_p;
  double* g_delta;         // per-observation Huber radius (implicit and DLM backward)
  double* adjoint_out;
};

__device__ __forceinline__ double huber_radius(const BAArgs& a, int b) { return a.delta_b ? a.delta_b[b] : a.delta; }

__device__ double block_sum_ba(double v, double* red) {
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

// 1. linearise observations (and the problem's priors in its first block).
// S = float (mixed precision): the Jacobians of the J^T J blocks are rounded
// to float, while the gradient contributions J~^T r~ of each observation
// (camera 6, point 3) are formed from the float64 residual and Jacobians and
// kept in float64 (a.gob): a float gradient moves the fixed point of the
// iteration by far more than the float curvature does.
template <class S>
__global__ void __launch_bounds__(kBT) k_ba_lin(BAArgs a) {
  __shared__ double red[kBT / 64];
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  double sacc = 0.0;
  if (!a.frozen[b]) {
    const int lo = blockIdx.x * kBT + threadIdx.x;
    if (lo < g.nobs) {
      const int o = g.obs0 + lo;
      double c[2], Jc[12], Jp[6];
      reproj<double>(a.cams + (size_t)a.obs_cam[o] * 12, a.pts + (size_t)a.obs_pt[o] * 3, a.obs_uv + (size_t)o * 2,
                     a, c, Jc, Jp);
      const double w = a.obs_w[o];
      double rho, drho;
      huber(w * w * (c[0] * c[0] + c[1] * c[1]), huber_radius(a, b), rho, drho);
      const double sw = ::sqrt(drho) * w;
      S* rec = reinterpret_cast<S*>(a.orec) + (size_t)o * kObsRec;
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
      sacc += 0.5 * rho;
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < g.nprior) {
      const int q = g.prior0 + threadIdx.x;
      double c[6], C[36];
      prior_cost<3, double>(a.cams + (size_t)a.prior_var[q] * 12, a.prior_meas + (size_t)q * 12, c, C);
      const double w = exp(a.prior_logw[q]);
      double* pr = a.prec + (size_t)q * kPriorRec;
      double cc = 0.0;
      for (int k = 0; k < 36; ++k) pr[k] = w * C[k];
      for (int k = 0; k < 6; ++k) {
        pr[36 + k] = w * c[k];
        cc += c[k] * c[k];
      }
      sacc += 0.5 * w * w * cc;
    }
  }
  const double tot = block_sum_ba(sacc, red);
  if (threadIdx.x == 0) a.partial[b * a.nx_lin + blockIdx.x] = tot;
}

__device__ __forceinline__ bool inv3(const double m[9], double r[9]) {
  r[0] = m[4] * m[8] - m[5] * m[7];
  r[1] = m[2] * m[7] - m[1] * m[8];
  r[2] = m[1] * m[5] - m[2] * m[4];
  r[3] = m[5] * m[6] - m[3] * m[8];
  r[4] = m[0] * m[8] - m[2] * m[6];
  r[5] = m[2] * m[3] - m[0] * m[5];
  r[6] = m[3] * m[7] - m[4] * m[6];
  r[7] = m[1] * m[6] - m[0] * m[7];
  r[8] = m[0] * m[4] - m[1] * m[3];
  const double det = m[0] * r[0] + m[1] * r[3] + m[2] * r[6];
  const double id = 1.0 / det;
#pragma unroll
  for (int k = 0; k < 9; ++k) r[k] *= id;
  return det > 0.0;
}

// 2. point blocks C = sum J~p^T J~p + lambda I, g_p, C^-1 (one thread per point)
template <class S>
__global__ void __launch_bounds__(kBT) k_ba_point(BAArgs a, double lambda) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  if (a.lam_g) lambda = a.lam_g[b];
  const int lp = blockIdx.x * kBT + threadIdx.x;
  if (lp >= g.npt) return;
  const int pt = g.pt0 + lp;
  const S* rec = reinterpret_cast<const S*>(a.orec);
  S C[9];
  double gg[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 9; ++k) C[k] = S(0);
  for (int s = a.pt_obs_off[pt]; s < a.pt_obs_off[pt + 1]; ++s) {
    const int o = a.pt_obs[s];
    const S* r = rec + (size_t)o * kObsRec;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j) C[i * 3 + j] += r[12 + i] * r[12 + j] + r[15 + i] * r[15 + j];
      if constexpr (std::is_same<S, double>::value) gg[i] += r[12 + i] * r[18] + r[15 + i] * r[19];
      else gg[i] += a.gob[(size_t)o * 9 + 6 + i];
    }
  }
  double Cd[9], Ci[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Cd[k] = double(C[k]) + ((k % 4 == 0) ? lambda : 0.0);
  inv3(Cd, Ci);
#pragma unroll
  for (int k = 0; k < 9; ++k) a.Cinv[(size_t)pt * 9 + k] = Ci[k];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    a.gp[(size_t)pt * 3 + k] = gg[k] - (a.dlm_eps > 0.0 && a.seed_p ? a.dlm_eps * a.seed_p[(size_t)pt * 3 + k] : 0.0);
}

// 2b. per observation: E_o = J~c^T J~p and F_o = E_o C^-1 of its point
// (after k_ba_point; one thread per observation)
template <class S>
__global__ void __launch_bounds__(kBT) k_ba_obs_ef(BAArgs a) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (t >= g.nobs) return;
  const int o = g.obs0 + t;
  const S* r = reinterpret_cast<const S*>(a.orec) + (size_t)o * kObsRec;
  const double* Ci = a.Cinv + (size_t)a.obs_pt[o] * 9;
  double Eo[18];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Eo[i * 3 + j] = double(r[i] * r[12 + j] + r[6 + i] * r[15 + j]);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      a.E[(size_t)o * 18 + i * 3 + j] = Eo[i * 3 + j];
      a.F[(size_t)o * 18 + i * 3 + j] = Eo[i * 3] * Ci[j] + Eo[i * 3 + 1] * Ci[3 + j] + Eo[i * 3 + 2] * Ci[6 + j];
    }
}

// sum over the 64 lanes of a wave (butterfly; every lane gets the total)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// 3. Schur complement S (lower blocks, all) and g_s into the right-hand-side row.
// One wave per camera-pair block: the lanes split the block's contribution
// list (observations of the camera for a diagonal block, point-sharing
// observation pairs for every block), then a butterfly sum.
constexpr int kSchurWaves = kBT / 64;
template <class S>
__global__ void __launch_bounds__(kBT) k_ba_schur(BAArgs a, double lambda) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  if (a.lam_g) lambda = a.lam_g[b];
  double* A = a.factor + g.fac_off;
  const int npad = g.npad;
  const S* rec = reinterpret_cast<const S*>(a.orec);
  // padding rows, the right-hand-side row and the padding rows after it
  if (blockIdx.x == 0) {
    for (int e = threadIdx.x; e < (npad - g.n) * npad; e += kBT) {
      const int r = g.n + e / npad, c = e % npad;
      A[(size_t)r * npad + c] = (r == c) ? 1.0 : 0.0;
    }
    for (int e = threadIdx.x; e < 16 * npad; e += kBT) {
      const int r = npad + e / npad, c = e % npad;
      if (r > npad || c >= g.n) A[(size_t)r * npad + c] = 0.0;
    }
  }
  const int lane = threadIdx.x & 63;
  const int lb = blockIdx.x * kSchurWaves + (threadIdx.x >> 6);
  if (lb >= g.nblk) return;
  const int4 blk = a.sblk[g.blk0 + lb];
  const int ca = blk.x, cb = blk.y;
  double v[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) v[k] = 0.0;
  double gs[6] = {0, 0, 0, 0, 0, 0};
  if (ca == cb) {
    const int cam = g.cam0 + ca;
    S h[36];
#pragma unroll
    for (int k = 0; k < 36; ++k) h[k] = S(0);
    double gsl[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int s = a.cam_obs_off[cam] + lane; s < a.cam_obs_off[cam + 1]; s += 64) {
      const int o = a.cam_obs[s];
      const S* r = rec + (size_t)o * kObsRec;
#pragma unroll
      for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) h[i * 6 + j] += r[i] * r[j] + r[6 + i] * r[6 + j];
        if constexpr (std::is_same<S, double>::value) gsl[i] += r[i] * r[18] + r[6 + i] * r[19];
        else gsl[i] += a.gob[(size_t)o * 9 + i];
      }
      // - F_o g_p
      const double* Fo = a.F + (size_t)o * 18;
      const double* gpp = a.gp + (size_t)a.obs_pt[o] * 3;
#pragma unroll
      for (int i = 0; i < 6; ++i) gs[i] -= Fo[i * 3] * gpp[0] + Fo[i * 3 + 1] * gpp[1] + Fo[i * 3 + 2] * gpp[2];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) v[i * 6 + j] = double(h[i * 6 + j]);
#pragma unroll
    for (int k = 0; k < 6; ++k) gs[k] += gsl[k];
  }
  for (int s = blk.z + lane; s < blk.z + blk.w; s += 64) {
    const int2 pr = a.spair[s];
    const double* Fa = a.F + (size_t)pr.x * 18;
    const double* Eb = a.E + (size_t)pr.y * 18;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < 6; ++j) v[i * 6 + j] -= Fa[i * 3] * Eb[j * 3] + Fa[i * 3 + 1] * Eb[j * 3 + 1] + Fa[i * 3 + 2] * Eb[j * 3 + 2];
  }
  // butterfly sums (the diagonal block's J^T J part is symmetric: lower half only)
#pragma unroll
  for (int k = 0; k < 36; ++k) v[k] = wave_sum(v[k]);
  if (ca == cb) {
#pragma unroll
    for (int k = 0; k < 6; ++k) gs[k] = wave_sum(gs[k]);
  }
  if (lane != 0) return;
  if (ca == cb) {
    const int cam = g.cam0 + ca;
    // the J^T J part was accumulated on the lower triangle; the E C^-1 E^T
    // part of a diagonal block is symmetric as well
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = i + 1; j < 6; ++j) v[i * 6 + j] = v[j * 6 + i];
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      if (a.prior_var[q] != cam) continue;
      const double* pr = a.prec + (size_t)q * kPriorRec;
      for (int i = 0; i < 6; ++i) {
        for (int j = 0; j < 6; ++j) {
          double t = 0.0;
          for (int k = 0; k < 6; ++k) t += pr[k * 6 + i] * pr[k * 6 + j];
          v[i * 6 + j] += t;
        }
        double t = 0.0;
        for (int k = 0; k < 6; ++k) t += pr[k * 6 + i] * pr[36 + k];
        gs[i] += t;
      }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i * 7] += lambda;
    if (a.dlm_eps > 0.0)
      for (int i = 0; i < 6; ++i) gs[i] -= a.dlm_eps * a.seed_c[(size_t)cam * 6 + i];
    double* aug = A + (size_t)npad * npad;
#pragma unroll
    for (int i = 0; i < 6; ++i) aug[ca * 6 + i] = gs[i];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) A[(size_t)(ca * 6 + i) * npad + cb * 6 + j] = v[i * 6 + j];
}

struct BALds {
  DenseLds dl;
  double red[kNW];
};

// 4. objective, factorisation and camera step (one workgroup per problem)
// MULTI: a cooperative launch of nway workgroups per problem (blocks b,
// b + B, ...): all of them take part in the factorisation (chol_dense_pair),
// the leader (role 0) does the rest.
template <bool MULTI>
__global__ void __launch_bounds__(kNT) k_ba_factor(BAArgs a, int final_lin) {
  extern __shared__ double dyn[];
  __shared__ BALds L;
  const int nslot = MULTI ? gridDim.x / a.nway : gridDim.x;
  const int b = blockIdx.x % nslot;
  const int role = blockIdx.x / nslot;
  const BADesc g = a.bd[b];
  double* obj = a.objective + (size_t)b * (a.K + 1);
  if (a.frozen[b]) {
    if (threadIdx.x == 0) obj[a.it] = a.lastobj[b];
    return;
  }
  double S = 0.0;
  for (int k = 0; k < a.nx_lin; ++k) S += a.partial[b * a.nx_lin + k];
  if (threadIdx.x == 0 && role == 0) {
    obj[a.it] = S;
    a.lastobj[b] = S;
  }
  if (!isfinite(S)) {
    if (threadIdx.x == 0 && role == 0) {
      a.frozen[b] = DNLS_GRAPH_NONFINITE;
      a.status[b] = DNLS_GRAPH_NONFINITE;
    }
    return;
  }
  double* A = a.factor + g.fac_off;
  double* winv = A + (size_t)(g.npad + 16) * g.npad;
  bool ok;
  if constexpr (MULTI) {
    unsigned long long* c = a.pair_ctr + (size_t)b * kBaCtr;
    const PairSync ps{nullptr, nullptr, c + 2, c + 3, a.pair_base, role, a.nway, a.pair_spin};
    bool bail = false;
    ok = chol_dense_pair(A, A, g.npad, winv, L.dl, ps, 0, bail);
    if (role != 0) return;
    if (bail) {
      if (threadIdx.x == 0) {
        a.frozen[b] = DNLS_GRAPH_TIMEOUT;
        a.status[b] = DNLS_GRAPH_TIMEOUT;
      }
      return;
    }
  } else {
    ok = chol_dense(A, A, g.npad, winv, L.dl);
  }
  if (!ok) {
    if (threadIdx.x == 0) {
      a.frozen[b] = DNLS_GRAPH_NOT_PD;
      a.status[b] = DNLS_GRAPH_NOT_PD;
    }
    return;
  }
  if (final_lin) return;
  double* x = dyn;
  for (int u = threadIdx.x; u < g.npad; u += kNT) x[u] = A[(size_t)g.npad * g.npad + u];
  __syncthreads();
  trsv_upper_t(A, g.npad, winv, x, L.dl);
  for (int u = threadIdx.x; u < g.npad; u += kNT) a.dc[(size_t)b * a.npad_max + u] = x[u];
}

// 5. point back-substitution and retraction of cameras and points
__global__ void __launch_bounds__(kBT) k_ba_update(BAArgs a) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  const double* dc = a.dc + (size_t)b * a.npad_max;
  if (t < g.npt) {
    const int pt = g.pt0 + t;
    double r[3] = {a.gp[(size_t)pt * 3], a.gp[(size_t)pt * 3 + 1], a.gp[(size_t)pt * 3 + 2]};
    for (int s = a.pt_obs_off[pt]; s < a.pt_obs_off[pt + 1]; ++s) {
      const int o = a.pt_obs[s];
      const double* Eo = a.E + (size_t)o * 18;
      const double* d = dc + (a.obs_cam[o] - g.cam0) * 6;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) acc += Eo[i * 3 + j] * d[i];
        r[j] -= acc;
      }
    }
    const double* Ci = a.Cinv + (size_t)pt * 9;
#pragma unroll
    for (int j = 0; j < 3; ++j) a.pts[(size_t)pt * 3 + j] -= Ci[j * 3] * r[0] + Ci[j * 3 + 1] * r[1] + Ci[j * 3 + 2] * r[2];
  }
  if (t < g.ncam) retract_minus<3>(a.cams + (size_t)(g.cam0 + t) * 12, dc + t * 6);
}

// adaptive damping (Levenberg-Marquardt, Section 3 optimizers): the step is
// kept iff the float64 objective at the trial point is strictly below S(theta_t)
// (lambda / 10, floor 1e-7), else cameras and points return to theta_t
// (lambda x 10, ceiling 1e7)
constexpr double kLambdaMin = 1e-7, kLambdaMax = 1e7;

__global__ void k_ba_lam_init(BAArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) a.lam_g[b] = a.lambda;
}

// theta_t -> backup (dir = 0) or backup -> theta_t for rejected steps (dir = 1)
__global__ void __launch_bounds__(kBT) k_ba_backup(BAArgs a, int dir) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b] || (dir && !a.rej[b])) return;
  for (int u = blockIdx.x * kBT + threadIdx.x; u < g.ncam * 12; u += gridDim.x * kBT) {
    const size_t k = (size_t)g.cam0 * 12 + u;
    if (dir) a.cams[k] = a.bak_c[k];
    else a.bak_c[k] = a.cams[k];
  }
  for (int u = blockIdx.x * kBT + threadIdx.x; u < g.npt * 3; u += gridDim.x * kBT) {
    const size_t k = (size_t)g.pt0 * 3 + u;
    if (dir) a.pts[k] = a.bak_p[k];
    else a.bak_p[k] = a.pts[k];
  }
}

// trial objective from the partials of k_ba_lin<double> at the retracted
// point against S(theta_t) (thread per problem)
__global__ void k_ba_decide(BAArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  a.rej[b] = 0;
  if (a.frozen[b]) return;
  double S = 0.0;
  for (int k = 0; k < a.nx_lin; ++k) S += a.partial[b * a.nx_lin + k];
  if (S < a.lastobj[b]) {
    a.lam_g[b] = fmax(a.lam_g[b] / 10.0, kLambdaMin);
  } else {
    a.lam_g[b] = fmin(a.lam_g[b] * 10.0, kLambdaMax);
    a.rej[b] = 1;
  }
}

// Powell's dogleg over cameras and points together (Section 3 optimizers):
// the Gauss-Newton step of H + lambda I if |delta| <= radius, else the
// gradient cut at the boundary if the Cauchy point lies outside, else the
// boundary point of the path from the Cauchy point to the Gauss-Newton step;
// kept iff the float64 objective strictly decreases; with rho = actual /
// predicted decrease the radius becomes |delta| / 4 if rho < 1/4 (or
// undefined) and min(2 radius, 1e4) if rho > 3/4 on the boundary
constexpr double kRadiusMax = 1e4;

__global__ void k_ba_dl_init(BAArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) a.dl[4 * b] = a.radius0;
}

// point part of the Gauss-Newton step, C^-1 (g_p - E^T dc), and the camera
// gradient sum J~c^T r~ + priors (thread per point / camera)
__global__ void __launch_bounds__(kBT) k_ba_dl_gn(BAArgs a) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  const double* dc = a.dc + (size_t)b * a.npad_max;
  if (t < g.npt) {
    const int pt = g.pt0 + t;
    double r[3] = {a.gp[(size_t)pt * 3], a.gp[(size_t)pt * 3 + 1], a.gp[(size_t)pt * 3 + 2]};
    for (int s = a.pt_obs_off[pt]; s < a.pt_obs_off[pt + 1]; ++s) {
      const int o = a.pt_obs[s];
      const double* Eo = a.E + (size_t)o * 18;
      const double* d = dc + (a.obs_cam[o] - g.cam0) * 6;
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int i = 0; i < 6; ++i) acc += Eo[i * 3 + j] * d[i];
        r[j] -= acc;
      }
    }
    const double* Ci = a.Cinv + (size_t)pt * 9;
    for (int j = 0; j < 3; ++j)
      a.dp[(size_t)pt * 3 + j] = Ci[j * 3] * r[0] + Ci[j * 3 + 1] * r[1] + Ci[j * 3 + 2] * r[2];
  }
  if (t < g.ncam) {
    const int cam = g.cam0 + t;
    const double* rec = reinterpret_cast<const double*>(a.orec);
    double gs[6] = {0, 0, 0, 0, 0, 0};
    for (int s = a.cam_obs_off[cam]; s < a.cam_obs_off[cam + 1]; ++s) {
      const double* r = rec + (size_t)a.cam_obs[s] * kObsRec;
      for (int i = 0; i < 6; ++i) gs[i] += r[i] * r[18] + r[6 + i] * r[19];
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      if (a.prior_var[q] != cam) continue;
      const double* pr = a.prec + (size_t)q * kPriorRec;
      for (int i = 0; i < 6; ++i)
        for (int k = 0; k < 6; ++k) gs[i] += pr[k * 6 + i] * pr[36 + k];
    }
    for (int i = 0; i < 6; ++i) a.gc[(size_t)cam * 6 + i] = gs[i];
  }
}

// y_o = J~c x_c + J~p x_p per observation; x = (camera part `xc` with the
// per-problem layout of dc when cam_local, else global [Vc][6]; points [Vp][3])
__global__ void __launch_bounds__(kBT) k_ba_dl_jx(BAArgs a, const double* xc, int cam_local, const double* xp) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (t >= g.nobs) return;
  const int o = g.obs0 + t;
  const double* r = reinterpret_cast<const double*>(a.orec) + (size_t)o * kObsRec;
  const double* x = cam_local ? xc + (size_t)b * a.npad_max + (a.obs_cam[o] - g.cam0) * 6 : xc + (size_t)a.obs_cam[o] * 6;
  const double* q = xp + (size_t)a.obs_pt[o] * 3;
  for (int k = 0; k < 2; ++k) {
    double acc = 0.0;
    for (int i = 0; i < 6; ++i) acc += r[k * 6 + i] * x[i];
    for (int j = 0; j < 3; ++j) acc += r[12 + k * 3 + j] * q[j];
    a.yo[(size_t)o * 2 + k] = acc;
  }
}

// (H + lambda I) x from y_o: cameras (with the priors) into hc, points into hp
__global__ void __launch_bounds__(kBT) k_ba_dl_hx(BAArgs a, const double* xc, int cam_local, const double* xp,
                                                  double lambda) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  const double* rec = reinterpret_cast<const double*>(a.orec);
  if (t < g.ncam) {
    const int cam = g.cam0 + t;
    const double* x = cam_local ? xc + (size_t)b * a.npad_max + t * 6 : xc + (size_t)cam * 6;
    double h[6];
    for (int i = 0; i < 6; ++i) h[i] = lambda * x[i];
    for (int s = a.cam_obs_off[cam]; s < a.cam_obs_off[cam + 1]; ++s) {
      const int o = a.cam_obs[s];
      const double* r = rec + (size_t)o * kObsRec;
      const double y0 = a.yo[(size_t)o * 2], y1 = a.yo[(size_t)o * 2 + 1];
      for (int i = 0; i < 6; ++i) h[i] += r[i] * y0 + r[6 + i] * y1;
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      if (a.prior_var[q] != cam) continue;
      const double* pr = a.prec + (size_t)q * kPriorRec;
      for (int k = 0; k < 6; ++k) {
        double cx = 0.0;
        for (int j = 0; j < 6; ++j) cx += pr[k * 6 + j] * x[j];
        for (int i = 0; i < 6; ++i) h[i] += pr[k * 6 + i] * cx;
      }
    }
    for (int i = 0; i < 6; ++i) a.hc[(size_t)cam * 6 + i] = h[i];
  }
  if (t < g.npt) {
    const int pt = g.pt0 + t;
    double h[3];
    for (int j = 0; j < 3; ++j) h[j] = lambda * xp[(size_t)pt * 3 + j];
    for (int s = a.pt_obs_off[pt]; s < a.pt_obs_off[pt + 1]; ++s) {
      const int o = a.pt_obs[s];
      const double* r = rec + (size_t)o * kObsRec;
      const double y0 = a.yo[(size_t)o * 2], y1 = a.yo[(size_t)o * 2 + 1];
      for (int j = 0; j < 3; ++j) h[j] += r[12 + j] * y0 + r[15 + j] * y1;
    }
    for (int j = 0; j < 3; ++j) a.hp[(size_t)pt * 3 + j] = h[j];
  }
}

// per-problem reductions over cameras then points: sum f(u, v, w) of three
// vectors given by (camera part, point part) with the camera layouts above
struct DlVec {
  const double* c;
  int cam_local;
  const double* p;
};

__device__ __forceinline__ double dl_at(const BAArgs& a, const BADesc& g, int b, const DlVec& v, int u) {
  const int nc = g.ncam * 6;
  if (u < nc) return v.cam_local ? v.c[(size_t)b * a.npad_max + u] : v.c[(size_t)g.cam0 * 6 + u];
  return v.p[(size_t)g.pt0 * 3 + (u - nc)];
}

// the dogleg step (one workgroup per problem): Gauss-Newton step in (dc, dp),
// g in (gc, gp), (H + lambda I) g in (hc, hp); the chosen step replaces (dc, dp)
__global__ void __launch_bounds__(kBT) k_ba_dogleg(BAArgs a) {
  __shared__ double red[kBT / 64];
  const int b = blockIdx.x;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const DlVec X{a.dc, 1, a.dp}, Gv{a.gc, 0, a.gp}, HG{a.hc, 0, a.hp};
  const int n = g.ncam * 6 + g.npt * 3, nc = g.ncam * 6;
  auto put = [&](int u, double v) {
    if (u < nc) a.dc[(size_t)b * a.npad_max + u] = v;
    else a.dp[(size_t)g.pt0 * 3 + (u - nc)] = v;
  };
  const double radius = a.dl[4 * b];
  double p0 = 0.0;
  for (int u = threadIdx.x; u < n; u += kBT) {
    const double x = dl_at(a, g, b, X, u);
    p0 += x * x;
  }
  const double n_gn = ::sqrt(block_sum_ba(p0, red));
  int boundary = 0;
  if (!(n_gn <= radius)) {
    boundary = 1;
    double p1 = 0.0, p2 = 0.0;
    for (int u = threadIdx.x; u < n; u += kBT) {
      const double gu = dl_at(a, g, b, Gv, u);
      p1 += gu * gu;
      p2 += gu * dl_at(a, g, b, HG, u);
    }
    const double gg = block_sum_ba(p1, red);
    const double gHg = block_sum_ba(p2, red);
    const double alpha = gg / gHg;
    if (alpha * ::sqrt(gg) >= radius) {
      const double sc = radius / ::sqrt(gg);
      for (int u = threadIdx.x; u < n; u += kBT) put(u, sc * dl_at(a, g, b, Gv, u));
    } else {
      double q1 = 0.0, q2 = 0.0;
      for (int u = threadIdx.x; u < n; u += kBT) {
        const double sd = alpha * dl_at(a, g, b, Gv, u), dd = dl_at(a, g, b, X, u) - sd;
        q1 += dd * dd;
        q2 += sd * dd;
      }
      const double qa = block_sum_ba(q1, red);
      const double qb = 2.0 * block_sum_ba(q2, red);
      const double qc = alpha * alpha * gg - radius * radius;
      const double beta = (-qb + ::sqrt(qb * qb - 4.0 * qa * qc)) / (2.0 * qa);
      for (int u = threadIdx.x; u < n; u += kBT) {
        const double sd = alpha * dl_at(a, g, b, Gv, u);
        put(u, sd + beta * (dl_at(a, g, b, X, u) - sd));
      }
    }
  }
  if (threadIdx.x == 0) a.dl[4 * b + 3] = boundary;
}

// predicted decrease g^T delta - 1/2 delta^T (H + lambda I) delta and |delta|
// (delta in (dc, dp), (H + lambda I) delta in (hc, hp)), one workgroup per problem
__global__ void __launch_bounds__(kBT) k_ba_dl_pred(BAArgs a) {
  __shared__ double red[kBT / 64];
  const int b = blockIdx.x;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const DlVec X{a.dc, 1, a.dp}, Gv{a.gc, 0, a.gp}, HX{a.hc, 0, a.hp};
  const int n = g.ncam * 6 + g.npt * 3;
  double r1 = 0.0, r2 = 0.0, r3 = 0.0;
  for (int u = threadIdx.x; u < n; u += kBT) {
    const double x = dl_at(a, g, b, X, u);
    r1 += dl_at(a, g, b, Gv, u) * x;
    r2 += x * dl_at(a, g, b, HX, u);
    r3 += x * x;
  }
  const double s1 = block_sum_ba(r1, red);
  const double s2 = block_sum_ba(r2, red);
  const double s3 = block_sum_ba(r3, red);
  if (threadIdx.x == 0) {
    a.dl[4 * b + 1] = s1 - 0.5 * s2;
    a.dl[4 * b + 2] = ::sqrt(s3);
  }
}

// theta <- theta (-) delta for cameras and points (delta in (dc, dp))
__global__ void __launch_bounds__(kBT) k_ba_dl_apply(BAArgs a) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.frozen[b]) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (t < g.npt)
    for (int j = 0; j < 3; ++j) a.pts[(size_t)(g.pt0 + t) * 3 + j] -= a.dp[(size_t)(g.pt0 + t) * 3 + j];
  if (t < g.ncam) retract_minus<3>(a.cams + (size_t)(g.cam0 + t) * 12, a.dc + (size_t)b * a.npad_max + t * 6);
}

// keep the trial step iff the objective decreased; radius update (thread per problem)
__global__ void k_ba_dl_decide(BAArgs a, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  a.rej[b] = 0;
  if (a.frozen[b]) return;
  double S = 0.0;
  for (int k = 0; k < a.nx_lin; ++k) S += a.partial[b * a.nx_lin + k];
  const double s_t = a.lastobj[b];
  const double rho = (s_t - S) / a.dl[4 * b + 1];
  if (!(S < s_t)) a.rej[b] = 1;
  if (!(rho >= 0.25)) a.dl[4 * b] = 0.25 * a.dl[4 * b + 2];
  else if (rho > 0.75 && a.dl[4 * b + 3] != 0.0) a.dl[4 * b] = fmin(2.0 * a.dl[4 * b], kRadiusMax);
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// u_c = S*^-1 (v_c - sum_o F_o v_p(o))  (one workgroup per problem)
__global__ void __launch_bounds__(kNT) k_ba_bwd_cam(BAArgs a) {
  extern __shared__ double dyn[];
  __shared__ BALds L;
  const int b = blockIdx.x;
  const BADesc g = a.bd[b];
  if (a.status[b] != DNLS_GRAPH_OK) return;
  const double* A = a.factor + g.fac_off;
  const double* winv = A + (size_t)(g.npad + 16) * g.npad;
  double* x = dyn;
  for (int u = threadIdx.x; u < g.npad; u += kNT) {
    double v = 0.0;
    if (u < g.n) {
      const int ca = u / 6, i = u % 6, cam = g.cam0 + ca;
      v = a.seed_c[(size_t)cam * 6 + i];
      if (a.seed_p)
        for (int s = a.cam_obs_off[cam]; s < a.cam_obs_off[cam + 1]; ++s) {
          const int o = a.cam_obs[s];
          const double* Fo = a.F + (size_t)o * 18 + i * 3;
          const double* vp = a.seed_p + (size_t)a.obs_pt[o] * 3;
          v -= Fo[0] * vp[0] + Fo[1] * vp[1] + Fo[2] * vp[2];
        }
    }
    x[u] = v;
  }
  __syncthreads();
  trsv_lower(A, g.npad, winv, x, L.dl);
  trsv_upper_t(A, g.npad, winv, x, L.dl);
  for (int u = threadIdx.x; u < g.npad; u += kNT) a.uc[(size_t)b * a.npad_max + u] = x[u];
  if (a.adjoint_out)
    for (int u = threadIdx.x; u < g.n; u += kNT) a.adjoint_out[(size_t)g.cam0 * 6 + u] = x[u];
}

// u_p = C^-1 (v_p - sum_o E_o^T u_c(o))
__global__ void __launch_bounds__(kBT) k_ba_bwd_pt(BAArgs a) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  if (a.status[b] != DNLS_GRAPH_OK) return;
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (t >= g.npt) return;
  const int pt = g.pt0 + t;
  const double* uc = a.uc + (size_t)b * a.npad_max;
  double r[3] = {0, 0, 0};
  if (a.seed_p)
    for (int j = 0; j < 3; ++j) r[j] = a.seed_p[(size_t)pt * 3 + j];
  for (int s = a.pt_obs_off[pt]; s < a.pt_obs_off[pt + 1]; ++s) {
    const int o = a.pt_obs[s];
    const double* Eo = a.E + (size_t)o * 18;
    const double* d = uc + (a.obs_cam[o] - g.cam0) * 6;
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int i = 0; i < 6; ++i) acc += Eo[i * 3 + j] * d[i];
      r[j] -= acc;
    }
  }
  const double* Ci = a.Cinv + (size_t)pt * 9;
  for (int j = 0; j < 3; ++j) a.up[(size_t)pt * 3 + j] = Ci[j * 3] * r[0] + Ci[j * 3 + 1] * r[1] + Ci[j * 3 + 2] * r[2];
}

// per-observation and per-prior VJP
__global__ void __launch_bounds__(kBT) k_ba_bwd_obs(BAArgs a) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  const bool ok = a.status[b] == DNLS_GRAPH_OK;
  const int t = blockIdx.x * kBT + threadIdx.x;
  const double* uc = a.uc + (size_t)b * a.npad_max;
  if (t < g.nobs && (a.g_w || a.g_delta)) {
    const int o = g.obs0 + t;
    double gw = 0.0, gd = 0.0;
    if (ok) {
      double c[2], Jc[12], Jp[6];
      reproj<double>(a.cams + (size_t)a.obs_cam[o] * 12, a.pts + (size_t)a.obs_pt[o] * 3, a.obs_uv + (size_t)o * 2, a,
                     c, Jc, Jp);
      const double* ucam = uc + (a.obs_cam[o] - g.cam0) * 6;
      const double* upt = a.up + (size_t)a.obs_pt[o] * 3;
      double y[2];
      for (int r = 0; r < 2; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 6; ++k) acc += Jc[r * 6 + k] * ucam[k];
        for (int k = 0; k < 3; ++k) acc += Jp[r * 3 + k] * upt[k];
        y[r] = acc;
      }
      const double w = a.obs_w[o];
      const double yc = y[0] * c[0] + y[1] * c[1];
      const double cn2 = c[0] * c[0] + c[1] * c[1];
      // g_o = rho'(s) w^2 C^T c with rho' = 1 inside, delta / sqrt(s) outside
      // (sqrt(s) = w |c|): d/dw and d/ddelta of -u^T g_o
      const double hd = huber_radius(a, b);
      if (w * w * cn2 <= hd * hd) {
        gw = -2.0 * w * yc;
      } else {
        gw = -hd * yc / ::sqrt(cn2);
        gd = -w * yc / ::sqrt(cn2);
      }
    }
    if (a.g_w) a.g_w[o] = gw;
    if (a.g_delta) a.g_delta[o] = gd;
  }
  if (blockIdx.x == 0 && (int)threadIdx.x < g.nprior && a.g_logw_p) {
    const int q = g.prior0 + threadIdx.x;
    double gl = 0.0;
    if (ok) {
      double c[6], C[36];
      prior_cost<3, double>(a.cams + (size_t)a.prior_var[q] * 12, a.prior_meas + (size_t)q * 12, c, C);
      const double w = exp(a.prior_logw[q]);
      const double* u = uc + (a.prior_var[q] - g.cam0) * 6;
      double yr = 0.0;
      for (int r = 0; r < 6; ++r) {
        double acc = 0.0;
        for (int k = 0; k < 6; ++k) acc += C[r * 6 + k] * u[k];
        yr += w * acc * w * c[r];
      }
      gl = -2.0 * yr;
    }
    a.g_logw_p[q] = gl;
  }
}

// DLM backward (Section 4.3, Appendix G), per observation and prior: dS/dphi
// at cameras `cams` and points `pts`, times `scale`, stored or added;
// S = 1/2 sum rho(w^2 |c|^2) + 1/2 sum exp(2 l) |c_p|^2 gives
// dS/dw = rho'(s) w |c|^2, dS/dl = exp(2 l) |c_p|^2 and, per observation,
// dS/ddelta = sqrt(s) - delta outside the quadratic branch (0 inside);
// problems marked frozen get zero gradients
__global__ void __launch_bounds__(kBT) k_ba_param_grads(BAArgs a, const double* cams, const double* pts, double scale,
                                                        int accumulate) {
  const int b = blockIdx.y;
  const BADesc g = a.bd[b];
  const bool zero = a.frozen[b] != 0;
  const int t = blockIdx.x * kBT + threadIdx.x;
  if (t < g.nobs && (a.g_w || a.g_delta)) {
    const int o = g.obs0 + t;
    double v = 0.0, vd = 0.0;
    if (!zero) {
      double c[2], Jc[12], Jp[6];
      reproj<double>(cams + (size_t)a.obs_cam[o] * 12, pts + (size_t)a.obs_pt[o] * 3, a.obs_uv + (size_t)o * 2, a, c,
                     Jc, Jp);
      const double w = a.obs_w[o], cn2 = c[0] * c[0] + c[1] * c[1];
      double rho, drho;
      const double hd = huber_radius(a, b);
      huber(w * w * cn2, hd, rho, drho);
      v = drho * w * cn2;
      // 1/2 d rho / d delta = sqrt(s) - delta outside the quadratic branch
      if (w * w * cn2 > hd * hd) vd = w * ::sqrt(cn2) - hd;
    }
    if (a.g_w) a.g_w[o] = zero ? 0.0 : (accumulate ? a.g_w[o] : 0.0) + scale * v;
    if (a.g_delta) a.g_delta[o] = zero ? 0.0 : (accumulate ? a.g_delta[o] : 0.0) + scale * vd;
  }
  if (blockIdx.x == 0 && (int)threadIdx.x < g.nprior && a.g_logw_p) {
    const int q = g.prior0 + threadIdx.x;
    double v = 0.0;
    if (!zero) {
      double c[6], C[36];
      prior_cost<3, double>(cams + (size_t)a.prior_var[q] * 12, a.prior_meas + (size_t)q * 12, c, C);
      const double w2 = exp(2.0 * a.prior_logw[q]);
      for (int r = 0; r < 6; ++r) v += w2 * c[r] * c[r];
    }
    a.g_logw_p[q] = zero ? 0.0 : (accumulate ? a.g_logw_p[q] : 0.0) + scale * v;
  }
}

__global__ void k_ba_frozen_from_status(int* frozen, const int* status, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) frozen[b] = status[b] != DNLS_GRAPH_OK;
}

__global__ void k_ba_reset(int* frozen, int* status, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    frozen[b] = 0;
    status[b] = DNLS_GRAPH_OK;
  }
}

bool offsets_ok(const int32_t* off, int B, int* total) {
  if (!off || off[0] != 0) return false;
  for (int b = 0; b < B; ++b)
    if (off[b + 1] < off[b]) return false;
  *total = off[B];
  return true;
}

BAArgs base_args(dnls_plan p) {
  BAArgs a{};
  a.bd = p->d_bd;
  a.obs_cam = p->d_obs_cam;
  a.obs_pt = p->d_obs_pt;
  a.cam_obs_off = p->d_cam_obs_off;
  a.cam_obs = p->d_cam_obs;
  a.pt_obs_off = p->d_pt_obs_off;
  a.pt_obs = p->d_pt_obs;
  a.sblk = p->d_sblk;
  a.spair = p->d_spair;
  a.prior_var = p->d_prior_var;
  a.fx = p->intr[0];
  a.fy = p->intr[1];
  a.cx = p->intr[2];
  a.cy = p->intr[3];
  a.delta = p->huber;
  a.K = p->opt.iterations;
  a.npad_max = p->npad_max;
  a.lambda = p->opt.lambda;
  return a;
}

int max_of(const std::vector<BADesc>& v, int BADesc::*f) {
  int m = 1;
  for (const auto& x : v) m = std::max(m, x.*f);
  return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
dnls_status ba_plan_create(dnls_plan p, const dnls_problem* pr, const dnls_options* op) {
  const int B = pr->batch;
  int Vc = 0, Vp = 0, O = 0, P = 0;
  if (!offsets_ok(pr->pose_off, B, &Vc) || !offsets_ok(pr->point_off, B, &Vp) || !offsets_ok(pr->obs_off, B, &O) ||
      !offsets_ok(pr->prior_off, B, &P))
    return fail(DNLS_ERR_INVALID_ARG, "bundle adjustment needs pose/point/obs/prior offsets starting at 0, non-decreasing");
  if (pr->group != DNLS_SE3) return fail(DNLS_ERR_UNSUPPORTED, "bundle adjustment uses SE3 cameras");
  if (O > 0 && (!pr->obs_cam || !pr->obs_pt)) return fail(DNLS_ERR_INVALID_ARG, "obs_cam / obs_pt are NULL");
  if (P > 0 && !pr->prior_var) return fail(DNLS_ERR_INVALID_ARG, "prior_var is NULL");
  if (!(pr->huber_delta > 0.0)) return fail(DNLS_ERR_INVALID_ARG, "huber_delta must be > 0");
  if (pr->edge_off && pr->edge_off[B] != 0) return fail(DNLS_ERR_UNSUPPORTED, "relative-pose costs are not part of the SCHUR path");
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
  std::vector<int> obs_cam(O), obs_pt(O), prior_var(P);
  std::vector<std::vector<int>> cam_obs(Vc), pt_obs(Vp);
  std::vector<int4> sblk;
  std::vector<int2> spair;
  p->bd.resize(B);
  long long fac = 0;
  for (int b = 0; b < B; ++b) {
    BADesc& g = p->bd[b];
    g.cam0 = pr->pose_off[b];
    g.ncam = pr->pose_off[b + 1] - g.cam0;
    g.pt0 = pr->point_off[b];
    g.npt = pr->point_off[b + 1] - g.pt0;
    g.obs0 = pr->obs_off[b];
    g.nobs = pr->obs_off[b + 1] - g.obs0;
    g.prior0 = pr->prior_off[b];
    g.nprior = pr->prior_off[b + 1] - g.prior0;
    if (g.nprior > kBT) return fail(DNLS_ERR_UNSUPPORTED, "at most 256 camera priors per problem");
    g.n = 6 * g.ncam;
    g.npad = std::max(kNB, (g.n + kNB - 1) / kNB * kNB);
    p->flops_alg += double(g.n) * g.n * g.n / 3.0;
    p->flops_exec += double(g.npad) * g.npad * g.npad / 3.0;
    if (g.npad > kMaxDenseN) return fail(DNLS_ERR_UNSUPPORTED, "camera system larger than the dense limit");
    g.fac_off = fac;
    fac += (long long)(g.npad + 16) * g.npad + (long long)(g.npad / kNB) * kNB * kNB;
    fac = (fac + 31) / 32 * 32;
    p->npad_max = std::max(p->npad_max, g.npad);
    for (int o = g.obs0; o < g.obs0 + g.nobs; ++o) {
      const int c = pr->obs_cam[o], q = pr->obs_pt[o];
      if (c < g.cam0 || c >= g.cam0 + g.ncam || q < g.pt0 || q >= g.pt0 + g.npt)
        return fail(DNLS_ERR_INVALID_ARG, "observation " + std::to_string(o) + " refers outside its problem");
      obs_cam[o] = c;
      obs_pt[o] = q;
      cam_obs[c].push_back(o);
      pt_obs[q].push_back(o);
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      const int v = pr->prior_var[q];
      if (v < g.cam0 || v >= g.cam0 + g.ncam)
        return fail(DNLS_ERR_INVALID_ARG, "prior " + std::to_string(q) + " refers outside its problem");
      prior_var[q] = v;
    }
    // Schur contributions F_oa E_ob^T of every point to camera pair (cam oa >= cam ob)
    std::map<std::pair<int, int>, std::vector<int2>> blocks;
    for (int q = g.pt0; q < g.pt0 + g.npt; ++q)
      for (int oa : pt_obs[q])
        for (int ob : pt_obs[q]) {
          const int ca = obs_cam[oa] - g.cam0, cb = obs_cam[ob] - g.cam0;
          if (ca >= cb) blocks[{ca, cb}].push_back(int2{oa, ob});
        }
    g.blk0 = (int)sblk.size();
    for (int ca = 0; ca < g.ncam; ++ca)
      for (int cb = 0; cb <= ca; ++cb) {
        auto it = blocks.find({ca, cb});
        const int start = (int)spair.size();
        int cnt = 0;
        if (it != blocks.end()) {
          for (const int2& x : it->second) spair.push_back(x);
          cnt = (int)it->second.size();
        }
        sblk.push_back(int4{ca, cb, start, cnt});
      }
    g.nblk = (int)sblk.size() - g.blk0;
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
  const int nx = (max_of(p->bd, &BADesc::nobs) + kBT - 1) / kBT;
  p->nlin_blocks = nx;
  dnls_status st;
  if ((st = upload(p, &p->d_bd, p->bd)) != DNLS_OK || (st = upload(p, &p->d_obs_cam, obs_cam)) != DNLS_OK ||
      (st = upload(p, &p->d_obs_pt, obs_pt)) != DNLS_OK || (st = upload(p, &p->d_prior_var, prior_var)) != DNLS_OK ||
      (st = upload(p, &p->d_cam_obs_off, cam_off)) != DNLS_OK || (st = upload(p, &p->d_cam_obs, cam_list)) != DNLS_OK ||
      (st = upload(p, &p->d_pt_obs_off, pt_off)) != DNLS_OK || (st = upload(p, &p->d_pt_obs, pt_list)) != DNLS_OK ||
      (st = upload(p, &p->d_sblk, sblk)) != DNLS_OK || (st = upload(p, &p->d_spair, spair)) != DNLS_OK)
    return st;
  // solve workspace: obs records, prior records, objective partials, camera steps, frozen flags
  size_t off = 0;
  // observation records: float64, or (mixed) float records followed by the
  // float64 gradient parts of each observation
  p->ba_off[0] = off;
  off += align256(std::max((size_t)O * kObsRec * sizeof(double),
                           align256((size_t)O * kObsRec * sizeof(float)) + (size_t)O * 9 * sizeof(double)));
  p->ba_off[1] = off; off += align256((size_t)P * kPriorRec * sizeof(double));
  p->ba_off[2] = off; off += align256((size_t)B * nx * sizeof(double));
  p->ba_off[3] = off; off += align256((size_t)B * p->npad_max * sizeof(double));
  p->ba_off[4] = off; off += align256((size_t)B * sizeof(int));
  p->ba_off[5] = off; off += align256((size_t)B * sizeof(double));
  p->ba_off[6] = off; off += align256((size_t)Vp * 3 * sizeof(double));   // u_p (backward)
  if (op->flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG)) {
    p->ba_off[7] = off; off += align256((size_t)B * sizeof(double));       // lambda per problem
    p->ba_off[8] = off; off += align256((size_t)B * sizeof(int));          // rejected
  }
  if (op->flags & DNLS_FLAG_DOGLEG) {
    p->ba_off[12] = off; off += align256((size_t)Vp * 3 * sizeof(double));       // point step
    p->ba_off[13] = off; off += align256((size_t)p->V * 6 * sizeof(double) * 2);  // camera gradient, (H + lambda I) x
    p->ba_off[14] = off; off += align256(((size_t)O * 2 + (size_t)Vp * 3) * sizeof(double));  // J x, points of (H + lambda I) x
    p->ba_off[15] = off; off += align256((size_t)B * 4 * sizeof(double));        // dogleg state
  }
  p->ba_off[9] = off; off += align256((size_t)p->V * 12 * sizeof(double));  // camera backup / DLM theta_direct
  p->ba_off[10] = off; off += align256((size_t)Vp * 3 * sizeof(double));    // point backup / DLM theta_direct
  p->ba_off[11] = off; off += align256((size_t)B * sizeof(int));            // DLM: status of its factorisations
  p->ba_off[16] = off; off += align256((size_t)O * sizeof(double));         // per-observation radius gradients
  p->ws_bytes = off;
  p->bwd_bytes = off;
  // factor cache: Schur factors, then E, F, C^-1, g_p of the final linearisation
  size_t fb = align256((size_t)fac * sizeof(double));
  p->ba_fac_off[0] = fb; fb += align256((size_t)O * 18 * sizeof(double));
  p->ba_fac_off[1] = fb; fb += align256((size_t)O * 18 * sizeof(double));
  p->ba_fac_off[2] = fb; fb += align256((size_t)Vp * 9 * sizeof(double));
  p->ba_fac_off[3] = fb; fb += align256((size_t)Vp * 3 * sizeof(double));
  p->fac_bytes = fb;
  // DNLS_FLAG_PAIR (not with HIP-graph capture, whose replays would reuse the
  // counter origin): six workgroups per problem share the camera-system
  // factorisation when they fit on the device at once
  p->ba_nway = 1;
  p->pair_spin = pair_spin_limit();
  if ((op->flags & DNLS_FLAG_PAIR) && !(op->flags & DNLS_FLAG_GRAPH)) {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    const size_t lds = (size_t)p->npad_max * sizeof(double);
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) == hipSuccess && coop &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_ba_factor<true>), kNT,
                                                     lds) == hipSuccess &&
        (long long)per_cu * cus >= (long long)kBaNway * B) {
      const size_t bytes = (size_t)B * kBaCtr * sizeof(unsigned long long);
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&p->d_pair), bytes));
      p->allocs.push_back(p->d_pair);
      HIP_TRY(hipMemset(p->d_pair, 0, bytes));
      p->ba_nway = kBaNway;
    }
  }
  return DNLS_OK;
}

static void bind_ws(dnls_plan p, BAArgs& a, void* ws, void* factor) {
  char* w = static_cast<char*>(ws);
  char* f = static_cast<char*>(factor);
  a.orec = w + p->ba_off[0];
  a.gob = reinterpret_cast<double*>(w + p->ba_off[0] + align256((size_t)p->O * kObsRec * sizeof(float)));
  a.prec = reinterpret_cast<double*>(w + p->ba_off[1]);
  a.partial = reinterpret_cast<double*>(w + p->ba_off[2]);
  a.dc = reinterpret_cast<double*>(w + p->ba_off[3]);
  a.uc = a.dc;
  a.frozen = reinterpret_cast<int*>(w + p->ba_off[4]);
  a.lastobj = reinterpret_cast<double*>(w + p->ba_off[5]);
  a.up = reinterpret_cast<double*>(w + p->ba_off[6]);
  a.factor = reinterpret_cast<double*>(f);
  a.E = reinterpret_cast<double*>(f + p->ba_fac_off[0]);
  a.F = reinterpret_cast<double*>(f + p->ba_fac_off[1]);
  a.Cinv = reinterpret_cast<double*>(f + p->ba_fac_off[2]);
  a.gp = reinterpret_cast<double*>(f + p->ba_fac_off[3]);
  a.nx_lin = p->nlin_blocks;
  a.bak_c = reinterpret_cast<double*>(w + p->ba_off[9]);
  a.bak_p = reinterpret_cast<double*>(w + p->ba_off[10]);
  if (p->opt.flags & DNLS_FLAG_ADAPTIVE_LM) a.lam_g = reinterpret_cast<double*>(w + p->ba_off[7]);
  if (p->opt.flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG)) a.rej = reinterpret_cast<int*>(w + p->ba_off[8]);
  if (p->opt.flags & DNLS_FLAG_DOGLEG) {
    a.dp = reinterpret_cast<double*>(w + p->ba_off[12]);
    a.gc = reinterpret_cast<double*>(w + p->ba_off[13]);
    a.hc = a.gc + (size_t)p->V * 6;
    a.yo = reinterpret_cast<double*>(w + p->ba_off[14]);
    a.hp = a.yo + (size_t)p->O * 2;
    a.dl = reinterpret_cast<double*>(w + p->ba_off[15]);
    a.radius0 = p->opt.trust_radius;
  }
}

// factorisation of the assembled camera systems (and, unless final_lin, the
// camera step): six co-resident workgroups per problem when the plan holds
// their counters, else one
static dnls_status launch_ba_factor(dnls_plan p, const BAArgs& a, bool final_lin, hipStream_t st) {
  const size_t lds = (size_t)p->npad_max * sizeof(double);
  if (p->ba_nway > 1) {
    BAArgs am = a;
    am.pair_ctr = p->d_pair;
    am.pair_base = (++p->pair_epoch) << 20;
    am.pair_spin = p->pair_spin;
    am.nway = p->ba_nway;
    int fl = final_lin ? 1 : 0;
    void* args[] = {&am, &fl};
    HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_ba_factor<true>), dim3(p->ba_nway * p->B),
                                       dim3(kNT), args, (unsigned)lds, st));
  } else {
    hipLaunchKernelGGL(k_ba_factor<false>, dim3(p->B), dim3(kNT), lds, st, a, final_lin ? 1 : 0);
  }
  return DNLS_OK;
}

dnls_status ba_solve(dnls_plan p, const dnls_solve_args* s, hipStream_t st) {
  if (!s->points || (p->O > 0 && (!s->obs_uv || !s->obs_w)) || (p->P > 0 && (!s->prior_meas || !s->prior_logw)))
    return fail(DNLS_ERR_INVALID_ARG, "points, obs_uv, obs_w and prior data are required");
  BAArgs a = base_args(p);
  bind_ws(p, a, s->workspace, s->factor);
  a.cams = s->poses;
  a.pts = s->points;
  a.delta_b = s->huber_delta;
  a.obs_uv = s->obs_uv;
  a.obs_w = s->obs_w;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.objective = s->objective;
  a.status = s->status;
  const int B = p->B;
  const dim3 blk(kBT);
  const dim3 g_lin(p->nlin_blocks, B);
  const dim3 g_pt((max_of(p->bd, &BADesc::npt) + kBT - 1) / kBT, B);
  const dim3 g_blk((max_of(p->bd, &BADesc::nblk) + kSchurWaves - 1) / kSchurWaves, B);
  const int nupd = std::max(max_of(p->bd, &BADesc::npt), max_of(p->bd, &BADesc::ncam));
  const dim3 g_upd((nupd + kBT - 1) / kBT, B);
  const size_t lds = (size_t)p->npad_max * sizeof(double);
  const bool mixed = p->opt.precision == DNLS_PREC_MIXED;
  const bool adaptive = (p->opt.flags & DNLS_FLAG_ADAPTIVE_LM) != 0;
  const bool dogleg = (p->opt.flags & DNLS_FLAG_DOGLEG) != 0;
  double* lam_g = a.lam_g;
  hipLaunchKernelGGL(k_ba_reset, dim3((B + 255) / 256), dim3(256), 0, st, a.frozen, a.status, B);
  if (adaptive) hipLaunchKernelGGL(k_ba_lam_init, dim3((B + 255) / 256), dim3(256), 0, st, a, B);
  if (dogleg) hipLaunchKernelGGL(k_ba_dl_init, dim3((B + 255) / 256), dim3(256), 0, st, a, B);
  const int nobs = std::max(max_of(p->bd, &BADesc::nobs), 1);
  const dim3 g_obs((nobs + kBT - 1) / kBT, B);
  for (int it = 0; it <= p->opt.iterations; ++it) {
    const bool final_lin = it == p->opt.iterations;
    const double lam = final_lin ? 0.0 : p->opt.lambda;
    a.it = it;
    a.lam_g = (adaptive && !final_lin) ? lam_g : nullptr;   // the final linearisation is undamped
    // the final (cached) linearisation is float64 in both precisions, and so
    // is every step of the dogleg (its model uses the records) and of adaptive
    // damping: the float curvature of the mixed steps moves an iterate that
    // is still far from convergence (the trajectory of refused and damped
    // steps) by more than 1e-5, and without float64 refinement on this path
    // the accept / reject decisions would follow that trajectory
    if (mixed && !final_lin && !dogleg && !adaptive) {
      hipLaunchKernelGGL(k_ba_lin<float>, g_lin, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_point<float>, g_pt, blk, 0, st, a, lam);
      hipLaunchKernelGGL(k_ba_obs_ef<float>, g_obs, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_schur<float>, g_blk, blk, 0, st, a, lam);
    } else {
      hipLaunchKernelGGL(k_ba_lin<double>, g_lin, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_point<double>, g_pt, blk, 0, st, a, lam);
      hipLaunchKernelGGL(k_ba_obs_ef<double>, g_obs, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_schur<double>, g_blk, blk, 0, st, a, lam);
    }
    const dnls_status fs = launch_ba_factor(p, a, final_lin, st);
    if (fs != DNLS_OK) return fs;
    if (!final_lin && dogleg) {
      hipLaunchKernelGGL(k_ba_dl_gn, g_upd, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_dl_jx, g_obs, blk, 0, st, a, (const double*)a.gc, 0, (const double*)a.gp);
      hipLaunchKernelGGL(k_ba_dl_hx, g_upd, blk, 0, st, a, (const double*)a.gc, 0, (const double*)a.gp, lam);
      hipLaunchKernelGGL(k_ba_dogleg, dim3(B), blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_dl_jx, g_obs, blk, 0, st, a, (const double*)a.dc, 1, (const double*)a.dp);
      hipLaunchKernelGGL(k_ba_dl_hx, g_upd, blk, 0, st, a, (const double*)a.dc, 1, (const double*)a.dp, lam);
      hipLaunchKernelGGL(k_ba_dl_pred, dim3(B), blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_backup, g_upd, blk, 0, st, a, 0);
      hipLaunchKernelGGL(k_ba_dl_apply, g_upd, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_lin<double>, g_lin, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_dl_decide, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
      hipLaunchKernelGGL(k_ba_backup, g_upd, blk, 0, st, a, 1);
    } else if (!final_lin && adaptive) {
      hipLaunchKernelGGL(k_ba_backup, g_upd, blk, 0, st, a, 0);
      hipLaunchKernelGGL(k_ba_update, g_upd, blk, 0, st, a);
      // the trial objective (float64 records at the trial point are rewritten
      // by the next step's linearisation anyway)
      hipLaunchKernelGGL(k_ba_lin<double>, g_lin, blk, 0, st, a);
      hipLaunchKernelGGL(k_ba_decide, dim3((B + 63) / 64), dim3(64), 0, st, a, B);
      hipLaunchKernelGGL(k_ba_backup, g_upd, blk, 0, st, a, 1);
    } else if (!final_lin) {
      hipLaunchKernelGGL(k_ba_update, g_upd, blk, 0, st, a);
    }
  }
  HIP_TRY(hipGetLastError());
  return DNLS_OK;
}

// Gradient of each problem's Huber radius: the sum of its observations'
// per-radius gradients (every observation of problem b uses the radius
// delta_b), one workgroup per problem, strided partial sums then a fixed
// tree in LDS (deterministic order).
__global__ void __launch_bounds__(kBT) k_ba_delta_sum(BAArgs a, const double* __restrict__ g_obs,
                                                      double* __restrict__ out) {
  __shared__ double red[kBT];
  const int b = blockIdx.x;
  const BADesc g = a.bd[b];
  double acc = 0.0;
  for (int t = threadIdx.x; t < g.nobs; t += kBT) acc += g_obs[g.obs0 + t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = red[0];
}

dnls_status ba_backward(dnls_plan p, const dnls_backward_args* s, hipStream_t st) {
  if (!s->points || (p->O > 0 && (!s->obs_uv || !s->obs_w)))
    return fail(DNLS_ERR_INVALID_ARG, "points, obs_uv and obs_w are required");
  BAArgs a = base_args(p);
  bind_ws(p, a, s->workspace, const_cast<void*>(s->factor));
  a.lam_g = nullptr;   // the backward's systems take the damping passed to the kernels
  a.cams = const_cast<double*>(s->poses);
  a.pts = const_cast<double*>(s->points);
  a.delta_b = s->huber_delta;
  a.obs_uv = s->obs_uv;
  a.obs_w = s->obs_w;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.status = const_cast<int*>(s->status);
  a.seed_c = s->seed_pose;
  a.seed_p = s->seed_point;
  a.g_w = s->grad_obs_w;
  a.g_logw_p = s->grad_prior_logw;
  a.g_delta = s->grad_obs_delta;
  // the per-problem radius gradient needs the per-observation ones: in the
  // workspace when the caller does not ask for them
  if (s->grad_huber_delta && !a.g_delta)
    a.g_delta = reinterpret_cast<double*>(static_cast<char*>(s->workspace) + p->ba_off[16]);
  a.adjoint_out = s->adjoint;
  const int B = p->B;
  const dim3 blk(kBT);
  const dim3 g_pt((max_of(p->bd, &BADesc::npt) + kBT - 1) / kBT, B);
  const int nobs = std::max(max_of(p->bd, &BADesc::nobs), 1);
  const dim3 g_obs((nobs + kBT - 1) / kBT, B);
  const size_t lds = (size_t)p->npad_max * sizeof(double);
  if (s->mode == DNLS_BACKWARD_DLM) {
    // one Gauss-Newton step from theta_K on S + ||eps theta - v/2||^2:
    // (H* + 2 eps^2 I) delta = -g* + eps v (cameras and points), by the solve's
    // Schur kernels with the right-hand side g* - eps v (so they produce
    // -delta and their update lands on theta_direct = theta_K (+) delta), in
    // copies of the cameras and points; the factor cache is then rebuilt at
    // theta_K by the same kernels as the solve's final linearisation
    const double eps = s->dlm_eps;
    const dim3 g_lin(p->nlin_blocks, B);
    const dim3 g_blk((max_of(p->bd, &BADesc::nblk) + kSchurWaves - 1) / kSchurWaves, B);
    const int nupd = std::max(max_of(p->bd, &BADesc::npt), max_of(p->bd, &BADesc::ncam));
    const dim3 g_upd((nupd + kBT - 1) / kBT, B);
    char* w = static_cast<char*>(s->workspace);
    a.status = reinterpret_cast<int*>(w + p->ba_off[11]);   // the caller's status stays untouched
    a.objective = a.lastobj;                                   // objective slot of the factor kernel
    a.K = 0;
    a.it = 0;
    hipLaunchKernelGGL(k_ba_frozen_from_status, dim3((B + 255) / 256), dim3(256), 0, st, a.frozen, s->status, B);
    hipLaunchKernelGGL(k_ba_param_grads, g_obs, blk, 0, st, a, (const double*)a.cams, (const double*)a.pts, 1.0 / eps,
                       0);
    BAArgs ad = a;
    ad.dlm_eps = eps;
    hipLaunchKernelGGL(k_ba_lin<double>, g_lin, blk, 0, st, ad);
    hipLaunchKernelGGL(k_ba_point<double>, g_pt, blk, 0, st, ad, 2.0 * eps * eps);
    hipLaunchKernelGGL(k_ba_obs_ef<double>, g_obs, blk, 0, st, ad);
    hipLaunchKernelGGL(k_ba_schur<double>, g_blk, blk, 0, st, ad, 2.0 * eps * eps);
    dnls_status fs = launch_ba_factor(p, ad, false, st);
    if (fs != DNLS_OK) return fs;
    HIP_TRY(hipMemcpyAsync(a.bak_c, a.cams, (size_t)p->V * 12 * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(a.bak_p, a.pts, (size_t)p->Vp * 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
    ad.cams = a.bak_c;
    ad.pts = a.bak_p;
    hipLaunchKernelGGL(k_ba_update, g_upd, blk, 0, st, ad);
    hipLaunchKernelGGL(k_ba_param_grads, g_obs, blk, 0, st, ad, (const double*)a.bak_c, (const double*)a.bak_p,
                       -1.0 / eps, 1);
    hipLaunchKernelGGL(k_ba_frozen_from_status, dim3((B + 255) / 256), dim3(256), 0, st, a.frozen, s->status, B);
    hipLaunchKernelGGL(k_ba_lin<double>, g_lin, blk, 0, st, a);
    hipLaunchKernelGGL(k_ba_point<double>, g_pt, blk, 0, st, a, 0.0);
    hipLaunchKernelGGL(k_ba_obs_ef<double>, g_obs, blk, 0, st, a);
    hipLaunchKernelGGL(k_ba_schur<double>, g_blk, blk, 0, st, a, 0.0);
    fs = launch_ba_factor(p, a, true, st);
    if (fs != DNLS_OK) return fs;
    if (s->grad_huber_delta)
      hipLaunchKernelGGL(k_ba_delta_sum, dim3(B), blk, 0, st, a, (const double*)a.g_delta, s->grad_huber_delta);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  hipLaunchKernelGGL(k_ba_bwd_cam, dim3(B), dim3(kNT), lds, st, a);
  hipLaunchKernelGGL(k_ba_bwd_pt, g_pt, blk, 0, st, a);
  hipLaunchKernelGGL(k_ba_bwd_obs, g_obs, blk, 0, st, a);
  if (s->grad_huber_delta)
    hipLaunchKernelGGL(k_ba_delta_sum, dim3(B), blk, 0, st, a, (const double*)a.g_delta, s->grad_huber_delta);
  HIP_TRY(hipGetLastError());
  return DNLS_OK;
}

}  // namespace dnls
