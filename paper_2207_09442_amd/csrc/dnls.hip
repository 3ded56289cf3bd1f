// C-ABI library of the batched DNLS inner step (dense pose-graph path).
//
// One workgroup owns one graph for the whole solve: it linearises the costs,
// gathers the normal equations H = sum J^T J, g = sum J^T r into the
// caller's factor buffer (Section 2 "Solving NLS"), damps the diagonal
// (Levenberg-Marquardt), factors with the MFMA Cholesky of dense.hpp, solves,
// retracts, and repeats K times before the undamped final linearisation whose
// factor is kept for the implicit backward (Section 4.2, Section 4.3,
// Proposition 1).  The normal equations are assembled by gathering, for every
// Hessian block, the Jacobian products of the costs incident to it (index
// lists built once by the plan), so no atomics are needed and every sum has a
// fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "costs.hpp"
#include "dense.hpp"
#include "plan.hpp"
#include "pose_costs.hpp"

using namespace dnls;

thread_local std::string dnls::g_err;

namespace {

// ---------------------------------------------------------------------------
// kernel arguments
// ---------------------------------------------------------------------------
struct DenseArgs {
  const GraphDesc* gd;
  const int* order;
  const int* edge_ij;
  const int* prior_var;
  const int* inc_off;
  const int* inc_slot;
  const int4* od_blk;
  const int* od_slot;
  double* poses;
  const double* edge_meas;
  const double* edge_logw;
  const double* edge_tau;
  const double* prior_meas;
  const double* prior_logw;
  const double* edge_logc;   // Welsch log-radii or null
  double* objective;
  int* status;
  double* factor;
  double* ws64;      // per-cost records, float64
  float* ws32;       // per-cost records, float32 (mixed)
  double* ycost;     // per-cost J delta (d values)
  double* hbuf;      // assembled systems (per graph at GraphDesc::h_off)
  double* pose_bak;  // adaptive damping: theta_t while the trial step is evaluated; DLM: theta_direct
  double* dlm_winv;  // DLM backward: inverses of the diagonal panels of the factor of H* + 2 eps^2 I
  double* hvp;       // exact / unrolled backward: [cost][2][d] per-cost pose terms
  double* traj;      // DNLS_FLAG_KEEP_ITERATES: theta_t, t < K, [K][V][sz] in the factor cache
  unsigned long long* pair_ctr;   // DNLS_FLAG_PAIR: 8 event counters per graph slot
  unsigned long long pair_base;   // this launch's counter origin
  int pair_spin;                  // poll limit of a pair wait
  int adaptive;      // DNLS_FLAG_ADAPTIVE_LM
  int dogleg;        // DNLS_FLAG_DOGLEG
  double radius0;    // dogleg: initial trust radius
  const double* seed;
  double* g_logw_e;
  double* g_tau;
  double* g_logw_p;
  double* g_logc;
  double* adjoint_out;
  int E;             // total edges (prior records follow the edge records)
  int V;             // total poses
  int K;
  int refine;
  int refine_from;   // mixed: steps refine_from <= it < refine_until run the refinement sweeps
  int refine_until;
  int adj_refine;    // backward: the float64 refinement step of the adjoint (float64 plans)
  double lambda;
};

// block-wide sum of one double per thread (all threads call)
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kNW; ++w) t += red[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ PoseCostData cost_data(const DenseArgs& a) {
  return PoseCostData{a.edge_ij, a.prior_var, a.poses, a.edge_meas, a.edge_logw,
                      a.edge_tau, a.prior_meas, a.prior_logw, a.E, a.edge_logc};
}

// Linearise every cost of graph g in precision S into `rec`; returns the
// objective 1/2 sum ||w c||^2 (block-reduced).
template <int G, class S>
__device__ double linearize_graph(const DenseArgs& a, const GraphDesc& g, S* rec, double* red) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const PoseCostData cd = cost_data(a);
  double sacc = 0.0;
  const int ncost = g.nedge + g.nprior;
  for (int k = threadIdx.x; k < ncost; k += kNT) {
    const int rk = (k < g.nedge) ? g.edge0 + k : a.E + g.prior0 + (k - g.nedge);
    sacc += linearize_cost<G, S>(cd, rk, rec + (size_t)rk * RN);
  }
  return block_sum(sacc, red);
}

// objective 1/2 sum w^2 ||c||^2 of the graph at the current poses, float64
template <int G>
__device__ double objective_graph(const DenseArgs& a, const GraphDesc& g, double* red) {
  const PoseCostData cd = cost_data(a);
  double sacc = 0.0;
  const int ncost = g.nedge + g.nprior;
  for (int k = threadIdx.x; k < ncost; k += kNT) {
    const int rk = (k < g.nedge) ? g.edge0 + k : a.E + g.prior0 + (k - g.nedge);
    sacc += cost_objective<G>(cd, rk);
  }
  return block_sum(sacc, red);
}

// Once per solve: zero every row of H up to the end of its 64-wide diagonal
// block (the part the factorisation reads) and the right-hand-side row with
// the padding rows after it, and put
// 1 on the diagonal of the padding.  The assembly then rewrites only the
// structurally non-zero blocks, so the zeros persist across iterations.
__device__ void init_H(const GraphDesc& g, double* A) {
  const int npad = g.npad;
  const int q4 = npad >> 2;
  for (int u = threadIdx.x; u < (npad + 16) * q4; u += kNT) {
    const int r = u / q4, c = 4 * (u - r * q4);
    if (r >= npad || c < kNB * (r / kNB + 1))
      *reinterpret_cast<d4v*>(A + (size_t)r * npad + c) = d4v{0.0, 0.0, 0.0, 0.0};
  }
  __syncthreads();
  for (int r = g.n + threadIdx.x; r < npad; r += kNT) A[(size_t)r * npad + r] = 1.0;
  __syncthreads();
}

// H = sum J^T J (+ lambda I) on the non-zero 6x6 / 3x3 blocks of the lower
// triangle (H prepared by init_H), one thread per block, products
// accumulated in precision S
template <int G, class S>
__device__ void assemble_H(const DenseArgs& a, const GraphDesc& g, const S* rec, double* A, double lambda) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const int npad = g.npad;
  for (int u = threadIdx.x; u < g.npose + g.nod; u += kNT) {
    S h[d * d];
#pragma unroll
    for (int q = 0; q < d * d; ++q) h[q] = S(0);
    int rb, cb;
    if (u < g.npose) {
      rb = cb = u;
      const int gp = g.pose0 + u;
      for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
        const int slot = a.inc_slot[s];
        const S* J = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
        S j[d * d];
#pragma unroll
        for (int q = 0; q < d * d; ++q) j[q] = J[q];
#pragma unroll
        for (int k = 0; k < d; ++k)
#pragma unroll
          for (int r = 0; r < d; ++r)
#pragma unroll
            for (int c = 0; c < d; ++c) h[r * d + c] += j[k * d + r] * j[k * d + c];
      }
    } else {
      const int4 blk = a.od_blk[g.od0 + (u - g.npose)];
      rb = blk.x;
      cb = blk.y;
      for (int s = blk.z; s < blk.z + blk.w; ++s) {
        const int slot = a.od_slot[s];
        const S* Jr = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
        const S* Jc = rec + (size_t)(slot >> 1) * RN + ((slot & 1) ^ 1) * d * d;
        S jr[d * d], jc[d * d];
#pragma unroll
        for (int q = 0; q < d * d; ++q) {
          jr[q] = Jr[q];
          jc[q] = Jc[q];
        }
#pragma unroll
        for (int k = 0; k < d; ++k)
#pragma unroll
          for (int r = 0; r < d; ++r)
#pragma unroll
            for (int c = 0; c < d; ++c) h[r * d + c] += jr[k * d + r] * jc[k * d + c];
      }
    }
#pragma unroll
    for (int r = 0; r < d; ++r)
#pragma unroll
      for (int c = 0; c < d; ++c)
        A[(size_t)(rb * d + r) * npad + cb * d + c] = double(h[r * d + c]) + ((rb == cb && r == c) ? lambda : 0.0);
  }
  __syncthreads();
}

// b[p*d + r] = sum over incident costs of J^T (w c), zero on the padding;
// with aug != nullptr also written to the right-hand-side row of the matrix.
template <int G, class S>
__device__ void assemble_g(const DenseArgs& a, const GraphDesc& g, const S* rec, double* b, double* aug) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  for (int p = threadIdx.x; p < g.npose; p += kNT) {
    const int gp = g.pose0 + p;
    S h[d];
#pragma unroll
    for (int r = 0; r < d; ++r) h[r] = S(0);
    for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
      const int slot = a.inc_slot[s];
      const S* J = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
      const S* res = rec + (size_t)(slot >> 1) * RN + 2 * d * d;
      S j[d * d], rr[d];
#pragma unroll
      for (int q = 0; q < d * d; ++q) j[q] = J[q];
#pragma unroll
      for (int q = 0; q < d; ++q) rr[q] = res[q];
#pragma unroll
      for (int k = 0; k < d; ++k)
#pragma unroll
        for (int r = 0; r < d; ++r) h[r] += j[k * d + r] * rr[k];
    }
#pragma unroll
    for (int r = 0; r < d; ++r) {
      b[p * d + r] = double(h[r]);
      if (aug) aug[p * d + r] = double(h[r]);
    }
  }
  for (int u = g.n + threadIdx.x; u < g.npad; u += kNT) b[u] = 0.0;
  __syncthreads();
}

// y = (H + lambda I) x with H = sum J^T J applied matrix-free in float64.
// Each cost's thread reads its record once, row by row, and forms both pose
// terms J_i^T (J x) and J_j^T (J x) into LDS (the staging buffers of s, free
// outside the factorisation); each unknown then sums the terms of its
// incident costs, four incidence entries per round of loads.  Costs go in
// chunks of what the buffers hold.
template <int G>
__device__ void matvec_H(const DenseArgs& a, const GraphDesc& g, const double* rec, const double* x,
                         double* y, double lambda, DenseLds& s) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  constexpr int kCh = (2 * kNB * kSP) / (2 * d);   // costs per chunk of zs
  double* zs = &s.stage[0][0];
  const int ncost = g.nedge + g.nprior;
  for (int c0 = 0; c0 == 0 || c0 < ncost; c0 += kCh) {
    const int c1 = min(ncost, c0 + kCh);
    for (int k = c0 + threadIdx.x; k < c1; k += kNT) {
      int cost, pi, pj;
      if (k < g.nedge) {
        cost = g.edge0 + k;
        pi = a.edge_ij[2 * cost] - g.pose0;
        pj = a.edge_ij[2 * cost + 1] - g.pose0;
      } else {
        const int p = g.prior0 + (k - g.nedge);
        cost = a.E + p;
        pi = -1;
        pj = a.prior_var[p] - g.pose0;
      }
      const double* J = rec + (size_t)cost * RN;
      double xi[d], xj[d], zi[d], zj[d];
#pragma unroll
      for (int q = 0; q < d; ++q) {
        xi[q] = pi >= 0 ? x[pi * d + q] : 0.0;
        xj[q] = x[pj * d + q];
        zi[q] = 0.0;
        zj[q] = 0.0;
      }
#pragma unroll
      for (int r = 0; r < d; ++r) {
        double ji[d], jj[d];
#pragma unroll
        for (int q = 0; q < d; ++q) {
          ji[q] = pi >= 0 ? J[r * d + q] : 0.0;
          jj[q] = J[d * d + r * d + q];
        }
        double yr = 0.0;
#pragma unroll
        for (int q = 0; q < d; ++q) yr += ji[q] * xi[q] + jj[q] * xj[q];
#pragma unroll
        for (int q = 0; q < d; ++q) {
          zi[q] += ji[q] * yr;
          zj[q] += jj[q] * yr;
        }
      }
      double* z = zs + (size_t)(k - c0) * 2 * d;
#pragma unroll
      for (int q = 0; q < d; ++q) {
        z[q] = zi[q];
        z[d + q] = zj[q];
      }
    }
    __syncthreads();
    for (int u = threadIdx.x; u < g.npad; u += kNT) {
      double v = c0 > 0 ? y[u] : (u < g.n ? lambda * x[u] : 0.0);
      if (u < g.n) {
        const int p = u / d, r = u % d, gp = g.pose0 + p;
        const int s0 = a.inc_off[gp], s1 = a.inc_off[gp + 1];
        for (int e = s0; e < s1; e += 4) {
          int sl[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) sl[j] = e + j < s1 ? a.inc_slot[e + j] : -1;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (sl[j] < 0) continue;
            const int rid = sl[j] >> 1;   // record: edge, or a.E + prior
            const int k = rid < a.E ? rid - g.edge0 : g.nedge + (rid - a.E - g.prior0);
            if (k >= c0 && k < c1) v += zs[(size_t)(k - c0) * 2 * d + (sl[j] & 1) * d + r];
          }
        }
      }
      y[u] = v;
    }
    __syncthreads();
  }
}

constexpr double kLambdaMin = 1e-7, kLambdaMax = 1e7;   // adaptive damping range
constexpr double kRadiusMax = 1e4;                         // dogleg: largest trust radius
constexpr int kMaxExactSweeps = 64;                        // exact-Hessian backward: refinement sweeps

struct KernelLds {
  DenseLds dl;
  double red[kNW];
  int flag;
};

// ---------------------------------------------------------------------------
// forward: K steps + final linearisation, one workgroup per graph
// ---------------------------------------------------------------------------
// GENERAL = false is the plain fixed/adaptive-damping solve with plain least
// squares; GENERAL = true adds the run-time options that would otherwise push
// the plain solve's registers into scratch: the dogleg (a.dogleg) and Welsch
// edges (a.edge_logc).
// PAIR: two co-resident workgroups per graph (blocks b and b + B of a
// cooperative launch): the follower only takes its share of every
// factorisation (chol_dense_pair), the leader runs everything else.
template <int G, bool MIXED, bool GENERAL, bool PAIR = false>
__global__ void __launch_bounds__(kNT) k_dense_solve(DenseArgs a) {
  if constexpr (!GENERAL) {
    a.edge_logc = nullptr;
    a.dogleg = 0;
  }
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  extern __shared__ double dyn[];
  __shared__ KernelLds L;
  const int nslot = PAIR ? gridDim.x / 2 : gridDim.x;
  const int slot = blockIdx.x % nslot;
  const int b = a.order[slot];
  const GraphDesc g = a.gd[b];
  double* A = a.factor + g.fac_off;
  double* winv = A + (size_t)(g.npad + 16) * g.npad;
  double* H = a.hbuf + g.h_off;    // assembled system (workspace), read by the factorisation
  PairSync ps{};
  PairLa pl{};
  bool timed_out = false;
  if constexpr (PAIR) {
    // counters of the slot: system assembled, leader stopped, then the
    // factorisation's diagonal / look-ahead / done / failed events
    unsigned long long* c = a.pair_ctr + (size_t)slot * 8;
    ps = PairSync{c, c + 1, nullptr, nullptr, a.pair_base, (int)(blockIdx.x / nslot), 2, a.pair_spin};
    pl = PairLa{c + 2, c + 3, c + 4, c + 5, a.pair_base, ps.role, a.pair_spin};
    if (ps.role == 1) {
      for (int f = 0; f <= a.K; ++f) {
        if (!pair_wait(ps.lead_h, ps.base + f + 1, ps.lead_stop, ps.spin, L.dl, ps.base + 1)) return;
        bool bail = false;
        chol_dense_pair_la(A, H, g.npad, winv, L.dl, pl, f, bail, g.n);
        if (bail) return;
      }
      return;
    }
  }
  // factorisation number f of this launch (the step index; K for the final one)
  auto factor = [&](int f) -> bool {
    if constexpr (PAIR) {
      pair_post(ps.lead_h, ps.base + f + 1);
      bool bail = false;
      const bool ok = chol_dense_pair_la(A, H, g.npad, winv, L.dl, pl, f, bail, g.n);
      timed_out = timed_out || bail;
      return ok && !bail;
    } else {
      return chol_dense(A, H, g.npad, winv, L.dl, g.n);
    }
  };
  double* vb = dyn;                // step
  double* vx = dyn + g.npad;       // refinement residual / matrix-free product
  double* vy = dyn + 2 * g.npad;   // right-hand side g
  int status = DNLS_GRAPH_OK;
  double last_obj = 0.0;
  int last_it = 0;
  double lam_cur = a.lambda;       // adaptive damping: this graph's lambda
  double radius = a.radius0;       // dogleg: this graph's trust radius
  init_H(g, H);
  for (int it = 0; it <= a.K; ++it) {
    const bool final_lin = (it == a.K);
    const double lam = final_lin ? 0.0 : lam_cur;
    if (a.traj && !final_lin) {
      double* dst = a.traj + ((size_t)it * a.V + g.pose0) * sz;
      for (int u = threadIdx.x; u < g.npose * sz; u += kNT) dst[u] = a.poses[(size_t)g.pose0 * sz + u];
    }
    double S = 0.0;
    // the mixed path linearises in float32 inside the loop; the float64
    // linearisation feeds its refinement sweeps and the final (cached) factor
    const bool lin32 = MIXED && !final_lin;
    const bool refine_now = MIXED && !final_lin && a.refine > 0 && it >= a.refine_from && it < a.refine_until;
    const bool lin64 = !MIXED || refine_now || final_lin || a.dogleg;
    if (lin32) S = linearize_graph<G, float>(a, g, a.ws32, L.red);
    if (lin64) S = linearize_graph<G, double>(a, g, a.ws64, L.red);
    last_obj = S;
    last_it = it;
    if (threadIdx.x == 0) a.objective[(size_t)b * (a.K + 1) + it] = S;
    if (!isfinite(S)) {
      status = DNLS_GRAPH_NONFINITE;
      break;
    }
    double* haug = H + (size_t)g.npad * g.npad;  // right-hand side row of the system
    double* aug = A + (size_t)g.npad * g.npad;   // ... and of the factor: y = L^-1 g
    if (final_lin) {
      // undamped factor of H* for the backward, assembled in float64
      assemble_H<G, double>(a, g, a.ws64, H, 0.0);
    } else if (MIXED) {
      assemble_H<G, float>(a, g, a.ws32, H, lam);
      if (refine_now || a.dogleg) assemble_g<G, double>(a, g, a.ws64, vy, haug);
      else assemble_g<G, float>(a, g, a.ws32, vy, haug);
    } else {
      assemble_H<G, double>(a, g, a.ws64, H, lam);
      assemble_g<G, double>(a, g, a.ws64, vy, haug);
    }
    // one factorisation site per step (the fused kernel keeps one inlined copy)
    if (!factor(it)) {
      status = DNLS_GRAPH_NOT_PD;
      break;
    }
    if (final_lin) break;
    // delta = L^-T y with y = L^-1 g from the right-hand-side row
    for (int u = threadIdx.x; u < g.npad; u += kNT) vb[u] = aug[u];
    __syncthreads();
    // the quarter form where its registers fit (the mixed pair kernels)
    if constexpr (MIXED && PAIR) trsv_upper_t(A, g.npad, winv, vb, L.dl);
    else trsv_upper_t_cols(A, g.npad, winv, vb, L.dl);
    if (MIXED) {
      for (int sweep = 0; sweep < (refine_now ? a.refine : 0); ++sweep) {
        // vx = g - (H64 + lambda I) delta ; delta += (L L^T)^-1 vx
        matvec_H<G>(a, g, a.ws64, vb, vx, lam, L.dl);
        for (int u = threadIdx.x; u < g.npad; u += kNT) vx[u] = vy[u] - vx[u];
        __syncthreads();
        trsv_lower(A, g.npad, winv, vx, L.dl);
        if constexpr (PAIR) trsv_upper_t(A, g.npad, winv, vx, L.dl);
        else trsv_upper_t_cols(A, g.npad, winv, vx, L.dl);
        for (int u = threadIdx.x; u < g.npad; u += kNT) vb[u] += vx[u];
        __syncthreads();
      }
    }
    if (GENERAL && a.dogleg) {
      // Powell's dogleg in the trust region ||delta|| <= radius for the model
      // S - g^T delta + 1/2 delta^T (H + lambda I) delta (float64 g and H)
      double part = 0.0;
      for (int u = threadIdx.x; u < g.n; u += kNT) part += vb[u] * vb[u];
      const double n_gn = sqrt(block_sum(part, L.red));
      bool boundary = false;
      if (!(n_gn <= radius)) {
        boundary = true;
        matvec_H<G>(a, g, a.ws64, vy, vx, lam, L.dl);   // (H + lambda I) g
        double p1 = 0.0, p2 = 0.0;
        for (int u = threadIdx.x; u < g.n; u += kNT) {
          p1 += vy[u] * vy[u];
          p2 += vy[u] * vx[u];
        }
        const double gg = block_sum(p1, L.red);
        const double gHg = block_sum(p2, L.red);
        const double alpha = gg / gHg;
        if (alpha * sqrt(gg) >= radius) {
          // the Cauchy point is outside: gradient direction cut at the boundary
          const double sc = radius / sqrt(gg);
          for (int u = threadIdx.x; u < g.n; u += kNT) vb[u] = sc * vy[u];
          __syncthreads();
        } else {
          // between the Cauchy point alpha g and the Gauss-Newton point
          double q1 = 0.0, q2 = 0.0;
          for (int u = threadIdx.x; u < g.n; u += kNT) {
            const double sd = alpha * vy[u], dd = vb[u] - sd;
            q1 += dd * dd;
            q2 += sd * dd;
          }
          const double qa = block_sum(q1, L.red);
          const double qb = 2.0 * block_sum(q2, L.red);
          const double qc = alpha * alpha * gg - radius * radius;
          const double beta = (-qb + sqrt(qb * qb - 4.0 * qa * qc)) / (2.0 * qa);
          for (int u = threadIdx.x; u < g.n; u += kNT) {
            const double sd = alpha * vy[u];
            vb[u] = sd + beta * (vb[u] - sd);
          }
          __syncthreads();
        }
      }
      // predicted decrease g^T delta - 1/2 delta^T (H + lambda I) delta
      matvec_H<G>(a, g, a.ws64, vb, vx, lam, L.dl);
      double r1 = 0.0, r2 = 0.0;
      for (int u = threadIdx.x; u < g.n; u += kNT) {
        r1 += vy[u] * vb[u];
        r2 += vb[u] * vx[u];
      }
      const double pred = block_sum(r1, L.red) - 0.5 * block_sum(r2, L.red);
      double r3 = 0.0;
      for (int u = threadIdx.x; u < g.n; u += kNT) r3 += vb[u] * vb[u];
      const double n_step = sqrt(block_sum(r3, L.red));
      double* bak = a.pose_bak + (size_t)g.pose0 * sz;
      for (int u = threadIdx.x; u < g.npose * sz; u += kNT) bak[u] = a.poses[(size_t)g.pose0 * sz + u];
      for (int p = threadIdx.x; p < g.npose; p += kNT)
        retract_minus<G>(a.poses + (size_t)(g.pose0 + p) * sz, vb + p * d);
      __syncthreads();
      const double s_trial = objective_graph<G>(a, g, L.red);
      const double rho = (S - s_trial) / pred;
      if (!(s_trial < S))
        for (int u = threadIdx.x; u < g.npose * sz; u += kNT) a.poses[(size_t)g.pose0 * sz + u] = bak[u];
      if (!(rho >= 0.25)) radius = 0.25 * n_step;
      else if (rho > 0.75 && boundary) radius = fmin(2.0 * radius, kRadiusMax);
      __syncthreads();
      continue;
    }
    if (a.adaptive) {
      // adaptive damping: keep the step iff the float64 objective strictly
      // decreases (lambda / 10), else restore theta_t (lambda x 10)
      const double s_t = lin64 ? S : objective_graph<G>(a, g, L.red);
      double* bak = a.pose_bak + (size_t)g.pose0 * sz;
      for (int u = threadIdx.x; u < g.npose * sz; u += kNT) bak[u] = a.poses[(size_t)g.pose0 * sz + u];
      for (int p = threadIdx.x; p < g.npose; p += kNT)
        retract_minus<G>(a.poses + (size_t)(g.pose0 + p) * sz, vb + p * d);
      __syncthreads();
      const double s_trial = objective_graph<G>(a, g, L.red);
      if (s_trial < s_t) {
        lam_cur = fmax(lam_cur / 10.0, kLambdaMin);
      } else {
        for (int u = threadIdx.x; u < g.npose * sz; u += kNT) a.poses[(size_t)g.pose0 * sz + u] = bak[u];
        lam_cur = fmin(lam_cur * 10.0, kLambdaMax);
      }
      __syncthreads();
      continue;
    }
    // retraction X <- X Exp(-delta)
    for (int p = threadIdx.x; p < g.npose; p += kNT)
      retract_minus<G>(a.poses + (size_t)(g.pose0 + p) * sz, vb + p * d);
    __syncthreads();
  }
  if constexpr (PAIR) {
    pair_post(ps.lead_stop, ps.base + 1);
    if (timed_out) status = DNLS_GRAPH_TIMEOUT;
  }
  if (threadIdx.x == 0) {
    // a failed graph repeats its last objective for the steps that did not run
    for (int t = last_it + 1; t <= a.K; ++t) a.objective[(size_t)b * (a.K + 1) + t] = last_obj;
    a.status[b] = status;
  }
}

// ---------------------------------------------------------------------------
// backward: adjoint solve with the cached factor, then per-cost VJP
// ---------------------------------------------------------------------------

// per-cost VJP of the implicit backward for the adjoint vu (LDS) of graph g
template <int G>
__device__ void vjp_graph(const DenseArgs& a, const GraphDesc& g, const double* vu) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const PoseCostData cd = cost_data(a);
  const int ncost = g.nedge + g.nprior;
  for (int k = threadIdx.x; k < ncost; k += kNT) {
    int rk;
    const double *ui = nullptr, *uj;
    if (k < g.nedge) {
      rk = g.edge0 + k;
      ui = vu + (a.edge_ij[2 * rk] - g.pose0) * d;
      uj = vu + (a.edge_ij[2 * rk + 1] - g.pose0) * d;
    } else {
      const int p = g.prior0 + (k - g.nedge);
      rk = a.E + p;
      uj = vu + (a.prior_var[p] - g.pose0) * d;
    }
    cost_vjp<G>(cd, rk, a.ws64 + (size_t)rk * RN, ui, uj, a.g_logw_e, a.g_tau, a.g_logw_p, a.g_logc);
  }
}

template <int G>
__device__ void zero_grads(const DenseArgs& a, const GraphDesc& g, bool adjoint) {
  constexpr int d = GroupTraits<G>::d;
  for (int k = threadIdx.x; k < g.nedge; k += kNT) {
    const int e = g.edge0 + k;
    if (a.g_logw_e) a.g_logw_e[e] = 0.0;
    if (a.g_logc) a.g_logc[e] = 0.0;
    if (a.g_tau)
      for (int q = 0; q < d; ++q) a.g_tau[(size_t)e * d + q] = 0.0;
  }
  for (int k = threadIdx.x; k < g.nprior; k += kNT)
    if (a.g_logw_p) a.g_logw_p[g.prior0 + k] = 0.0;
  if (adjoint && a.adjoint_out)
    for (int u = threadIdx.x; u < g.n; u += kNT) a.adjoint_out[(size_t)g.pose0 * d + u] = 0.0;
}

// y = Hx x with Hx the exact Hessian of S(theta_K Exp(delta)) at delta = 0:
//   Hx x = sum J^T J x + sum w^2 (dC/ds)^T c - 1/2 [ad(x_p)^T g_p]_p
// (Gauss-Newton part from the float64 records, second-order cost terms by
// one dual-number pass per cost, and the term of the retraction's right
// Jacobian Jr(delta) = I - ad(delta)/2 + ...); gvec is the gradient at theta_K.
template <int G>
__device__ void hvp_exact(const DenseArgs& a, const GraphDesc& g, const double* rec, const double* x,
                          double* y, const double* gvec) {
  constexpr int d = GroupTraits<G>::d, RN = CostRec<d>::n;
  const PoseCostData cd = cost_data(a);
  const int ncost = g.nedge + g.nprior;
  for (int k = threadIdx.x; k < ncost; k += kNT) {
    int cost, pi, pj;
    if (k < g.nedge) {
      cost = g.edge0 + k;
      pi = a.edge_ij[2 * cost] - g.pose0;
      pj = a.edge_ij[2 * cost + 1] - g.pose0;
    } else {
      const int p = g.prior0 + (k - g.nedge);
      cost = a.E + p;
      pi = -1;
      pj = a.prior_var[p] - g.pose0;
    }
    const double* J = rec + (size_t)cost * RN;
#pragma unroll
    for (int r = 0; r < d; ++r) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < d; ++q) {
        if (pi >= 0) acc += J[r * d + q] * x[pi * d + q];
        acc += J[d * d + r * d + q] * x[pj * d + q];
      }
      a.ycost[(size_t)cost * d + r] = acc;
    }
    double* o = a.hvp + (size_t)cost * 2 * d;
    cost_hvp_residual<G>(cd, cost, J, pi >= 0 ? x + pi * d : nullptr, x + pj * d, o, o + d);
  }
  __syncthreads();
  for (int u = threadIdx.x; u < g.npad; u += kNT) {
    double v = 0.0;
    if (u < g.n) {
      const int p = u / d, r = u % d, gp = g.pose0 + p;
      for (int s = a.inc_off[gp]; s < a.inc_off[gp + 1]; ++s) {
        const int slot = a.inc_slot[s];
        const double* J = rec + (size_t)(slot >> 1) * RN + (slot & 1) * d * d;
        const double* yc = a.ycost + (size_t)(slot >> 1) * d;
#pragma unroll
        for (int k = 0; k < d; ++k) v += J[k * d + r] * yc[k];
        v += a.hvp[(size_t)(slot >> 1) * 2 * d + (slot & 1) * d + r];
      }
      double c[d];
      ad_transpose_mul<G>(x + p * d, gvec + p * d, c);
      v -= 0.5 * c[r];
    }
    y[u] = v;
  }
  __syncthreads();
}

// The adjoint u = H*^-1 v of the implicit backward: the two triangular
// solves with the cached factor, then one step of float64 iterative
// refinement u <- u + H*^-1 (v - H* u) with H* applied matrix-free from the
// float64 records at theta_K, so that u carries the rounding of that product
// rather than the factorisation's rounding amplified by cond(H*).  Mixed
// plans skip the refinement: their results are held to 1e-5 of the float64
// ones, and the adjoint through the float64 factor of H* is within
// cond(H*) eps64 of it.  vu holds v on entry and u on return; vx is scratch
// (npad each, LDS).
template <int G>
__device__ void adjoint_solve(const DenseArgs& a, const GraphDesc& g, const double* A, const double* winv,
                              double* vu, double* vx, KernelLds& L) {
  constexpr int d = GroupTraits<G>::d;
  const double* seed = a.seed + (size_t)g.pose0 * d;
  trsv_lower(A, g.npad, winv, vu, L.dl);
  trsv_upper_t(A, g.npad, winv, vu, L.dl);
  if (!a.adj_refine) return;
  matvec_H<G>(a, g, a.ws64, vu, vx, 0.0, L.dl);
  for (int u = threadIdx.x; u < g.npad; u += kNT) vx[u] = ((u < g.n) ? seed[u] : 0.0) - vx[u];
  __syncthreads();
  trsv_lower(A, g.npad, winv, vx, L.dl);
  trsv_upper_t(A, g.npad, winv, vx, L.dl);
  for (int u = threadIdx.x; u < g.npad; u += kNT) vu[u] += vx[u];
  __syncthreads();
}

template <int G>
__global__ void __launch_bounds__(kNT) k_dense_backward(DenseArgs a) {
  constexpr int d = GroupTraits<G>::d;
  extern __shared__ double dyn[];
  __shared__ KernelLds L;
  const int b = a.order[blockIdx.x];
  const GraphDesc g = a.gd[b];
  if (a.status[b] != DNLS_GRAPH_OK) {
    zero_grads<G>(a, g, true);
    return;
  }
  const double* A = a.factor + g.fac_off;
  const double* winv = A + (size_t)(g.npad + 16) * g.npad;
  double* vu = dyn;
  double* vx = dyn + g.npad;
  for (int u = threadIdx.x; u < g.npad; u += kNT) vu[u] = (u < g.n) ? a.seed[(size_t)g.pose0 * d + u] : 0.0;
  __syncthreads();
  // float64 linearisation at theta_K: residuals and Jacobians for the
  // refinement of the adjoint and for the VJP
  linearize_graph<G, double>(a, g, a.ws64, L.red);
  adjoint_solve<G>(a, g, A, winv, vu, vx, L);
  if (a.adjoint_out)
    for (int u = threadIdx.x; u < g.n; u += kNT) a.adjoint_out[(size_t)g.pose0 * d + u] = vu[u];
  // per-cost VJP:  dL/dphi = -d/dphi [ (J u)^T r ]
  vjp_graph<G>(a, g, vu);
}

// Implicit backward with the exact Hessian: u = Hx^-1 v by iterative
// refinement preconditioned by the cached Gauss-Newton factor,
// u <- u + H*^-1 (v - Hx u) from u = H*^-1 v, then the per-cost VJP.
template <int G>
__global__ void __launch_bounds__(kNT) k_dense_backward_exact(DenseArgs a, int sweeps) {
  constexpr int d = GroupTraits<G>::d;
  extern __shared__ double dyn[];
  __shared__ KernelLds L;
  const int b = a.order[blockIdx.x];
  const GraphDesc g = a.gd[b];
  if (a.status[b] != DNLS_GRAPH_OK) {
    zero_grads<G>(a, g, true);
    return;
  }
  const double* A = a.factor + g.fac_off;
  const double* winv = A + (size_t)(g.npad + 16) * g.npad;
  double* vu = dyn;
  double* vx = dyn + g.npad;
  double* vg = dyn + 2 * g.npad;
  const double* seed = a.seed + (size_t)g.pose0 * d;
  for (int u = threadIdx.x; u < g.npad; u += kNT) vu[u] = (u < g.n) ? seed[u] : 0.0;
  __syncthreads();
  linearize_graph<G, double>(a, g, a.ws64, L.red);
  assemble_g<G, double>(a, g, a.ws64, vg, nullptr);
  // the Gauss-Newton adjoint of the implicit mode, then the exact sweeps
  adjoint_solve<G>(a, g, A, winv, vu, vx, L);
  for (int it = 0; it < sweeps; ++it) {
    hvp_exact<G>(a, g, a.ws64, vu, vx, vg);
    for (int u = threadIdx.x; u < g.npad; u += kNT) vx[u] = ((u < g.n) ? seed[u] : 0.0) - vx[u];
    __syncthreads();
    trsv_lower(A, g.npad, winv, vx, L.dl);
    trsv_upper_t(A, g.npad, winv, vx, L.dl);
    for (int u = threadIdx.x; u < g.npad; u += kNT) vu[u] += vx[u];
    __syncthreads();
  }
  if (a.adjoint_out)
    for (int u = threadIdx.x; u < g.n; u += kNT) a.adjoint_out[(size_t)g.pose0 * d + u] = vu[u];
  vjp_graph<G>(a, g, vu);
}

// Unrolled backward (truncated to the last T steps): reverse sweep through
// theta_{t+1} = theta_t Exp(-delta_t), delta_t = (H_t + lambda I)^-1 g_t, from
// the kept iterates.  Per step, with abar the cotangent at theta_{t+1}:
//   dbar_p = -Jr(-delta_p)^T abar_p,  abar_p <- Ad(Exp(delta_p))^T abar_p,
//   y = (H_t + lambda I)^-1 dbar, then the gradient of
//   s = y^T g_t - y^T (H_t + lambda I) delta_t (y, delta_t fixed) is added to
//   abar (poses) and to the parameter gradients (cost_unroll_vjp).
template <int G>
__global__ void __launch_bounds__(kNT) k_dense_backward_unroll(DenseArgs a, int T) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  extern __shared__ double dyn[];
  __shared__ KernelLds L;
  const int b = a.order[blockIdx.x];
  const GraphDesc g = a.gd[b];
  zero_grads<G>(a, g, true);
  if (a.status[b] != DNLS_GRAPH_OK) return;
  double* va = dyn;                // cotangent of the iterate
  double* vd = dyn + g.npad;       // delta_t
  double* vw = dyn + 2 * g.npad;   // dbar, then y
  double* H = a.hbuf + g.h_off;
  double* haug = H + (size_t)g.npad * g.npad;
  double* winv = a.dlm_winv + g.dlm_winv_off;
  for (int u = threadIdx.x; u < g.npad; u += kNT) va[u] = (u < g.n) ? a.seed[(size_t)g.pose0 * d + u] : 0.0;
  __syncthreads();
  const int ncost = g.nedge + g.nprior;
  for (int t = a.K - 1; t >= a.K - T; --t) {
    DenseArgs at = a;
    at.poses = a.traj + (size_t)t * a.V * sz;
    const PoseCostData cd = cost_data(at);
    linearize_graph<G, double>(at, g, a.ws64, L.red);
    init_H(g, H);
    assemble_H<G, double>(at, g, a.ws64, H, a.lambda);
    assemble_g<G, double>(at, g, a.ws64, vd, haug);
    if (!chol_dense(H, H, g.npad, winv, L.dl, g.n)) {
      // the forward factored this system (in float32 on the mixed path): give up on the graph
      zero_grads<G>(a, g, true);
      return;
    }
    for (int u = threadIdx.x; u < g.npad; u += kNT) vd[u] = haug[u];
    __syncthreads();
    trsv_upper_t(H, g.npad, winv, vd, L.dl);
    // through the retraction
    for (int p = threadIdx.x; p < g.npose; p += kNT) {
      double dl[d], md[d], Jr[d * d], Ad[d * d], ab[d];
      for (int q = 0; q < d; ++q) {
        dl[q] = vd[p * d + q];
        md[q] = -dl[q];
        ab[q] = va[p * d + q];
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
        vw[p * d + m] = -s1;
        va[p * d + m] = s2;
      }
    }
    for (int u = g.n + threadIdx.x; u < g.npad; u += kNT) vw[u] = 0.0;
    __syncthreads();
    trsv_lower(H, g.npad, winv, vw, L.dl);
    trsv_upper_t(H, g.npad, winv, vw, L.dl);
    // per-cost gradient of s: pose terms to the per-cost buffer, parameters accumulated
    for (int k = threadIdx.x; k < ncost; k += kNT) {
      int cost, pi, pj;
      if (k < g.nedge) {
        cost = g.edge0 + k;
        pi = a.edge_ij[2 * cost] - g.pose0;
        pj = a.edge_ij[2 * cost + 1] - g.pose0;
      } else {
        const int pq = g.prior0 + (k - g.nedge);
        cost = a.E + pq;
        pi = -1;
        pj = a.prior_var[pq] - g.pose0;
      }
      double* o = a.hvp + (size_t)cost * 2 * d;
      double dlw, dt[d];
      cost_unroll_vjp<G>(cd, cost, pi >= 0 ? vw + pi * d : nullptr, vw + pj * d, pi >= 0 ? vd + pi * d : nullptr,
                         vd + pj * d, o, o + d, &dlw, k < g.nedge ? dt : nullptr);
      if (pi < 0)
        for (int q = 0; q < d; ++q) o[q] = 0.0;
      if (k < g.nedge) {
        if (a.g_logw_e) a.g_logw_e[cost] += dlw;
        if (a.g_tau)
          for (int q = 0; q < d; ++q) a.g_tau[(size_t)cost * d + q] += dt[q];
      } else if (a.g_logw_p) {
        a.g_logw_p[cost - a.E] += dlw;
      }
    }
    __syncthreads();
    for (int u = threadIdx.x; u < g.n; u += kNT) {
      const int p = u / d, r = u % d, gp = g.pose0 + p;
      double v = 0.0;
      for (int s2 = a.inc_off[gp]; s2 < a.inc_off[gp + 1]; ++s2) {
        const int slot = a.inc_slot[s2];
        v += a.hvp[(size_t)(slot >> 1) * 2 * d + (slot & 1) * d + r];
      }
      va[u] += v;
    }
    __syncthreads();
  }
  if (a.adjoint_out)
    for (int u = threadIdx.x; u < g.n; u += kNT) a.adjoint_out[(size_t)g.pose0 * d + u] = va[u];
}

// ---------------------------------------------------------------------------
// backward by direct loss minimisation (Section 4.3, Appendix G): one
// Gauss-Newton step from theta_K on S + ||eps theta - v / 2||^2,
//   (H* + 2 eps^2 I) delta = -g* + eps v,  theta_direct = theta_K (+) delta,
// then dL/dphi = (dS/dphi(theta_K) - dS/dphi(theta_direct)) / eps
// ---------------------------------------------------------------------------
template <int G>
__device__ void param_grads(const DenseArgs& a, const GraphDesc& g, const double* poses, double scale, bool accumulate) {
  constexpr int d = GroupTraits<G>::d;
  PoseCostData cd = cost_data(a);
  cd.poses = poses;
  for (int k = threadIdx.x; k < g.nedge + g.nprior; k += kNT) {
    double dl, dt[d], dlc = 0.0;
    if (k < g.nedge) {
      const int e = g.edge0 + k;
      cost_param_grad<G>(cd, e, &dl, dt, &dlc);
      if (a.g_logw_e) a.g_logw_e[e] = (accumulate ? a.g_logw_e[e] : 0.0) + scale * dl;
      if (a.g_logc) a.g_logc[e] = (accumulate ? a.g_logc[e] : 0.0) + scale * dlc;
      if (a.g_tau)
#pragma unroll
        for (int q = 0; q < d; ++q) a.g_tau[(size_t)e * d + q] = (accumulate ? a.g_tau[(size_t)e * d + q] : 0.0) + scale * dt[q];
    } else {
      const int pq = g.prior0 + (k - g.nedge);
      cost_param_grad<G>(cd, a.E + pq, &dl, dt, nullptr);
      if (a.g_logw_p) a.g_logw_p[pq] = (accumulate ? a.g_logw_p[pq] : 0.0) + scale * dl;
    }
  }
  __syncthreads();
}

template <int G>
__global__ void __launch_bounds__(kNT) k_dense_backward_dlm(DenseArgs a, double eps) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  extern __shared__ double dyn[];
  __shared__ KernelLds L;
  const int b = a.order[blockIdx.x];
  const GraphDesc g = a.gd[b];
  if (a.status[b] != DNLS_GRAPH_OK) {
    zero_grads<G>(a, g, false);
    return;
  }
  // dS/dphi at theta_K, scaled by 1 / eps
  param_grads<G>(a, g, a.poses, 1.0 / eps, false);
  // H* + 2 eps^2 I and -g* + eps v, factored in the workspace
  double* H = a.hbuf + g.h_off;
  double* winv = a.dlm_winv + g.dlm_winv_off;
  double* vb = dyn;
  double* vy = dyn + g.npad;
  linearize_graph<G, double>(a, g, a.ws64, L.red);
  init_H(g, H);
  assemble_H<G, double>(a, g, a.ws64, H, 2.0 * eps * eps);
  double* haug = H + (size_t)g.npad * g.npad;
  assemble_g<G, double>(a, g, a.ws64, vy, haug);
  for (int u = threadIdx.x; u < g.n; u += kNT) haug[u] = -haug[u] + eps * a.seed[(size_t)g.pose0 * d + u];
  __syncthreads();
  const bool ok = chol_dense(H, H, g.npad, winv, L.dl, g.n);
  if (!ok) {
    // cannot happen for a positive definite H* (it was factored in the solve)
    zero_grads<G>(a, g, false);
    return;
  }
  for (int u = threadIdx.x; u < g.npad; u += kNT) vb[u] = haug[u];
  __syncthreads();
  trsv_upper_t(H, g.npad, winv, vb, L.dl);
  // theta_direct = theta_K Exp(delta), i.e. retract_minus by -delta
  double* Xd = a.pose_bak + (size_t)g.pose0 * sz;
  for (int u = threadIdx.x; u < g.npose * sz; u += kNT) Xd[u] = a.poses[(size_t)g.pose0 * sz + u];
  for (int u = threadIdx.x; u < g.n; u += kNT) vb[u] = -vb[u];
  __syncthreads();
  for (int p = threadIdx.x; p < g.npose; p += kNT) retract_minus<G>(Xd + (size_t)p * sz, vb + p * d);
  __syncthreads();
  // minus dS/dphi at theta_direct, scaled by 1 / eps
  param_grads<G>(a, g, a.pose_bak, -1.0 / eps, true);
}

// projection operator of Appendix D (one thread per element)
template <int G>
__global__ void k_project(long long n, const double* X, const double* Gr, double* out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= n) return;
  if constexpr (G == 3) {
    const double* x = X + e * 12;
    const double* gr = Gr + e * 12;
    double M[9];
    // M = R^T G_R
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) M[r * 3 + q] = x[0 * 4 + r] * gr[0 * 4 + q] + x[1 * 4 + r] * gr[1 * 4 + q] + x[2 * 4 + r] * gr[2 * 4 + q];
    double* o = out + e * 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) o[k] = x[0 * 4 + k] * gr[3] + x[1 * 4 + k] * gr[7] + x[2 * 4 + k] * gr[11];
    o[3] = M[7] - M[5];
    o[4] = M[2] - M[6];
    o[5] = M[3] - M[1];
  } else {
    const double* x = X + e * 4;
    const double* gr = Gr + e * 4;
    const double c = x[2], s = x[3];
    double* o = out + e * 3;
    o[0] = c * gr[0] + s * gr[1];
    o[1] = -s * gr[0] + c * gr[1];
    o[2] = -s * gr[2] + c * gr[3];
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
bool check_off(const int32_t* off, int B, int total_hint, int* total) {
  if (!off || off[0] != 0) return false;
  for (int b = 0; b < B; ++b)
    if (off[b + 1] < off[b]) return false;
  *total = off[B];
  (void)total_hint;
  return true;
}


// Whether the pair kernel of this plan can be launched with every pair
// co-resident: two workgroups per graph within what the device holds at once.
template <int G, bool MIXED>
bool pair_fits(dnls_plan p) {
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return false;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
  const size_t lds = 3 * (size_t)p->npad_max * sizeof(double);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_dense_solve<G, MIXED, false, true>),
                                                   kNT, lds) != hipSuccess)
    return false;
  return (long long)per_cu * cus >= 2LL * p->B;
}

template <int G, bool MIXED>
dnls_status launch_solve(dnls_plan p, const DenseArgs& a, hipStream_t st) {
  const size_t lds = 3 * (size_t)p->npad_max * sizeof(double);
  if (a.dogleg || a.edge_logc) {
    hipLaunchKernelGGL((k_dense_solve<G, MIXED, true>), dim3(p->B), dim3(kNT), lds, st, a);
  } else if ((p->opt.flags & DNLS_FLAG_PAIR) && p->pair_ok) {
    DenseArgs ap = a;
    ap.pair_ctr = p->d_pair;
    ap.pair_base = (++p->pair_epoch) << 20;   // counters only grow: no reset between launches
    ap.pair_spin = p->pair_spin;
    void* args[] = {&ap};
    HIP_TRY(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_dense_solve<G, MIXED, false, true>),
                                       dim3(2 * p->B), dim3(kNT), args, (unsigned)lds, st));
  } else {
    hipLaunchKernelGGL((k_dense_solve<G, MIXED, false>), dim3(p->B), dim3(kNT), lds, st, a);
  }
  HIP_TRY(hipGetLastError());
  return DNLS_OK;
}

template <int G>
dnls_status launch_backward(dnls_plan p, const DenseArgs& a, hipStream_t st, int mode, double eps, int sweeps) {
  if (mode == DNLS_BACKWARD_UNROLL) {
    const size_t lds3 = 3 * (size_t)p->npad_max * sizeof(double);
    hipLaunchKernelGGL((k_dense_backward_unroll<G>), dim3(p->B), dim3(kNT), lds3, st, a, sweeps);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  if (mode == DNLS_BACKWARD_EXACT) {
    const size_t lds3 = 3 * (size_t)p->npad_max * sizeof(double);
    hipLaunchKernelGGL((k_dense_backward_exact<G>), dim3(p->B), dim3(kNT), lds3, st, a, sweeps);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  if (mode == DNLS_BACKWARD_DLM) {
    const size_t lds2 = 2 * (size_t)p->npad_max * sizeof(double);
    hipLaunchKernelGGL((k_dense_backward_dlm<G>), dim3(p->B), dim3(kNT), lds2, st, a, eps);
    HIP_TRY(hipGetLastError());
    return DNLS_OK;
  }
  const size_t lds = 2 * (size_t)p->npad_max * sizeof(double);
  hipLaunchKernelGGL((k_dense_backward<G>), dim3(p->B), dim3(kNT), lds, st, a);
  HIP_TRY(hipGetLastError());
  return DNLS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* dnls_last_error(void) { return g_err.c_str(); }

const char* dnls_version(void) { return "dnls-gfx950 0.1"; }

dnls_status dnls_plan_create(dnls_plan* out, const dnls_problem* pr, const dnls_options* op) {
  g_err.clear();
  if (!out || !pr || !op) return fail(DNLS_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (pr->batch < 1) return fail(DNLS_ERR_INVALID_ARG, "batch must be >= 1");
  if (pr->group != DNLS_SE2 && pr->group != DNLS_SE3) return fail(DNLS_ERR_INVALID_ARG, "group must be SE2 or SE3");
  if (op->iterations < 0) return fail(DNLS_ERR_INVALID_ARG, "iterations must be >= 0");
  if (!(op->lambda >= 0.0)) return fail(DNLS_ERR_INVALID_ARG, "lambda must be >= 0");
  if (op->precision != DNLS_PREC_FP64 && op->precision != DNLS_PREC_MIXED)
    return fail(DNLS_ERR_INVALID_ARG, "unknown precision");
  if (op->refine < 0 || op->refine > 4) return fail(DNLS_ERR_INVALID_ARG, "refine must be in 0..4");
  if (op->refine_last < -op->iterations || op->refine_last > op->iterations)
    return fail(DNLS_ERR_INVALID_ARG, "refine_last must be in 0..iterations");
  if (op->sparse_solve < DNLS_SPSOLVE_AUTO || op->sparse_solve > DNLS_SPSOLVE_BLOCK)
    return fail(DNLS_ERR_INVALID_ARG, "unknown sparse_solve");
  if (op->flags & ~int32_t(DNLS_FLAG_GRAPH | DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG | DNLS_FLAG_KEEP_ITERATES |
                           DNLS_FLAG_PAIR))
    return fail(DNLS_ERR_INVALID_ARG, "unknown flags");
  if (op->flags & DNLS_FLAG_KEEP_ITERATES) {
    if (op->solver == DNLS_SOLVER_SCHUR)
      return fail(DNLS_ERR_UNSUPPORTED, "kept iterates (unrolled backward) are implemented for the pose-graph solvers");
    if (op->flags & (DNLS_FLAG_ADAPTIVE_LM | DNLS_FLAG_DOGLEG))
      return fail(DNLS_ERR_UNSUPPORTED, "the unrolled backward differentiates the fixed-damping step only");
  }
  if (op->flags & DNLS_FLAG_DOGLEG) {
    if ((op->flags & DNLS_FLAG_ADAPTIVE_LM))
      return fail(DNLS_ERR_INVALID_ARG, "adaptive damping and dogleg exclude each other");
    if (!(op->trust_radius > 0.0) || !std::isfinite(op->trust_radius))
      return fail(DNLS_ERR_INVALID_ARG, "dogleg needs a positive finite trust_radius");
  }
  if (op->solver == DNLS_SOLVER_SCHUR || (op->solver == DNLS_SOLVER_SPARSE && pr->point_off)) {
    auto* p = new dnls_plan_s();
    p->B = pr->batch;
    p->group = pr->group;
    p->d = 6;
    p->sz = 12;
    p->opt = *op;
    const dnls_status st = op->solver == DNLS_SOLVER_SCHUR ? ba_plan_create(p, pr, op) : sp_plan_create_ba(p, pr);
    if (st != DNLS_OK) {
      const std::string msg = g_err;
      dnls_plan_destroy(p);
      return fail(st, msg);
    }
    *out = p;
    return DNLS_OK;
  }
  if (op->solver != DNLS_SOLVER_DENSE && op->solver != DNLS_SOLVER_SPARSE)
    return fail(DNLS_ERR_UNSUPPORTED, "unknown solver");
  const int B = pr->batch;
  int V = 0, E = 0, P = 0;
  if (!check_off(pr->pose_off, B, 0, &V) || !check_off(pr->edge_off, B, 0, &E) ||
      !check_off(pr->prior_off, B, 0, &P))
    return fail(DNLS_ERR_INVALID_ARG, "offsets must start at 0 and be non-decreasing");
  if (E > 0 && !pr->edge_ij) return fail(DNLS_ERR_INVALID_ARG, "edge_ij is NULL");
  if (P > 0 && !pr->prior_var) return fail(DNLS_ERR_INVALID_ARG, "prior_var is NULL");

  auto* p = new dnls_plan_s();
  p->B = B;
  p->group = pr->group;
  p->d = pr->group == DNLS_SE3 ? 6 : 3;
  p->sz = pr->group == DNLS_SE3 ? 12 : 4;
  p->opt = *op;
  p->V = V;
  p->E = E;
  p->P = P;
  const int d = p->d;
  if (op->solver == DNLS_SOLVER_SPARSE) {
    const dnls_status st = sp_plan_create(p, pr);
    if (st != DNLS_OK) {
      const std::string msg = g_err;
      dnls_plan_destroy(p);
      return fail(st, msg);
    }
    *out = p;
    return DNLS_OK;
  }

  // per-pose incidence (slots = cost * 2 + side) and off-diagonal blocks
  std::vector<std::vector<int>> inc(V);
  std::vector<int> edge_ij(2 * (size_t)E), prior_var(P);
  std::vector<int4> od_blk;
  std::vector<int> od_slot;
  p->gd.resize(B);
  long long fac = 0, hsz = 0, dlmw = 0;
  for (int b = 0; b < B; ++b) {
    GraphDesc& g = p->gd[b];
    g.pose0 = pr->pose_off[b];
    g.npose = pr->pose_off[b + 1] - g.pose0;
    g.edge0 = pr->edge_off[b];
    g.nedge = pr->edge_off[b + 1] - g.edge0;
    g.prior0 = pr->prior_off[b];
    g.nprior = pr->prior_off[b + 1] - g.prior0;
    g.n = g.npose * d;
    g.npad = std::max(kNB, (g.n + kNB - 1) / kNB * kNB);
    if (g.npad > kMaxDenseN) {
      delete p;
      return fail(DNLS_ERR_UNSUPPORTED, "dense solver supports at most " + std::to_string(kMaxDenseN) +
                                            " unknowns per graph");
    }
    p->flops_alg += double(g.n) * g.n * g.n / 3.0;
    p->flops_exec += double(g.npad) * g.npad * g.npad / 3.0;
    g.fac_off = fac;
    g.h_off = hsz;
    hsz += (long long)(g.npad + 16) * g.npad;
    g.dlm_winv_off = dlmw;
    dlmw += (long long)(g.npad / kNB) * kNB * kNB;
    // L (npad x npad) + right-hand-side row and 15 padding rows (16 x npad) + panel inverses
    fac += (long long)(g.npad + 16) * g.npad + (long long)(g.npad / kNB) * kNB * kNB;
    fac = (fac + 31) / 32 * 32;
    p->npad_max = std::max(p->npad_max, g.npad);
    std::map<std::pair<int, int>, std::vector<int>> blocks;
    for (int e = g.edge0; e < g.edge0 + g.nedge; ++e) {
      const int i = pr->edge_ij[2 * (size_t)e], j = pr->edge_ij[2 * (size_t)e + 1];
      if (i < g.pose0 || i >= g.pose0 + g.npose || j < g.pose0 || j >= g.pose0 + g.npose || i == j) {
        delete p;
        return fail(DNLS_ERR_INVALID_ARG, "edge " + std::to_string(e) + " has an index outside its graph or i == j");
      }
      edge_ij[2 * (size_t)e] = i;
      edge_ij[2 * (size_t)e + 1] = j;
      inc[i].push_back(2 * e + 0);
      inc[j].push_back(2 * e + 1);
      const int li = i - g.pose0, lj = j - g.pose0;
      if (li > lj) blocks[{li, lj}].push_back(2 * e + 0);   // row side = i
      else blocks[{lj, li}].push_back(2 * e + 1);           // row side = j
    }
    for (int q = g.prior0; q < g.prior0 + g.nprior; ++q) {
      const int v = pr->prior_var[q];
      if (v < g.pose0 || v >= g.pose0 + g.npose) {
        delete p;
        return fail(DNLS_ERR_INVALID_ARG, "prior " + std::to_string(q) + " refers to a pose outside its graph");
      }
      prior_var[q] = v;
      inc[v].push_back(2 * (E + q) + 1);
    }
    g.od0 = (int)od_blk.size();
    for (auto& kv : blocks) {
      od_blk.push_back(int4{kv.first.first, kv.first.second, (int)od_slot.size(), (int)kv.second.size()});
      for (int s : kv.second) od_slot.push_back(s);
    }
    g.nod = (int)od_blk.size() - g.od0;
  }
  std::vector<int> inc_off(V + 1, 0), inc_slot;
  for (int v = 0; v < V; ++v) {
    inc_off[v + 1] = inc_off[v] + (int)inc[v].size();
    for (int s : inc[v]) inc_slot.push_back(s);
  }
  // largest graphs first
  std::vector<int> order(B);
  for (int b = 0; b < B; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return p->gd[x].npad > p->gd[y].npad; });

  dnls_status st;
  if ((st = upload(p, &p->d_gd, p->gd)) != DNLS_OK ||
      (st = upload(p, &p->d_order, order)) != DNLS_OK ||
      (st = upload(p, &p->d_edge_ij, edge_ij)) != DNLS_OK ||
      (st = upload(p, &p->d_prior_var, prior_var)) != DNLS_OK ||
      (st = upload(p, &p->d_inc_off, inc_off)) != DNLS_OK ||
      (st = upload(p, &p->d_inc_slot, inc_slot)) != DNLS_OK ||
      (st = upload(p, &p->d_od_blk, od_blk)) != DNLS_OK ||
      (st = upload(p, &p->d_od_slot, od_slot)) != DNLS_OK) {
    std::string msg = g_err;
    dnls_plan_destroy(p);
    return fail(st, msg);
  }
  const size_t ncost = (size_t)E + P;
  const size_t rn = 2 * (size_t)d * d + d;
  size_t ws = align256(ncost * rn * sizeof(double));
  p->ws32_off = ws;
  if (op->precision == DNLS_PREC_MIXED) ws += align256(ncost * rn * sizeof(float));
  p->ycost_off = ws;
  ws += align256(ncost * d * sizeof(double));
  p->h_off = ws;
  ws += align256((size_t)hsz * sizeof(double));
  p->bak_off = ws;
  ws += align256((size_t)V * p->sz * sizeof(double));   // adaptive damping backup / DLM theta_direct
  p->dlmw_off = ws;
  ws += align256((size_t)dlmw * sizeof(double));        // DLM backward: panel inverses
  p->hvp_off = ws;
  ws += align256(ncost * 2 * d * sizeof(double));       // exact backward: residual terms per cost side
  p->ws_bytes = ws;
  p->bwd_bytes = ws;
  p->traj_off = fac;   // doubles
  if (op->flags & DNLS_FLAG_KEEP_ITERATES) fac += (long long)op->iterations * V * p->sz;
  p->fac_bytes = (size_t)fac * sizeof(double);
  if (op->flags & DNLS_FLAG_PAIR) {
    p->pair_spin = pair_spin_limit();
    const bool mixed = op->precision == DNLS_PREC_MIXED;
    // a pair needs a second row group to share: with one 64-wide panel per
    // graph the follower would only add its synchronisation to every step
    p->pair_ok = p->npad_max > kNB &&
                 (p->group == DNLS_SE3 ? (mixed ? pair_fits<3, true>(p) : pair_fits<3, false>(p))
                                       : (mixed ? pair_fits<2, true>(p) : pair_fits<2, false>(p)));
    if (p->pair_ok) {
      const size_t bytes = (size_t)p->B * 8 * sizeof(unsigned long long);
      if (hipMalloc(reinterpret_cast<void**>(&p->d_pair), bytes) != hipSuccess ||
          (p->allocs.push_back(p->d_pair), hipMemset(p->d_pair, 0, bytes)) != hipSuccess) {
        dnls_plan_destroy(p);
        return fail(DNLS_ERR_HIP, "allocating the pair counters failed");
      }
    }
  }
  *out = p;
  return DNLS_OK;
}

dnls_status dnls_plan_schedule(dnls_plan p, int32_t* dense_pair, int32_t* sparse_solve) {
  if (!p) return fail(DNLS_ERR_INVALID_ARG, "null plan");
  if (dense_pair)
    *dense_pair = ((p->opt.solver == DNLS_SOLVER_DENSE && (p->opt.flags & DNLS_FLAG_PAIR) && p->pair_ok) ||
                   (p->opt.solver == DNLS_SOLVER_SCHUR && p->ba_nway > 1)) ? 1 : 0;
  if (sparse_solve) {
    *sparse_solve = DNLS_SPSOLVE_AUTO;
    if (p->opt.solver == DNLS_SOLVER_SPARSE)
      *sparse_solve = p->sp_ts != 48 ? DNLS_SPSOLVE_BLOCK
                      : p->sp_persistent ? DNLS_SPSOLVE_PERSISTENT
                      : p->sp_factor_wg ? DNLS_SPSOLVE_WORKGROUP
                      : (p->sp_solve_wg ? DNLS_SPSOLVE_HYBRID : DNLS_SPSOLVE_SWEEPS);
  }
  return DNLS_OK;
}

dnls_status dnls_plan_flops(dnls_plan p, double* algorithmic, double* executed) {
  if (!p) return fail(DNLS_ERR_INVALID_ARG, "null plan");
  if (algorithmic) *algorithmic = p->flops_alg;
  if (executed) *executed = p->flops_exec;
  return DNLS_OK;
}

dnls_status dnls_plan_workspace(dnls_plan p, size_t* solve_ws, size_t* factor_bytes, size_t* backward_ws) {
  if (!p) return fail(DNLS_ERR_INVALID_ARG, "null plan");
  if (solve_ws) *solve_ws = p->ws_bytes;
  if (factor_bytes) *factor_bytes = p->fac_bytes;
  if (backward_ws) *backward_ws = p->bwd_bytes;
  return DNLS_OK;
}

static DenseArgs base_args(dnls_plan p) {
  DenseArgs a{};
  a.gd = p->d_gd;
  a.order = p->d_order;
  a.edge_ij = p->d_edge_ij;
  a.prior_var = p->d_prior_var;
  a.inc_off = p->d_inc_off;
  a.inc_slot = p->d_inc_slot;
  a.od_blk = p->d_od_blk;
  a.od_slot = p->d_od_slot;
  a.E = p->E;
  a.V = p->V;
  a.K = p->opt.iterations;
  a.refine = p->opt.precision == DNLS_PREC_MIXED ? p->opt.refine : 0;
  a.refine_from = p->opt.refine_last > 0 ? p->opt.iterations - p->opt.refine_last : 0;
  a.refine_until = p->opt.refine_last < 0 ? -p->opt.refine_last : p->opt.iterations;
  a.lambda = p->opt.lambda;
  return a;
}

// Enqueue the launch sequence of a multi-kernel solver (SPARSE, SCHUR) on
// `st`, through a captured HIP graph when DNLS_FLAG_GRAPH is set: the
// sequence is recorded once on a private stream and replayed while the
// argument pointers stay the same.
static dnls_status solve_multi(dnls_plan p, const dnls_solve_args* s, hipStream_t st) {
  auto enqueue = [&](hipStream_t q) {
    return p->opt.solver == DNLS_SOLVER_SCHUR ? ba_solve(p, s, q) : sp_solve(p, s, q);
  };
  if (!(p->opt.flags & DNLS_FLAG_GRAPH)) return enqueue(st);
  const std::vector<const void*> key = {s->poses, s->points, s->edge_meas, s->edge_logw, s->edge_tau,
                                        s->prior_meas, s->prior_logw, s->obs_uv, s->obs_w,
                                        s->objective, s->status, s->factor, s->workspace,
                                        s->edge_logc, s->huber_delta};
  std::lock_guard<std::mutex> lock(p->graph_mu);
  if (!p->graph_exec || p->graph_key != key) {
    if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const dnls_status est = enqueue(p->cap_stream);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(p->cap_stream, &graph);
    if (est != DNLS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return est;
    }
    if (ce != hipSuccess) return fail(DNLS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ce));
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return fail(DNLS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = exec;
    p->graph_key = key;
  }
  HIP_TRY(hipGraphLaunch(p->graph_exec, st));
  return DNLS_OK;
}

dnls_status dnls_solve(dnls_plan p, const dnls_solve_args* s, void* stream) {
  g_err.clear();
  if (!p || !s) return fail(DNLS_ERR_INVALID_ARG, "null argument");
  if (!s->poses || !s->objective || !s->status || !s->factor || !s->workspace)
    return fail(DNLS_ERR_INVALID_ARG, "poses, objective, status, factor and workspace are required");
  if ((reinterpret_cast<uintptr_t>(s->factor) & 255) || (reinterpret_cast<uintptr_t>(s->workspace) & 255))
    return fail(DNLS_ERR_WORKSPACE, "factor and workspace must be 256-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (p->opt.solver == DNLS_SOLVER_SCHUR || p->sp_ba) {
    if (!s->points || (p->O > 0 && (!s->obs_uv || !s->obs_w)) || (p->P > 0 && (!s->prior_meas || !s->prior_logw)))
      return fail(DNLS_ERR_INVALID_ARG, "points, obs_uv, obs_w and prior data are required");
    return solve_multi(p, s, st);
  }
  if ((p->E > 0 && (!s->edge_meas || !s->edge_logw)) || (p->P > 0 && (!s->prior_meas || !s->prior_logw)))
    return fail(DNLS_ERR_INVALID_ARG, "cost data pointers are required");
  if (p->opt.solver == DNLS_SOLVER_SPARSE) return solve_multi(p, s, st);
  DenseArgs a = base_args(p);
  a.poses = s->poses;
  a.edge_logc = s->edge_logc;
  a.edge_meas = s->edge_meas;
  a.edge_logw = s->edge_logw;
  a.edge_tau = s->edge_tau;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.objective = s->objective;
  a.status = s->status;
  a.factor = static_cast<double*>(s->factor);
  char* ws = static_cast<char*>(s->workspace);
  a.ws64 = reinterpret_cast<double*>(ws);
  a.ws32 = reinterpret_cast<float*>(ws + p->ws32_off);
  a.ycost = reinterpret_cast<double*>(ws + p->ycost_off);
  a.hbuf = reinterpret_cast<double*>(ws + p->h_off);
  a.pose_bak = reinterpret_cast<double*>(ws + p->bak_off);
  a.dlm_winv = reinterpret_cast<double*>(ws + p->dlmw_off);
  a.adaptive = (p->opt.flags & DNLS_FLAG_ADAPTIVE_LM) ? 1 : 0;
  a.dogleg = (p->opt.flags & DNLS_FLAG_DOGLEG) ? 1 : 0;
  a.radius0 = p->opt.trust_radius;
  a.traj = (p->opt.flags & DNLS_FLAG_KEEP_ITERATES) ? a.factor + p->traj_off : nullptr;
  const bool mixed = p->opt.precision == DNLS_PREC_MIXED;
  if (p->group == DNLS_SE3) return mixed ? launch_solve<3, true>(p, a, st) : launch_solve<3, false>(p, a, st);
  return mixed ? launch_solve<2, true>(p, a, st) : launch_solve<2, false>(p, a, st);
}

// ---------------------------------------------------------------------------
// dnls_solve_noalloc: dnls_solve with its workspace in a file-scope device
// array, for callers that cannot allocate (graph capture, serving loops).
// Each device that loads the library holds its own copy until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_addr;   // per device ordinal, set on the first call there

static dnls_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_addr.size()) g_scratch_addr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(DNLS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return DNLS_OK;
}

dnls_status dnls_solve_noalloc(dnls_plan p, const dnls_solve_args* s, void* stream) {
  g_err.clear();
  if (!p || !s) return fail(DNLS_ERR_INVALID_ARG, "null argument");
  if (s->workspace)
    return fail(DNLS_ERR_INVALID_ARG, "workspace must be NULL: dnls_solve_noalloc uses the library's scratch");
  if (p->opt.flags & DNLS_FLAG_GRAPH)
    return fail(DNLS_ERR_UNSUPPORTED, "dnls_solve_noalloc does not take DNLS_FLAG_GRAPH plans (instantiating "
                                      "a HIP graph allocates)");
  if (p->ws_bytes > kScratchBytes)
    return fail(DNLS_ERR_WORKSPACE, "the plan's solve workspace (" + std::to_string(p->ws_bytes) +
                                        " bytes) exceeds the scratch of dnls_solve_noalloc (" +
                                        std::to_string(kScratchBytes) + " bytes)");
  void* ws = nullptr;
  const dnls_status st = scratch_address(&ws);
  if (st != DNLS_OK) return st;
  dnls_solve_args a = *s;
  a.workspace = ws;
  return dnls_solve(p, &a, stream);
}

dnls_status dnls_backward(dnls_plan p, const dnls_backward_args* s, void* stream) {
  g_err.clear();
  if (!p || !s) return fail(DNLS_ERR_INVALID_ARG, "null argument");
  if (!s->poses || !s->status || !s->factor || !s->workspace || !s->seed_pose)
    return fail(DNLS_ERR_INVALID_ARG, "poses, status, factor, seed_pose and workspace are required");
  if ((reinterpret_cast<uintptr_t>(s->factor) & 255) || (reinterpret_cast<uintptr_t>(s->workspace) & 255))
    return fail(DNLS_ERR_WORKSPACE, "factor and workspace must be 256-byte aligned");
  if (s->mode < DNLS_BACKWARD_IMPLICIT || s->mode > DNLS_BACKWARD_UNROLL)
    return fail(DNLS_ERR_INVALID_ARG, "unknown backward mode");
  if (s->edge_logc && (s->mode == DNLS_BACKWARD_EXACT || s->mode == DNLS_BACKWARD_UNROLL))
    return fail(DNLS_ERR_UNSUPPORTED, "the exact-Hessian and unrolled backward do not take Welsch edges");
  if (s->mode == DNLS_BACKWARD_UNROLL) {
    if (!(p->opt.flags & DNLS_FLAG_KEEP_ITERATES))
      return fail(DNLS_ERR_INVALID_ARG, "the unrolled backward needs a plan with DNLS_FLAG_KEEP_ITERATES");
    if (s->steps < 1 || s->steps > p->opt.iterations)
      return fail(DNLS_ERR_INVALID_ARG, "steps must be in [1, iterations]");
  }
  if (s->mode == DNLS_BACKWARD_EXACT) {
    if (p->opt.solver == DNLS_SOLVER_SCHUR)
      return fail(DNLS_ERR_UNSUPPORTED, "the exact-Hessian backward is implemented for the pose-graph solvers");
    if (s->sweeps < 0 || s->sweeps > kMaxExactSweeps)
      return fail(DNLS_ERR_INVALID_ARG, "sweeps must be in [0, 64]");
  }
  if (s->mode == DNLS_BACKWARD_DLM) {
    if (!(s->dlm_eps > 0.0) || !std::isfinite(s->dlm_eps))
      return fail(DNLS_ERR_INVALID_ARG, "dlm_eps must be positive and finite");
  }
  if (p->opt.solver == DNLS_SOLVER_SCHUR) return ba_backward(p, s, static_cast<hipStream_t>(stream));
  if (p->opt.solver == DNLS_SOLVER_SPARSE) return sp_backward(p, s, static_cast<hipStream_t>(stream));
  DenseArgs a = base_args(p);
  a.poses = const_cast<double*>(s->poses);
  a.edge_meas = s->edge_meas;
  a.edge_logw = s->edge_logw;
  a.edge_tau = s->edge_tau;
  a.prior_meas = s->prior_meas;
  a.prior_logw = s->prior_logw;
  a.status = const_cast<int*>(s->status);
  a.factor = const_cast<double*>(static_cast<const double*>(s->factor));
  char* ws = static_cast<char*>(s->workspace);
  a.ws64 = reinterpret_cast<double*>(ws);
  a.ycost = reinterpret_cast<double*>(ws + p->ycost_off);
  a.hbuf = reinterpret_cast<double*>(ws + p->h_off);
  a.pose_bak = reinterpret_cast<double*>(ws + p->bak_off);
  a.dlm_winv = reinterpret_cast<double*>(ws + p->dlmw_off);
  a.hvp = reinterpret_cast<double*>(ws + p->hvp_off);
  a.traj = (p->opt.flags & DNLS_FLAG_KEEP_ITERATES) ? a.factor + p->traj_off : nullptr;
  a.seed = s->seed_pose;
  a.adj_refine = p->opt.precision == DNLS_PREC_MIXED ? 0 : 1;
  a.g_logw_e = s->grad_edge_logw;
  a.g_tau = s->grad_edge_tau;
  a.g_logw_p = s->grad_prior_logw;
  a.edge_logc = s->edge_logc;
  a.g_logc = s->grad_edge_logc;
  a.adjoint_out = s->adjoint;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the cached factor is float64-assembled in both precisions
  const int count = s->mode == DNLS_BACKWARD_UNROLL ? s->steps : s->sweeps;
  if (p->group == DNLS_SE3) return launch_backward<3>(p, a, st, s->mode, s->dlm_eps, count);
  return launch_backward<2>(p, a, st, s->mode, s->dlm_eps, count);
}

dnls_status dnls_project_grad(int32_t group, int64_t n, const double* poses, const double* grad, double* out,
                              void* stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!poses || !grad || !out))) return fail(DNLS_ERR_INVALID_ARG, "bad arguments");
  if (group != DNLS_SE2 && group != DNLS_SE3) return fail(DNLS_ERR_INVALID_ARG, "group must be SE2 or SE3");
  if (n == 0) return DNLS_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nt = 256;
  const unsigned nb = (unsigned)((n + nt - 1) / nt);
  if (group == DNLS_SE3) hipLaunchKernelGGL(k_project<3>, dim3(nb), dim3(nt), 0, st, (long long)n, poses, grad, out);
  else hipLaunchKernelGGL(k_project<2>, dim3(nb), dim3(nt), 0, st, (long long)n, poses, grad, out);
  HIP_TRY(hipGetLastError());
  return DNLS_OK;
}

dnls_status dnls_plan_destroy(dnls_plan p) {
  if (!p) return DNLS_OK;
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  for (void* q : p->allocs) (void)hipFree(q);
  delete p;
  return DNLS_OK;
}

}  // extern "C"
