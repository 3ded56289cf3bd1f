// Per-cost kernels of the pose-graph objective shared by the dense and the
// block-sparse paths: linearisation of one cost into its record
// (w C_i, w C_j, w c) and the per-cost vector-Jacobian product of the
// implicit backward (Proposition 1):
//   dL/dl_e   = -2 (J u)^T r                        (w = exp(l), J = w C, r = w c)
//   dL/dtau_e = w^2 d/ds [Jl^-1(c(s))^T c(s)]        along c' = C u, then the
//               chain rule Jr(tau)^T for a non-zero base tau
// The tau formula follows from dc/dtau = -Jl^-1(c) and the symmetry of
// mixed partial derivatives of 1/2 ||c(theta (+) s u, tau)||^2.
#pragma once

#include "costs.hpp"

namespace dnls {

struct PoseCostData {
  const int* edge_ij;       // [E][2] global pose indices
  const int* prior_var;     // [P]
  const double* poses;
  const double* edge_meas;
  const double* edge_logw;
  const double* edge_tau;   // may be null
  const double* prior_meas;
  const double* prior_logw;
  int E;                    // records: edges [0, E), priors [E, E + P)
};

// Linearise cost k (record index) into rec (CostRec<d>::n values of S);
// returns 1/2 w^2 ||c||^2.
template <int G, class S>
__device__ __forceinline__ double linearize_cost(const PoseCostData& a, int k, S* rec) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  S c[d], Ci[d * d], Cj[d * d];
  double w;
  if (k < a.E) {
    const int i = a.edge_ij[2 * k], j = a.edge_ij[2 * k + 1];
    double Z[sz];
    perturbed_meas<G>(a.edge_meas + (size_t)k * sz, a.edge_tau ? a.edge_tau + (size_t)k * d : nullptr, Z);
    between_cost<G, S>(a.poses + (size_t)i * sz, a.poses + (size_t)j * sz, Z, c, Ci, Cj);
    w = exp(a.edge_logw[k]);
  } else {
    const int p = k - a.E;
    prior_cost<G, S>(a.poses + (size_t)a.prior_var[p] * sz, a.prior_meas + (size_t)p * sz, c, Cj);
#pragma unroll
    for (int q = 0; q < d * d; ++q) Ci[q] = S(0);
    w = exp(a.prior_logw[p]);
  }
  const S ws = S(w);
  double cc = 0.0;
#pragma unroll
  for (int q = 0; q < d * d; ++q) {
    rec[q] = ws * Ci[q];
    rec[d * d + q] = ws * Cj[q];
  }
#pragma unroll
  for (int q = 0; q < d; ++q) {
    rec[2 * d * d + q] = ws * c[q];
    cc += double(c[q]) * double(c[q]);
  }
  return 0.5 * w * w * cc;
}

// 1/2 w^2 ||c||^2 of cost k in float64 (residual only: the Jacobian outputs
// of the cost functions are dead and removed by the compiler).
template <int G>
__device__ __forceinline__ double cost_objective(const PoseCostData& a, int k) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  double c[d], Ci[d * d], Cj[d * d];
  double w;
  if (k < a.E) {
    const int i = a.edge_ij[2 * k], j = a.edge_ij[2 * k + 1];
    double Z[sz];
    perturbed_meas<G>(a.edge_meas + (size_t)k * sz, a.edge_tau ? a.edge_tau + (size_t)k * d : nullptr, Z);
    between_cost<G, double>(a.poses + (size_t)i * sz, a.poses + (size_t)j * sz, Z, c, Ci, Cj);
    w = exp(a.edge_logw[k]);
  } else {
    const int p = k - a.E;
    prior_cost<G, double>(a.poses + (size_t)a.prior_var[p] * sz, a.prior_meas + (size_t)p * sz, c, Cj);
    w = exp(a.prior_logw[p]);
  }
  double cc = 0.0;
#pragma unroll
  for (int q = 0; q < d; ++q) cc += c[q] * c[q];
  return 0.5 * w * w * cc;
}

// Parameter gradient of the cost's 1/2 w^2 ||c||^2 at the current poses
// (direct loss minimisation): dS/dl = w^2 ||c||^2 and, for an edge,
//   dS/dtau = -w^2 Jr(tau0)^T Jl^-1(c)^T c,  Jl^-1(c) = Jr^-1(-c),
// from dc/dtau = -Jl^-1(c) Jr(tau0) for Z <- Z Exp(tau) at the base tau0.
template <int G>
__device__ __forceinline__ void cost_param_grad(const PoseCostData& a, int k, double* dl, double* dtau) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  double c[d], Ci[d * d], Cj[d * d];
  double w;
  const bool edge = k < a.E;
  if (edge) {
    const int i = a.edge_ij[2 * k], j = a.edge_ij[2 * k + 1];
    double Z[sz];
    perturbed_meas<G>(a.edge_meas + (size_t)k * sz, a.edge_tau ? a.edge_tau + (size_t)k * d : nullptr, Z);
    between_cost<G, double>(a.poses + (size_t)i * sz, a.poses + (size_t)j * sz, Z, c, Ci, Cj);
    w = exp(a.edge_logw[k]);
  } else {
    const int p = k - a.E;
    prior_cost<G, double>(a.poses + (size_t)a.prior_var[p] * sz, a.prior_meas + (size_t)p * sz, c, Cj);
    w = exp(a.prior_logw[p]);
  }
  double cc = 0.0;
#pragma unroll
  for (int q = 0; q < d; ++q) cc += c[q] * c[q];
  *dl = w * w * cc;
  if (!edge) return;
  double mc[d], Jl[d * d], t[d];
#pragma unroll
  for (int q = 0; q < d; ++q) mc[q] = -c[q];
  if constexpr (G == 3) se3_jr_inv(mc, Jl);
  else se2_jr_inv(mc, Jl);
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) acc += Jl[q * d + m] * c[q];
    t[m] = acc;
  }
  if (a.edge_tau) {
    double Jr[d * d], t0[d];
    const double* tau0 = a.edge_tau + (size_t)k * d;
#pragma unroll
    for (int q = 0; q < d; ++q) t0[q] = tau0[q];
    if constexpr (G == 3) se3_jr(t0, Jr);
    else se2_jr(t0, Jr);
    double u[d];
#pragma unroll
    for (int m = 0; m < d; ++m) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < d; ++q) acc += Jr[q * d + m] * t[q];
      u[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < d; ++m) t[m] = u[m];
  }
#pragma unroll
  for (int m = 0; m < d; ++m) dtau[m] = -w * w * t[m];
}

// Per-cost VJP of cost k from its float64 record and the adjoint u of its
// poses (ui is null for a prior).  Null gradient outputs are skipped.
template <int G>
__device__ __forceinline__ void cost_vjp(const PoseCostData& a, int k, const double* rec, const double* ui,
                                         const double* uj, double* g_logw_e, double* g_tau, double* g_logw_p) {
  constexpr int d = GroupTraits<G>::d;
  const double* r = rec + 2 * d * d;
  double y[d], yr = 0.0;
#pragma unroll
  for (int q = 0; q < d; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < d; ++m) {
      if (ui) acc += rec[q * d + m] * ui[m];
      acc += rec[d * d + q * d + m] * uj[m];
    }
    y[q] = acc;
    yr += acc * r[q];
  }
  if (k >= a.E) {
    if (g_logw_p) g_logw_p[k - a.E] = -2.0 * yr;
    return;
  }
  if (g_logw_e) g_logw_e[k] = -2.0 * yr;
  if (!g_tau) return;
  const double w = exp(a.edge_logw[k]);
  double c[d], cd[d], out[d];
#pragma unroll
  for (int q = 0; q < d; ++q) {
    c[q] = r[q] / w;
    cd[q] = y[q] / w;
  }
  dual_jlinvT_c<G>(c, cd, out);
  double gt[d];
#pragma unroll
  for (int q = 0; q < d; ++q) gt[q] = w * w * out[q];
  if (a.edge_tau) {
    // Exp(tau + dt) = Exp(tau) Exp(Jr(tau) dt)  =>  dL/dtau = Jr(tau)^T dL/dxi
    double tau[d], Jt[d * d];
#pragma unroll
    for (int q = 0; q < d; ++q) tau[q] = a.edge_tau[(size_t)k * d + q];
    if constexpr (G == 3)
      se3_jr(tau, Jt);
    else
      se2_jr(tau, Jt);
#pragma unroll
    for (int q = 0; q < d; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < d; ++m) acc += Jt[m * d + q] * gt[m];
      g_tau[(size_t)k * d + q] = acc;
    }
  } else {
#pragma unroll
    for (int q = 0; q < d; ++q) g_tau[(size_t)k * d + q] = gt[q];
  }
}

}  // namespace dnls
