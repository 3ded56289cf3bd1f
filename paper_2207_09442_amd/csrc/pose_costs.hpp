// Per-cost kernels of the pose-graph objective shared by the dense and the
// block-sparse paths: linearisation of one cost into its record
// (w C_i, w C_j, w c) and the per-cost vector-Jacobian product of the
// implicit backward (Proposition 1):
//   dL/dl_e   = -2 (J u)^T r                        (w = exp(l), J = w C, r = w c)
//   dL/dtau_e = w^2 d/ds [Jl^-1(c(s))^T c(s)]        along c' = C u, then the
//               chain rule Jr(tau)^T for a non-zero base tau
// The tau formula follows from dc/dtau = -Jl^-1(c) and the symmetry of
// mixed partial derivatives of 1/2 ||c(theta (+) s u, tau)||^2.
//
// Edges may carry a Welsch robust loss with radius c_e = exp(logc_e):
// rho(s) = c^2 (1 - exp(-s / c^2)) on s = ||w c||^2, applied by first-order
// reweighting (J and r scaled by sqrt(rho'(s)), rho'(s) = exp(-s / c^2)) and
// objective 1/2 rho(s).
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
  const double* edge_logc;  // [E] Welsch log-radii, or null (plain least squares)
};

// Welsch reweighting of edge k at squared weighted residual s: returns
// rho'(s) and sets *half_rho = rho(s) / 2, *x = s / c^2.
DNLS_HD double welsch_weight(const PoseCostData& a, int k, double s, double* half_rho, double* x) {
  const double c2 = exp(2.0 * a.edge_logc[k]);
  *x = s / c2;
  *half_rho = -0.5 * c2 * expm1(-*x);
  return exp(-*x);
}

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
  double cc = 0.0;
#pragma unroll
  for (int q = 0; q < d; ++q) cc += double(c[q]) * double(c[q]);
  double obj = 0.5 * w * w * cc;
  if (k < a.E && a.edge_logc) {
    double x;
    w *= ::sqrt(welsch_weight(a, k, w * w * cc, &obj, &x));
  }
  const S ws = S(w);
#pragma unroll
  for (int q = 0; q < d * d; ++q) {
    rec[q] = ws * Ci[q];
    rec[d * d + q] = ws * Cj[q];
  }
#pragma unroll
  for (int q = 0; q < d; ++q) rec[2 * d * d + q] = ws * c[q];
  return obj;
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
  double obj = 0.5 * w * w * cc;
  if (k < a.E && a.edge_logc) {
    double x;
    welsch_weight(a, k, w * w * cc, &obj, &x);
  }
  return obj;
}

// t = Jr(tau0)^T Jl^-1(c)^T c for edge k, Jl^-1(c) = Jr^-1(-c): minus the
// tau-gradient of 1/2 ||c||^2 through dc/dtau = -Jl^-1(c) Jr(tau0) for
// Z <- Z Exp(tau) at the base tau0 (the chain factor is I when tau is absent).
template <int G>
DNLS_HD void tau_pullback_c(const PoseCostData& a, int k, const double* c, double* t) {
  constexpr int d = GroupTraits<G>::d;
  double mc[d], Jl[d * d];
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
    double Jr[d * d], t0[d], u[d];
#pragma unroll
    for (int q = 0; q < d; ++q) t0[q] = a.edge_tau[(size_t)k * d + q];
    if constexpr (G == 3) se3_jr(t0, Jr);
    else se2_jr(t0, Jr);
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
}

// Parameter gradient of the cost's share of the objective at the current
// poses (direct loss minimisation): plain cost 1/2 w^2 ||c||^2 gives
// dS/dl = w^2 ||c||^2 = s and, for an edge, dS/dtau = -w^2 Jr(tau0)^T Jl^-1(c)^T c;
// a Welsch edge 1/2 rho(s) gives dS/dl = rho'(s) s, dS/dtau = rho'(s) x the
// plain one and dS/dlogc = rho(s) - rho'(s) s (dlc may be null).
template <int G>
__device__ __forceinline__ void cost_param_grad(const PoseCostData& a, int k, double* dl, double* dtau, double* dlc) {
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
  const double s = w * w * cc;
  *dl = s;
  if (!edge) return;
  double rp = 1.0;
  if (a.edge_logc) {
    double half_rho, x;
    rp = welsch_weight(a, k, s, &half_rho, &x);
    *dl = rp * s;
    if (dlc) *dlc = 2.0 * half_rho - rp * s;
  }
  double t[d];
  tau_pullback_c<G>(a, k, c, t);
#pragma unroll
  for (int m = 0; m < d; ++m) dtau[m] = -rp * w * w * t[m];
}

// out = ad(x)^T v, with ad(x) the linearisation of Ad(Exp(s x)) = I + s ad(x):
// SE(3), x = (rho, phi): ad = [[phi^, rho^], [0, phi^]], so
//   ad^T v = (-phi x v_rho, -rho x v_rho - phi x v_phi);
// SE(2), x = (x, y, th): ad = [[0, -th, y], [th, 0, -x], [0, 0, 0]].
template <int G>
DNLS_HD void ad_transpose_mul(const double* x, const double* v, double* out) {
  if constexpr (G == 3) {
    double a[3], b[3];
    cross3(x + 3, v, a);
    cross3(x, v, b);
    out[0] = -a[0];
    out[1] = -a[1];
    out[2] = -a[2];
    cross3(x + 3, v + 3, a);
    out[3] = -b[0] - a[0];
    out[4] = -b[1] - a[1];
    out[5] = -b[2] - a[2];
  } else {
    out[0] = x[2] * v[1];
    out[1] = -x[2] * v[0];
    out[2] = x[1] * v[0] - x[0] * v[1];
  }
}

// Second-order (residual) part of the exact Hessian-vector product for cost
// k along the pose directions xi, xj (xi null for a prior): with
// c(s) = c at X_i Exp(s xi), X_j Exp(s xj), this is w^2 (dC/ds)^T c for each
// side, the term that the Gauss-Newton product w^2 C^T C x leaves out.
//   dC_j/ds = D Jr^-1(c)[c'],  c' = C_i xi + C_j xj   (one dual-number pass)
//   dC_i/ds = -D Jr^-1(c)[c'] Ad(T) - Jr^-1(c) (Ad(T) ad(xi) - ad(xj) Ad(T)),
//   T = X_j^-1 X_i, from Ad(Exp(-s xj) T Exp(s xi)).
// rec is the cost's float64 record (w C_i, w C_j, w c).
template <int G>
DNLS_HD void cost_hvp_residual(const PoseCostData& a, int k, const double* rec, const double* xi,
                               const double* xj, double* oi, double* oj) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  const bool edge = k < a.E;
  const double w = exp(edge ? a.edge_logw[k] : a.prior_logw[k - a.E]);
  const double* r = rec + 2 * d * d;
  Dual<double> cd[d];
#pragma unroll
  for (int q = 0; q < d; ++q) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < d; ++m) {
      if (edge) acc += rec[q * d + m] * xi[m];
      acc += rec[d * d + q * d + m] * xj[m];
    }
    cd[q] = Dual<double>(r[q] / w, acc / w);
  }
  Dual<double> J[d * d];
  if constexpr (G == 3) se3_jr_inv(cd, J);
  else se2_jr_inv(cd, J);
  // av = Jr^-T c, bv = (D Jr^-1)^T c, scaled by w^2 through r = w c
  double av[d], bv[d];
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      sa += J[q * d + m].v * r[q];
      sb += J[q * d + m].d * r[q];
    }
    av[m] = w * sa;
    bv[m] = w * sb;
  }
#pragma unroll
  for (int m = 0; m < d; ++m) oj[m] = bv[m];
  if (!edge) return;
  const int i = a.edge_ij[2 * k], j = a.edge_ij[2 * k + 1];
  double Ad[d * d];
  if constexpr (G == 3) {
    double Xji[12], M[12];
    se3_inv(a.poses + (size_t)j * sz, Xji);
    se3_mul(Xji, a.poses + (size_t)i * sz, M);
    double RM[9], tM[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
#pragma unroll
      for (int q = 0; q < 3; ++q) RM[rr * 3 + q] = M[rr * 4 + q];
      tM[rr] = M[rr * 4 + 3];
    }
    se3_adjoint(RM, tM, Ad);
  } else {
    double Xji[4], M[4];
    se2_inv(a.poses + (size_t)j * sz, Xji);
    se2_mul(Xji, a.poses + (size_t)i * sz, M);
    se2_adjoint(M[0], M[1], M[2], M[3], Ad);
  }
  // oi = Ad^T (ad(xj)^T av - bv) - ad(xi)^T Ad^T av
  double ta[d], tj[d], ti[d];
  ad_transpose_mul<G>(xj, av, tj);
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      s1 += Ad[q * d + m] * av[q];
      s2 += Ad[q * d + m] * (tj[q] - bv[q]);
    }
    ta[m] = s1;
    oi[m] = s2;
  }
  ad_transpose_mul<G>(xi, ta, ti);
#pragma unroll
  for (int m = 0; m < d; ++m) oi[m] -= ti[m];
}

// One cost's part of the reverse step through delta = (H + lambda I)^-1 g
// (unrolled differentiation): with y = (H + lambda I)^-1 dL/ddelta and delta
// held fixed, the gradient of s = (J y)^T (r - J delta) = w^2 (C y)^T e,
// e = c - C delta, with respect to right perturbations of the cost's poses
// (oi, oj; oi unused for a prior), its log-weight (2 s) and its measurement
// tangent.  With u1 = y_j - Ad(T) y_i and u2 = delta_j - Ad(T) delta_i
// (T = X_j^-1 X_i; y_j and delta_j alone for a prior), C y = Jr^-1(c) u1 and
// C delta = Jr^-1(c) u2, so through c
//   ds/dc = w^2 (C y + G),  G_m = e^T (dJr^-1/dc_m) u1 - (C y)^T (dJr^-1/dc_m) u2
// (one dual-number pass per component of c), moved to the poses by C^T; the
// pose dependence of Ad(T), d/ds Ad = Ad ad(x_i) - ad(x_j) Ad, adds
//   oi += w^2 (ad(y_i)^T Ad^T p - ad(delta_i)^T Ad^T q),
//   oj += w^2 (-ad(Ad y_i)^T p + ad(Ad delta_i)^T q),  p = Jr^-T e, q = Jr^-T C y;
// and dc/dtau = -Jl^-1(c) Jr(tau0) gives the tangent gradient.
template <int G>
DNLS_HD void cost_unroll_vjp(const PoseCostData& a, int k, const double* yi, const double* yj, const double* di,
                             const double* dj, double* oi, double* oj, double* dlogw, double* dtau) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  const bool edge = k < a.E;
  double c[d], Ci[d * d], Jinv[d * d], Ad[d * d], w;
  if (edge) {
    const int i = a.edge_ij[2 * k], j = a.edge_ij[2 * k + 1];
    double Z[sz];
    perturbed_meas<G>(a.edge_meas + (size_t)k * sz, a.edge_tau ? a.edge_tau + (size_t)k * d : nullptr, Z);
    between_cost<G, double>(a.poses + (size_t)i * sz, a.poses + (size_t)j * sz, Z, c, Ci, Jinv);
    w = exp(a.edge_logw[k]);
    if constexpr (G == 3) {
      double Xji[12], M[12], RM[9], tM[3];
      se3_inv(a.poses + (size_t)j * sz, Xji);
      se3_mul(Xji, a.poses + (size_t)i * sz, M);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int q = 0; q < 3; ++q) RM[r * 3 + q] = M[r * 4 + q];
        tM[r] = M[r * 4 + 3];
      }
      se3_adjoint(RM, tM, Ad);
    } else {
      double Xji[4], M[4];
      se2_inv(a.poses + (size_t)j * sz, Xji);
      se2_mul(Xji, a.poses + (size_t)i * sz, M);
      se2_adjoint(M[0], M[1], M[2], M[3], Ad);
    }
  } else {
    const int p = k - a.E;
    prior_cost<G, double>(a.poses + (size_t)a.prior_var[p] * sz, a.prior_meas + (size_t)p * sz, c, Jinv);
    w = exp(a.prior_logw[p]);
  }
  const double w2 = w * w;
  double u1[d], u2[d], Ayi[d], Adi[d];
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double s1 = 0.0, s2 = 0.0;
    if (edge)
#pragma unroll
      for (int q = 0; q < d; ++q) {
        s1 += Ad[m * d + q] * yi[q];
        s2 += Ad[m * d + q] * di[q];
      }
    Ayi[m] = s1;
    Adi[m] = s2;
    u1[m] = yj[m] - s1;
    u2[m] = dj[m] - s2;
  }
  double Cy[d], e[d];
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      s1 += Jinv[m * d + q] * u1[q];
      s2 += Jinv[m * d + q] * u2[q];
    }
    Cy[m] = s1;
    e[m] = c[m] - s2;
  }
  double sval = 0.0;
#pragma unroll
  for (int m = 0; m < d; ++m) sval += Cy[m] * e[m];
  *dlogw = 2.0 * w2 * sval;
  // ds/dc
  double gc[d];
#pragma unroll 1
  for (int m = 0; m < d; ++m) {
    Dual<double> cd[d], J[d * d];
#pragma unroll
    for (int q = 0; q < d; ++q) cd[q] = Dual<double>(c[q], q == m ? 1.0 : 0.0);
    if constexpr (G == 3) se3_jr_inv(cd, J);
    else se2_jr_inv(cd, J);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < d; ++r) {
      double t1 = 0.0, t2 = 0.0;
#pragma unroll
      for (int q = 0; q < d; ++q) {
        t1 += J[r * d + q].d * u1[q];
        t2 += J[r * d + q].d * u2[q];
      }
      acc += e[r] * t1 - Cy[r] * t2;
    }
    gc[m] = w2 * (Cy[m] + acc);
  }
  // through c: C_j = Jr^-1, C_i = -Jr^-1 Ad
  double jg[d];
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) acc += Jinv[q * d + m] * gc[q];
    jg[m] = acc;
    oj[m] = acc;
  }
  if (!edge) return;
  double pv[d], qv[d];
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      s1 += Jinv[q * d + m] * e[q];
      s2 += Jinv[q * d + m] * Cy[q];
    }
    pv[m] = s1;
    qv[m] = s2;
  }
  double Ap[d], Aq[d], t1[d], t2[d];
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      s1 += Ad[q * d + m] * jg[q];
      s2 += Ad[q * d + m] * pv[q];
      s3 += Ad[q * d + m] * qv[q];
    }
    oi[m] = -s1;
    Ap[m] = s2;
    Aq[m] = s3;
  }
  ad_transpose_mul<G>(yi, Ap, t1);
  ad_transpose_mul<G>(di, Aq, t2);
#pragma unroll
  for (int m = 0; m < d; ++m) oi[m] += w2 * (t1[m] - t2[m]);
  ad_transpose_mul<G>(Ayi, pv, t1);
  ad_transpose_mul<G>(Adi, qv, t2);
#pragma unroll
  for (int m = 0; m < d; ++m) oj[m] += w2 * (t2[m] - t1[m]);
  if (!dtau) return;
  // dtau = -Jr(tau0)^T Jl^-T(c) ds/dc,  Jl^-1(c) = Jr^-1(-c)
  double mc[d], Jl[d * d], tt[d];
#pragma unroll
  for (int q = 0; q < d; ++q) mc[q] = -c[q];
  if constexpr (G == 3) se3_jr_inv(mc, Jl);
  else se2_jr_inv(mc, Jl);
#pragma unroll
  for (int m = 0; m < d; ++m) {
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) acc += Jl[q * d + m] * gc[q];
    tt[m] = acc;
  }
  if (a.edge_tau) {
    double Jr[d * d], t0[d];
#pragma unroll
    for (int q = 0; q < d; ++q) t0[q] = a.edge_tau[(size_t)k * d + q];
    if constexpr (G == 3) se3_jr(t0, Jr);
    else se2_jr(t0, Jr);
#pragma unroll
    for (int m = 0; m < d; ++m) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < d; ++q) acc += Jr[q * d + m] * tt[q];
      dtau[m] = -acc;
    }
  } else {
#pragma unroll
    for (int m = 0; m < d; ++m) dtau[m] = -tt[m];
  }
}

// Per-cost VJP of cost k from its float64 record and the adjoint u of its
// poses (ui is null for a prior).  Null gradient outputs are skipped.  For a
// Welsch edge the record holds the reweighted J~, r~ (factor sqrt(rho')), so
// (J~ u)^T r~ = rho'(s) (J u)^T r =: yr and, with x = s / c^2,
//   dL/dl = -2 yr (1 - x),  dL/dlogc = -2 x yr,
//   dL/dtau = rho' x (plain formula) - (2 w^2 / c^2) yr Jr(tau0)^T Jl^-1(c)^T c,
// the last term from rho'' = -rho' / c^2 and ds/dtau.
template <int G>
__device__ __forceinline__ void cost_vjp(const PoseCostData& a, int k, const double* rec, const double* ui,
                                         const double* uj, double* g_logw_e, double* g_tau, double* g_logw_p,
                                         double* g_logc) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
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
  const double w = exp(a.edge_logw[k]);
  double w2eff = w * w, c[d], cd[d];   // w^2 (rho'(s) w^2 for a Welsch edge); c; c' = C u
  double robust_tau = 0.0;             // coefficient of Jr(tau0)^T Jl^-1(c)^T c in dL/dtau
  if (a.edge_logc) {
    // the raw residual and Jacobians (the record holds the reweighted ones,
    // which vanish where rho' underflows on a gross outlier)
    const int i = a.edge_ij[2 * k], j = a.edge_ij[2 * k + 1];
    double Z[sz], Ci[d * d], Cj[d * d];
    perturbed_meas<G>(a.edge_meas + (size_t)k * sz, a.edge_tau ? a.edge_tau + (size_t)k * d : nullptr, Z);
    between_cost<G, double>(a.poses + (size_t)i * sz, a.poses + (size_t)j * sz, Z, c, Ci, Cj);
    double cc = 0.0;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      cc += c[q] * c[q];
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < d; ++m) acc += Ci[q * d + m] * ui[m] + Cj[q * d + m] * uj[m];
      cd[q] = acc;
    }
    double half_rho, x;
    const double rp = welsch_weight(a, k, w * w * cc, &half_rho, &x);
    w2eff = rp * w * w;
    if (g_logw_e) g_logw_e[k] = -2.0 * yr * (1.0 - x);
    if (g_logc) g_logc[k] = -2.0 * x * yr;
    robust_tau = -2.0 * w * w * exp(-2.0 * a.edge_logc[k]) * yr;
  } else {
    if (g_logw_e) g_logw_e[k] = -2.0 * yr;
#pragma unroll
    for (int q = 0; q < d; ++q) {
      c[q] = r[q] / w;
      cd[q] = y[q] / w;
    }
  }
  if (!g_tau) return;
  double out[d];
  dual_jlinvT_c<G>(c, cd, out);
  double gt[d];
#pragma unroll
  for (int q = 0; q < d; ++q) gt[q] = w2eff * out[q];
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
  if (robust_tau != 0.0) {
    double t[d];
    tau_pullback_c<G>(a, k, c, t);
#pragma unroll
    for (int q = 0; q < d; ++q) g_tau[(size_t)k * d + q] += robust_tau * t[q];
  }
}

}  // namespace dnls
