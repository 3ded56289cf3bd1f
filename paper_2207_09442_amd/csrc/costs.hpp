// Cost functions of the DNLS objective (Eq. nls): residual blocks and their
// Jacobians with respect to right perturbations (Appendix D).
//
//   relative pose  c = Log(Z^-1 X_i^-1 X_j)          (Appendix E.1)
//                  dc/dxi_j = Jr^-1(c),  dc/dxi_i = -Jr^-1(c) Ad(X_j^-1 X_i)
//   prior          c = Log(P^-1 X),       dc/dxi = Jr^-1(c)
//
// Group products of the float64 poses (the relative transforms) are formed
// in float64; the logarithm and Jacobians are then evaluated in the working
// precision S (float for the mixed path, double otherwise).  A cost writes
// its weighted Jacobians w C_i, w C_j (d x d, row-major: row = residual
// component) and its weighted residual w c into a record of kCost<d> values.
#pragma once

#include "lie.hpp"

namespace dnls {

template <int G> struct GroupTraits;
template <> struct GroupTraits<3> { static constexpr int d = 6, sz = 12; };
template <> struct GroupTraits<2> { static constexpr int d = 3, sz = 4; };

template <int d> struct CostRec { static constexpr int n = 2 * d * d + d; };

// measurement with an optional tangent perturbation: Z Exp(tau)
template <int G>
DNLS_HD void perturbed_meas(const double* Z, const double* tau, double* out) {
  constexpr int sz = GroupTraits<G>::sz;
  if (!tau) {
#pragma unroll
    for (int k = 0; k < sz; ++k) out[k] = Z[k];
    return;
  }
  double E[sz];
  if constexpr (G == 3) {
    se3_exp(tau, E);
    se3_mul(Z, E, out);
  } else {
    se2_exp(tau, E);
    se2_mul(Z, E, out);
  }
}

// Between cost.  Xi, Xj, Z in storage layout.  Outputs (unweighted) c[d],
// Ci[d*d], Cj[d*d] in precision S.
template <int G, class S>
DNLS_HD void between_cost(const double* Xi, const double* Xj, const double* Z, S* c, S* Ci, S* Cj) {
  if constexpr (G == 3) {
    double Xii[12], D[12], Zi[12], E[12], M[12];
    se3_inv(Xi, Xii);
    se3_mul(Xii, Xj, D);     // X_i^-1 X_j
    se3_inv(Z, Zi);
    se3_mul(Zi, D, E);       // Z^-1 X_i^-1 X_j
    se3_inv(D, M);           // X_j^-1 X_i
    S R[9], t[3], RM[9], tM[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        R[r * 3 + q] = S(E[r * 4 + q]);
        RM[r * 3 + q] = S(M[r * 4 + q]);
      }
      t[r] = S(E[r * 4 + 3]);
      tM[r] = S(M[r * 4 + 3]);
    }
    se3_log(R, t, c);
    S Jr[36], Ad[36];
    se3_jr_inv(c, Jr);
    se3_adjoint(RM, tM, Ad);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        S acc = S(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += Jr[r * 6 + k] * Ad[k * 6 + q];
        Ci[r * 6 + q] = -acc;
        Cj[r * 6 + q] = Jr[r * 6 + q];
      }
  } else {
    double Xii[4], D[4], Zi[4], E[4], M[4];
    se2_inv(Xi, Xii);
    se2_mul(Xii, Xj, D);
    se2_inv(Z, Zi);
    se2_mul(Zi, D, E);
    se2_inv(D, M);
    se2_log(S(E[0]), S(E[1]), S(E[2]), S(E[3]), c);
    S Jr[9], Ad[9];
    se2_jr_inv(c, Jr);
    se2_adjoint(S(M[0]), S(M[1]), S(M[2]), S(M[3]), Ad);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        S acc = S(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc += Jr[r * 3 + k] * Ad[k * 3 + q];
        Ci[r * 3 + q] = -acc;
        Cj[r * 3 + q] = Jr[r * 3 + q];
      }
  }
}

template <int G, class S>
DNLS_HD void prior_cost(const double* X, const double* P, S* c, S* C) {
  if constexpr (G == 3) {
    double Pi[12], E[12];
    se3_inv(P, Pi);
    se3_mul(Pi, X, E);
    S R[9], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int q = 0; q < 3; ++q) R[r * 3 + q] = S(E[r * 4 + q]);
      t[r] = S(E[r * 4 + 3]);
    }
    se3_log(R, t, c);
    se3_jr_inv(c, C);
  } else {
    double Pi[4], E[4];
    se2_inv(P, Pi);
    se2_mul(Pi, X, E);
    se2_log(S(E[0]), S(E[1]), S(E[2]), S(E[3]), c);
    se2_jr_inv(c, C);
  }
}

// Right retraction X <- X Exp(-delta) in float64.
template <int G>
DNLS_HD void retract_minus(double* X, const double* delta) {
  constexpr int d = GroupTraits<G>::d, sz = GroupTraits<G>::sz;
  double m[d], E[sz], Y[sz];
#pragma unroll
  for (int k = 0; k < d; ++k) m[k] = -delta[k];
  if constexpr (G == 3) {
    se3_exp(m, E);
    se3_mul(X, E, Y);
  } else {
    se2_exp(m, E);
    se2_mul(X, E, Y);
    // keep (cos, sin) on the unit circle
    const double n = ::sqrt(Y[2] * Y[2] + Y[3] * Y[3]);
    Y[2] /= n;
    Y[3] /= n;
  }
#pragma unroll
  for (int k = 0; k < sz; ++k) X[k] = Y[k];
}

// d/ds [Jl^-1(c(s))^T c(s)] at s = 0 along cdot = dc/ds, by one pass of
// forward-mode dual numbers through the closed-form inverse left Jacobian
// (Jl^-1(c) = Jr^-1(-c)).
template <int G>
DNLS_HD void dual_jlinvT_c(const double* c, const double* cdot, double* out) {
  constexpr int d = GroupTraits<G>::d;
  using D = Dual<double>;
  D xi[d], J[d * d];
#pragma unroll
  for (int k = 0; k < d; ++k) xi[k] = D(-c[k], -cdot[k]);
  if constexpr (G == 3)
    se3_jr_inv(xi, J);
  else
    se2_jr_inv(xi, J);
#pragma unroll
  for (int q = 0; q < d; ++q) {
    D acc(0.0);
#pragma unroll
    for (int k = 0; k < d; ++k) acc += J[k * d + q] * D(c[k], cdot[k]);
    out[q] = acc.d;
  }
}

}  // namespace dnls
