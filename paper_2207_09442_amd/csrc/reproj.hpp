// Pinhole reprojection cost of bundle adjustment and the Huber robust loss,
// shared by the Schur solver and the block-sparse solver.
//   c = pi(R q + t) - uv,  pi(x) = (fx x0 / x2 + cx, fy x1 / x2 + cy)
// with Jacobians with respect to the camera's right perturbation
// [translation; rotation] (Appendix D's convention) and the point.  Huber on
// s = ||w c||^2: rho = s inside (s <= delta^2), 2 delta sqrt(s) - delta^2
// outside; Gauss-Newton uses rho'(s) only (first-order reweighting).
#pragma once

#include <hip/hip_runtime.h>

namespace dnls {

// Reprojection residual and Jacobians; camera/point in float64 storage,
// derivatives in precision S (the point's depth is not checked).
template <class S, class A>
__device__ __forceinline__ void reproj(const double* T, const double* q, const double* uv, const A& a,
                                       double c[2], S Jc[12], S Jp[6]) {
  double pc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) pc[r] = T[r * 4] * q[0] + T[r * 4 + 1] * q[1] + T[r * 4 + 2] * q[2] + T[r * 4 + 3];
  const double iz = 1.0 / pc[2];
  c[0] = a.fx * pc[0] * iz + a.cx - uv[0];
  c[1] = a.fy * pc[1] * iz + a.cy - uv[1];
  // dpi/dpc (2x3)
  const S d00 = S(a.fx * iz), d02 = S(-a.fx * pc[0] * iz * iz);
  const S d11 = S(a.fy * iz), d12 = S(-a.fy * pc[1] * iz * iz);
  S R[9], Q[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int k = 0; k < 3; ++k) R[r * 3 + k] = S(T[r * 4 + k]);
    Q[r] = S(q[r]);
  }
  // Jp = dpi R
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Jp[k] = d00 * R[k] + d02 * R[6 + k];
    Jp[3 + k] = d11 * R[3 + k] + d12 * R[6 + k];
  }
  // Jc = dpi R [I, -q^] = [Jp, -Jp q^];  (Jp q^)_k = (q x Jp_row)... written out:
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const S* jp = Jp + 3 * r;
    Jc[r * 6 + 0] = jp[0];
    Jc[r * 6 + 1] = jp[1];
    Jc[r * 6 + 2] = jp[2];
    // -(jp^T q^) = -(q^T ... ): row vector jp * (-q^) = (jp x q)... explicit:
    // (-q^) = [[0, q2, -q1], [-q2, 0, q0], [q1, -q0, 0]]
    Jc[r * 6 + 3] = -jp[1] * Q[2] + jp[2] * Q[1];
    Jc[r * 6 + 4] = jp[0] * Q[2] - jp[2] * Q[0];
    Jc[r * 6 + 5] = -jp[0] * Q[1] + jp[1] * Q[0];
  }
}

__device__ __forceinline__ void huber(double s, double delta, double& rho, double& drho) {
  if (s <= delta * delta) {
    rho = s;
    drho = 1.0;
  } else {
    const double r = ::sqrt(s);
    rho = 2.0 * delta * r - delta * delta;
    drho = delta / r;
  }
}

}  // namespace dnls
