// Lie-group algebra for the DNLS kernels: SO(3), SE(3), SE(2) in closed form.
//
// The paper evaluates exponential / logarithm maps and their tangent-space
// derivatives in closed form (Section 3 "Differentiable Lie groups",
// Appendix D).  Here every map is written for a scalar type S that is float,
// double, or Dual<double> (first-order forward mode, used by the backward
// pass to differentiate the inverse left Jacobian along a tangent direction).
//
// Tangent order is [translation; rotation]; perturbations act on the right,
// X <- X Exp(xi).  Closed forms (Barfoot, "State Estimation for Robotics",
// 2017; Sola et al., 2018, both cited by the paper):
//   SO(3): R = I + A W + B W^2,  W = phi^,  A = sin t/t, B = (1-cos t)/t^2
//   SE(3): t = V rho,  V = I + B W + C W^2,  C = (t - sin t)/t^3
//          V^-1 = I - W/2 + D W^2,  D = (1 - (t/2) cot(t/2)) / t^2
//          Jr^-1(rho, phi) = [[Ar, -Ar Qr Ar], [0, Ar]],  Ar = I + W/2 + D W^2
//          Qr(rho, phi) = Q(-rho, -phi), with Barfoot's
//          Q(rho, phi) = rho^/2 + C (W P + P W + W P W)
//                        + a2 (W^2 P + P W^2 - 3 W P W)
//                        + a3 (W P W^2 + W^2 P W),   P = rho^,
//          a2 = (t^2 + 2 cos t - 2) / (2 t^4),  a3 = (2t - 3 sin t + t cos t) / (2 t^5)
//   SE(2): Jr = [[A, tB, x t C - y B], [-tB, A, x B + y t C], [0, 0, 1]]
// Every coefficient switches to its Taylor series below a threshold chosen
// per precision so that neither the series truncation nor the cancellation
// of the closed form exceeds the working precision.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#define DNLS_HD __host__ __device__ __forceinline__

namespace dnls {

// ---------------------------------------------------------------------------
// first-order dual numbers
// ---------------------------------------------------------------------------
template <class T>
struct Dual {
  T v, d;
  DNLS_HD Dual() : v(0), d(0) {}
  DNLS_HD Dual(T a) : v(a), d(0) {}
  DNLS_HD Dual(T a, T b) : v(a), d(b) {}
};
template <class T> DNLS_HD Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> DNLS_HD Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> DNLS_HD Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> DNLS_HD Dual<T> operator*(Dual<T> a, Dual<T> b) { return {a.v * b.v, a.v * b.d + a.d * b.v}; }
template <class T> DNLS_HD Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
template <class T> DNLS_HD Dual<T> operator*(T s, Dual<T> a) { return {s * a.v, s * a.d}; }
template <class T> DNLS_HD Dual<T> operator*(Dual<T> a, T s) { return {s * a.v, s * a.d}; }
template <class T> DNLS_HD Dual<T> operator+(Dual<T> a, T s) { return {a.v + s, a.d}; }
template <class T> DNLS_HD Dual<T> operator+(T s, Dual<T> a) { return {a.v + s, a.d}; }
template <class T> DNLS_HD Dual<T> operator-(Dual<T> a, T s) { return {a.v - s, a.d}; }
template <class T> DNLS_HD Dual<T> operator-(T s, Dual<T> a) { return {s - a.v, -a.d}; }
template <class T> DNLS_HD Dual<T> operator/(Dual<T> a, T s) { return {a.v / s, a.d / s}; }
template <class T> DNLS_HD Dual<T>& operator+=(Dual<T>& a, Dual<T> b) { a.v += b.v; a.d += b.d; return a; }
template <class T> DNLS_HD Dual<T>& operator-=(Dual<T>& a, Dual<T> b) { a.v -= b.v; a.d -= b.d; return a; }
template <class T> DNLS_HD Dual<T> sqrt(Dual<T> a) {
  T s = ::sqrt(a.v);
  return {s, a.d / (T(2) * s)};
}
template <class T> DNLS_HD Dual<T> sin(Dual<T> a) { return {::sin(a.v), ::cos(a.v) * a.d}; }
template <class T> DNLS_HD Dual<T> cos(Dual<T> a) { return {::cos(a.v), -::sin(a.v) * a.d}; }

template <class S> struct Real { using type = S; };
template <class T> struct Real<Dual<T>> { using type = T; };
DNLS_HD double val(double x) { return x; }
DNLS_HD float val(float x) { return x; }
template <class T> DNLS_HD T val(Dual<T> x) { return x.v; }

// Below th2 < series_limit the coefficients use their Taylor series.
template <class T> struct SeriesLimit;
template <> struct SeriesLimit<double> { static constexpr double v = 1e-2; };
template <> struct SeriesLimit<float> { static constexpr float v = 0.25f; };

// ---------------------------------------------------------------------------
// scalar coefficients as functions of th2 = t^2
// ---------------------------------------------------------------------------
template <class S>
struct Coefs {
  S A, B, C, D, a2, a3;
};

template <class S>
DNLS_HD Coefs<S> coefs(S th2) {
  using R = typename Real<S>::type;
  using std::cos;
  using std::sin;
  using std::sqrt;
  Coefs<S> k;
  if (val(th2) < SeriesLimit<R>::v) {
    const S u = th2, u2 = u * u, u3 = u2 * u;
    k.A = R(1) - u * R(1.0 / 6) + u2 * R(1.0 / 120) - u3 * R(1.0 / 5040);
    k.B = R(0.5) - u * R(1.0 / 24) + u2 * R(1.0 / 720) - u3 * R(1.0 / 40320);
    k.C = R(1.0 / 6) - u * R(1.0 / 120) + u2 * R(1.0 / 5040) - u3 * R(1.0 / 362880);
    k.D = R(1.0 / 12) + u * R(1.0 / 720) + u2 * R(1.0 / 30240) + u3 * R(1.0 / 1209600);
    k.a2 = R(1.0 / 24) - u * R(1.0 / 720) + u2 * R(1.0 / 40320) - u3 * R(1.0 / 3628800);
    k.a3 = R(1.0 / 120) - u * R(1.0 / 2520) + u2 * R(1.0 / 120960) - u3 * R(1.0 / 9979200);
  } else {
    const S t = sqrt(th2), s = sin(t), c = cos(t);
    const S th4 = th2 * th2;
    k.A = s / t;
    k.B = (R(1) - c) / th2;
    k.C = (t - s) / (th2 * t);
    k.D = (R(1) - (t * s) / (R(2) * (R(1) - c))) / th2;
    k.a2 = (th2 + R(2) * c - R(2)) / (R(2) * th4);
    k.a3 = (R(2) * t - R(3) * s + t * c) / (R(2) * th4 * t);
  }
  return k;
}

// ---------------------------------------------------------------------------
// 3-vectors and 3x3 matrices (row-major S[9])
// ---------------------------------------------------------------------------
template <class S> DNLS_HD void hat3(const S w[3], S M[9]) {
  M[0] = S(0);  M[1] = -w[2]; M[2] = w[1];
  M[3] = w[2];  M[4] = S(0);  M[5] = -w[0];
  M[6] = -w[1]; M[7] = w[0];  M[8] = S(0);
}
template <class S> DNLS_HD void mm3(const S a[9], const S b[9], S c[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) c[r * 3 + q] = a[r * 3] * b[q] + a[r * 3 + 1] * b[3 + q] + a[r * 3 + 2] * b[6 + q];
}
template <class S> DNLS_HD void mv3(const S a[9], const S x[3], S y[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) y[r] = a[r * 3] * x[0] + a[r * 3 + 1] * x[1] + a[r * 3 + 2] * x[2];
}
template <class S> DNLS_HD void cross3(const S a[3], const S b[3], S c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// ---------------------------------------------------------------------------
// SE(3) elements in float64 storage: 3x4 row-major [R | t]
// ---------------------------------------------------------------------------
DNLS_HD void se3_inv(const double X[12], double Y[12]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) Y[r * 4 + q] = X[q * 4 + r];
#pragma unroll
  for (int r = 0; r < 3; ++r) Y[r * 4 + 3] = -(X[r] * X[3] + X[4 + r] * X[7] + X[8 + r] * X[11]);
}
DNLS_HD void se3_mul(const double X[12], const double Y[12], double Z[12]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      Z[r * 4 + q] = X[r * 4] * Y[q] + X[r * 4 + 1] * Y[4 + q] + X[r * 4 + 2] * Y[8 + q];
    Z[r * 4 + 3] = X[r * 4] * Y[3] + X[r * 4 + 1] * Y[7] + X[r * 4 + 2] * Y[11] + X[r * 4 + 3];
  }
}

// Log of SO(3) for a rotation in working precision S (float or double).
template <class S>
DNLS_HD void so3_log(const S R[9], S phi[3]) {
  S w[3] = {S(0.5) * (R[7] - R[5]), S(0.5) * (R[2] - R[6]), S(0.5) * (R[3] - R[1])};
  const S cos_t = S(0.5) * (R[0] + R[4] + R[8] - S(1));
  const S s2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const S s = ::sqrt(s2);
  if (cos_t < S(-0.9)) {
    // angle near pi: (R + R^T)/2 - cos(t) I = (1 - cos t) a a^T
    const S omc = S(1) - cos_t;
    S Bm[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 3; ++q) Bm[r * 3 + q] = S(0.5) * (R[r * 3 + q] + R[q * 3 + r]) - (r == q ? cos_t : S(0));
    int k = 0;
    if (Bm[4] > Bm[k * 4]) k = 1;
    if (Bm[8] > Bm[k * 4]) k = 2;
    const S inv = S(1) / ::sqrt(Bm[k * 4] * omc);
    S a[3] = {Bm[0 * 3 + k] * inv, Bm[1 * 3 + k] * inv, Bm[2 * 3 + k] * inv};
    if (a[0] * w[0] + a[1] * w[1] + a[2] * w[2] < S(0)) { a[0] = -a[0]; a[1] = -a[1]; a[2] = -a[2]; }
    const S th = ::atan2(s, cos_t);
    phi[0] = th * a[0]; phi[1] = th * a[1]; phi[2] = th * a[2];
    return;
  }
  S f;
  if (s2 < S(1e-12)) {
    f = S(1) + s2 * S(1.0 / 6) + s2 * s2 * S(3.0 / 40);  // t / sin t in powers of sin t
  } else {
    f = ::atan2(s, cos_t) / s;
  }
  phi[0] = f * w[0]; phi[1] = f * w[1]; phi[2] = f * w[2];
}

// Log of SE(3): xi = (V^-1 t, phi)
template <class S>
DNLS_HD void se3_log(const S R[9], const S t[3], S xi[6]) {
  S phi[3];
  so3_log(R, phi);
  const Coefs<S> k = coefs(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  S a[3], b[3];
  cross3(phi, t, a);
  cross3(phi, a, b);
#pragma unroll
  for (int r = 0; r < 3; ++r) xi[r] = t[r] - S(0.5) * a[r] + k.D * b[r];
  xi[3] = phi[0]; xi[4] = phi[1]; xi[5] = phi[2];
}

// Exp of SE(3) in float64, result in storage layout.
DNLS_HD void se3_exp(const double xi[6], double X[12]) {
  const double* rho = xi;
  const double* phi = xi + 3;
  const Coefs<double> k = coefs(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  double W[9], W2[9];
  hat3(phi, W);
  mm3(W, W, W2);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) X[r * 4 + q] = (r == q ? 1.0 : 0.0) + k.A * W[r * 3 + q] + k.B * W2[r * 3 + q];
  double a[3], b[3];
  cross3(phi, rho, a);
  cross3(phi, a, b);
#pragma unroll
  for (int r = 0; r < 3; ++r) X[r * 4 + 3] = rho[r] + k.B * a[r] + k.C * b[r];
}

// Q_r(rho, phi) = Q(-rho, -phi): the off-diagonal block of the SE(3) right
// Jacobian (odd-degree terms of Barfoot's Q change sign).
template <class S>
DNLS_HD void se3_Qr(const S rho[3], const S phi[3], const Coefs<S>& k, S Q[9]) {
  S W[9], P[9], W2[9];
  hat3(phi, W);
  hat3(rho, P);
  mm3(W, W, W2);
  S WP[9], PW[9], WPW[9], W2P[9], PW2[9], WPW2[9], W2PW[9];
  mm3(W, P, WP);
  mm3(P, W, PW);
  mm3(WP, W, WPW);
  mm3(W2, P, W2P);
  mm3(P, W2, PW2);
  mm3(WPW, W, WPW2);
  mm3(W2, PW, W2PW);
#pragma unroll
  for (int i = 0; i < 9; ++i)
    Q[i] = S(-0.5) * P[i] + k.C * (WP[i] + PW[i] - WPW[i]) - k.a2 * (W2P[i] + PW2[i] - S(3) * WPW[i]) +
           k.a3 * (WPW2[i] + W2PW[i]);
}

// Inverse right Jacobian of SE(3) at xi: J[6][6] row-major.
// (the inverse left Jacobian is jr_inv at -xi)
template <class S>
DNLS_HD void se3_jr_inv(const S xi[6], S J[36]) {
  const S* rho = xi;
  const S* phi = xi + 3;
  const Coefs<S> k = coefs(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  S W[9], W2[9];
  hat3(phi, W);
  mm3(W, W, W2);
  S Ar[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Ar[i] = (i % 4 == 0 ? S(1) : S(0)) + S(0.5) * W[i] + k.D * W2[i];
  S Q[9];
  se3_Qr(rho, phi, k, Q);
  S T1[9], T2[9];
  mm3(Ar, Q, T1);
  mm3(T1, Ar, T2);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      J[r * 6 + q] = Ar[r * 3 + q];
      J[r * 6 + 3 + q] = -T2[r * 3 + q];
      J[(r + 3) * 6 + q] = S(0);
      J[(r + 3) * 6 + 3 + q] = Ar[r * 3 + q];
    }
}

// Right Jacobian of SE(3): [[Jr(phi), Qr], [0, Jr(phi)]], Jr(phi) = I - B W + C W^2.
template <class S>
DNLS_HD void se3_jr(const S xi[6], S J[36]) {
  const S* rho = xi;
  const S* phi = xi + 3;
  const Coefs<S> k = coefs(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  S W[9], W2[9];
  hat3(phi, W);
  mm3(W, W, W2);
  S Q[9];
  se3_Qr(rho, phi, k, Q);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const S a = (r == q ? S(1) : S(0)) - k.B * W[r * 3 + q] + k.C * W2[r * 3 + q];
      J[r * 6 + q] = a;
      J[r * 6 + 3 + q] = Q[r * 3 + q];
      J[(r + 3) * 6 + q] = S(0);
      J[(r + 3) * 6 + 3 + q] = a;
    }
}

// Adjoint of an SE(3) element: [[R, t^ R], [0, R]].
template <class S>
DNLS_HD void se3_adjoint(const S R[9], const S t[3], S Ad[36]) {
  S T[9], TR[9];
  hat3(t, T);
  mm3(T, R, TR);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Ad[r * 6 + q] = R[r * 3 + q];
      Ad[r * 6 + 3 + q] = TR[r * 3 + q];
      Ad[(r + 3) * 6 + q] = S(0);
      Ad[(r + 3) * 6 + 3 + q] = R[r * 3 + q];
    }
}

// ---------------------------------------------------------------------------
// SE(2) elements in float64 storage: (x, y, cos, sin)
// ---------------------------------------------------------------------------
DNLS_HD void se2_inv(const double X[4], double Y[4]) {
  const double c = X[2], s = X[3];
  Y[0] = -(c * X[0] + s * X[1]);
  Y[1] = -(-s * X[0] + c * X[1]);
  Y[2] = c;
  Y[3] = -s;
}
DNLS_HD void se2_mul(const double X[4], const double Y[4], double Z[4]) {
  const double c = X[2], s = X[3];
  Z[0] = c * Y[0] - s * Y[1] + X[0];
  Z[1] = s * Y[0] + c * Y[1] + X[1];
  Z[2] = c * Y[2] - s * Y[3];
  Z[3] = s * Y[2] + c * Y[3];
}

template <class S>
DNLS_HD void se2_log(S x, S y, S c, S s, S xi[3]) {
  const S th = ::atan2(s, c);
  const Coefs<S> k = coefs(th * th);
  // V = [[A, -tB], [tB, A]], det V = A^2 + t^2 B^2 = 2B
  const S tb = th * k.B, inv = S(1) / (S(2) * k.B);
  xi[0] = inv * (k.A * x + tb * y);
  xi[1] = inv * (-tb * x + k.A * y);
  xi[2] = th;
}

DNLS_HD void se2_exp(const double xi[3], double X[4]) {
  const double th = xi[2];
  const Coefs<double> k = coefs(th * th);
  const double tb = th * k.B;
  X[0] = k.A * xi[0] - tb * xi[1];
  X[1] = tb * xi[0] + k.A * xi[1];
  X[2] = ::cos(th);
  X[3] = ::sin(th);
}

template <class S>
DNLS_HD void se2_jr_inv(const S xi[3], S J[9]) {
  const S x = xi[0], y = xi[1], th = xi[2];
  const Coefs<S> k = coefs(th * th);
  // Jr = [[A, tB, v0], [-tB, A, v1], [0, 0, 1]]
  const S tb = th * k.B;
  const S v0 = x * th * k.C - y * k.B;
  const S v1 = x * k.B + y * th * k.C;
  const S det = k.A * k.A + tb * tb;
  const S m00 = k.A / det, m01 = -tb / det, m10 = tb / det, m11 = k.A / det;
  J[0] = m00; J[1] = m01; J[2] = -(m00 * v0 + m01 * v1);
  J[3] = m10; J[4] = m11; J[5] = -(m10 * v0 + m11 * v1);
  J[6] = S(0); J[7] = S(0); J[8] = S(1);
}

template <class S>
DNLS_HD void se2_jr(const S xi[3], S J[9]) {
  const S x = xi[0], y = xi[1], th = xi[2];
  const Coefs<S> k = coefs(th * th);
  const S tb = th * k.B;
  J[0] = k.A;  J[1] = tb;   J[2] = x * th * k.C - y * k.B;
  J[3] = -tb;  J[4] = k.A;  J[5] = x * k.B + y * th * k.C;
  J[6] = S(0); J[7] = S(0); J[8] = S(1);
}

template <class S>
DNLS_HD void se2_adjoint(S x, S y, S c, S s, S Ad[9]) {
  Ad[0] = c;    Ad[1] = -s;   Ad[2] = y;
  Ad[3] = s;    Ad[4] = c;    Ad[5] = -x;
  Ad[6] = S(0); Ad[7] = S(0); Ad[8] = S(1);
}

}  // namespace dnls
