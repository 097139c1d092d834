// Euler physics for the HIP kernels: perfect-gas flux, Rusanov numerical
// flux, slip-wall and characteristic far-field ghost states (arXiv:1807.01151,
// Section 3, eq. (euler) with a non-rotating frame; Section 3.3 boundary
// fluxes F~(U_L, U_ghost(U_L))).
//
// Everything is templated on the scalar type S: a real type R (double, or
// float in the FP32 smoother), or the forward-mode dual number Dual<M, R>
// below, which carries M tangent components and so returns exact flux and
// ghost Jacobians (the paper evaluates these Jacobians by automatic
// differentiation).  Constants and geometry are of the real type R of S.
// Branches decide on the value.
#pragma once

#include <hip/hip_runtime.h>

namespace eg {

template <int M, class R = double>
struct Dual {
  R v;
  R d[M];
  __device__ __forceinline__ Dual() {}
  __device__ __forceinline__ Dual(R c) : v(c) {
#pragma unroll
    for (int k = 0; k < M; ++k) d[k] = R(0);
  }
};

// real type underlying a scalar type
template <class S> struct RealOf { using type = S; };
template <int M, class R> struct RealOf<Dual<M, R>> { using type = R; };
template <class S> using real_t = typename RealOf<S>::type;

__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ float val(float x) { return x; }
template <int M, class R> __device__ __forceinline__ R val(const Dual<M, R>& x) { return x.v; }

#define EG_DUAL template <int M, class R> __device__ __forceinline__
EG_DUAL Dual<M, R> operator+(const Dual<M, R>& a, const Dual<M, R>& b) {
  Dual<M, R> r; r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
EG_DUAL Dual<M, R> operator-(const Dual<M, R>& a, const Dual<M, R>& b) {
  Dual<M, R> r; r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
EG_DUAL Dual<M, R> operator-(const Dual<M, R>& a) {
  Dual<M, R> r; r.v = -a.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = -a.d[k];
  return r;
}
EG_DUAL Dual<M, R> operator*(const Dual<M, R>& a, const Dual<M, R>& b) {
  Dual<M, R> r; r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
EG_DUAL Dual<M, R> operator/(const Dual<M, R>& a, const Dual<M, R>& b) {
  Dual<M, R> r; R ib = R(1) / b.v; r.v = a.v * ib;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
EG_DUAL Dual<M, R> operator+(const Dual<M, R>& a, R b) { Dual<M, R> r = a; r.v += b; return r; }
EG_DUAL Dual<M, R> operator+(R b, const Dual<M, R>& a) { return a + b; }
EG_DUAL Dual<M, R> operator-(const Dual<M, R>& a, R b) { Dual<M, R> r = a; r.v -= b; return r; }
EG_DUAL Dual<M, R> operator-(R b, const Dual<M, R>& a) {
  Dual<M, R> r; r.v = b - a.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = -a.d[k];
  return r;
}
EG_DUAL Dual<M, R> operator*(const Dual<M, R>& a, R b) {
  Dual<M, R> r; r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = a.d[k] * b;
  return r;
}
EG_DUAL Dual<M, R> operator*(R b, const Dual<M, R>& a) { return a * b; }
EG_DUAL Dual<M, R> operator/(const Dual<M, R>& a, R b) {
  Dual<M, R> r; R ib = R(1) / b; r.v = a.v * ib;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = a.d[k] * ib;
  return r;
}
EG_DUAL Dual<M, R> operator/(R a, const Dual<M, R>& b) {
  Dual<M, R> r; R ib = R(1) / b.v; r.v = a * ib; R s = -r.v * ib;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = s * b.d[k];
  return r;
}

__device__ __forceinline__ double dsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float dsqrt(float x) { return sqrtf(x); }
EG_DUAL Dual<M, R> dsqrt(const Dual<M, R>& a) {
  Dual<M, R> r; r.v = dsqrt(a.v); R s = R(0.5) / r.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = s * a.d[k];
  return r;
}
__device__ __forceinline__ double dpow(double x, double c) { return pow(x, c); }
__device__ __forceinline__ float dpow(float x, float c) { return powf(x, c); }
EG_DUAL Dual<M, R> dpow(const Dual<M, R>& a, R c) {
  Dual<M, R> r; r.v = dpow(a.v, c); R s = c * r.v / a.v;
#pragma unroll
  for (int k = 0; k < M; ++k) r.d[k] = s * a.d[k];
  return r;
}
// |x| and max(a, b): plain values; their dual-number derivatives take the
// symmetric subgradient where the function is not differentiable (zero slope
// for |x| <= 1e-13, the average of both slopes at a relative tie <= 1e-12 of
// max), so a face's Jacobian does not depend on which side evaluates it.
__device__ __forceinline__ double dabs(double x) { return fabs(x); }
__device__ __forceinline__ float dabs(float x) { return fabsf(x); }
EG_DUAL Dual<M, R> dabs(const Dual<M, R>& x) {
  if (dabs(x.v) <= R(1e-13)) return Dual<M, R>(dabs(x.v));
  return x.v < R(0) ? -x : x;
}
__device__ __forceinline__ double dmax(double a, double b) { return a >= b ? a : b; }
__device__ __forceinline__ float dmax(float a, float b) { return a >= b ? a : b; }
EG_DUAL Dual<M, R> dmax(const Dual<M, R>& a, const Dual<M, R>& b) {
  if (dabs(a.v - b.v) <= R(1e-12) * dmax(dabs(a.v), dabs(b.v))) {
    Dual<M, R> r;
    r.v = a.v >= b.v ? a.v : b.v;
#pragma unroll
    for (int k = 0; k < M; ++k) r.d[k] = R(0.5) * (a.d[k] + b.d[k]);
    return r;
  }
  return a.v >= b.v ? a : b;
}
#undef EG_DUAL

// Pressure of the perfect gas, p = (g - 1)(rho E - |rho v|^2 / (2 rho)).
template <int D, class S> __device__ __forceinline__ S pressure(const S* U, real_t<S> g) {
  using R = real_t<S>;
  S m2 = U[1] * U[1];
#pragma unroll
  for (int a = 1; a < D; ++a) m2 = m2 + U[1 + a] * U[1 + a];
  return (g - R(1)) * (U[D + 1] - R(0.5) * m2 / U[0]);
}

// F(U) . n for an arbitrary (not necessarily unit) vector n.
template <int D, class S>
__device__ __forceinline__ void flux_n(const S* U, const real_t<S>* n, S* F, real_t<S> g) {
  using R = real_t<S>;
  S irho = R(1) / U[0];
  S un = U[1] * n[0];
#pragma unroll
  for (int a = 1; a < D; ++a) un = un + U[1 + a] * n[a];
  S vn = un * irho;
  S p = pressure<D>(U, g);
  F[0] = un;
#pragma unroll
  for (int a = 0; a < D; ++a) F[1 + a] = U[1 + a] * vn + p * n[a];
  F[D + 1] = (U[D + 1] + p) * vn;
}

// Rusanov flux: 1/2 (F(UL) + F(UR)) . n - 1/2 lambda (UR - UL),
// lambda = max over the two sides of |v . n| + c, n a unit vector.
template <int D, class SL, class SR, class S>
__device__ __forceinline__ void rusanov(const SL* UL, const SR* UR, const real_t<S>* nh, S* F, real_t<S> g) {
  using R = real_t<S>;
  S ul[D + 2], ur[D + 2];
#pragma unroll
  for (int v = 0; v < D + 2; ++v) { ul[v] = S(UL[v]); ur[v] = S(UR[v]); }
  S FL[D + 2], FR[D + 2];
  flux_n<D>(ul, nh, FL, g);
  flux_n<D>(ur, nh, FR, g);
  S unl = ul[1] * nh[0], unr = ur[1] * nh[0];
#pragma unroll
  for (int a = 1; a < D; ++a) { unl = unl + ul[1 + a] * nh[a]; unr = unr + ur[1 + a] * nh[a]; }
  S cl = dsqrt(g * pressure<D>(ul, g) / ul[0]);
  S cr = dsqrt(g * pressure<D>(ur, g) / ur[0]);
  S lam = dmax(S(dabs(S(unl / ul[0])) + cl), S(dabs(S(unr / ur[0])) + cr));
#pragma unroll
  for (int v = 0; v < D + 2; ++v) F[v] = R(0.5) * (FL[v] + FR[v]) - R(0.5) * lam * (ur[v] - ul[v]);
}

// Roe's approximate Riemann solver (the paper's flux, Section 3.1 after
// eq. (euler3), Section 3.3): 1/2 (F(UL) + F(UR)) . n minus half the sum
// over the waves of the Jacobian at the Roe-averaged state (sqrt(rho)
// weights for velocity and total enthalpy) of |lambda| x strength x
// eigenvector: acoustic waves v_n -+ c with strengths (dp -+ rho c dv_n) /
// (2 c^2), the entropy wave v_n with drho - dp / c^2, the shear waves v_n
// carrying rho (dv - dv_n n).  Entropy fix (the paper names none; the
// reading taken): Harten's on the acoustic waves, |lambda| ->
// (lambda^2 + delta^2) / (2 delta) for |lambda| < delta = c / 10.
template <class S>
__device__ __forceinline__ S harten_abs(const S& lam, const S& delta) {
  using R = real_t<S>;
  if (dabs(val(lam)) < val(delta)) return (lam * lam + delta * delta) / (R(2) * delta);
  return dabs(lam);
}

template <int D, class SL, class SR, class S>
__device__ __forceinline__ void roe(const SL* UL, const SR* UR, const real_t<S>* nh, S* F, real_t<S> g) {
  using R = real_t<S>;
  S ul[D + 2], ur[D + 2];
#pragma unroll
  for (int v = 0; v < D + 2; ++v) { ul[v] = S(UL[v]); ur[v] = S(UR[v]); }
  S FL[D + 2], FR[D + 2];
  flux_n<D>(ul, nh, FL, g);
  flux_n<D>(ur, nh, FR, g);
  const S rl = ul[0], rr = ur[0];
  const S pl = pressure<D>(ul, g), pr = pressure<D>(ur, g);
  S vl[D], vr[D];
#pragma unroll
  for (int a = 0; a < D; ++a) { vl[a] = ul[1 + a] / rl; vr[a] = ur[1 + a] / rr; }
  const S hl = (ul[D + 1] + pl) / rl, hr = (ur[D + 1] + pr) / rr;
  const S sl = dsqrt(rl), sr = dsqrt(rr);
  const S wsum = sl + sr;
  S v[D];
  S q2 = S(R(0)), vn = S(R(0));
#pragma unroll
  for (int a = 0; a < D; ++a) {
    v[a] = (sl * vl[a] + sr * vr[a]) / wsum;
    q2 = q2 + v[a] * v[a];
    vn = vn + v[a] * nh[a];
  }
  const S H = (sl * hl + sr * hr) / wsum;
  const S c2 = (g - R(1)) * (H - R(0.5) * q2);
  const S c = dsqrt(c2);
  const S rho = sl * sr;
  const S drho = rr - rl, dp = pr - pl;
  S dv[D];
  S dvn = S(R(0));
#pragma unroll
  for (int a = 0; a < D; ++a) { dv[a] = vr[a] - vl[a]; dvn = dvn + dv[a] * nh[a]; }
  const S a1 = (dp - rho * c * dvn) / (R(2) * c2);
  const S a5 = (dp + rho * c * dvn) / (R(2) * c2);
  const S a2 = drho - dp / c2;
  const S delta = R(0.1) * c;
  const S l1 = harten_abs(S(vn - c), delta), l5 = harten_abs(S(vn + c), delta), l2 = dabs(vn);
  const S w1 = l1 * a1, w5 = l5 * a5;
  S Dd[D + 2];
  Dd[0] = w1 + w5 + l2 * a2;
  S vdt = S(R(0));
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const S dvt = dv[a] - dvn * nh[a];
    vdt = vdt + v[a] * dvt;
    Dd[1 + a] = w1 * (v[a] - c * nh[a]) + w5 * (v[a] + c * nh[a]) + l2 * (a2 * v[a] + rho * dvt);
  }
  Dd[D + 1] = w1 * (H - c * vn) + w5 * (H + c * vn) + l2 * (a2 * (R(0.5) * q2) + rho * vdt);
#pragma unroll
  for (int k = 0; k < D + 2; ++k) F[k] = R(0.5) * (FL[k] + FR[k]) - R(0.5) * Dd[k];
}

// Slip wall: mirror the momentum about the face, rho v_g = rho v - 2 (rho v . n) n.
template <int D, class S> __device__ __forceinline__ void ghost_wall(const S* U, const real_t<S>* nh, S* G) {
  using R = real_t<S>;
  S mn = U[1] * nh[0];
#pragma unroll
  for (int a = 1; a < D; ++a) mn = mn + U[1 + a] * nh[a];
  G[0] = U[0];
#pragma unroll
  for (int a = 0; a < D; ++a) G[1 + a] = U[1 + a] - R(2) * (mn * nh[a]);
  G[D + 1] = U[D + 1];
}

// Characteristic far field from the Riemann invariants normal to the face:
// the outgoing one (v_n + 2c/(g-1)) from inside, the incoming one from the
// free stream; on outflow (boundary normal velocity > 0) tangential velocity
// and entropy p / rho^g come from inside, else from the free stream.
template <int D, class S>
__device__ __forceinline__ void ghost_far(const S* U, const real_t<S>* nh, S* G, const real_t<S>* Uinf,
                                          real_t<S> g) {
  using R = real_t<S>;
  S irho = R(1) / U[0];
  S vi[D];
#pragma unroll
  for (int a = 0; a < D; ++a) vi[a] = U[1 + a] * irho;
  S vni = vi[0] * nh[0];
#pragma unroll
  for (int a = 1; a < D; ++a) vni = vni + vi[a] * nh[a];
  S pin = pressure<D>(U, g);
  S ci = dsqrt(g * pin * irho);
  R rinf = Uinf[0];
  R vinf[D];
  R vninf = R(0);
#pragma unroll
  for (int a = 0; a < D; ++a) { vinf[a] = Uinf[1 + a] / rinf; vninf += vinf[a] * nh[a]; }
  R pinf = pressure<D>(Uinf, g);
  R cinf = dsqrt(g * pinf / rinf);
  S rp = vni + (R(2) / (g - R(1))) * ci;
  R rm = vninf - (R(2) / (g - R(1))) * cinf;
  S vnb = R(0.5) * (rp + rm);
  S cb = (R(0.25) * (g - R(1))) * (rp - rm);
  S vt[D];
  S ent;
  if (val(vnb) > R(0)) {
#pragma unroll
    for (int a = 0; a < D; ++a) vt[a] = vi[a] - vni * nh[a];
    ent = pin / dpow(U[0], g);
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) vt[a] = S(vinf[a] - vninf * nh[a]);
    ent = S(pinf / dpow(rinf, g));
  }
  S rb = dpow(S(cb * cb / (g * ent)), R(1) / (g - R(1)));
  S pb = rb * cb * cb / g;
  S ke = S(R(0));
  G[0] = rb;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S vb = vt[a] + vnb * nh[a];
    G[1 + a] = rb * vb;
    ke = ke + vb * vb;
  }
  G[D + 1] = pb / (g - R(1)) + R(0.5) * rb * ke;
}

}  // namespace eg
