// FP64 CPU oracle for the exponential p-multigrid (eMG) hot path.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, deliberately
// unoptimised statement of what the method computes.  It is loaded by the
// test-suite, by the smoke check and by the CPU-baseline leg of the benchmark;
// the product library never links, loads or calls it, and it shares no code,
// header, table or helper with the HIP path.
//
// Every function states the passage of the paper (arXiv:1807.01151) it
// follows.  Where the paper is silent or garbled, the reading taken is named
// in the comment (the same reading binds the HIP path).
//
// Conventions:
//   * d = 2 or 3, V = d + 2 conserved variables (rho, rho v, rho E).
//   * Level-p vectors are [E][V][N_p], N_p = (p+1)^d, modes in hierarchical
//     order (sort key (max degree, a0, a1, a2)), so level p-1 is a leading
//     slice of level p.
//   * Basis: tensor Legendre phi_k on the reference cube, orthonormalised per
//     element in the physical L2 inner product: psi = T phi with T = L^{-1},
//     G = L L^T the element Gram matrix (Section 3.2, eq. (basis): psi_i is
//     s_i [chi_i + sum_{j<i} c_ij chi_j], i.e. a lower-triangular transform).
//   * Numerical flux: Rusanov (local Lax-Friedrichs); boundary fluxes use the
//     same flux with a ghost state (Section 3.3, boundary flux equation).
//   * Element map: multilinear through the 2^d vertices, or, when the mesh
//     carries 3^d nodes per element, the tensor quadratic Lagrange map through
//     them (quadratic curved elements, Sections 5.1 and 5.2).
//
// Build: g++ -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cd = std::complex<double>;
using cd_t = std::complex<double>;

// ---------------------------------------------------------------------------
// Scalar helpers usable with double and with complex<double> (complex-step
// differentiation).  Branches decide on the real part.  Where |x| and
// max(a, b) are not differentiable the Jacobian takes the symmetric
// subgradient, so that it does not depend on which side of a face is called
// L: d|x|/dx = 0 for |x| <= 1e-13, and at a tie of max (relative gap
// <= 1e-12) the derivative is the average of both arguments' derivatives.
// Values are unchanged.
// ---------------------------------------------------------------------------
inline double re(double x) { return x; }
inline double re(const cd& z) { return z.real(); }
inline double cs_abs(double x) { return std::fabs(x); }
inline cd cs_abs(const cd& x) {
  if (std::fabs(x.real()) <= 1e-13) return cd(std::fabs(x.real()), 0.0);
  return x.real() < 0.0 ? -x : x;
}
inline double cs_max(double a, double b) { return a >= b ? a : b; }
inline cd cs_max(const cd& a, const cd& b) {
  const double ra = a.real(), rb = b.real();
  if (std::fabs(ra - rb) <= 1e-12 * std::max(std::fabs(ra), std::fabs(rb)))
    return cd(ra >= rb ? ra : rb, 0.5 * (a.imag() + b.imag()));
  return ra >= rb ? a : b;
}
inline double cs_sqrt(double x) { return std::sqrt(x); }
inline cd cs_sqrt(const cd& z) { return std::sqrt(z); }
inline double cs_pow(double x, double y) { return std::pow(x, y); }
inline cd cs_pow(const cd& z, double y) { return std::exp(y * std::log(z)); }

constexpr int MAXD = 3;
constexpr int MAXV = 5;

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [-1, 1] (the paper's "Gaussian quadrature points",
// Section 3.2).  Newton iteration on P_Q from the Chebyshev-like guess; nodes
// ascending, symmetric pairs made exactly symmetric.
// ---------------------------------------------------------------------------
void gauss_legendre(int Q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(Q, 0.0);
  w.assign(Q, 0.0);
  for (int i = 0; i < Q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (Q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= Q; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (Q == 1) { p0 = 1.0; p1 = z; }
      dp = Q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= Q; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (Q == 1) { p0 = 1.0; p1 = z; }
      dp = Q * (z * p1 - p0) / (z * z - 1.0);
    }
    x[Q - 1 - i] = z;
    w[Q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  for (int i = 0; i < Q / 2; ++i) {
    x[i] = -x[Q - 1 - i];
    w[i] = w[Q - 1 - i];
  }
  if (Q % 2 == 1) x[Q / 2] = 0.0;
}

// Orthonormal Legendre L_a = sqrt((2a+1)/2) P_a and its derivative, a <= pm.
void legendre_on(int pm, double x, double* L, double* dL) {
  double P[16], dP[16];
  P[0] = 1.0; dP[0] = 0.0;
  if (pm >= 1) { P[1] = x; dP[1] = 1.0; }
  for (int n = 1; n < pm; ++n) {
    P[n + 1] = ((2.0 * n + 1.0) * x * P[n] - n * P[n - 1]) / (n + 1.0);
    dP[n + 1] = dP[n - 1] + (2.0 * n + 1.0) * P[n];
  }
  for (int a = 0; a <= pm; ++a) {
    double s = std::sqrt((2.0 * a + 1.0) / 2.0);
    L[a] = s * P[a];
    dL[a] = s * dP[a];
  }
}

int nmodes(int d, int p) { int n = 1; for (int r = 0; r < d; ++r) n *= (p + 1); return n; }

// Multi-indices of the tensor space Q_p, hierarchical order.
std::vector<std::array<int, 3>> mode_list(int d, int p) {
  std::vector<std::array<int, 3>> m;
  int n = nmodes(d, p);
  for (int k = 0; k < n; ++k) {
    std::array<int, 3> a{0, 0, 0};
    int t = k;
    for (int r = 0; r < d; ++r) { a[r] = t % (p + 1); t /= (p + 1); }
    m.push_back(a);
  }
  std::sort(m.begin(), m.end(), [](const std::array<int, 3>& x, const std::array<int, 3>& y) {
    int mx = std::max(x[0], std::max(x[1], x[2]));
    int my = std::max(y[0], std::max(y[1], y[2]));
    if (mx != my) return mx < my;
    return x < y;
  });
  return m;
}

// ---------------------------------------------------------------------------
// Mesh, faces and per-element basis
// ---------------------------------------------------------------------------
struct Face {
  int eL, fL, eR, fR, tag;
  int M[2][2];  // face-local coordinates of R = M * face-local coordinates of L
};

struct Oracle {
  int d = 2, V = 4, nv = 0, ne = 0, pmax = 1;
  double gam = 1.4, mach = 0.3, alpha = 0.0, beta = 0.0;
  std::vector<double> xyz;
  std::vector<int> ev;
  std::vector<signed char> tag;
  std::vector<double> geo;  // curved: [E][3^d][d], node digits (a, b[, c]) at (a-1, b-1[, c-1]); empty = straight
  std::vector<Face> faces;
  std::vector<int> efc, eside;  // [E][2d] face id and side (0 = L, 1 = R)
  std::vector<double> T;        // [E][N][N], N = N_pmax, lower triangular
  std::vector<double> vol, surf, hE;
  double omega = 0.0;
  std::vector<std::array<int, 3>> modes;  // at pmax
  int Nmax = 0;
  double Uinf[MAXV];
  int flux = 0;  // numerical flux: 0 Rusanov, 1 Roe
  std::string err;
};

int nface(const Oracle& O) { return 2 * O.d; }

// Tangential axes of face f = 2 r + s, ascending.
void face_axes(int d, int f, int* ax) {
  int r = f / 2, k = 0;
  for (int a = 0; a < d; ++a) if (a != r) ax[k++] = a;
}

void embed(int d, int f, const double* s, double* xi) {
  int ax[2];
  face_axes(d, f, ax);
  xi[f / 2] = (f % 2) ? 1.0 : -1.0;
  for (int k = 0; k < d - 1; ++k) xi[ax[k]] = s[k];
}

// Multilinear map x(xi), tangents t[r] = dx/dxi_r, det and the vectors
// c[r] with c[r] . t[r'] = det delta_{r r'} (det * grad_x = sum_r c[r] d/dxi_r;
// the scaled outward normal of face (r, s) is (2s - 1) c[r]).
// One-dimensional Lagrange polynomial of node a over the nodes -1, 0, 1, and
// its derivative (product rule over the factors).
double lagrange3(int a, double z) {
  const double zn[3] = {-1.0, 0.0, 1.0};
  double v = 1.0;
  for (int m = 0; m < 3; ++m) if (m != a) v *= (z - zn[m]) / (zn[a] - zn[m]);
  return v;
}
double lagrange3_deriv(int a, double z) {
  const double zn[3] = {-1.0, 0.0, 1.0};
  double sum = 0.0;
  for (int j = 0; j < 3; ++j) {
    if (j == a) continue;
    double v = 1.0 / (zn[a] - zn[j]);
    for (int m = 0; m < 3; ++m) if (m != a && m != j) v *= (z - zn[m]) / (zn[a] - zn[m]);
    sum += v;
  }
  return sum;
}

void geom(const Oracle& O, int e, const double* xi, double* x, double t[MAXD][MAXD],
          double& det, double c[MAXD][MAXD]) {
  const int d = O.d, nc = 1 << d;
  for (int a = 0; a < d; ++a) { x[a] = 0.0; for (int r = 0; r < d; ++r) t[r][a] = 0.0; }
  if (!O.geo.empty()) {
    // x(xi) = sum over the 3^d nodes n (digits n_r in 0..2) of
    // prod_r l_{n_r}(xi_r) X_n, and dx/dxi_r with l' in factor r
    const int ng = d == 2 ? 9 : 27;
    for (int k = 0; k < ng; ++k) {
      int dig[MAXD];
      for (int r = 0, kk = k; r < d; ++r, kk /= 3) dig[r] = kk % 3;
      const double* X = &O.geo[((size_t)e * ng + k) * d];
      double N = 1.0;
      for (int r = 0; r < d; ++r) N *= lagrange3(dig[r], xi[r]);
      for (int r = 0; r < d; ++r) {
        double dN = 1.0;
        for (int q = 0; q < d; ++q) dN *= (q == r) ? lagrange3_deriv(dig[q], xi[q]) : lagrange3(dig[q], xi[q]);
        for (int a = 0; a < d; ++a) t[r][a] += dN * X[a];
      }
      for (int a = 0; a < d; ++a) x[a] += N * X[a];
    }
  } else {
    for (int k = 0; k < nc; ++k) {
      const double* X = &O.xyz[(size_t)O.ev[(size_t)e * nc + k] * d];
      double N = 1.0, dN[MAXD];
      for (int r = 0; r < d; ++r) {
        double sg = ((k >> r) & 1) ? 1.0 : -1.0;
        N *= 0.5 * (1.0 + sg * xi[r]);
      }
      for (int r = 0; r < d; ++r) {
        double v = 1.0;
        for (int q = 0; q < d; ++q) {
          double sg = ((k >> q) & 1) ? 1.0 : -1.0;
          v *= (q == r) ? 0.5 * sg : 0.5 * (1.0 + sg * xi[q]);
        }
        dN[r] = v;
      }
      for (int a = 0; a < d; ++a) {
        x[a] += N * X[a];
        for (int r = 0; r < d; ++r) t[r][a] += dN[r] * X[a];
      }
    }
  }
  if (d == 2) {
    det = t[0][0] * t[1][1] - t[0][1] * t[1][0];
    c[0][0] = t[1][1]; c[0][1] = -t[1][0];
    c[1][0] = -t[0][1]; c[1][1] = t[0][0];
  } else {
    auto cross = [](const double* a, const double* b, double* o) {
      o[0] = a[1] * b[2] - a[2] * b[1];
      o[1] = a[2] * b[0] - a[0] * b[2];
      o[2] = a[0] * b[1] - a[1] * b[0];
    };
    cross(t[1], t[2], c[0]);
    cross(t[2], t[0], c[1]);
    cross(t[0], t[1], c[2]);
    det = t[0][0] * c[0][0] + t[0][1] * c[0][1] + t[0][2] * c[0][2];
  }
}

// Reference basis phi_k and its reference gradient at xi (level-p modes are
// the first N_p of O.modes).
void ref_basis(const Oracle& O, int N, const double* xi, double* phi, double* dphi /*[N][d]*/) {
  const int d = O.d;
  double L[MAXD][16], dL[MAXD][16];
  for (int r = 0; r < d; ++r) legendre_on(O.pmax, xi[r], L[r], dL[r]);
  for (int k = 0; k < N; ++k) {
    const auto& a = O.modes[k];
    double v = 1.0;
    for (int r = 0; r < d; ++r) v *= L[r][a[r]];
    phi[k] = v;
    if (dphi) {
      for (int r = 0; r < d; ++r) {
        double g = 1.0;
        for (int q = 0; q < d; ++q) g *= (q == r) ? dL[q][a[q]] : L[q][a[q]];
        dphi[k * d + r] = g;
      }
    }
  }
}

// psi_i(x(xi)) = sum_j T_ij phi_j(xi) and det * grad_x psi_i.
void elem_basis(const Oracle& O, int e, int N, const double* xi, double* psi, double* gpsi /*[N][d] or null*/,
                double* xout = nullptr, double* detout = nullptr, double cout_[MAXD][MAXD] = nullptr) {
  const int d = O.d;
  double phi[128], dphi[128 * MAXD];
  ref_basis(O, N, xi, phi, gpsi ? dphi : nullptr);
  const double* T = &O.T[(size_t)e * O.Nmax * O.Nmax];
  for (int i = 0; i < N; ++i) {
    double s = 0.0;
    for (int j = 0; j <= i; ++j) s += T[i * O.Nmax + j] * phi[j];
    psi[i] = s;
  }
  if (gpsi || xout || detout || cout_) {
    double x[MAXD], t[MAXD][MAXD], det, c[MAXD][MAXD];
    geom(O, e, xi, x, t, det, c);
    if (xout) for (int a = 0; a < d; ++a) xout[a] = x[a];
    if (detout) *detout = det;
    if (cout_) for (int r = 0; r < d; ++r) for (int a = 0; a < d; ++a) cout_[r][a] = c[r][a];
    if (gpsi) {
      for (int i = 0; i < N; ++i) {
        double gr[MAXD];
        for (int r = 0; r < d; ++r) {
          double s = 0.0;
          for (int j = 0; j <= i; ++j) s += T[i * O.Nmax + j] * dphi[j * d + r];
          gr[r] = s;
        }
        for (int a = 0; a < d; ++a) {
          double s = 0.0;
          for (int r = 0; r < d; ++r) s += c[r][a] * gr[r];
          gpsi[i * d + a] = s;
        }
      }
    }
  }
}

// Cholesky G = L L^T and T = L^{-1} (dense, row-major, n x n).
bool chol_inverse(int n, const double* G, double* T) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = G[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = G[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  for (int i = 0; i < n * n; ++i) T[i] = 0.0;
  for (int c = 0; c < n; ++c) {  // solve L x = e_c by forward substitution
    for (int i = 0; i < n; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) s -= L[i * n + k] * T[k * n + c];
      T[i * n + c] = s / L[i * n + i];
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Physics (Section 3, eq. (euler) with omega = 0; perfect gas, gamma = 7/5)
// ---------------------------------------------------------------------------
template <class S> S pressure(int d, double g, const S* U) {
  S ke = 0.0;
  for (int a = 0; a < d; ++a) ke += U[1 + a] * U[1 + a];
  return (g - 1.0) * (U[d + 1] - 0.5 * ke / U[0]);
}

// F(U) . n for any vector n.
template <class S> void flux_n(int d, double g, const S* U, const double* n, S* Fn) {
  S rho = U[0];
  S vn = 0.0;
  for (int a = 0; a < d; ++a) vn += (U[1 + a] / rho) * n[a];
  S p = pressure(d, g, U);
  Fn[0] = rho * vn;
  for (int a = 0; a < d; ++a) Fn[1 + a] = U[1 + a] * vn + p * n[a];
  Fn[d + 1] = (U[d + 1] + p) * vn;
}

// Rusanov flux F~(UL, UR; n^) = 1/2 (F(UL) + F(UR)) . n^ - 1/2 lambda (UR - UL),
// lambda = max(|vL . n^| + cL, |vR . n^| + cR).
template <class S> void rusanov(int d, double g, const S* UL, const S* UR, const double* nh, S* F) {
  S FL[MAXV], FR[MAXV];
  flux_n(d, g, UL, nh, FL);
  flux_n(d, g, UR, nh, FR);
  S vnL = 0.0, vnR = 0.0;
  for (int a = 0; a < d; ++a) { vnL += (UL[1 + a] / UL[0]) * nh[a]; vnR += (UR[1 + a] / UR[0]) * nh[a]; }
  S cL = cs_sqrt(g * pressure(d, g, UL) / UL[0]);
  S cR = cs_sqrt(g * pressure(d, g, UR) / UR[0]);
  S lam = cs_max(S(cs_abs(vnL) + cL), S(cs_abs(vnR) + cR));
  for (int v = 0; v < d + 2; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * lam * (UR[v] - UL[v]);
}

// Roe's approximate Riemann solver (Roe 1981; the paper's flux, Section 3.1
// after eq. (euler3) and Section 3.3): F~ = 1/2 (F(UL) + F(UR)) . n
// - 1/2 sum_k |lambda_k| alpha_k r_k over the waves of the Jacobian at the
// Roe-averaged state (sqrt(rho)-weighted velocity and total enthalpy), n a
// unit vector: acoustic waves v_n -+ c with strengths
// (dp -+ rho c dv_n) / (2 c^2), the entropy wave v_n with strength
// drho - dp / c^2, and the shear waves v_n carrying rho (dv - dv_n n).  The
// paper names no entropy fix; the reading taken is Harten's on the two
// acoustic waves, |lambda| -> (lambda^2 + delta^2) / (2 delta) for
// |lambda| < delta = 0.1 c (inactive in subsonic flow away from sonic
// points); the entropy and shear waves keep |v_n| (zero slope at v_n = 0 by
// the tie rule of cs_abs).
template <class S> S harten_abs(const S& lam, const S& delta) {
  if (std::fabs(re(lam)) < re(delta)) return (lam * lam + delta * delta) / (2.0 * delta);
  return cs_abs(lam);
}

template <class S> void roe(int d, double g, const S* UL, const S* UR, const double* nh, S* F) {
  const int V = d + 2;
  S FL[MAXV], FR[MAXV];
  flux_n(d, g, UL, nh, FL);
  flux_n(d, g, UR, nh, FR);
  S rl = UL[0], rr = UR[0];
  S pl = pressure(d, g, UL), pr = pressure(d, g, UR);
  S vl[MAXD], vr[MAXD];
  for (int a = 0; a < d; ++a) { vl[a] = UL[1 + a] / rl; vr[a] = UR[1 + a] / rr; }
  S hl = (UL[d + 1] + pl) / rl, hr = (UR[d + 1] + pr) / rr;
  // Roe averages
  S sl = cs_sqrt(rl), sr = cs_sqrt(rr);
  S wsum = sl + sr;
  S v[MAXD], q2 = 0.0, vn = 0.0;
  for (int a = 0; a < d; ++a) {
    v[a] = (sl * vl[a] + sr * vr[a]) / wsum;
    q2 += v[a] * v[a];
    vn += v[a] * nh[a];
  }
  S H = (sl * hl + sr * hr) / wsum;
  S c2 = (g - 1.0) * (H - 0.5 * q2);
  S c = cs_sqrt(c2);
  S rho = sl * sr;
  // jumps and wave strengths
  S drho = rr - rl, dp = pr - pl, dv[MAXD], dvn = 0.0;
  for (int a = 0; a < d; ++a) { dv[a] = vr[a] - vl[a]; dvn += dv[a] * nh[a]; }
  S a1 = (dp - rho * c * dvn) / (2.0 * c2);
  S a5 = (dp + rho * c * dvn) / (2.0 * c2);
  S a2 = drho - dp / c2;
  S delta = 0.1 * c;
  S l1 = harten_abs(S(vn - c), delta), l5 = harten_abs(S(vn + c), delta), l2 = cs_abs(vn);
  // dissipation sum_k |lambda_k| alpha_k r_k
  S Dd[MAXV];
  Dd[0] = l1 * a1 + l5 * a5 + l2 * a2;
  S vdt = 0.0;
  for (int a = 0; a < d; ++a) {
    S dvt = dv[a] - dvn * nh[a];
    vdt += v[a] * dvt;
    Dd[1 + a] = l1 * a1 * (v[a] - c * nh[a]) + l5 * a5 * (v[a] + c * nh[a]) + l2 * (a2 * v[a] + rho * dvt);
  }
  Dd[d + 1] = l1 * a1 * (H - c * vn) + l5 * a5 * (H + c * vn) + l2 * (a2 * 0.5 * q2 + rho * vdt);
  for (int w = 0; w < V; ++w) F[w] = 0.5 * (FL[w] + FR[w]) - 0.5 * Dd[w];
}

// The numerical flux of the oracle (Rusanov unless the Roe flux is selected).
template <class S> void num_flux(const Oracle& O, const S* UL, const S* UR, const double* nh, S* F) {
  if (O.flux == 1) roe(O.d, O.gam, UL, UR, nh, F);
  else rusanov(O.d, O.gam, UL, UR, nh, F);
}

// Manufactured smooth state (tests of the convergence rate only).
template <class S> void mms_state(int d, double g, const S* x, S* U) {
  const double pi = M_PI;
  S sx = std::sin(pi * x[0]), cx = std::cos(pi * x[0]);
  S sy = std::sin(pi * x[1]), cy = std::cos(pi * x[1]);
  S cz = (d == 3) ? S(std::cos(pi * x[2])) : S(1.0);
  S rho = 1.0 + 0.1 * sx * cy * cz;
  S vel[3];
  vel[0] = 0.3 + 0.05 * cx * sy;
  vel[1] = 0.1 + 0.05 * sx * sy * cz;
  vel[2] = 0.05 + 0.03 * cx * cy;
  S p = 1.0 / g + 0.05 * cx * cy * cz;
  S ke = 0.0;
  for (int a = 0; a < d; ++a) ke += vel[a] * vel[a];
  U[0] = rho;
  for (int a = 0; a < d; ++a) U[1 + a] = rho * vel[a];
  U[d + 1] = p / (g - 1.0) + 0.5 * rho * ke;
}

// Ghost state for boundary faces (Section 3.3: U_ghost is a function of U_L).
//  tag 1 slip wall: mirror state, rho v_g = rho v - 2 (rho v . n^) n^.
//  tag 4 symmetry plane (Section 5.2): the same mirror state; only the drag
//        integral tells it from a wall.
//  tag 2 far-field: Riemann invariants R+ = v_n + 2c/(g-1) from inside,
//        R- = v_n,inf - 2 c_inf/(g-1) from the free stream; outflow iff the
//        boundary normal velocity is > 0, taking tangential velocity and
//        entropy p/rho^g from inside, else from the free stream.
//  tag 3 exact state of the manufactured solution (tests only).
template <class S> void ghost(const Oracle& O, int tg, const S* U, const double* nh, const double* x, S* Ug) {
  const int d = O.d;
  const double g = O.gam;
  if (tg == 1 || tg == 4) {
    S mn = 0.0;
    for (int a = 0; a < d; ++a) mn += U[1 + a] * nh[a];
    Ug[0] = U[0];
    for (int a = 0; a < d; ++a) Ug[1 + a] = U[1 + a] - 2.0 * mn * nh[a];
    Ug[d + 1] = U[d + 1];
  } else if (tg == 2) {
    const double* Ui = O.Uinf;
    S rho = U[0];
    S vi[MAXD];
    S vni = 0.0;
    for (int a = 0; a < d; ++a) { vi[a] = U[1 + a] / rho; vni += vi[a] * nh[a]; }
    S pi = pressure(d, g, U);
    S ci = cs_sqrt(g * pi / rho);
    double rinf = Ui[0], vinf[MAXD], vninf = 0.0;
    for (int a = 0; a < d; ++a) { vinf[a] = Ui[1 + a] / rinf; vninf += vinf[a] * nh[a]; }
    double pinf = pressure(d, g, Ui);
    double cinf = std::sqrt(g * pinf / rinf);
    S Rp = vni + 2.0 * ci / (g - 1.0);
    double Rm = vninf - 2.0 * cinf / (g - 1.0);
    S vnb = 0.5 * (Rp + Rm);
    S cb = 0.25 * (g - 1.0) * (Rp - Rm);
    S vt[MAXD], ent;
    if (re(vnb) > 0.0) {
      for (int a = 0; a < d; ++a) vt[a] = vi[a] - vni * nh[a];
      ent = pi / cs_pow(rho, g);
    } else {
      for (int a = 0; a < d; ++a) vt[a] = S(vinf[a] - vninf * nh[a]);
      ent = S(pinf / std::pow(rinf, g));
    }
    S rb = cs_pow(S(cb * cb / (g * ent)), 1.0 / (g - 1.0));
    S pb = rb * cb * cb / g;
    S ke = 0.0;
    Ug[0] = rb;
    for (int a = 0; a < d; ++a) {
      S vb = vt[a] + vnb * nh[a];
      Ug[1 + a] = rb * vb;
      ke += vb * vb;
    }
    Ug[d + 1] = pb / (g - 1.0) + 0.5 * rb * ke;
  } else {
    (void)x;
    for (int v = 0; v < d + 2; ++v) Ug[v] = U[v];
  }
}

// The exact-state ghost cannot go through the template above for complex S
// (it does not depend on U), so it is handled here.
template <class S> void ghost_any(const Oracle& O, int tg, const S* U, const double* nh, const double* x, S* Ug) {
  if (tg == 3) {
    double Um[MAXV];
    mms_state<double>(O.d, O.gam, x, Um);
    for (int v = 0; v < O.V; ++v) Ug[v] = Um[v];
  } else {
    ghost(O, tg, U, nh, x, Ug);
  }
}

// Euler flux Jacobian contracted with a vector g: sum_a g_a dF_a/dU
// (Appendix A, eq. (dfdu), omega = 0, with a_1 read as gamma E - a_0 = H, the
// total enthalpy, which is what differentiating the energy flux gives).
void flux_jac(int d, double gm, const double* U, const double* gv, double* K /*[V][V]*/) {
  const int V = d + 2;
  double rho = U[0], vel[MAXD], q2 = 0.0;
  for (int a = 0; a < d; ++a) { vel[a] = U[1 + a] / rho; q2 += vel[a] * vel[a]; }
  double E = U[d + 1] / rho;
  double a0 = 0.5 * (gm - 1.0) * q2;
  double a1 = gm * E - a0;
  double a2 = gm - 1.0, a3 = gm - 2.0;
  double B1 = 0.0;
  for (int a = 0; a < d; ++a) B1 += vel[a] * gv[a];
  for (int i = 0; i < V * V; ++i) K[i] = 0.0;
  for (int a = 0; a < d; ++a) K[0 * V + 1 + a] = gv[a];
  for (int r = 0; r < d; ++r) {
    K[(1 + r) * V + 0] = a0 * gv[r] - B1 * vel[r];
    for (int c = 0; c < d; ++c) {
      if (c == r) K[(1 + r) * V + 1 + c] = B1 - a3 * vel[r] * gv[r];
      else K[(1 + r) * V + 1 + c] = vel[r] * gv[c] - a2 * vel[c] * gv[r];
    }
    K[(1 + r) * V + d + 1] = a2 * gv[r];
  }
  K[(d + 1) * V + 0] = (a0 - a1) * B1;
  for (int c = 0; c < d; ++c) K[(d + 1) * V + 1 + c] = a1 * gv[c] - a2 * B1 * vel[c];
  K[(d + 1) * V + d + 1] = gm * B1;
}

// Complex-step derivative of a map R^V -> R^V at U: Jac[v][w] = dF_v/dU_w.
template <class Fn> void cs_jac(int V, const double* U, Fn f, double* Jac) {
  const double h = 1e-30;
  for (int w = 0; w < V; ++w) {
    cd Uc[MAXV], Fc[MAXV];
    for (int v = 0; v < V; ++v) Uc[v] = cd(U[v], 0.0);
    Uc[w] = cd(U[w], h);
    f(Uc, Fc);
    for (int v = 0; v < V; ++v) Jac[v * V + w] = Fc[v].imag() / h;
  }
}

// ---------------------------------------------------------------------------
// Set-up: faces (matched through shared vertices), geometry, Gram / T.
// ---------------------------------------------------------------------------
bool setup(Oracle& O) {
  const int d = O.d, nfc = 2 * d, nc = 1 << d, ncf = 1 << (d - 1);
  O.V = d + 2;
  O.modes = mode_list(d, O.pmax);
  O.Nmax = nmodes(d, O.pmax);
  O.efc.assign((size_t)O.ne * nfc, -1);
  O.eside.assign((size_t)O.ne * nfc, 0);
  // face vertices in face-local lexicographic order
  auto fverts = [&](int e, int f, int* vv) {
    int ax[2];
    face_axes(d, f, ax);
    for (int c = 0; c < ncf; ++c) {
      int k = (f % 2) << (f / 2);
      for (int q = 0; q < d - 1; ++q) if ((c >> q) & 1) k |= 1 << ax[q];
      vv[c] = O.ev[(size_t)e * nc + k];
    }
  };
  std::map<std::vector<int>, std::pair<int, int>> open;
  for (int e = 0; e < O.ne; ++e) {
    for (int f = 0; f < nfc; ++f) {
      int tg = O.tag[(size_t)e * nfc + f];
      if (tg != 0) {
        Face F{e, f, -1, -1, tg, {{1, 0}, {0, 1}}};
        O.efc[(size_t)e * nfc + f] = (int)O.faces.size();
        O.eside[(size_t)e * nfc + f] = 0;
        O.faces.push_back(F);
        continue;
      }
      int vv[4];
      fverts(e, f, vv);
      std::vector<int> key(vv, vv + ncf);
      std::sort(key.begin(), key.end());
      auto it = open.find(key);
      if (it == open.end()) { open[key] = {e, f}; continue; }
      int e0 = it->second.first, f0 = it->second.second;
      open.erase(it);
      // L = earlier element, R = this one; build the signed permutation M
      int vL[4], vR[4];
      fverts(e0, f0, vL);
      fverts(e, f, vR);
      auto corner_of = [&](int vid, const int* vlist, double* s) {
        for (int c = 0; c < ncf; ++c) if (vlist[c] == vid) {
          for (int q = 0; q < d - 1; ++q) s[q] = ((c >> q) & 1) ? 1.0 : -1.0;
          return true;
        }
        return false;
      };
      Face F{e0, f0, e, f, 0, {{0, 0}, {0, 0}}};
      double s0[2] = {0, 0}, sq[2] = {0, 0};
      if (!corner_of(vL[0], vR, s0)) { O.err = "face matching failed"; return false; }
      for (int q = 0; q < d - 1; ++q) {
        if (!corner_of(vL[1 << q], vR, sq)) { O.err = "face matching failed"; return false; }
        for (int k = 0; k < d - 1; ++k) F.M[k][q] = (int)std::lround(0.5 * (sq[k] - s0[k]));
      }
      // check every corner maps through M (offset must vanish)
      for (int c = 0; c < ncf; ++c) {
        double sl[2], sr[2], sm[2];
        for (int q = 0; q < d - 1; ++q) sl[q] = ((c >> q) & 1) ? 1.0 : -1.0;
        if (!corner_of(vL[c], vR, sr)) { O.err = "face matching failed"; return false; }
        for (int k = 0; k < d - 1; ++k) {
          sm[k] = 0.0;
          for (int q = 0; q < d - 1; ++q) sm[k] += F.M[k][q] * sl[q];
          if (sm[k] != sr[k]) { O.err = "non-conforming face"; return false; }
        }
      }
      int id = (int)O.faces.size();
      O.faces.push_back(F);
      O.efc[(size_t)e0 * nfc + f0] = id; O.eside[(size_t)e0 * nfc + f0] = 0;
      O.efc[(size_t)e * nfc + f] = id; O.eside[(size_t)e * nfc + f] = 1;
    }
  }
  if (!open.empty()) { O.err = "unmatched interior face"; return false; }
  if (!O.geo.empty()) {
    // curved elements: the nodes at the corners are the vertices, and the two
    // sides of an interior face place its 3^(d-1) nodes at the same points
    const int ng = d == 2 ? 9 : 27;
    auto same = [&](const double* a, const double* b) {
      for (int q = 0; q < d; ++q)
        if (std::fabs(a[q] - b[q]) > 1e-12 * std::max(1.0, std::fabs(a[q]))) return false;
      return true;
    };
    auto node = [&](int e, int k) { return &O.geo[((size_t)e * ng + k) * d]; };
    auto digit = [](int k, int r) { for (int q = 0; q < r; ++q) k /= 3; return k % 3; };
    for (int e = 0; e < O.ne; ++e)
      for (int v = 0; v < nc; ++v) {
        int k = 0;
        for (int r = 0, p3 = 1; r < d; ++r, p3 *= 3) k += 2 * ((v >> r) & 1) * p3;
        if (!same(node(e, k), &O.xyz[(size_t)O.ev[(size_t)e * nc + v] * d])) {
          O.err = "curved element node at a corner differs from its vertex";
          return false;
        }
      }
    for (const Face& F : O.faces) {
      if (F.eR < 0) continue;
      for (int k = 0; k < ng; ++k) {
        if (digit(k, F.fL / 2) != 2 * (F.fL % 2)) continue;
        bool found = false;
        for (int k2 = 0; k2 < ng; ++k2)
          if (digit(k2, F.fR / 2) == 2 * (F.fR % 2) && same(node(F.eL, k), node(F.eR, k2))) found = true;
        if (!found) {
          O.err = "non-conforming curved face";
          return false;
        }
      }
    }
  }

  // Geometry and per-element orthonormalisation with the (pmax+2)-point rule,
  // which integrates phi_i phi_j det exactly on multilinear elements.
  const int N = O.Nmax, Q = O.pmax + 2;
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  O.T.assign((size_t)O.ne * N * N, 0.0);
  O.vol.assign(O.ne, 0.0);
  O.surf.assign(O.ne, 0.0);
  O.hE.assign(O.ne, 0.0);
  int nq = 1;
  for (int r = 0; r < d; ++r) nq *= Q;
  int nqf = nq / Q;
  bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
  for (int e = 0; e < O.ne; ++e) {
    std::vector<double> G((size_t)N * N, 0.0), phi(N);
    double vol = 0.0;
    for (int q = 0; q < nq; ++q) {
      double xi[MAXD], w = 1.0;
      int t = q;
      for (int r = 0; r < d; ++r) { xi[r] = xg[t % Q]; w *= wg[t % Q]; t /= Q; }
      double x[MAXD], tt[MAXD][MAXD], det, c[MAXD][MAXD];
      geom(O, e, xi, x, tt, det, c);
      if (!(det > 0.0)) ok = false;
      ref_basis(O, N, xi, phi.data(), nullptr);
      vol += w * det;
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) G[i * N + j] += w * det * phi[i] * phi[j];
    }
    double surf = 0.0;
    for (int f = 0; f < nfc; ++f) {
      for (int k = 0; k < nqf; ++k) {
        double s[2], w = 1.0, xi[MAXD];
        int t = k;
        for (int q = 0; q < d - 1; ++q) { s[q] = xg[t % Q]; w *= wg[t % Q]; t /= Q; }
        embed(d, f, s, xi);
        double x[MAXD], tt[MAXD][MAXD], det, c[MAXD][MAXD];
        geom(O, e, xi, x, tt, det, c);
        double a2 = 0.0;
        for (int a = 0; a < d; ++a) a2 += c[f / 2][a] * c[f / 2][a];
        surf += w * std::sqrt(a2);
      }
    }
    O.vol[e] = vol;
    O.surf[e] = surf;
    O.hE[e] = 2.0 * d * vol / surf;
    if (!chol_inverse(N, G.data(), &O.T[(size_t)e * N * N])) ok = false;
  }
  if (!ok) { O.err = "non-positive Jacobian or Gram matrix"; return false; }
  O.omega = 0.0;
  for (int e = 0; e < O.ne; ++e) O.omega += O.vol[e];
  // free stream (rho = 1, p = 1/gamma so c = 1)
  double vinf[3] = {O.mach * std::cos(O.alpha) * std::cos(O.beta), O.mach * std::sin(O.alpha) * std::cos(O.beta),
                    O.mach * std::sin(O.beta)};
  O.Uinf[0] = 1.0;
  double ke = 0.0;
  for (int a = 0; a < d; ++a) { O.Uinf[1 + a] = vinf[a]; ke += vinf[a] * vinf[a]; }
  O.Uinf[d + 1] = (1.0 / O.gam) / (O.gam - 1.0) + 0.5 * ke;
  return true;
}

// Reference coordinates of face point k (tensor order, first axis fastest)
// for the L side and, through M, for the R side.
void face_point(const Oracle& O, const Face& F, int Q, const std::vector<double>& xg, const std::vector<double>& wg,
                int k, double* xiL, double* xiR, double& w) {
  const int d = O.d;
  double s[2] = {0, 0};
  w = 1.0;
  int t = k;
  for (int q = 0; q < d - 1; ++q) { s[q] = xg[t % Q]; w *= wg[t % Q]; t /= Q; }
  embed(d, F.fL, s, xiL);
  if (F.eR >= 0) {
    double sr[2] = {0, 0};
    for (int a = 0; a < d - 1; ++a) {
      sr[a] = 0.0;
      for (int b = 0; b < d - 1; ++b) sr[a] += F.M[a][b] * s[b];
    }
    embed(d, F.fR, sr, xiR);
  }
}

template <class S> void eval_state(const Oracle& O, int e, int N, const S* u, const double* psi, S* U) {
  for (int v = 0; v < O.V; ++v) {
    S s = 0.0;
    for (int i = 0; i < N; ++i) s += u[((size_t)e * O.V + v) * N + i] * psi[i];
    U[v] = s;
  }
}

// ---------------------------------------------------------------------------
// DG residual R_p(u) (Section 3.1, eq. (euler3), S = 0):
//   R_{E,i} = - sum_faces int psi_i F~ . n^ dsigma + int_E F . grad psi_i dx,
// with (p+2)^d Gauss points in the volume and (p+2)^(d-1) per face.  Each
// interior face flux is computed once with the L element's normal and added to
// both sides.
// ---------------------------------------------------------------------------
template <class S> void residual_t(const Oracle& O, int p, const S* u, S* r) {
  const int d = O.d, V = O.V, N = nmodes(d, p), Q = p + 2, nfc = 2 * d;
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  int nq = 1;
  for (int k = 0; k < d; ++k) nq *= Q;
  const int nqf = nq / Q;
  // volume term
#pragma omp parallel for schedule(static)
  for (int e = 0; e < O.ne; ++e) {
    S* re_ = r + (size_t)e * V * N;
    for (int i = 0; i < V * N; ++i) re_[i] = 0.0;
    double psi[128], gpsi[128 * MAXD];
    for (int q = 0; q < nq; ++q) {
      double xi[MAXD], w = 1.0;
      int t = q;
      for (int k = 0; k < d; ++k) { xi[k] = xg[t % Q]; w *= wg[t % Q]; t /= Q; }
      elem_basis(O, e, N, xi, psi, gpsi);
      S U[MAXV];
      eval_state(O, e, N, u, psi, U);
      S F[MAXD][MAXV];
      for (int a = 0; a < d; ++a) {
        double ea[MAXD] = {0, 0, 0};
        ea[a] = 1.0;
        flux_n(d, O.gam, U, ea, F[a]);
      }
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < N; ++i) {
          S s = 0.0;
          for (int a = 0; a < d; ++a) s += F[a][v] * gpsi[i * d + a];
          re_[v * N + i] += w * s;
        }
    }
  }
  // face fluxes, weighted by w |n dsigma|
  const int nf = (int)O.faces.size();
  std::vector<S> flux((size_t)nf * nqf * V);
#pragma omp parallel for schedule(static)
  for (int fc = 0; fc < nf; ++fc) {
    const Face& F = O.faces[fc];
    double psiL[128], psiR[128];
    for (int k = 0; k < nqf; ++k) {
      double xiL[MAXD], xiR[MAXD], w;
      face_point(O, F, Q, xg, wg, k, xiL, xiR, w);
      double x[MAXD], det, c[MAXD][MAXD];
      elem_basis(O, F.eL, N, xiL, psiL, nullptr, x, &det, c);
      double sg = (F.fL % 2) ? 1.0 : -1.0, nh[MAXD], area2 = 0.0;
      for (int a = 0; a < d; ++a) { nh[a] = sg * c[F.fL / 2][a]; area2 += nh[a] * nh[a]; }
      double area = std::sqrt(area2);
      for (int a = 0; a < d; ++a) nh[a] /= area;
      S UL[MAXV], UR[MAXV], Fl[MAXV];
      eval_state(O, F.eL, N, u, psiL, UL);
      if (F.eR >= 0) {
        elem_basis(O, F.eR, N, xiR, psiR, nullptr);
        eval_state(O, F.eR, N, u, psiR, UR);
      } else {
        ghost_any(O, F.tag, UL, nh, x, UR);
      }
      num_flux(O, UL, UR, nh, Fl);
      for (int v = 0; v < V; ++v) flux[((size_t)fc * nqf + k) * V + v] = (w * area) * Fl[v];
    }
  }
  // lift to the elements
#pragma omp parallel for schedule(static)
  for (int e = 0; e < O.ne; ++e) {
    S* re_ = r + (size_t)e * V * N;
    double psi[128];
    for (int lf = 0; lf < nfc; ++lf) {
      int fc = O.efc[(size_t)e * nfc + lf], side = O.eside[(size_t)e * nfc + lf];
      const Face& F = O.faces[fc];
      for (int k = 0; k < nqf; ++k) {
        double xiL[MAXD], xiR[MAXD], w;
        face_point(O, F, Q, xg, wg, k, xiL, xiR, w);
        elem_basis(O, e, N, side == 0 ? xiL : xiR, psi, nullptr);
        double sg = side == 0 ? -1.0 : 1.0;
        for (int v = 0; v < V; ++v)
          for (int i = 0; i < N; ++i) re_[v * N + i] += sg * psi[i] * flux[((size_t)fc * nqf + k) * V + v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Exact Jacobian blocks (Section 3.3, eqs. (jac1) and (jac2)).
//   D_E = dR_E/du_E:  volume  int psi_j grad psi_i . dF/dU dx   (Appendix A)
//                     faces  -int psi_i psi_j dF~/dU_own dsigma (with the
//                     boundary chain rule dF~/dU_L + dF~/dU_g dU_g/dU_L)
//   O_{E,f} = dR_E/du_nb(f):  -int psi_i^E psi_j^nb dF~/dU_nb dsigma.
// The Riemann-flux and ghost Jacobians are obtained by complex-step
// differentiation, which is exact to rounding (the paper uses AD).
// Blocks are [(v,i)][(w,j)], n = V N_p.
// ---------------------------------------------------------------------------
void jacobian_blocks(const Oracle& O, int p, const double* u, double* D, double* Off /*nullable [E][2d][n][n]*/) {
  const int d = O.d, V = O.V, N = nmodes(d, p), Q = p + 2, nfc = 2 * d, n = V * N;
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  int nq = 1;
  for (int k = 0; k < d; ++k) nq *= Q;
  const int nqf = nq / Q;
#pragma omp parallel for schedule(dynamic)
  for (int e = 0; e < O.ne; ++e) {
    double* De = D + (size_t)e * n * n;
    for (int i = 0; i < n * n; ++i) De[i] = 0.0;
    if (Off) for (size_t i = 0; i < (size_t)nfc * n * n; ++i) Off[(size_t)e * nfc * n * n + i] = 0.0;
    double psi[128], gpsi[128 * MAXD];
    for (int q = 0; q < nq; ++q) {
      double xi[MAXD], w = 1.0;
      int t = q;
      for (int k = 0; k < d; ++k) { xi[k] = xg[t % Q]; w *= wg[t % Q]; t /= Q; }
      elem_basis(O, e, N, xi, psi, gpsi);
      double U[MAXV];
      eval_state(O, e, N, u, psi, U);
      for (int i = 0; i < N; ++i) {
        double K[MAXV * MAXV];
        flux_jac(d, O.gam, U, &gpsi[i * d], K);
        for (int v = 0; v < V; ++v)
          for (int wv = 0; wv < V; ++wv)
            for (int j = 0; j < N; ++j) De[(v * N + i) * n + wv * N + j] += w * K[v * V + wv] * psi[j];
      }
    }
    double psiE[128], psiO[128];
    for (int lf = 0; lf < nfc; ++lf) {
      int fc = O.efc[(size_t)e * nfc + lf], side = O.eside[(size_t)e * nfc + lf];
      const Face& F = O.faces[fc];
      for (int k = 0; k < nqf; ++k) {
        double xiL[MAXD], xiR[MAXD], w;
        face_point(O, F, Q, xg, wg, k, xiL, xiR, w);
        double x[MAXD], det, c[MAXD][MAXD], psiL[128];
        elem_basis(O, F.eL, N, xiL, psiL, nullptr, x, &det, c);
        double sg = (F.fL % 2) ? 1.0 : -1.0, nh[MAXD], area2 = 0.0;
        for (int a = 0; a < d; ++a) { nh[a] = sg * c[F.fL / 2][a]; area2 += nh[a] * nh[a]; }
        double area = std::sqrt(area2);
        for (int a = 0; a < d; ++a) nh[a] /= area;
        double UL[MAXV], UR[MAXV];
        eval_state(O, F.eL, N, u, psiL, UL);
        double Jown[MAXV * MAXV], Joth[MAXV * MAXV];
        int other = -1;
        if (F.eR >= 0) {
          double psiR[128];
          elem_basis(O, F.eR, N, xiR, psiR, nullptr);
          eval_state(O, F.eR, N, u, psiR, UR);
          // dF~/dUL and dF~/dUR
          double JL[MAXV * MAXV], JR[MAXV * MAXV];
          cs_jac(V, UL, [&](const cd* Uc, cd* Fc) {
            cd URc[MAXV];
            for (int v = 0; v < V; ++v) URc[v] = UR[v];
            num_flux(O, Uc, URc, nh, Fc);
          }, JL);
          cs_jac(V, UR, [&](const cd* Uc, cd* Fc) {
            cd ULc[MAXV];
            for (int v = 0; v < V; ++v) ULc[v] = UL[v];
            num_flux(O, ULc, Uc, nh, Fc);
          }, JR);
          if (side == 0) { std::memcpy(Jown, JL, sizeof JL); std::memcpy(Joth, JR, sizeof JR); other = F.eR; for (int i = 0; i < N; ++i) psiE[i] = psiL[i], psiO[i] = psiR[i]; }
          else { std::memcpy(Jown, JR, sizeof JR); std::memcpy(Joth, JL, sizeof JL); other = F.eL; for (int i = 0; i < N; ++i) psiE[i] = psiR[i], psiO[i] = psiL[i]; }
        } else {
          double Ug[MAXV];
          ghost_any(O, F.tag, UL, nh, x, Ug);
          double JL[MAXV * MAXV], Jg[MAXV * MAXV], Gg[MAXV * MAXV];
          cs_jac(V, UL, [&](const cd* Uc, cd* Fc) {
            cd Ugc[MAXV];
            for (int v = 0; v < V; ++v) Ugc[v] = Ug[v];
            num_flux(O, Uc, Ugc, nh, Fc);
          }, JL);
          cs_jac(V, Ug, [&](const cd* Uc, cd* Fc) {
            cd ULc[MAXV];
            for (int v = 0; v < V; ++v) ULc[v] = UL[v];
            num_flux(O, ULc, Uc, nh, Fc);
          }, Jg);
          cs_jac(V, UL, [&](const cd* Uc, cd* Fc) { ghost_any(O, F.tag, Uc, nh, x, Fc); }, Gg);
          for (int v = 0; v < V; ++v)
            for (int wv = 0; wv < V; ++wv) {
              double s = JL[v * V + wv];
              for (int k2 = 0; k2 < V; ++k2) s += Jg[v * V + k2] * Gg[k2 * V + wv];
              Jown[v * V + wv] = s;
            }
          for (int i = 0; i < N; ++i) psiE[i] = psiL[i];
        }
        double sgn = side == 0 ? -1.0 : 1.0, wa = w * area;
        for (int v = 0; v < V; ++v)
          for (int wv = 0; wv < V; ++wv)
            for (int i = 0; i < N; ++i)
              for (int j = 0; j < N; ++j)
                De[(v * N + i) * n + wv * N + j] += sgn * wa * psiE[i] * psiE[j] * Jown[v * V + wv];
        if (Off && other >= 0) {
          double* Oe = Off + ((size_t)e * nfc + lf) * n * n;
          for (int v = 0; v < V; ++v)
            for (int wv = 0; wv < V; ++wv)
              for (int i = 0; i < N; ++i)
                for (int j = 0; j < N; ++j)
                  Oe[(v * N + i) * n + wv * N + j] += sgn * wa * psiE[i] * psiO[j] * Joth[v * V + wv];
        }
      }
    }
  }
}

int neighbour(const Oracle& O, int e, int lf) {
  const Face& F = O.faces[O.efc[(size_t)e * 2 * O.d + lf]];
  if (F.eR < 0) return -1;
  return O.eside[(size_t)e * 2 * O.d + lf] == 0 ? F.eR : F.eL;
}

// ---------------------------------------------------------------------------
// Pseudo-time step (Section 4, eq. (x3d)): dtau_E = CFL h_E / ((2p+1)(|v| + c))
// with h_E = 2 d |E| / |dE| and v, c from the cell-mean state u_0 psi_0.
// ---------------------------------------------------------------------------
void timestep(const Oracle& O, int p, int Np, double cfl, const double* u, double* dtau) {
  const int d = O.d, V = O.V;
  for (int e = 0; e < O.ne; ++e) {
    double phi0 = std::pow(0.5, 0.5 * d);  // phi_0 = L_0^d, constant
    double psi0 = O.T[(size_t)e * O.Nmax * O.Nmax] * phi0;
    double U[MAXV];
    for (int v = 0; v < V; ++v) U[v] = u[((size_t)e * V + v) * Np] * psi0;
    double q2 = 0.0;
    for (int a = 0; a < d; ++a) q2 += (U[1 + a] / U[0]) * (U[1 + a] / U[0]);
    double c = std::sqrt(O.gam * pressure(d, O.gam, U) / U[0]);
    dtau[e] = cfl * O.hE[e] / ((2.0 * p + 1.0) * (std::sqrt(q2) + c));
  }
}

// Density-residual norm (Section 4, eq. (cfl)): (1/|Omega|) [int R(rho)^2]^(1/2);
// with an orthonormal basis the integral is the sum of squared coefficients.
double rnorm(const Oracle& O, int Np, const double* r) {
  double s = 0.0;
  for (int e = 0; e < O.ne; ++e)
    for (int i = 0; i < Np; ++i) {
      double x = r[((size_t)e * O.V + 0) * Np + i];
      s += x * x;
    }
  return std::sqrt(s) / O.omega;
}

// ---------------------------------------------------------------------------
// Pressure drag coefficient, the functional of the adjoint study: the force
// of the fluid on the slip walls projected on the direction dir,
//   C_D = -(1 / (q_inf S_ref)) sum_{wall faces} int p(U) n^ . dir dsigma,
// n^ the element's outward unit normal (it points into the body, so -p n^ is
// the pressure force on the body), q_inf = rho_inf |v_inf|^2 / 2 (rho_inf =
// 1, |v_inf| = Ma), U the element's trace, with the face quadrature of the
// residual at level p.  grad (nullable, [E][V][N_p]) receives dC_D/du: the
// pressure's derivative by complex step at each quadrature point times
// psi_i(x_k) and the same weight.
// ---------------------------------------------------------------------------
double drag(const Oracle& O, int p, const double* u, const double* dir, double sref, double* grad) {
  const int d = O.d, V = O.V, N = nmodes(d, p), Q = p + 2;
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  int nq = 1;
  for (int k = 0; k < d; ++k) nq *= Q;
  const int nqf = nq / Q;
  const double scale = -1.0 / (0.5 * O.mach * O.mach * sref);
  if (grad) for (size_t i = 0; i < (size_t)O.ne * V * N; ++i) grad[i] = 0.0;
  double cd = 0.0;
  for (const Face& F : O.faces) {
    if (F.tag != 1) continue;
    double psi[128];
    for (int k = 0; k < nqf; ++k) {
      double xiL[MAXD], xiR[MAXD], w;
      face_point(O, F, Q, xg, wg, k, xiL, xiR, w);
      double x[MAXD], det, c[MAXD][MAXD];
      elem_basis(O, F.eL, N, xiL, psi, nullptr, x, &det, c);
      double sg = (F.fL % 2) ? 1.0 : -1.0, nh[MAXD], area2 = 0.0;
      for (int a = 0; a < d; ++a) { nh[a] = sg * c[F.fL / 2][a]; area2 += nh[a] * nh[a]; }
      double area = std::sqrt(area2), nd = 0.0;
      for (int a = 0; a < d; ++a) nd += nh[a] / area * dir[a];
      double U[MAXV];
      eval_state(O, F.eL, N, u, psi, U);
      const double wt = scale * w * area * nd;
      cd += wt * pressure(d, O.gam, U);
      if (grad) {
        double dp[MAXV];
        for (int v = 0; v < V; ++v) {
          cd_t Uc[MAXV];
          for (int q = 0; q < V; ++q) Uc[q] = cd_t(U[q], q == v ? 1e-30 : 0.0);
          dp[v] = pressure(d, O.gam, Uc).imag() / 1e-30;
        }
        for (int v = 0; v < V; ++v)
          for (int i = 0; i < N; ++i) grad[((size_t)F.eL * V + v) * N + i] += wt * dp[v] * psi[i];
      }
    }
  }
  return cd;
}

// Dense LU with partial pivoting (row-major), and solve.
bool lu_factor(int n, double* A, int* piv) {
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double mx = std::fabs(A[k * n + k]);
    for (int i = k + 1; i < n; ++i) if (std::fabs(A[i * n + k]) > mx) { mx = std::fabs(A[i * n + k]); pr = i; }
    piv[k] = pr;
    if (mx == 0.0) return false;
    if (pr != k) for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[pr * n + j]);
    for (int i = k + 1; i < n; ++i) {
      A[i * n + k] /= A[k * n + k];
      double l = A[i * n + k];
      for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
    }
  }
  return true;
}
void lu_solve(int n, const double* A, const int* piv, double* b) {
  for (int k = 0; k < n; ++k) if (piv[k] != k) std::swap(b[k], b[piv[k]]);
  for (int i = 0; i < n; ++i) { double s = b[i]; for (int j = 0; j < i; ++j) s -= A[i * n + j] * b[j]; b[i] = s; }
  for (int i = n - 1; i >= 0; --i) { double s = b[i]; for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j]; b[i] = s / A[i * n + i]; }
}

void add_forcing(size_t n, double* r, const double* f) { if (f) for (size_t i = 0; i < n; ++i) r[i] += f[i]; }

// ---------------------------------------------------------------------------
// s-stage preconditioned Runge-Kutta step (Section 2.3, eq. (prk_scalar)):
//   u^(k) = u^n + beta_k P^{-1}(u^n) [R(u^(k-1)) + f],  beta_k = 1/(s-k+1),
// with P the element block of I/dtau - dR/du (the diagonal shift of the end of
// Section 2.3; sign read so that P is the backward-Euler block of du/dt = R),
// frozen at u^n.  R1 (optional) is the stage-1 residual R(u^n) + f.
// ---------------------------------------------------------------------------
bool prk(const Oracle& O, int p, int s, double cfl, double* u, const double* f, const double* R1) {
  const int V = O.V, N = nmodes(O.d, p), n = V * N;
  const size_t K = (size_t)O.ne * n;
  std::vector<double> dtau(O.ne), D((size_t)O.ne * n * n), un(u, u + K), R(K);
  std::vector<int> piv((size_t)O.ne * n);
  timestep(O, p, N, cfl, u, dtau.data());
  jacobian_blocks(O, p, u, D.data(), nullptr);
  bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
  for (int e = 0; e < O.ne; ++e) {
    double* P = &D[(size_t)e * n * n];
    for (int i = 0; i < n * n; ++i) P[i] = -P[i];
    for (int i = 0; i < n; ++i) P[i * n + i] += 1.0 / dtau[e];
    if (!lu_factor(n, P, &piv[(size_t)e * n])) ok = false;
  }
  if (!ok) return false;
  for (int k = 1; k <= s; ++k) {
    if (k == 1 && R1) {
      std::copy(R1, R1 + K, R.begin());
    } else {
      residual_t<double>(O, p, u, R.data());
      add_forcing(K, R.data(), f);
    }
    double bk = 1.0 / (s - k + 1.0);
#pragma omp parallel for schedule(static)
    for (int e = 0; e < O.ne; ++e) {
      double x[640];
      for (int i = 0; i < n; ++i) x[i] = R[(size_t)e * n + i];
      lu_solve(n, &D[(size_t)e * n * n], &piv[(size_t)e * n], x);
      for (int i = 0; i < n; ++i) u[(size_t)e * n + i] = un[(size_t)e * n + i] + bk * x[i];
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// Small dense matrix exponential: diagonal Pade approximant of degree 13 with
// scaling and squaring (Higham, SIAM J. Matrix Anal. Appl. 26 (2005) 1179).
// This stands in for the paper's rational approximation of exp(dt H_m)
// (end of Section 2.2).
// ---------------------------------------------------------------------------
void matmul(int n, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      C[i * n + j] = s;
    }
}

bool expm(int n, const double* A, double* E) {
  static const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                               1187353796428800.0,  129060195264000.0,   10559470521600.0,
                               670442572800.0,      33522128640.0,       1323241920.0,
                               40840800.0,          960960.0,            16380.0,
                               182.0,               1.0};
  const double theta13 = 5.371920351148152;
  double nrm = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(A[i * n + j]);
    nrm = std::max(nrm, s);
  }
  int sq = 0;
  if (nrm > theta13) sq = std::max(0, (int)std::ceil(std::log2(nrm / theta13)));
  const size_t nn = (size_t)n * n;
  std::vector<double> B(nn), B2(nn), B4(nn), B6(nn), U(nn), Vm(nn), W(nn), Tm(nn);
  double sc = std::ldexp(1.0, -sq);
  for (size_t i = 0; i < nn; ++i) B[i] = A[i] * sc;
  matmul(n, B.data(), B.data(), B2.data());
  matmul(n, B2.data(), B2.data(), B4.data());
  matmul(n, B4.data(), B2.data(), B6.data());
  for (size_t i = 0; i < nn; ++i) W[i] = b[13] * B6[i] + b[11] * B4[i] + b[9] * B2[i];
  matmul(n, B6.data(), W.data(), Tm.data());
  for (size_t i = 0; i < nn; ++i) Tm[i] += b[7] * B6[i] + b[5] * B4[i] + b[3] * B2[i];
  for (int i = 0; i < n; ++i) Tm[(size_t)i * n + i] += b[1];
  matmul(n, B.data(), Tm.data(), U.data());
  for (size_t i = 0; i < nn; ++i) W[i] = b[12] * B6[i] + b[10] * B4[i] + b[8] * B2[i];
  matmul(n, B6.data(), W.data(), Vm.data());
  for (size_t i = 0; i < nn; ++i) Vm[i] += b[6] * B6[i] + b[4] * B4[i] + b[2] * B2[i];
  for (int i = 0; i < n; ++i) Vm[(size_t)i * n + i] += b[0];
  // (V - U) X = (V + U)
  std::vector<double> Pm(nn), Rhs(nn);
  for (size_t i = 0; i < nn; ++i) { Pm[i] = Vm[i] - U[i]; Rhs[i] = Vm[i] + U[i]; }
  std::vector<int> piv(n);
  if (!lu_factor(n, Pm.data(), piv.data())) return false;
  std::vector<double> col(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) col[i] = Rhs[(size_t)i * n + j];
    lu_solve(n, Pm.data(), piv.data(), col.data());
    for (int i = 0; i < n; ++i) E[(size_t)i * n + j] = col[i];
  }
  for (int k = 0; k < sq; ++k) {
    matmul(n, E, E, Tm.data());
    std::copy(Tm.begin(), Tm.end(), E);
  }
  return true;
}

// phi_1(H) e_1 for an m x m matrix H (row-major), from the exponential of the
// augmented matrix [[H, e_1], [0, 0]] whose last column holds phi_1(H) e_1.
bool phi1_e1(int m, const double* H, double* y) {
  const int n = m + 1;
  std::vector<double> A((size_t)n * n, 0.0), E((size_t)n * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) A[(size_t)i * n + j] = H[(size_t)i * m + j];
  A[(size_t)0 * n + m] = 1.0;
  if (!expm(n, A.data(), E.data())) return false;
  for (int i = 0; i < m; ++i) y[i] = E[(size_t)i * n + m];
  return true;
}

// ---------------------------------------------------------------------------
// Arnoldi with (twice-swept) modified Gram-Schmidt (Section 2.2, eqs. (vm)-(vm2)):
// A V_m = V_{m+1} H~_m, v_1 = b / ||b||.  Stops early (happy breakdown) when
// h_{j+1,j} <= 1e-12 ||A v_j||.  Returns the number of columns used.
// ---------------------------------------------------------------------------
template <class MatVec>
int arnoldi(size_t K, int m, const double* b, MatVec Av, std::vector<double>& Vb, std::vector<double>& H, double& beta) {
  Vb.assign(K * (m + 1), 0.0);
  H.assign((size_t)(m + 1) * m, 0.0);
  double s = 0.0;
  for (size_t i = 0; i < K; ++i) s += b[i] * b[i];
  beta = std::sqrt(s);
  if (beta == 0.0) return 0;
  for (size_t i = 0; i < K; ++i) Vb[i] = b[i] / beta;
  std::vector<double> w(K);
  for (int j = 0; j < m; ++j) {
    Av(&Vb[(size_t)j * K], w.data());
    double w0 = 0.0;
    for (size_t i = 0; i < K; ++i) w0 += w[i] * w[i];
    w0 = std::sqrt(w0);
    // modified Gram-Schmidt, swept twice so that V_m^T V_m = I holds to
    // rounding (eq. (vm2) relies on it; one sweep loses orthogonality once
    // the Krylov space is nearly exhausted)
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (int i = 0; i <= j; ++i) {
        double h = 0.0;
        const double* vi = &Vb[(size_t)i * K];
        for (size_t k = 0; k < K; ++k) h += w[k] * vi[k];
        H[(size_t)i * m + j] += h;
        for (size_t k = 0; k < K; ++k) w[k] -= h * vi[k];
      }
    }
    double hn = 0.0;
    for (size_t k = 0; k < K; ++k) hn += w[k] * w[k];
    hn = std::sqrt(hn);
    H[(size_t)(j + 1) * m + j] = hn;
    if (hn <= 1e-12 * w0) return j + 1;
    for (size_t k = 0; k < K; ++k) Vb[(size_t)(j + 1) * K + k] = w[k] / hn;
  }
  return m;
}

// ---------------------------------------------------------------------------
// EXP1 step on the p = 0 level (Section 2.1, eq. (EXP1); Section 2.2,
// eq. (final)):  u <- u + phi_1(A) b with A = T J_0, b = T (R_0(u) + f),
// T = diag(dt_E), dt_E = (pmax+1) dtau_E (Section 4; dtau with p = pmax,
// element-local), J_0 the exact first-order Jacobian.  phi_1(A) b is
// approximated by beta V_m phi_1(H_m) e_1.
// ---------------------------------------------------------------------------
struct Exp1Info { int m_used; double beta; };

bool exp1(const Oracle& O, int pmax, int m, double cfl, double* u0, const double* f0, Exp1Info* info) {
  const int d = O.d, V = O.V, nfc = 2 * d;
  const size_t K = (size_t)O.ne * V;
  std::vector<double> dtau(O.ne), R(K), Dg((size_t)O.ne * V * V), Off((size_t)O.ne * nfc * V * V), b(K);
  timestep(O, pmax, 1, cfl, u0, dtau.data());
  for (int e = 0; e < O.ne; ++e) dtau[e] *= (pmax + 1.0);
  residual_t<double>(O, 0, u0, R.data());
  add_forcing(K, R.data(), f0);
  jacobian_blocks(O, 0, u0, Dg.data(), Off.data());
  for (int e = 0; e < O.ne; ++e) for (int v = 0; v < V; ++v) b[(size_t)e * V + v] = dtau[e] * R[(size_t)e * V + v];
  auto Av = [&](const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int e = 0; e < O.ne; ++e) {
      for (int v = 0; v < V; ++v) {
        double s = 0.0;
        for (int w = 0; w < V; ++w) s += Dg[((size_t)e * V + v) * V + w] * x[(size_t)e * V + w];
        for (int lf = 0; lf < nfc; ++lf) {
          int nb = neighbour(O, e, lf);
          if (nb < 0) continue;
          for (int w = 0; w < V; ++w) s += Off[(((size_t)e * nfc + lf) * V + v) * V + w] * x[(size_t)nb * V + w];
        }
        y[(size_t)e * V + v] = dtau[e] * s;
      }
    }
  };
  std::vector<double> Vb, H;
  double beta = 0.0;
  int mu = arnoldi(K, m, b.data(), Av, Vb, H, beta);
  if (info) { info->m_used = mu; info->beta = beta; }
  if (mu == 0) return true;
  std::vector<double> Hm((size_t)mu * mu), y(mu);
  for (int i = 0; i < mu; ++i)
    for (int j = 0; j < mu; ++j) Hm[(size_t)i * mu + j] = H[(size_t)i * m + j];
  if (!phi1_e1(mu, Hm.data(), y.data())) return false;
  for (size_t k = 0; k < K; ++k) {
    double s = 0.0;
    for (int j = 0; j < mu; ++j) s += Vb[(size_t)j * K + k] * y[j];
    u0[k] += beta * s;
  }
  return true;
}

// Modal restriction (truncation) and prolongation (zero padding) between
// levels p and p-1 (Section 2.4, steps 2 and 6): with a hierarchical
// orthonormal basis these are the L2 projection and the natural injection.
void truncate(const Oracle& O, int Nf, int Nc, const double* x, double* y) {
  for (int e = 0; e < O.ne; ++e)
    for (int v = 0; v < O.V; ++v)
      for (int i = 0; i < Nc; ++i) y[((size_t)e * O.V + v) * Nc + i] = x[((size_t)e * O.V + v) * Nf + i];
}
void add_padded(const Oracle& O, int Nf, int Nc, const double* x, double* y) {
  for (int e = 0; e < O.ne; ++e)
    for (int v = 0; v < O.V; ++v)
      for (int i = 0; i < Nc; ++i) y[((size_t)e * O.V + v) * Nf + i] += x[((size_t)e * O.V + v) * Nc + i];
}

struct Cyc { int pmax, s, m; double cfl_max; };

// ---------------------------------------------------------------------------
// V-cycle (Section 2.4): PRK on p >= 1, EXP1 on p = 0, FAS coarse forcing.
// The forcing is read as f_{p-1} = Trunc(R_p(u) + f_p) - R_{p-1}(Trunc u), so
// the coarse residual at the restricted state equals the restricted fine
// residual (the printed s^{p-1} has its sign garbled).  One PRK step before
// restriction, no post-smoothing.
// ---------------------------------------------------------------------------
bool vcycle_rec(const Oracle& O, const Cyc& C, int p, double cfl, double* u, const double* f, const double* R1) {
  const int V = O.V, N = nmodes(O.d, p);
  if (p == 0) return exp1(O, C.pmax, C.m, cfl, u, f, nullptr);
  if (!prk(O, p, C.s, cfl, u, f, R1)) return false;
  const int Nc = nmodes(O.d, p - 1);
  const size_t K = (size_t)O.ne * V * N, Kc = (size_t)O.ne * V * Nc;
  std::vector<double> r(K), v0(Kc), rc(Kc), fc(Kc), Rc(Kc);
  residual_t<double>(O, p, u, r.data());
  add_forcing(K, r.data(), f);
  truncate(O, N, Nc, u, v0.data());
  truncate(O, N, Nc, r.data(), rc.data());
  residual_t<double>(O, p - 1, v0.data(), Rc.data());
  for (size_t i = 0; i < Kc; ++i) fc[i] = rc[i] - Rc[i];
  std::vector<double> v(v0);
  if (!vcycle_rec(O, C, p - 1, cfl, v.data(), fc.data(), (p - 1 >= 1) ? rc.data() : nullptr)) return false;
  for (size_t i = 0; i < Kc; ++i) v[i] -= v0[i];
  add_padded(O, N, Nc, v.data(), u);
  return true;
}

// CFL ramp (Section 4, eq. (cfl)).  The residual norm entering the ramp is
// divided by rref: rref = 1 is the literal formula; rref = r_1 (the norm at
// the first iteration) makes the ramp start at CFL = 1 and grow as the
// residual falls, which is the behaviour the text describes.
double cfl_ramp(double cfl_max, double rn, double rref, int n, int pmax) {
  double a = (rn > 0.0) ? rref / rn : HUGE_VAL;
  double b = 1.0 + (n - 1.0) / (2.0 * pmax + 1.0);
  return std::min(cfl_max, std::max(a, b));
}

}  // namespace

// ===========================================================================
// C interface (used by the tests through ctypes)
// ===========================================================================
extern "C" {

void* orc_create(int dim, int n_vert, const double* xyz, int n_elem, const int32_t* ev, const int8_t* tag,
                 const double* geo, int pmax, double gamma, double mach, double alpha_deg, double beta_deg,
                 char* errbuf, int errlen) {
  Oracle* O = new Oracle;
  O->d = dim;
  O->nv = n_vert;
  O->ne = n_elem;
  O->pmax = pmax;
  O->gam = gamma;
  O->mach = mach;
  O->alpha = alpha_deg * M_PI / 180.0;
  O->beta = beta_deg * M_PI / 180.0;
  O->xyz.assign(xyz, xyz + (size_t)n_vert * dim);
  O->ev.assign(ev, ev + (size_t)n_elem * (1 << dim));
  O->tag.assign(tag, tag + (size_t)n_elem * 2 * dim);
  if (geo && (dim == 2 || dim == 3)) O->geo.assign(geo, geo + (size_t)n_elem * (dim == 2 ? 18 : 81));
  if ((dim != 2 && dim != 3) || pmax < 0 || pmax > 6 || !setup(*O)) {
    if (errbuf && errlen > 0) std::snprintf(errbuf, errlen, "%s", O->err.c_str());
    delete O;
    return nullptr;
  }
  return O;
}

void orc_free(void* h) { delete static_cast<Oracle*>(h); }

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int orc_get_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int orc_nmodes(int dim, int p) { return nmodes(dim, p); }
int orc_nfaces(void* h) { return (int)static_cast<Oracle*>(h)->faces.size(); }

void orc_gauss(int Q, double* x, double* w) {
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  for (int i = 0; i < Q; ++i) { x[i] = xg[i]; w[i] = wg[i]; }
}

void orc_modes(int dim, int p, int32_t* a /*[N][3]*/) {
  auto m = mode_list(dim, p);
  for (size_t k = 0; k < m.size(); ++k) for (int r = 0; r < 3; ++r) a[k * 3 + r] = m[k][r];
}

void orc_geometry(void* h, double* vol, double* surf, double* hE, double* omega) {
  Oracle& O = *static_cast<Oracle*>(h);
  for (int e = 0; e < O.ne; ++e) { vol[e] = O.vol[e]; surf[e] = O.surf[e]; hE[e] = O.hE[e]; }
  *omega = O.omega;
}

void orc_basis_T(void* h, double* T) {
  Oracle& O = *static_cast<Oracle*>(h);
  std::memcpy(T, O.T.data(), O.T.size() * sizeof(double));
}

void orc_neighbours(void* h, int32_t* nb /*[E][2d]*/) {
  Oracle& O = *static_cast<Oracle*>(h);
  for (int e = 0; e < O.ne; ++e) for (int f = 0; f < 2 * O.d; ++f) nb[(size_t)e * 2 * O.d + f] = neighbour(O, e, f);
}

// Evaluate the level-p state of element e at reference point xi.
void orc_eval_point(void* h, int p, int e, const double* u, const double* xi, double* U, double* x) {
  Oracle& O = *static_cast<Oracle*>(h);
  int N = nmodes(O.d, p);
  double psi[128], det, c[MAXD][MAXD];
  elem_basis(O, e, N, xi, psi, nullptr, x, &det, c);
  eval_state(O, e, N, u, psi, U);
}

void orc_freestream_state(void* h, double* U) {
  Oracle& O = *static_cast<Oracle*>(h);
  for (int v = 0; v < O.V; ++v) U[v] = O.Uinf[v];
}

// Uniform free stream as a level-p coefficient vector: u_{E,v,0} = U_v / psi_0.
void orc_freestream(void* h, int p, double* u) {
  Oracle& O = *static_cast<Oracle*>(h);
  int N = nmodes(O.d, p);
  double phi0 = std::pow(0.5, 0.5 * O.d);
  for (int e = 0; e < O.ne; ++e) {
    double psi0 = O.T[(size_t)e * O.Nmax * O.Nmax] * phi0;
    for (int v = 0; v < O.V; ++v)
      for (int i = 0; i < N; ++i) u[((size_t)e * O.V + v) * N + i] = (i == 0) ? O.Uinf[v] / psi0 : 0.0;
  }
}

void orc_residual(void* h, int p, const double* u, double* r) {
  residual_t<double>(*static_cast<Oracle*>(h), p, u, r);
}

// Complex residual for brute-force complex-step tests.
void orc_residual_complex(void* h, int p, const double* ure, const double* uim, double* rre, double* rim) {
  Oracle& O = *static_cast<Oracle*>(h);
  size_t K = (size_t)O.ne * O.V * nmodes(O.d, p);
  std::vector<cd> u(K), r(K);
  for (size_t i = 0; i < K; ++i) u[i] = cd(ure[i], uim[i]);
  residual_t<cd>(O, p, u.data(), r.data());
  for (size_t i = 0; i < K; ++i) { rre[i] = r[i].real(); rim[i] = r[i].imag(); }
}

void orc_jacobian_blocks(void* h, int p, const double* u, double* D, double* Off) {
  jacobian_blocks(*static_cast<Oracle*>(h), p, u, D, Off);
}

void orc_flux_jac(int dim, double gamma, const double* U, const double* g, double* K) { flux_jac(dim, gamma, U, g, K); }

void orc_rusanov(int dim, double gamma, const double* UL, const double* UR, const double* nh, double* F) {
  rusanov<double>(dim, gamma, UL, UR, nh, F);
}

// Jacobians of the Rusanov flux with respect to each trace, by complex step
// through the same templated flux the element Jacobians use (tests of the
// derivative tie semantics).  JL[v][w] = dF_v/dUL_w, JR likewise.
void orc_rusanov_jac(int dim, double gamma, const double* UL, const double* UR, const double* nh, double* JL,
                     double* JR) {
  const int V = dim + 2;
  cs_jac(V, UL, [&](const cd* Uc, cd* Fc) {
    cd Ur[MAXV];
    for (int v = 0; v < V; ++v) Ur[v] = cd(UR[v], 0.0);
    rusanov<cd>(dim, gamma, Uc, Ur, nh, Fc);
  }, JL);
  cs_jac(V, UR, [&](const cd* Uc, cd* Fc) {
    cd Ul[MAXV];
    for (int v = 0; v < V; ++v) Ul[v] = cd(UL[v], 0.0);
    rusanov<cd>(dim, gamma, Ul, Uc, nh, Fc);
  }, JR);
}

void orc_set_flux(void* h, int flux) { static_cast<Oracle*>(h)->flux = flux; }

void orc_roe(int dim, double gamma, const double* UL, const double* UR, const double* nh, double* F) {
  roe<double>(dim, gamma, UL, UR, nh, F);
}

// Jacobians of the Roe flux with respect to each trace by complex step.
void orc_roe_jac(int dim, double gamma, const double* UL, const double* UR, const double* nh, double* JL,
                 double* JR) {
  const int V = dim + 2;
  cs_jac(V, UL, [&](const cd* Uc, cd* Fc) {
    cd Ur[MAXV];
    for (int v = 0; v < V; ++v) Ur[v] = cd(UR[v], 0.0);
    roe<cd>(dim, gamma, Uc, Ur, nh, Fc);
  }, JL);
  cs_jac(V, UR, [&](const cd* Uc, cd* Fc) {
    cd Ul[MAXV];
    for (int v = 0; v < V; ++v) Ul[v] = cd(UL[v], 0.0);
    roe<cd>(dim, gamma, Ul, Uc, nh, Fc);
  }, JR);
}

void orc_ghost(void* h, int tg, const double* U, const double* nh, const double* x, double* Ug) {
  ghost_any<double>(*static_cast<Oracle*>(h), tg, U, nh, x, Ug);
}

// dtau for order p from a level vector with Nu modes per variable.
void orc_timestep(void* h, int p, int Nu, double cfl, const double* u, double* dtau) {
  Oracle& O = *static_cast<Oracle*>(h);
  timestep(O, p, Nu, cfl, u, dtau);
}

double orc_rnorm(void* h, int p, const double* r) {
  Oracle& O = *static_cast<Oracle*>(h);
  return rnorm(O, nmodes(O.d, p), r);
}

double orc_cfl_ramp(double cfl_max, double rn, double rref, int n, int pmax) { return cfl_ramp(cfl_max, rn, rref, n, pmax); }

double orc_drag(void* h, int p, const double* u, const double* dir, double sref, double* grad) {
  return drag(*static_cast<Oracle*>(h), p, u, dir, sref, grad);
}

int orc_prk(void* h, int p, int s, double cfl, double* u, const double* f) {
  return prk(*static_cast<Oracle*>(h), p, s, cfl, u, f, nullptr) ? 0 : 1;
}

int orc_exp1(void* h, int pmax, int m, double cfl, double* u0, const double* f0, int* m_used, double* beta) {
  Exp1Info inf{0, 0.0};
  bool ok = exp1(*static_cast<Oracle*>(h), pmax, m, cfl, u0, f0, &inf);
  if (m_used) *m_used = inf.m_used;
  if (beta) *beta = inf.beta;
  return ok ? 0 : 1;
}

int orc_expm(int n, const double* A, double* E) { return expm(n, A, E) ? 0 : 1; }
int orc_phi1_e1(int m, const double* H, double* y) { return phi1_e1(m, H, y) ? 0 : 1; }

// Arnoldi on an explicit dense matrix (tests of the Krylov identities).
int orc_arnoldi_dense(int K, int m, const double* A, const double* b, double* Vout, double* Hout, double* beta) {
  std::vector<double> Vb, H;
  auto Av = [&](const double* x, double* y) {
    for (int i = 0; i < K; ++i) { double s = 0.0; for (int j = 0; j < K; ++j) s += A[(size_t)i * K + j] * x[j]; y[i] = s; }
  };
  int mu = arnoldi((size_t)K, m, b, Av, Vb, H, *beta);
  std::memcpy(Vout, Vb.data(), Vb.size() * sizeof(double));
  std::memcpy(Hout, H.data(), H.size() * sizeof(double));
  return mu;
}

// One V-cycle.  rn_out receives r_n = ||R_rho(u)||/|Omega| of the state on
// entry; the CFL number of the cycle follows the ramp with that r_n.
int orc_vcycle(void* h, int pmax, int s, int m, double cfl_max, double rref, int n, double* u, const double* f,
               double* rn_out, double* cfl_out) {
  Oracle& O = *static_cast<Oracle*>(h);
  const size_t K = (size_t)O.ne * O.V * nmodes(O.d, pmax);
  std::vector<double> R(K);
  residual_t<double>(O, pmax, u, R.data());
  add_forcing(K, R.data(), f);
  double rn = rnorm(O, nmodes(O.d, pmax), R.data());
  if (rn_out) *rn_out = rn;
  if (!std::isfinite(rn)) return 2;
  double cfl = cfl_ramp(cfl_max, rn, rref, n, pmax);
  if (cfl_out) *cfl_out = cfl;
  Cyc C{pmax, s, m, cfl_max};
  return vcycle_rec(O, C, pmax, cfl, u, f, R.data()) ? 0 : 1;
}

// Steady solve: cycle n computes r_n at its entry state, stops if
// r_n <= drop r_1, else performs the V-cycle.  hist[0..] = r_1, r_2, ...
// relative_ramp != 0 feeds r_n / r_1 to the CFL ramp (else r_n).
// Returns 0 converged, 3 not converged after max_cycles, 2 diverged, 1 error.
int orc_solve(void* h, int pmax, int s, int m, double cfl_max, int relative_ramp, double drop, int max_cycles, double* u,
              const double* f, double* hist, int* n_cycles) {
  Oracle& O = *static_cast<Oracle*>(h);
  const size_t K = (size_t)O.ne * O.V * nmodes(O.d, pmax);
  std::vector<double> R(K);
  double r1 = 0.0;
  Cyc C{pmax, s, m, cfl_max};
  for (int n = 1;; ++n) {
    residual_t<double>(O, pmax, u, R.data());
    add_forcing(K, R.data(), f);
    double rn = rnorm(O, nmodes(O.d, pmax), R.data());
    hist[n - 1] = rn;
    if (n == 1) r1 = rn;
    *n_cycles = n - 1;
    if (!std::isfinite(rn)) return 2;
    if (rn <= drop * r1) return 0;
    if (n - 1 == max_cycles) return 3;
    double cfl = cfl_ramp(cfl_max, rn, relative_ramp ? r1 : 1.0, n, pmax);
    if (!vcycle_rec(O, C, pmax, cfl, u, f, R.data())) return 1;
  }
}

// Manufactured-solution support: L2 projection of the exact state, source
// forcing f_i = int psi_i div F(U_m) dx (divergence by complex step in x),
// and the L2 error of a level-p state, all with a (p+4)-point rule.
static void mms_loop(Oracle& O, int p, int mode, const double* uin, double* out, double* err) {
  const int d = O.d, V = O.V, N = nmodes(d, p), Q = p + 4;
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  int nq = 1;
  for (int k = 0; k < d; ++k) nq *= Q;
  double esum = 0.0;
  for (int e = 0; e < O.ne; ++e) {
    if (out) for (int i = 0; i < V * N; ++i) out[(size_t)e * V * N + i] = 0.0;
    double psi[128];
    for (int q = 0; q < nq; ++q) {
      double xi[MAXD], w = 1.0;
      int t = q;
      for (int k = 0; k < d; ++k) { xi[k] = xg[t % Q]; w *= wg[t % Q]; t /= Q; }
      double x[MAXD], det, c[MAXD][MAXD];
      elem_basis(O, e, N, xi, psi, nullptr, x, &det, c);
      double val[MAXV];
      if (mode == 0) {
        mms_state<double>(d, O.gam, x, val);
      } else if (mode == 1) {
        for (int v = 0; v < V; ++v) val[v] = 0.0;
        for (int a = 0; a < d; ++a) {
          cd xc[MAXD], Uc[MAXV], Fc[MAXV];
          for (int b = 0; b < d; ++b) xc[b] = x[b];
          xc[a] = cd(x[a], 1e-30);
          mms_state<cd>(d, O.gam, xc, Uc);
          double ea[MAXD] = {0, 0, 0};
          ea[a] = 1.0;
          flux_n<cd>(d, O.gam, Uc, ea, Fc);
          for (int v = 0; v < V; ++v) val[v] += Fc[v].imag() / 1e-30;
        }
      } else {
        double Um[MAXV], Uh[MAXV];
        mms_state<double>(d, O.gam, x, Um);
        eval_state(O, e, N, uin, psi, Uh);
        for (int v = 0; v < V; ++v) esum += w * det * (Uh[v] - Um[v]) * (Uh[v] - Um[v]);
        continue;
      }
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < N; ++i) out[((size_t)e * V + v) * N + i] += w * det * psi[i] * val[v];
    }
  }
  if (err) *err = std::sqrt(esum);
}

void orc_mms_project(void* h, int p, double* u) { mms_loop(*static_cast<Oracle*>(h), p, 0, nullptr, u, nullptr); }
void orc_mms_forcing(void* h, int p, double* f) { mms_loop(*static_cast<Oracle*>(h), p, 1, nullptr, f, nullptr); }
double orc_mms_error(void* h, int p, const double* u) {
  double e = 0.0;
  mms_loop(*static_cast<Oracle*>(h), p, 2, u, nullptr, &e);
  return e;
}

}  // extern "C"

// ===========================================================================
// Unstructured tetrahedra and prisms with the paper's basis (Section 3.2):
// normalised Cartesian monomials chi_j(x) = prod_k ((x_k - xc_k) / L_k)^a_k
// of total degree <= p (eq. (basis2)), orthonormalised per element by modified
// Gram-Schmidt in the element's L2 inner product (eq. (basis)).  xc is the
// element centroid (the integral of x over |E|), L_k half the element's extent
// along axis k.  Straight-sided elements; the residual follows eq. (euler3)
// exactly as for the tensor elements above.
//
// Readings (the paper is silent on them):
//  * Monomial order: total degree, then a_x descending, then a_y descending,
//    so the level-(p-1) space is a leading slice and MGS makes the basis
//    hierarchical.
//  * Quadrature: collapsed (Duffy) products of the (p+2)-point Gauss-Legendre
//    rule on [0, 1].  Tetrahedron: barycentric l1 = t1 (1-t2)(1-t3),
//    l2 = t2 (1-t3), l3 = t3, weight factor (1-t2)(1-t3)^2; prism: the
//    triangle l1 = t1 (1-t2), l2 = t2 times zeta = t3, weight (1-t2) |det|;
//    triangular face: l1 = t1 (1-t2), l2 = t2 over its vertices sorted by
//    global id; quadrilateral face: tensor rule on the bilinear patch of its
//    corners (cyclic, starting at the lowest id, towards the lower-id
//    neighbour).  The volume rule is exact to degree 2p+1 on tetrahedra.
//  * MGS, xc, and the basis of every level use the volume rule of p_max.
// ===========================================================================

namespace {

struct PFace {
  int eL, fL, eR, fR, tag, nv;
  int cv[4];   // canonical vertex ids
  double sgn;  // +1 if the canonical normal points out of eL, else -1
};

struct Poly {
  Oracle base;  // parameters, free stream, flux selection (d = 3, V = 5)
  int nv = 0, ne = 0, pmax = 0, Nmax = 0;
  std::vector<double> xyz;
  std::vector<int> typ, ev;          // [E], [E][6]
  std::vector<signed char> tag;      // [E][5]
  std::vector<PFace> faces;
  std::vector<int> efc, eside;       // [E][5]
  std::vector<double> xc, Ls, vol;   // [E][3], [E][3], [E]
  std::vector<double> surf, hE;      // [E]: |dE|, h_E = 2 d |E| / |dE|
  double omega = 0.0;                // |Omega|
  std::vector<double> S;             // [E][Nmax][Nmax], lower triangular
  std::vector<std::array<int, 3>> mono;
  std::string err;
};

const int TETF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
const int PRIF[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};

int pnmodes(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
int pnfaces(int t) { return t == 0 ? 4 : 5; }
int pnverts(int t) { return t == 0 ? 4 : 6; }

std::vector<std::array<int, 3>> poly_monomials(int p) {
  std::vector<std::array<int, 3>> m;
  for (int k = 0; k <= p; ++k)
    for (int a = k; a >= 0; --a)
      for (int b = k - a; b >= 0; --b) m.push_back({a, b, k - a - b});
  return m;
}

void face_vertices(const Poly& P, int e, int lf, int* vv, int* n) {
  const int t = P.typ[e];
  if (t == 0) {
    *n = 3;
    for (int k = 0; k < 3; ++k) vv[k] = P.ev[(size_t)e * 6 + TETF[lf][k]];
  } else {
    *n = lf < 2 ? 3 : 4;
    for (int k = 0; k < *n; ++k) vv[k] = P.ev[(size_t)e * 6 + PRIF[lf][k]];
  }
}

// Canonical order of a face's vertices (see the readings above).
void canonical(int n, const int* vv, int* cv) {
  if (n == 3) {
    for (int k = 0; k < 3; ++k) cv[k] = vv[k];
    std::sort(cv, cv + 3);
    return;
  }
  int k0 = 0;
  for (int k = 1; k < 4; ++k) if (vv[k] < vv[k0]) k0 = k;
  int nxt = vv[(k0 + 1) % 4], prv = vv[(k0 + 3) % 4];
  int dir = nxt < prv ? 1 : 3;
  for (int k = 0; k < 4; ++k) cv[k] = vv[(k0 + dir * k) % 4];
}

const double* pvx(const Poly& P, int v) { return &P.xyz[(size_t)v * 3]; }

// Volume rule of element e with Q points per direction: points and weights.
void poly_vol_rule(const Poly& P, int e, int Q, std::vector<double>& X, std::vector<double>& W) {
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  for (int k = 0; k < Q; ++k) { xg[k] = 0.5 * (1.0 + xg[k]); wg[k] *= 0.5; }
  X.clear();
  W.clear();
  const int* v = &P.ev[(size_t)e * 6];
  if (P.typ[e] == 0) {
    const double *A = pvx(P, v[0]), *B = pvx(P, v[1]), *C = pvx(P, v[2]), *D = pvx(P, v[3]);
    double J[3][3];
    for (int k = 0; k < 3; ++k) { J[k][0] = B[k] - A[k]; J[k][1] = C[k] - A[k]; J[k][2] = D[k] - A[k]; }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    for (int i3 = 0; i3 < Q; ++i3)
      for (int i2 = 0; i2 < Q; ++i2)
        for (int i1 = 0; i1 < Q; ++i1) {
          double t1 = xg[i1], t2 = xg[i2], t3 = xg[i3];
          double l1 = t1 * (1.0 - t2) * (1.0 - t3), l2 = t2 * (1.0 - t3), l3 = t3;
          for (int k = 0; k < 3; ++k) X.push_back(A[k] + l1 * J[k][0] + l2 * J[k][1] + l3 * J[k][2]);
          W.push_back(wg[i1] * wg[i2] * wg[i3] * (1.0 - t2) * (1.0 - t3) * (1.0 - t3) * std::fabs(det));
        }
  } else {
    const double* Vx[6];
    for (int a = 0; a < 6; ++a) Vx[a] = pvx(P, v[a]);
    for (int i3 = 0; i3 < Q; ++i3)
      for (int i2 = 0; i2 < Q; ++i2)
        for (int i1 = 0; i1 < Q; ++i1) {
          double t1 = xg[i1], t2 = xg[i2], z = xg[i3];
          double l1 = t1 * (1.0 - t2), l2 = t2, l0 = 1.0 - l1 - l2;
          double lam[3] = {l0, l1, l2};
          double J[3][3];
          for (int k = 0; k < 3; ++k) {
            double x = 0.0;
            for (int a = 0; a < 3; ++a) x += lam[a] * ((1.0 - z) * Vx[a][k] + z * Vx[a + 3][k]);
            X.push_back(x);
            J[k][0] = (1.0 - z) * (Vx[1][k] - Vx[0][k]) + z * (Vx[4][k] - Vx[3][k]);
            J[k][1] = (1.0 - z) * (Vx[2][k] - Vx[0][k]) + z * (Vx[5][k] - Vx[3][k]);
            J[k][2] = 0.0;
            for (int a = 0; a < 3; ++a) J[k][2] += lam[a] * (Vx[a + 3][k] - Vx[a][k]);
          }
          double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
          W.push_back(wg[i1] * wg[i2] * wg[i3] * (1.0 - t2) * std::fabs(det));
        }
  }
}

// Face rule over the canonical vertices: points, weights times |n dsigma|
// factor (so sum W = area) and unit normals (canonical orientation).
void poly_face_rule(const Poly& P, const PFace& F, int Q, std::vector<double>& X, std::vector<double>& W,
                    std::vector<double>& Nh) {
  std::vector<double> xg, wg;
  gauss_legendre(Q, xg, wg);
  for (int k = 0; k < Q; ++k) { xg[k] = 0.5 * (1.0 + xg[k]); wg[k] *= 0.5; }
  X.clear();
  W.clear();
  Nh.clear();
  const double *C0 = pvx(P, F.cv[0]), *C1 = pvx(P, F.cv[1]), *C2 = pvx(P, F.cv[2]);
  auto cross = [](const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
  };
  if (F.nv == 3) {
    double e1[3], e2[3], nv[3];
    for (int k = 0; k < 3; ++k) { e1[k] = C1[k] - C0[k]; e2[k] = C2[k] - C0[k]; }
    cross(e1, e2, nv);
    double a = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int i2 = 0; i2 < Q; ++i2)
      for (int i1 = 0; i1 < Q; ++i1) {
        double t1 = xg[i1], t2 = xg[i2], l1 = t1 * (1.0 - t2), l2 = t2;
        for (int k = 0; k < 3; ++k) X.push_back(C0[k] + l1 * e1[k] + l2 * e2[k]);
        W.push_back(wg[i1] * wg[i2] * (1.0 - t2) * a);
        for (int k = 0; k < 3; ++k) Nh.push_back(nv[k] / a);
      }
  } else {
    const double* C3 = pvx(P, F.cv[3]);
    for (int i2 = 0; i2 < Q; ++i2)
      for (int i1 = 0; i1 < Q; ++i1) {
        double s = xg[i1], t = xg[i2];
        double xs[3], xt[3], nv[3];
        for (int k = 0; k < 3; ++k) {
          X.push_back((1 - s) * (1 - t) * C0[k] + s * (1 - t) * C1[k] + s * t * C2[k] + (1 - s) * t * C3[k]);
          xs[k] = (1 - t) * (C1[k] - C0[k]) + t * (C2[k] - C3[k]);
          xt[k] = (1 - s) * (C3[k] - C0[k]) + s * (C2[k] - C1[k]);
        }
        cross(xs, xt, nv);
        double a = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        W.push_back(wg[i1] * wg[i2] * a);
        for (int k = 0; k < 3; ++k) Nh.push_back(nv[k] / a);
      }
  }
}

// Monomials chi_j and their x-gradients at x for element e (N of them).
void poly_chi(const Poly& P, int e, int N, const double* x, double* chi, double* gchi /*[N][3] or null*/) {
  double X[3];
  for (int k = 0; k < 3; ++k) X[k] = (x[k] - P.xc[(size_t)e * 3 + k]) / P.Ls[(size_t)e * 3 + k];
  for (int j = 0; j < N; ++j) {
    const auto& a = P.mono[j];
    double pw[3], dp[3];
    for (int k = 0; k < 3; ++k) {
      pw[k] = 1.0;
      for (int r = 0; r < a[k]; ++r) pw[k] *= X[k];
      dp[k] = 0.0;
      if (a[k] > 0) {
        double t = 1.0;
        for (int r = 0; r < a[k] - 1; ++r) t *= X[k];
        dp[k] = a[k] * t;
      }
    }
    chi[j] = pw[0] * pw[1] * pw[2];
    if (gchi) {
      gchi[j * 3 + 0] = dp[0] * pw[1] * pw[2] / P.Ls[(size_t)e * 3 + 0];
      gchi[j * 3 + 1] = pw[0] * dp[1] * pw[2] / P.Ls[(size_t)e * 3 + 1];
      gchi[j * 3 + 2] = pw[0] * pw[1] * dp[2] / P.Ls[(size_t)e * 3 + 2];
    }
  }
}

// psi_i = sum_j S_ij chi_j (and gradients).
void poly_psi(const Poly& P, int e, int N, const double* x, double* psi, double* gpsi) {
  double chi[64], gchi[64 * 3];
  poly_chi(P, e, N, x, chi, gpsi ? gchi : nullptr);
  const double* S = &P.S[(size_t)e * P.Nmax * P.Nmax];
  for (int i = 0; i < N; ++i) {
    double s = 0.0, g[3] = {0, 0, 0};
    for (int j = 0; j <= i; ++j) {
      s += S[i * P.Nmax + j] * chi[j];
      if (gpsi) for (int k = 0; k < 3; ++k) g[k] += S[i * P.Nmax + j] * gchi[j * 3 + k];
    }
    psi[i] = s;
    if (gpsi) for (int k = 0; k < 3; ++k) gpsi[i * 3 + k] = g[k];
  }
}

bool poly_setup(Poly& P) {
  Oracle& O = P.base;
  O.d = 3;
  O.V = 5;
  P.mono = poly_monomials(P.pmax);
  P.Nmax = pnmodes(P.pmax);
  P.efc.assign((size_t)P.ne * 5, -1);
  P.eside.assign((size_t)P.ne * 5, 0);
  std::map<std::vector<int>, int> open;
  for (int e = 0; e < P.ne; ++e) {
    if (P.typ[e] != 0 && P.typ[e] != 1) { P.err = "unknown element type"; return false; }
    for (int lf = 0; lf < pnfaces(P.typ[e]); ++lf) {
      int vv[4], n;
      face_vertices(P, e, lf, vv, &n);
      int tg = P.tag[(size_t)e * 5 + lf];
      if (tg != 0) {
        PFace F{e, lf, -1, -1, tg, n, {0, 0, 0, 0}, 1.0};
        canonical(n, vv, F.cv);
        P.efc[(size_t)e * 5 + lf] = (int)P.faces.size();
        P.faces.push_back(F);
        continue;
      }
      std::vector<int> key(vv, vv + n);
      std::sort(key.begin(), key.end());
      auto it = open.find(key);
      if (it == open.end()) {
        PFace F{e, lf, -1, -1, 0, n, {0, 0, 0, 0}, 1.0};
        canonical(n, vv, F.cv);
        open[key] = (int)P.faces.size();
        P.efc[(size_t)e * 5 + lf] = (int)P.faces.size();
        P.faces.push_back(F);
      } else {
        PFace& F = P.faces[it->second];
        F.eR = e;
        F.fR = lf;
        P.efc[(size_t)e * 5 + lf] = it->second;
        P.eside[(size_t)e * 5 + lf] = 1;
        open.erase(it);
      }
    }
  }
  if (!open.empty()) { P.err = "unmatched interior face"; return false; }
  // element extents, centroids and the MGS basis
  const int N = P.Nmax, Q = P.pmax + 2;
  P.xc.assign((size_t)P.ne * 3, 0.0);
  P.Ls.assign((size_t)P.ne * 3, 0.0);
  P.vol.assign(P.ne, 0.0);
  P.S.assign((size_t)P.ne * N * N, 0.0);
  bool ok = true;
  for (int e = 0; e < P.ne; ++e) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int a = 0; a < pnverts(P.typ[e]); ++a)
      for (int k = 0; k < 3; ++k) {
        double c = pvx(P, P.ev[(size_t)e * 6 + a])[k];
        lo[k] = std::min(lo[k], c);
        hi[k] = std::max(hi[k], c);
      }
    for (int k = 0; k < 3; ++k) P.Ls[(size_t)e * 3 + k] = 0.5 * (hi[k] - lo[k]);
    std::vector<double> X, W;
    poly_vol_rule(P, e, Q, X, W);
    const int nq = (int)W.size();
    double v = 0.0, m[3] = {0, 0, 0};
    for (int q = 0; q < nq; ++q) {
      v += W[q];
      for (int k = 0; k < 3; ++k) m[k] += W[q] * X[q * 3 + k];
    }
    P.vol[e] = v;
    for (int k = 0; k < 3; ++k) P.xc[(size_t)e * 3 + k] = m[k] / v;
    // modified Gram-Schmidt on the monomial values at the points, applying
    // the same operations to the coefficient rows
    std::vector<double> chi((size_t)nq * N), psiv((size_t)nq * N);
    for (int q = 0; q < nq; ++q) poly_chi(P, e, N, &X[q * 3], &chi[(size_t)q * N], nullptr);
    double* S = &P.S[(size_t)e * N * N];
    for (int i = 0; i < N; ++i) {
      std::vector<double> w(nq), c(N, 0.0);
      for (int q = 0; q < nq; ++q) w[q] = chi[(size_t)q * N + i];
      c[i] = 1.0;
      for (int j = 0; j < i; ++j) {
        double h = 0.0;
        for (int q = 0; q < nq; ++q) h += W[q] * w[q] * psiv[(size_t)q * N + j];
        for (int q = 0; q < nq; ++q) w[q] -= h * psiv[(size_t)q * N + j];
        for (int k = 0; k <= j; ++k) c[k] -= h * S[j * N + k];
      }
      double nn = 0.0;
      for (int q = 0; q < nq; ++q) nn += W[q] * w[q] * w[q];
      if (!(nn > 0.0)) { ok = false; break; }
      double s = 1.0 / std::sqrt(nn);
      for (int q = 0; q < nq; ++q) psiv[(size_t)q * N + i] = s * w[q];
      for (int k = 0; k <= i; ++k) S[i * N + k] = s * c[k];
    }
  }
  if (!ok) { P.err = "degenerate element (MGS)"; return false; }
  // outward orientation of the canonical face normal for the L element
  for (auto& F : P.faces) {
    double cE[3] = {0, 0, 0}, cF[3] = {0, 0, 0};
    int nve = pnverts(P.typ[F.eL]);
    for (int a = 0; a < nve; ++a)
      for (int k = 0; k < 3; ++k) cE[k] += pvx(P, P.ev[(size_t)F.eL * 6 + a])[k] / nve;
    for (int a = 0; a < F.nv; ++a)
      for (int k = 0; k < 3; ++k) cF[k] += pvx(P, F.cv[a])[k] / F.nv;
    std::vector<double> X, W, Nh;
    poly_face_rule(P, F, 2, X, W, Nh);
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += Nh[k] * (cF[k] - cE[k]);
    F.sgn = s < 0.0 ? -1.0 : 1.0;
  }
  // surfaces (the face rule of p_max) and the length scale of the
  // pseudo-time step, as on the hexahedra: h_E = 2 d |E| / |dE|
  P.surf.assign(P.ne, 0.0);
  for (const auto& F : P.faces) {
    std::vector<double> X, W, Nh;
    poly_face_rule(P, F, Q, X, W, Nh);
    double a = 0.0;
    for (double w : W) a += w;
    P.surf[F.eL] += a;
    if (F.eR >= 0) P.surf[F.eR] += a;
  }
  P.hE.assign(P.ne, 0.0);
  P.omega = 0.0;
  for (int e = 0; e < P.ne; ++e) {
    P.hE[e] = 6.0 * P.vol[e] / P.surf[e];
    P.omega += P.vol[e];
  }
  double vinf[3] = {O.mach * std::cos(O.alpha) * std::cos(O.beta), O.mach * std::sin(O.alpha) * std::cos(O.beta),
                    O.mach * std::sin(O.beta)};
  O.Uinf[0] = 1.0;
  double ke = 0.0;
  for (int a = 0; a < 3; ++a) { O.Uinf[1 + a] = vinf[a]; ke += vinf[a] * vinf[a]; }
  O.Uinf[4] = (1.0 / O.gam) / (O.gam - 1.0) + 0.5 * ke;
  return true;
}

template <class S> void poly_state(const Poly& P, int e, int N, const S* u, const double* psi, S* U) {
  for (int v = 0; v < 5; ++v) {
    S s = 0.0;
    for (int i = 0; i < N; ++i) s += u[((size_t)e * 5 + v) * N + i] * psi[i];
    U[v] = s;
  }
  (void)P;
}

// DG residual R_p(u) of eq. (euler3) on the tetrahedra and prisms:
//   R_{E,i} = - sum_faces int psi_i F~ . n^ dsigma + int_E F . grad psi_i dx,
// (p+2)-point collapsed rules in the volume and on every face; each face flux
// computed once with eL's outward normal and lifted to both sides.
template <class S> void poly_residual_t(const Poly& P, int p, const S* u, S* r) {
  const Oracle& O = P.base;
  const int V = 5, N = pnmodes(p), Q = p + 2;
#pragma omp parallel for schedule(static)
  for (int e = 0; e < P.ne; ++e) {
    S* re_ = r + (size_t)e * V * N;
    for (int i = 0; i < V * N; ++i) re_[i] = 0.0;
    std::vector<double> X, W;
    poly_vol_rule(P, e, Q, X, W);
    double psi[64], gpsi[64 * 3];
    for (size_t q = 0; q < W.size(); ++q) {
      poly_psi(P, e, N, &X[q * 3], psi, gpsi);
      S U[MAXV], F[3][MAXV];
      poly_state(P, e, N, u, psi, U);
      for (int a = 0; a < 3; ++a) {
        double ea[3] = {0, 0, 0};
        ea[a] = 1.0;
        flux_n(3, O.gam, U, ea, F[a]);
      }
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < N; ++i) {
          S s = 0.0;
          for (int a = 0; a < 3; ++a) s += F[a][v] * gpsi[i * 3 + a];
          re_[v * N + i] += W[q] * s;
        }
    }
  }
  const int nf = (int)P.faces.size(), nqf = Q * Q;
  std::vector<S> flux((size_t)nf * nqf * V);
#pragma omp parallel for schedule(static)
  for (int fc = 0; fc < nf; ++fc) {
    const PFace& F = P.faces[fc];
    std::vector<double> X, W, Nh;
    poly_face_rule(P, F, Q, X, W, Nh);
    double psiL[64], psiR[64];
    for (int k = 0; k < nqf; ++k) {
      double nh[3];
      for (int a = 0; a < 3; ++a) nh[a] = F.sgn * Nh[k * 3 + a];
      S UL[MAXV], UR[MAXV], Fl[MAXV];
      poly_psi(P, F.eL, N, &X[k * 3], psiL, nullptr);
      poly_state(P, F.eL, N, u, psiL, UL);
      if (F.eR >= 0) {
        poly_psi(P, F.eR, N, &X[k * 3], psiR, nullptr);
        poly_state(P, F.eR, N, u, psiR, UR);
      } else {
        ghost_any(O, F.tag, UL, nh, &X[k * 3], UR);
      }
      num_flux(O, UL, UR, nh, Fl);
      for (int v = 0; v < V; ++v) flux[((size_t)fc * nqf + k) * V + v] = W[k] * Fl[v];
    }
  }
#pragma omp parallel for schedule(static)
  for (int e = 0; e < P.ne; ++e) {
    S* re_ = r + (size_t)e * V * N;
    double psi[64];
    for (int lf = 0; lf < pnfaces(P.typ[e]); ++lf) {
      int fc = P.efc[(size_t)e * 5 + lf], side = P.eside[(size_t)e * 5 + lf];
      std::vector<double> X, W, Nh;
      poly_face_rule(P, P.faces[fc], Q, X, W, Nh);
      double sg = side == 0 ? -1.0 : 1.0;
      for (int k = 0; k < nqf; ++k) {
        poly_psi(P, e, N, &X[k * 3], psi, nullptr);
        for (int v = 0; v < V; ++v)
          for (int i = 0; i < N; ++i) re_[v * N + i] += sg * psi[i] * flux[((size_t)fc * nqf + k) * V + v];
      }
    }
  }
}

// Manufactured solution on the tetrahedra and prisms: L2 projection (mode 0)
// and the source f_i = int psi_i div F(U_m) dx (mode 1, divergence by complex
// step in x), with the (p+4)-point volume rule.
void poly_mms(const Poly& P, int p, int mode, double* out) {
  const int V = 5, N = pnmodes(p), Q = p + 4;
  const double g = P.base.gam;
  for (int e = 0; e < P.ne; ++e) {
    for (int i = 0; i < V * N; ++i) out[(size_t)e * V * N + i] = 0.0;
    std::vector<double> X, W;
    poly_vol_rule(P, e, Q, X, W);
    double psi[64];
    for (size_t q = 0; q < W.size(); ++q) {
      const double* x = &X[q * 3];
      poly_psi(P, e, N, x, psi, nullptr);
      double val[MAXV];
      if (mode == 0) {
        mms_state<double>(3, g, x, val);
      } else {
        for (int v = 0; v < V; ++v) val[v] = 0.0;
        for (int a = 0; a < 3; ++a) {
          cd xcx[3], Uc[MAXV], Fc[MAXV];
          for (int b = 0; b < 3; ++b) xcx[b] = x[b];
          xcx[a] = cd(x[a], 1e-30);
          mms_state<cd>(3, g, xcx, Uc);
          double ea[3] = {0, 0, 0};
          ea[a] = 1.0;
          flux_n<cd>(3, g, Uc, ea, Fc);
          for (int v = 0; v < V; ++v) val[v] += Fc[v].imag() / 1e-30;
        }
      }
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < N; ++i) out[((size_t)e * V + v) * N + i] += W[q] * psi[i] * val[v];
    }
  }
}

// Pseudo-time step on the tetrahedra and prisms (Section 4, eq. (x3d)), the
// definition of the hexahedra: dtau_E = CFL h_E / ((2p+1)(|v| + c)) with v, c
// from the cell-mean state u_0 psi_0 (psi_0 = S_00, chi_0 = 1).
// Np: modes per row of u (the cell mean is mode 0); p enters the formula.
void porc_timestep_impl(const Poly& P, int p, int Np, double cfl, const double* u, double* dtau) {
  for (int e = 0; e < P.ne; ++e) {
    const double psi0 = P.S[(size_t)e * P.Nmax * P.Nmax];
    double U[MAXV];
    for (int v = 0; v < 5; ++v) U[v] = u[((size_t)e * 5 + v) * Np] * psi0;
    double q2 = 0.0;
    for (int a = 0; a < 3; ++a) q2 += (U[1 + a] / U[0]) * (U[1 + a] / U[0]);
    const double c = std::sqrt(P.base.gam * pressure(3, P.base.gam, U) / U[0]);
    dtau[e] = cfl * P.hE[e] / ((2.0 * p + 1.0) * (std::sqrt(q2) + c));
  }
}

// The residual of element e alone (Section 3.1, eq. (euler3)): its volume
// term and its faces, with the flux taken from e's side (own state first,
// e's outward normal); the neighbours' states are real.  Equal to the rows
// of e in poly_residual_t up to rounding (the numerical fluxes are
// conservative: F~(a, b; n) = -F~(b, a; -n)).
template <class S> void poly_elem_residual(const Poly& P, int p, int e, const S* ue, const double* u, S* re) {
  const Oracle& O = P.base;
  const int V = 5, N = pnmodes(p), Q = p + 2;
  for (int i = 0; i < V * N; ++i) re[i] = 0.0;
  std::vector<double> X, W, Nh;
  poly_vol_rule(P, e, Q, X, W);
  double psi[64], gpsi[64 * 3];
  auto state = [&](const auto* c, S* U) {
    for (int v = 0; v < V; ++v) {
      S t = 0.0;
      for (int i = 0; i < N; ++i) t += c[v * N + i] * psi[i];
      U[v] = t;
    }
  };
  for (size_t q = 0; q < W.size(); ++q) {
    poly_psi(P, e, N, &X[q * 3], psi, gpsi);
    S U[MAXV], F[3][MAXV];
    state(ue, U);
    for (int a = 0; a < 3; ++a) {
      double ea[3] = {0, 0, 0};
      ea[a] = 1.0;
      flux_n(3, O.gam, U, ea, F[a]);
    }
    for (int v = 0; v < V; ++v)
      for (int i = 0; i < N; ++i) {
        S t = 0.0;
        for (int a = 0; a < 3; ++a) t += F[a][v] * gpsi[i * 3 + a];
        re[v * N + i] += W[q] * t;
      }
  }
  for (int lf = 0; lf < pnfaces(P.typ[e]); ++lf) {
    const int fc = P.efc[(size_t)e * 5 + lf], side = P.eside[(size_t)e * 5 + lf];
    const PFace& F = P.faces[fc];
    poly_face_rule(P, F, Q, X, W, Nh);
    const double so = (side == 0 ? 1.0 : -1.0) * F.sgn;  // e's outward orientation
    const int nb = side == 0 ? F.eR : F.eL;
    double psin[64];
    for (size_t k = 0; k < W.size(); ++k) {
      double nh[3];
      for (int a = 0; a < 3; ++a) nh[a] = so * Nh[k * 3 + a];
      poly_psi(P, e, N, &X[k * 3], psi, nullptr);
      S Ue[MAXV], Un[MAXV], Fl[MAXV];
      state(ue, Ue);
      if (nb >= 0) {
        poly_psi(P, nb, N, &X[k * 3], psin, nullptr);
        for (int v = 0; v < V; ++v) {
          double t = 0.0;
          for (int i = 0; i < N; ++i) t += u[((size_t)nb * V + v) * N + i] * psin[i];
          Un[v] = t;
        }
      } else {
        ghost_any(O, F.tag, Ue, nh, &X[k * 3], Un);
      }
      num_flux(O, Ue, Un, nh, Fl);
      for (int v = 0; v < V; ++v)
        for (int i = 0; i < N; ++i) re[v * N + i] -= W[k] * psi[i] * Fl[v];
    }
  }
}

// Element blocks D_E = dR_E/du_E (Section 3.3, eq. (jac1)) by complex step
// on poly_elem_residual, one column per own coefficient; [E][n][n] row-major,
// n = 5 N, rows and columns (v, i).
void poly_blocks(const Poly& P, int p, const double* u, double* D) {
  const int N = pnmodes(p), n = 5 * N;
  const double h = 1e-30;
#pragma omp parallel for schedule(dynamic)
  for (int e = 0; e < P.ne; ++e) {
    std::vector<cd> ue(n), re(n);
    for (int c = 0; c < n; ++c) {
      for (int i = 0; i < n; ++i) ue[i] = cd(u[(size_t)e * n + i], i == c ? h : 0.0);
      poly_elem_residual<cd>(P, p, e, ue.data(), u, re.data());
      for (int i = 0; i < n; ++i) D[((size_t)e * n + i) * n + c] = re[i].imag() / h;
    }
  }
}

// s-stage preconditioned Runge-Kutta step on the tetrahedra and prisms
// (Section 2.3, eq. (prk_scalar)), the same step as on the hexahedra:
//   u^(k) = u^n + beta_k P^{-1}(u^n) [R(u^(k-1)) + f],  beta_k = 1/(s-k+1),
// P = I/dtau_E - D_E frozen at u^n (the basis is orthonormal: mass = I).
bool poly_prk(const Poly& P, int p, int s, double cfl, double* u, const double* f) {
  const int N = pnmodes(p), n = 5 * N;
  const size_t K = (size_t)P.ne * n;
  std::vector<double> dtau(P.ne), D((size_t)P.ne * n * n), un(u, u + K), R(K);
  std::vector<int> piv((size_t)P.ne * n);
  porc_timestep_impl(P, p, pnmodes(p), cfl, u, dtau.data());
  poly_blocks(P, p, u, D.data());
  bool ok = true;
  for (int e = 0; e < P.ne; ++e) {
    double* A = &D[(size_t)e * n * n];
    for (int i = 0; i < n * n; ++i) A[i] = -A[i];
    for (int i = 0; i < n; ++i) A[i * n + i] += 1.0 / dtau[e];
    if (!lu_factor(n, A, &piv[(size_t)e * n])) ok = false;
  }
  if (!ok) return false;
  for (int k = 1; k <= s; ++k) {
    poly_residual_t<double>(P, p, u, R.data());
    add_forcing(K, R.data(), f);
    const double bk = 1.0 / (s - k + 1.0);
    for (int e = 0; e < P.ne; ++e) {
      std::vector<double> x(R.begin() + (size_t)e * n, R.begin() + (size_t)(e + 1) * n);
      lu_solve(n, &D[(size_t)e * n * n], &piv[(size_t)e * n], x.data());
      for (int i = 0; i < n; ++i) u[(size_t)e * n + i] = un[(size_t)e * n + i] + bk * x[i];
    }
  }
  return true;
}

// EXP1 on the p = 0 level of the tetrahedra and prisms (Section 2.1,
// eq. (EXP1); Section 2.2), the step of the hexahedra: u <- u + phi_1(A) b,
// A = T J_0, b = T (R_0(u) + f), T = diag((p_max+1) dtau_E) with dtau at
// p_max from the cell means; J_0 applied as the complex-step derivative of
// the p = 0 residual (exact for the linearisation).
bool poly_exp1(const Poly& P, int pmax, int m, double cfl, double* u0, const double* f0) {
  const size_t K = (size_t)P.ne * 5;
  std::vector<double> dt(P.ne), R(K), b(K);
  // the cell-mean state at level p_max has the coefficients of level 0
  porc_timestep_impl(P, pmax, 1, cfl, u0, dt.data());
  for (int e = 0; e < P.ne; ++e) dt[e] *= (pmax + 1.0);
  poly_residual_t<double>(P, 0, u0, R.data());
  add_forcing(K, R.data(), f0);
  for (size_t k = 0; k < K; ++k) b[k] = dt[k / 5] * R[k];
  const double h = 1e-30;
  std::vector<cd> uc(K), rc(K);
  auto Av = [&](const double* x, double* y) {
    for (size_t k = 0; k < K; ++k) uc[k] = cd(u0[k], h * x[k]);
    poly_residual_t<cd>(P, 0, uc.data(), rc.data());
    for (size_t k = 0; k < K; ++k) y[k] = dt[k / 5] * rc[k].imag() / h;
  };
  std::vector<double> Vb, H;
  double beta = 0.0;
  const int mu = arnoldi(K, m, b.data(), Av, Vb, H, beta);
  if (mu == 0) return true;
  std::vector<double> Hm((size_t)mu * mu), y(mu);
  for (int i = 0; i < mu; ++i)
    for (int j = 0; j < mu; ++j) Hm[(size_t)i * mu + j] = H[(size_t)i * m + j];
  if (!phi1_e1(mu, Hm.data(), y.data())) return false;
  for (size_t k = 0; k < K; ++k) {
    double t = 0.0;
    for (int j = 0; j < mu; ++j) t += Vb[(size_t)j * K + k] * y[j];
    u0[k] += beta * t;
  }
  return true;
}

// V-cycle on the tetrahedra and prisms (Section 2.4), the cycle of the
// hexahedra: PRK on p >= 1, FAS forcing f_{p-1} = Trunc(R_p(u) + f_p) -
// R_{p-1}(Trunc u), EXP1 on p = 0, prolongation of the coarse correction.
bool poly_vcycle_rec(const Poly& P, int pmax, int s, int m, int p, double cfl, double* u, const double* f) {
  if (p == 0) return poly_exp1(P, pmax, m, cfl, u, f);
  if (!poly_prk(P, p, s, cfl, u, f)) return false;
  const int N = pnmodes(p), Nc = pnmodes(p - 1);
  const size_t K = (size_t)P.ne * 5 * N, Kc = (size_t)P.ne * 5 * Nc;
  std::vector<double> r(K), v0(Kc), rc(Kc), fc(Kc), Rc(Kc);
  poly_residual_t<double>(P, p, u, r.data());
  add_forcing(K, r.data(), f);
  for (size_t ev = 0; ev < (size_t)P.ne * 5; ++ev)
    for (int i = 0; i < Nc; ++i) {
      v0[ev * Nc + i] = u[ev * N + i];
      rc[ev * Nc + i] = r[ev * N + i];
    }
  poly_residual_t<double>(P, p - 1, v0.data(), Rc.data());
  for (size_t i = 0; i < Kc; ++i) fc[i] = rc[i] - Rc[i];
  std::vector<double> v(v0);
  if (!poly_vcycle_rec(P, pmax, s, m, p - 1, cfl, v.data(), fc.data())) return false;
  for (size_t ev = 0; ev < (size_t)P.ne * 5; ++ev)
    for (int i = 0; i < Nc; ++i) u[ev * N + i] += v[ev * Nc + i] - v0[ev * Nc + i];
  return true;
}

double poly_rnorm_impl(const Poly& P, int p, const double* r) {
  const int Np = pnmodes(p);
  double t = 0.0;
  for (int e = 0; e < P.ne; ++e)
    for (int i = 0; i < Np; ++i) {
      const double x = r[((size_t)e * 5 + 0) * Np + i];
      t += x * x;
    }
  return std::sqrt(t) / P.omega;
}

}  // namespace

extern "C" {

void* porc_create(int n_vert, const double* xyz, int n_elem, const int8_t* typ, const int32_t* ev,
                  const int8_t* tag, int pmax, double gamma, double mach, double alpha_deg, double beta_deg,
                  char* errbuf, int errlen) {
  Poly* P = new Poly;
  P->nv = n_vert;
  P->ne = n_elem;
  P->pmax = pmax;
  P->base.gam = gamma;
  P->base.mach = mach;
  P->base.alpha = alpha_deg * M_PI / 180.0;
  P->base.beta = beta_deg * M_PI / 180.0;
  P->xyz.assign(xyz, xyz + (size_t)n_vert * 3);
  P->typ.assign(typ, typ + n_elem);
  P->ev.assign(ev, ev + (size_t)n_elem * 6);
  P->tag.assign(tag, tag + (size_t)n_elem * 5);
  if (pmax < 0 || pmax > 4 || !poly_setup(*P)) {
    if (pmax < 0 || pmax > 4) P->err = "pmax out of range";
    if (errbuf && errlen > 0) std::snprintf(errbuf, errlen, "%s", P->err.c_str());
    delete P;
    return nullptr;
  }
  return P;
}

void porc_free(void* h) { delete static_cast<Poly*>(h); }
void porc_set_flux(void* h, int flux) { static_cast<Poly*>(h)->base.flux = flux; }
int porc_nmodes(int p) { return pnmodes(p); }
int porc_nfaces(void* h) { return (int)static_cast<Poly*>(h)->faces.size(); }

void porc_monomials(int p, int32_t* a /*[N][3]*/) {
  auto m = poly_monomials(p);
  for (size_t j = 0; j < m.size(); ++j)
    for (int k = 0; k < 3; ++k) a[j * 3 + k] = m[j][k];
}

void porc_geometry(void* h, double* vol, double* xc, double* L) {
  const Poly& P = *static_cast<Poly*>(h);
  for (int e = 0; e < P.ne; ++e) {
    vol[e] = P.vol[e];
    for (int k = 0; k < 3; ++k) { xc[e * 3 + k] = P.xc[e * 3 + k]; L[e * 3 + k] = P.Ls[e * 3 + k]; }
  }
}

void porc_basis_S(void* h, double* S) {
  const Poly& P = *static_cast<Poly*>(h);
  std::memcpy(S, P.S.data(), P.S.size() * sizeof(double));
}

// Volume rule of element e with Q points per direction (Q^3 points).
void porc_vol_rule(void* h, int e, int Q, double* X, double* W) {
  std::vector<double> x, w;
  poly_vol_rule(*static_cast<Poly*>(h), e, Q, x, w);
  std::memcpy(X, x.data(), x.size() * sizeof(double));
  std::memcpy(W, w.data(), w.size() * sizeof(double));
}

// Faces: info[f] = (eL, fL, eR, fR, tag, nv), cv[f] canonical vertices, sgn[f].
void porc_faces(void* h, int32_t* info, int32_t* cv, double* sgn) {
  const Poly& P = *static_cast<Poly*>(h);
  for (size_t f = 0; f < P.faces.size(); ++f) {
    const PFace& F = P.faces[f];
    int32_t r[6] = {F.eL, F.fL, F.eR, F.fR, F.tag, F.nv};
    for (int k = 0; k < 6; ++k) info[f * 6 + k] = r[k];
    for (int k = 0; k < 4; ++k) cv[f * 4 + k] = k < F.nv ? F.cv[k] : -1;
    sgn[f] = F.sgn;
  }
}

// Face rule of face f with Q points per direction (Q^2 points), unit normals
// out of the face's L element.
void porc_face_rule(void* h, int f, int Q, double* X, double* W, double* Nh) {
  const Poly& P = *static_cast<Poly*>(h);
  std::vector<double> x, w, n;
  poly_face_rule(P, P.faces[f], Q, x, w, n);
  for (auto& c : n) c *= P.faces[f].sgn;
  std::memcpy(X, x.data(), x.size() * sizeof(double));
  std::memcpy(W, w.data(), w.size() * sizeof(double));
  std::memcpy(Nh, n.data(), n.size() * sizeof(double));
}

void porc_psi(void* h, int e, int N, const double* x, double* psi, double* gpsi) {
  poly_psi(*static_cast<Poly*>(h), e, N, x, psi, gpsi);
}

void porc_freestream(void* h, int p, double* u) {
  const Poly& P = *static_cast<Poly*>(h);
  const int N = pnmodes(p);
  for (int e = 0; e < P.ne; ++e) {
    double s00 = P.S[(size_t)e * P.Nmax * P.Nmax];
    for (int v = 0; v < 5; ++v)
      for (int i = 0; i < N; ++i) u[((size_t)e * 5 + v) * N + i] = i == 0 ? P.base.Uinf[v] / s00 : 0.0;
  }
}

void porc_residual(void* h, int p, const double* u, double* r) { poly_residual_t(*static_cast<Poly*>(h), p, u, r); }

void porc_residual_complex(void* h, int p, const double* ure, const double* uim, double* rre, double* rim) {
  const Poly& P = *static_cast<Poly*>(h);
  size_t n = (size_t)P.ne * 5 * pnmodes(p);
  std::vector<cd> u(n), r(n);
  for (size_t i = 0; i < n; ++i) u[i] = cd(ure[i], uim[i]);
  poly_residual_t(P, p, u.data(), r.data());
  for (size_t i = 0; i < n; ++i) { rre[i] = r[i].real(); rim[i] = r[i].imag(); }
}

void porc_timestep(void* h, int p, double cfl, const double* u, double* dtau) {
  porc_timestep_impl(*static_cast<Poly*>(h), p, pnmodes(p), cfl, u, dtau);
}

void porc_element_blocks(void* h, int p, const double* u, double* D) { poly_blocks(*static_cast<Poly*>(h), p, u, D); }

int porc_prk(void* h, int p, int s, double cfl, double* u, const double* f) {
  return poly_prk(*static_cast<Poly*>(h), p, s, cfl, u, f) ? 0 : 1;
}

// Density-residual norm (Section 4, norm under eq. (cfl)): with the
// orthonormal basis, (1/|Omega|) (sum of the squared density coefficients)^(1/2).
double porc_rnorm(void* h, int p, const double* r) {
  const Poly& P = *static_cast<Poly*>(h);
  const int Np = pnmodes(p);
  double s = 0.0;
  for (int e = 0; e < P.ne; ++e)
    for (int i = 0; i < Np; ++i) {
      const double x = r[((size_t)e * 5 + 0) * Np + i];
      s += x * x;
    }
  return std::sqrt(s) / P.omega;
}

void porc_surface(void* h, double* surf, double* hE) {
  const Poly& P = *static_cast<Poly*>(h);
  for (int e = 0; e < P.ne; ++e) { surf[e] = P.surf[e]; hE[e] = P.hE[e]; }
}

int porc_exp1(void* h, int pmax, int m, double cfl, double* u0, const double* f0) {
  return poly_exp1(*static_cast<Poly*>(h), pmax, m, cfl, u0, f0) ? 0 : 1;
}

// One V-cycle (entry norm and CFL as on the hexahedra) and the steady solve
// (same stopping rules: r_n <= drop r_1 -> 0, max_cycles -> 3, non-finite
// norm -> 2, failed step -> 1).
int porc_vcycle(void* h, int pmax, int s, int m, double cfl_max, double rref, int n, double* u, double* rn_out,
                double* cfl_out) {
  const Poly& P = *static_cast<Poly*>(h);
  const size_t K = (size_t)P.ne * 5 * pnmodes(pmax);
  std::vector<double> R(K);
  poly_residual_t<double>(P, pmax, u, R.data());
  const double rn = poly_rnorm_impl(P, pmax, R.data());
  if (rn_out) *rn_out = rn;
  if (!std::isfinite(rn)) return 2;
  const double cfl = cfl_ramp(cfl_max, rn, rref > 0.0 ? rref : rn, n, pmax);
  if (cfl_out) *cfl_out = cfl;
  return poly_vcycle_rec(P, pmax, s, m, pmax, cfl, u, nullptr) ? 0 : 1;
}

int porc_solve(void* h, int pmax, int s, int m, double cfl_max, double drop, int max_cycles, double* u, double* hist,
               int* n_cycles) {
  const Poly& P = *static_cast<Poly*>(h);
  const size_t K = (size_t)P.ne * 5 * pnmodes(pmax);
  std::vector<double> R(K);
  double r1 = 0.0;
  for (int n = 1;; ++n) {
    poly_residual_t<double>(P, pmax, u, R.data());
    const double rn = poly_rnorm_impl(P, pmax, R.data());
    hist[n - 1] = rn;
    if (n == 1) r1 = rn;
    *n_cycles = n - 1;
    if (!std::isfinite(rn)) return 2;
    if (rn <= drop * r1) return 0;
    if (n - 1 == max_cycles) return 3;
    const double cfl = cfl_ramp(cfl_max, rn, r1, n, pmax);
    if (!poly_vcycle_rec(P, pmax, s, m, pmax, cfl, u, nullptr)) return 1;
  }
}

void porc_mms_project(void* h, int p, double* u) { poly_mms(*static_cast<Poly*>(h), p, 0, u); }
void porc_mms_forcing(void* h, int p, double* f) { poly_mms(*static_cast<Poly*>(h), p, 1, f); }

}  // extern "C"
