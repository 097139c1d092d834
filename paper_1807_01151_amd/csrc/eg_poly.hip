// Tetrahedra and prisms with the paper's Cartesian basis (arXiv:1807.01151,
// Section 3.2): set-up (face matching, centroids, extents, the per-element
// modified Gram-Schmidt basis, quadrature tables) and the DG residual of
// eq. (euler3) on the device.
//
// Design.  Because the basis is a polynomial in the global coordinates, the
// residual never needs a reference map at face points: a state is evaluated
// from its monomial coefficients a = S^T u (U_v(x) = sum_j a_vj chi_j(x)),
// and the residual is formed in monomial moments
//   m_vj = int_E F_v . grad chi_j dx - sum_faces int chi_j F~_v dsigma,
// then R = S m.  k_poly_mono writes a for every element (one FP64 vector per
// element, read back by the element and its face neighbours); k_poly_residual
// runs one wavefront per element: the lanes first take the quadrature points
// (state, flux, weight into LDS), then the outputs (v, j), which contract the
// staged values with the monomial derivatives recomputed from the scaled
// coordinates.  Face points are generated on the fly from the face's
// canonically ordered vertices, so both sides of a face evaluate bit-identical
// points; a per-face sign turns the canonical normal outward.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/eg.h"
#include "eg_common.h"
#include "eg_device.h"
#include "eg_launch.h"
#include "eg_physics.h"

namespace eg {
void gauss_rule01(int Q, double* x, double* w);
}

namespace {

constexpr int PV = 5;         // conserved variables in 3D
constexpr int PMAX_POLY = 3;  // highest order (N = 20)
constexpr int NMAX_POLY = 20;
// boundary codes in the neighbour table
constexpr int PB_WALL = -1, PB_FAR = -2, PB_SYM = -4;

__host__ __device__ constexpr int pn(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Exponents of monomial j: total degree, then a_x descending, then a_y
// descending.
__host__ __device__ inline void mono_exp(int j, int& ax, int& ay, int& az) {
  int idx = 0;
  for (int k = 0; k <= PMAX_POLY; ++k)
    for (int a = k; a >= 0; --a)
      for (int b = k - a; b >= 0; --b) {
        if (idx == j) { ax = a; ay = b; az = k - a - b; return; }
        ++idx;
      }
  ax = ay = az = 0;
}

struct PolyDev {
  const double* xyz;     // [nv][3]
  const int32_t* ev;     // [E][6]
  const int8_t* typ;     // [E]
  const int32_t* nbr;    // [E][5] neighbour or PB_* code
  const int32_t* fcv;    // [E][5][4] canonical face vertices (-1 pads a triangle)
  const int8_t* fsg;     // [E][5] +1 / -1: orientation of the canonical normal
  const double* geo;     // [E][6]: xc, L
  const double* S;       // [E][spk]: row-major packed lower triangle of S, spk = Nmax (Nmax+1) / 2
  int ne, spk;
};

// Reference tables of one order: tetrahedron and prism volume points
// (l1, l2, l3 or zeta, weight factor), triangle and quad face points
// (coordinates 1, 2, weight factor).
struct PolyRule {
  const double* tet;   // [Q^3][4]
  const double* pri;   // [Q^3][4]
  const double* tri;   // [Q^2][3]
  const double* quad;  // [Q^2][3]
};

__device__ __forceinline__ double det3(const double* c0, const double* c1, const double* c2) {
  return c0[0] * (c1[1] * c2[2] - c1[2] * c2[1]) - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1]) +
         c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]);
}

// a[e][v][j] = sum_{i >= j} S[e][i][j] u[e][v][i] (monomial coefficients).
// One wavefront per element: the element's packed triangle of S (the level-p
// block is its leading N(N+1)/2 entries) and its state are staged in LDS
// with contiguous loads, then the lanes take the outputs (v, j).
template <int P>
__global__ __launch_bounds__(64) void k_poly_mono(PolyDev M, const double* __restrict__ u, double* __restrict__ a) {
  constexpr int N = pn(P), NO = PV * N, NS = N * (N + 1) / 2;
  __shared__ double sS[NS], su[NO];
  const int e = blockIdx.x, t = threadIdx.x;
  if (e >= M.ne) return;
  for (int k = t; k < NS; k += 64) sS[k] = M.S[(size_t)e * M.spk + k];
  for (int k = t; k < NO; k += 64) su[k] = u[(size_t)e * NO + k];
  __syncthreads();
  for (int o = t; o < NO; o += 64) {
    const int v = o / N, j = o % N;
    double s = 0.0;
    for (int i = j; i < N; ++i) s += sS[i * (i + 1) / 2 + j] * su[v * N + i];
    a[(size_t)e * NO + o] = s;
  }
}

// Scaled coordinates and monomial powers at a point.
template <int P>
__device__ __forceinline__ void powers(const double* x, const double* g, double pw[3][P + 1]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double X = (x[k] - g[k]) / g[3 + k];
    pw[k][0] = 1.0;
#pragma unroll
    for (int r = 1; r <= P; ++r) pw[k][r] = pw[k][r - 1] * X;
  }
}

template <int P>
__device__ __forceinline__ void state_at(const double (*pw)[P + 1], const double* a, double* U) {
  constexpr int N = pn(P);
#pragma unroll
  for (int v = 0; v < PV; ++v) U[v] = 0.0;
  int j = 0;
#pragma unroll
  for (int k = 0; k <= P; ++k)
#pragma unroll
    for (int ax = k; ax >= 0; --ax)
#pragma unroll
      for (int ay = k - ax; ay >= 0; --ay) {
        const double c = pw[0][ax] * pw[1][ay] * pw[2][k - ax - ay];
#pragma unroll
        for (int v = 0; v < PV; ++v) U[v] += a[v * N + j] * c;
        ++j;
      }
}

// Exponents of monomial j and the index of chi_{j - e_d} (the monomial whose
// x_d-derivative is a_d chi_{j - e_d} up to 1/L_d; -1 when a_d = 0).
struct MonoTab {
  int8_t ex[NMAX_POLY][3];
  int8_t lo[NMAX_POLY][3];
};
constexpr MonoTab make_mono_tab() {
  MonoTab t{};
  int idx = 0;
  for (int k = 0; k <= PMAX_POLY; ++k)
    for (int a = k; a >= 0; --a)
      for (int b = k - a; b >= 0; --b) {
        t.ex[idx][0] = (int8_t)a;
        t.ex[idx][1] = (int8_t)b;
        t.ex[idx][2] = (int8_t)(k - a - b);
        ++idx;
      }
  for (int j = 0; j < NMAX_POLY; ++j)
    for (int d = 0; d < 3; ++d) {
      t.lo[j][d] = -1;
      if (t.ex[j][d] == 0) continue;
      for (int i = 0; i < NMAX_POLY; ++i) {
        bool same = true;
        for (int c = 0; c < 3; ++c) same = same && t.ex[i][c] == t.ex[j][c] - (c == d ? 1 : 0);
        if (same) t.lo[j][d] = (int8_t)i;
      }
    }
  return t;
}
__constant__ MonoTab kMono = make_mono_tab();

// The monomials of total degree <= K at a point, in basis order, from the
// powers table of order P >= K (indices fixed at compile time).
template <int P, int K>
__device__ __forceinline__ void mono_values(const double (*pw)[P + 1], double* out) {
  int j = 0;
#pragma unroll
  for (int k = 0; k <= K; ++k)
#pragma unroll
    for (int ax = k; ax >= 0; --ax)
#pragma unroll
      for (int ay = k - ax; ay >= 0; --ay) out[j++] = pw[0][ax] * pw[1][ay] * pw[2][k - ax - ay];
}

// One wavefront per element, in five phases:
//  1. volume points, in chunks of 64 (one per lane): state from the monomial
//     coefficients, Euler fluxes; LDS gets G[q][d*5+v] = w F_dv / L_d and the
//     monomials of degree < p at the point;
//  2. after each chunk, flux moments M[d*5+v][k] += sum_q G[q][.] chi_k(q),
//     accumulated in registers over the chunks: at p = 3 on the FP64 matrix
//     cores (one 16 x 16 tile, 16 steps of 4 points), at p <= 2 by the lanes
//     over (d*5+v, k) -- since
//     grad chi_j = (a_d chi_{j-e_d} / L_d)_d, they carry the whole volume term;
//  3. face points of every face, in chunks of 64: own and neighbour (or
//     ghost) traces, the numerical flux; LDS gets w F~_v and all monomials at
//     the point, in the space phase 1 used;
//  4. after each chunk, the face moments sum_q w F~_v chi_j (p = 3: matrix
//     cores, rows v, one 16-column tile per 16 modes; p <= 2: lanes over
//     (v, j)); then
//     m_vj = sum_d a_d M[d*5+v][j-e_d] - face moments;
//  5. R = S m.
// Blocks are mapped to elements so that each XCD (blocks b, b+8, ...) gets a
// contiguous range of elements, whose neighbours' coefficients then share
// that XCD's L2.
template <int P>
__global__ __launch_bounds__(64) void k_poly_residual(PolyDev M, PolyRule R, eg::Gas gas,
                                                     const double* __restrict__ a_all, double* __restrict__ r) {
  constexpr int N = pn(P), NL = pn(P - 1), NL1 = NL > 0 ? NL : 1, Q = P + 2, QV = Q * Q * Q, QF = Q * Q;
  constexpr int NO = PV * N;
  static_assert(NL <= 16, "the flux moments fit one 16 x 16 tile (15 rows d*5+v, NL columns)");
  constexpr int CH = 64;  // points per chunk: one per lane
  constexpr int W1 = 15 + NL, W3 = PV + N;
  __shared__ double sbuf[CH * (W1 > W3 ? W1 : W3)];
  __shared__ double sa[NO], sm[NO], sM[15 * NL1];
  __shared__ double sn[5][NO];
  __shared__ double sg[6], sgn[5][6];
  __shared__ int snb[5];
  const int t = threadIdx.x;
  const int per = (M.ne + 7) / 8;
  const int e = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (e >= M.ne) return;
  const int typ = M.typ[e];
  const int nf = typ == 0 ? 4 : 5;
  for (int o = t; o < NO; o += 64) sa[o] = a_all[(size_t)e * NO + o];
  if (t < 6) sg[t] = M.geo[(size_t)e * 6 + t];
  if (t < 5) snb[t] = t < nf ? M.nbr[(size_t)e * 5 + t] : PB_WALL;
  __syncthreads();
  for (int f = 0; f < nf; ++f) {
    const int nb = snb[f];
    if (nb < 0) continue;
    for (int o = t; o < NO; o += 64) sn[f][o] = a_all[(size_t)nb * NO + o];
    if (t < 6) sgn[f][t] = M.geo[(size_t)nb * 6 + t];
  }
  double Xv[6][3];
  const int nvt = typ == 0 ? 4 : 6;
  for (int k = 0; k < 6; ++k)
    for (int c = 0; c < 3; ++c) Xv[k][c] = k < nvt ? M.xyz[(size_t)M.ev[(size_t)e * 6 + k] * 3 + c] : 0.0;
  // ---- 1 + 2. volume points and flux moments
  double* sG = sbuf;               // [CH][15]
  double* sC = sbuf + CH * 15;     // [CH][NL]
  const int li = t & 15, lk = t >> 4;
  // the contractions run on the matrix cores at p = 3; at p <= 2 the padded
  // 16 x 16 tiles cost more registers (one wavefront per SIMD less) than
  // they save, and the lanes contract over the points directly
  constexpr bool MF = P >= 3;
  constexpr int NM = 15 * NL, MPL = (NM + 63) / 64 > 0 ? (NM + 63) / 64 : 1, OPL = (NO + 63) / 64;
  eg::dbl4_t accM = {0.0, 0.0, 0.0, 0.0};
  double accV[MF ? 1 : MPL];
#pragma unroll
  for (int m = 0; m < (MF ? 1 : MPL); ++m) accV[m] = 0.0;
  for (int q0 = 0; NL > 0 && q0 < QV; q0 += CH) {
    // keeps the coefficient reads from LDS inside the loop (hoisted, they
    // would hold V N registers for the whole loop)
    asm volatile("" ::: "memory");
    __syncthreads();
    const int q = q0 + t;
    if (q < QV) {
      double x[3], w;
      if (typ == 0) {
        const double* rq = R.tet + q * 4;
        double J[3][3];
        for (int c = 0; c < 3; ++c) {
          J[0][c] = Xv[1][c] - Xv[0][c];
          J[1][c] = Xv[2][c] - Xv[0][c];
          J[2][c] = Xv[3][c] - Xv[0][c];
          x[c] = Xv[0][c] + rq[0] * J[0][c] + rq[1] * J[1][c] + rq[2] * J[2][c];
        }
        w = rq[3] * fabs(det3(J[0], J[1], J[2]));
      } else {
        const double* rq = R.pri + q * 4;
        const double l1 = rq[0], l2 = rq[1], z = rq[2], l0 = 1.0 - l1 - l2;
        const double lam[3] = {l0, l1, l2};
        double J[3][3];
        for (int c = 0; c < 3; ++c) {
          double xs = 0.0, dz = 0.0;
          for (int k = 0; k < 3; ++k) {
            xs += lam[k] * ((1.0 - z) * Xv[k][c] + z * Xv[k + 3][c]);
            dz += lam[k] * (Xv[k + 3][c] - Xv[k][c]);
          }
          x[c] = xs;
          J[0][c] = (1.0 - z) * (Xv[1][c] - Xv[0][c]) + z * (Xv[4][c] - Xv[3][c]);
          J[1][c] = (1.0 - z) * (Xv[2][c] - Xv[0][c]) + z * (Xv[5][c] - Xv[3][c]);
          J[2][c] = dz;
        }
        w = rq[3] * fabs(det3(J[0], J[1], J[2]));
      }
      double pw[3][P + 1];
      powers<P>(x, sg, pw);
      double U[PV];
      state_at<P>(pw, sa, U);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double nd[3] = {0.0, 0.0, 0.0};
        nd[d] = 1.0;
        double F[PV];
        eg::flux_n<3>(U, nd, F, gas.g);
        const double s = w / sg[3 + d];
#pragma unroll
        for (int v = 0; v < PV; ++v) sG[t * 15 + d * 5 + v] = s * F[v];
      }
      double cv_[NL1];
      mono_values<P, (P > 0 ? P - 1 : 0)>(pw, cv_);
#pragma unroll
      for (int k = 0; k < NL; ++k) sC[t * NL1 + k] = cv_[k];
    }
    __syncthreads();
    // M (16 x 16, rows d*5+v, columns k) += G^T (16 x 64) C (64 x 16) on the
    // FP64 matrix cores: at step st lane l supplies G[4 st + l/16][l%16] and
    // C[4 st + l/16][l%16] (zero past the chunk, row 15 and column NL)
    const int nq = QV - q0 < CH ? QV - q0 : CH;
    if constexpr (MF) {
#pragma unroll
      for (int st = 0; st < CH / 4; ++st) {
        const int qq = 4 * st + lk;
        const double av = (li < 15 && qq < nq) ? sG[qq * 15 + li] : 0.0;
        const double bv = (li < NL && qq < nq) ? sC[qq * NL1 + li] : 0.0;
        accM = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, accM, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int m = 0; m < MPL; ++m) {
        const int o = t + 64 * m;
        if (o < NM) {
          const int c = o / NL1, k = o % NL1;
          double acc = accV[m];
          for (int qq = 0; qq < nq; ++qq) acc += sG[qq * 15 + c] * sC[qq * NL1 + k];
          accV[m] = acc;
        }
      }
    }
  }
  if constexpr (MF) {
    // lane l holds rows l/16 + 4 r of column l%16
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int c = lk + 4 * rr;
      if (c < 15 && li < NL) sM[c * NL1 + li] = accM[rr];
    }
  } else {
#pragma unroll
    for (int m = 0; m < MPL; ++m)
      if (t + 64 * m < NM) sM[t + 64 * m] = accV[m];
  }
  // ---- 3 + 4. face points of all faces and their moments
  double* sH = sbuf;               // [CH][5]
  double* sX = sbuf + CH * PV;     // [CH][N]
  constexpr int NT = MF ? (N + 15) / 16 : 1;  // 16-column tiles of the face moments
  eg::dbl4_t accF[NT];
#pragma unroll
  for (int T = 0; T < NT; ++T) accF[T] = eg::dbl4_t{0.0, 0.0, 0.0, 0.0};
  double accW[MF ? 1 : OPL];
#pragma unroll
  for (int m = 0; m < (MF ? 1 : OPL); ++m) accW[m] = 0.0;
  const int nfq = nf * QF;
  for (int q0 = 0; q0 < nfq; q0 += CH) {
    asm volatile("" ::: "memory");
    __syncthreads();
    const int fq = q0 + t;
    if (fq < nfq) {
    const int f = fq / QF, q = fq % QF;
    const int nb = snb[f];
    const int32_t* cv = M.fcv + ((size_t)e * 5 + f) * 4;
    const double sgnf = (double)M.fsg[(size_t)e * 5 + f];
    const int ncv = cv[3] < 0 ? 3 : 4;
    double C[4][3];
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) C[k][c] = k < ncv ? M.xyz[(size_t)cv[k] * 3 + c] : 0.0;
    double x[3], nv[3], w;
    if (ncv == 3) {
      const double* rq = R.tri + q * 3;
      double e1[3], e2[3];
      for (int c = 0; c < 3; ++c) {
        e1[c] = C[1][c] - C[0][c];
        e2[c] = C[2][c] - C[0][c];
        x[c] = C[0][c] + rq[0] * e1[c] + rq[1] * e2[c];
      }
      nv[0] = e1[1] * e2[2] - e1[2] * e2[1];
      nv[1] = e1[2] * e2[0] - e1[0] * e2[2];
      nv[2] = e1[0] * e2[1] - e1[1] * e2[0];
      w = rq[2];
    } else {
      const double* rq = R.quad + q * 3;
      const double s = rq[0], tt = rq[1];
      double xs[3], xt[3];
      for (int c = 0; c < 3; ++c) {
        x[c] = (1 - s) * (1 - tt) * C[0][c] + s * (1 - tt) * C[1][c] + s * tt * C[2][c] + (1 - s) * tt * C[3][c];
        xs[c] = (1 - tt) * (C[1][c] - C[0][c]) + tt * (C[2][c] - C[3][c]);
        xt[c] = (1 - s) * (C[3][c] - C[0][c]) + s * (C[2][c] - C[1][c]);
      }
      nv[0] = xs[1] * xt[2] - xs[2] * xt[1];
      nv[1] = xs[2] * xt[0] - xs[0] * xt[2];
      nv[2] = xs[0] * xt[1] - xs[1] * xt[0];
      w = rq[2];
    }
    const double area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    double nh[3];
    for (int c = 0; c < 3; ++c) nh[c] = sgnf * (nv[c] / area);
    w *= area;
    double pw[3][P + 1];
    powers<P>(x, sg, pw);
    double UL[PV], UR[PV], Fl[PV];
    state_at<P>(pw, sa, UL);
    if (nb >= 0) {
      double pn_[3][P + 1];
      powers<P>(x, sgn[f], pn_);
      state_at<P>(pn_, sn[f], UR);
    } else if (nb == PB_FAR) {
      eg::ghost_far<3>(UL, nh, UR, gas.Uinf, gas.g);
    } else {
      eg::ghost_wall<3>(UL, nh, UR);
    }
    if (gas.flux == eg::FLUX_ROE) eg::roe<3>(UL, UR, nh, Fl, gas.g);
    else eg::rusanov<3>(UL, UR, nh, Fl, gas.g);
#pragma unroll
    for (int v = 0; v < PV; ++v) sH[t * PV + v] = w * Fl[v];
    double xv_[N];
    mono_values<P, P>(pw, xv_);
#pragma unroll
    for (int j = 0; j < N; ++j) sX[t * N + j] = xv_[j];
    }
    __syncthreads();
    // F (16 x 16 per tile, rows v, columns j) += H^T (16 x 64) X (64 x 16)
    const int nq = nfq - q0 < CH ? nfq - q0 : CH;
    if constexpr (MF) {
#pragma unroll
      for (int st = 0; st < CH / 4; ++st) {
        const int qq = 4 * st + lk;
        const double av = (li < PV && qq < nq) ? sH[qq * PV + li] : 0.0;
#pragma unroll
        for (int T = 0; T < NT; ++T) {
          const int j = 16 * T + li;
          const double bv = (j < N && qq < nq) ? sX[qq * N + j] : 0.0;
          accF[T] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, accF[T], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < OPL; ++m) {
        const int o = t + 64 * m;
        if (o < NO) {
          const int v = o / N, j = o % N;
          double acc = accW[m];
          for (int qq = 0; qq < nq; ++qq) acc += sH[qq * PV + v] * sX[qq * N + j];
          accW[m] = acc;
        }
      }
    }
  }
  __syncthreads();  // sM complete (written before the face loop)
  // m_vj = sum_d a_d M[d*5+v][j-e_d] - (face moments)_vj
  auto finish = [&](int v, int j, double fm) {
    double acc = -fm;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lo = kMono.lo[j][d];
      if (lo >= 0) acc += (double)kMono.ex[j][d] * sM[(d * 5 + v) * NL1 + lo];
    }
    sm[v * N + j] = acc;
  };
  if constexpr (MF) {
    // lane l holds rows v = l/16 + 4 r of column j = 16 T + l%16
#pragma unroll
    for (int T = 0; T < NT; ++T)
#pragma unroll
      for (int rr = 0; rr < 2; ++rr) {
        const int v = lk + 4 * rr, j = 16 * T + li;
        if (v < PV && j < N) finish(v, j, accF[T][rr]);
      }
  } else {
#pragma unroll
    for (int m = 0; m < OPL; ++m) {
      const int o = t + 64 * m;
      if (o < NO) finish(o / N, o % N, accW[m]);
    }
  }
  __syncthreads();
  // ---- 5. R = S m
  const double* Se = M.S + (size_t)e * M.spk;
  for (int o = t; o < NO; o += 64) {
    const int v = o / N, i = o % N;
    const double* Si = Se + i * (i + 1) / 2;
    double s = 0.0;
    for (int j = 0; j <= i; ++j) s += Si[j] * sm[v * N + j];
    r[(size_t)e * NO + o] = s;
  }
}

// Element block D_E = dR_E / du_E (Section 3.3, eq. (jac1): the volume
// term and the own-side derivative of every face flux, ghost states
// included) on the tetrahedra and prisms, one workgroup of four wavefronts
// per element.  In monomial coordinates, with A_d = dF_d/dU at the volume
// points and B = dF~/dU_own at the face points (forward-mode dual numbers),
//   K_vw[k][l] = sum_d a_d(k) sum_q w A_d,vw chi_{k-e_d} chi_l / L_d
//              - sum_faces sum_q w B_vw chi_k chi_l,
// and D_vw = S K_vw S^T (R = S m, a = S^T u).  The pointwise Jacobians and
// monomials are staged in LDS, the K entries accumulated by the threads that
// own them; D is written row-major, n = 5 N, rows and columns (v, i).
template <int P>
__global__ __launch_bounds__(256) void k_poly_block(PolyDev M, PolyRule R, eg::Gas gas,
                                                   const double* __restrict__ a_all, double* __restrict__ Dout) {
  constexpr int N = pn(P), Q = P + 2, QV = Q * Q * Q, QF = Q * Q, NO = PV * N, NB = NO * NO;
  constexpr int NK = 25 * N * N, OPT = (NK + 255) / 256, NFQ = 5 * QF;
  constexpr int NN = N * N, NG0 = NN >= 256 ? 1 : 256 / NN, NG = NG0 > 25 ? 25 : NG0;
  constexpr int VPT = (25 + NG - 1) / NG, OPT2 = (NN * NG + 255) / 256;
  constexpr int RJ = QV * 75 + QV * N;          // volume: w A_d / L_d and monomials per point
  constexpr int RF = NFQ * 25 + NFQ * N;        // faces: w B and monomials per point
  // at p <= 2 a thread takes one (volume point, direction) pair, so each
  // thread makes one dual-number flux evaluation; at p <= 1 both stagings
  // also fit in LDS side by side (faces and K first, the volume points after
  // them), and the face points run at the same time on wavefronts of their
  // own (a wavefront that took both would run the two one after the other)
  constexpr bool VSPLIT = 3 * QV <= 256;
  constexpr int NVT = VSPLIT ? 3 * QV : QV;
  constexpr bool CONC = P <= 1;
  constexpr int VOFF = CONC ? RF + NK : 0;
  constexpr int FOFF = CONC ? (NVT + 63) / 64 * 64 : 0;
  constexpr int REG = CONC ? RF + NK + RJ : (RJ > RF + NK ? RJ : RF + NK);
  static_assert(NVT <= 256 && NFQ <= 256, "one point per thread");
  static_assert(!CONC || FOFF + NFQ <= 256, "volume and face points side by side");
  __shared__ double sbuf[REG];
  __shared__ double sa[NO], sS[N * (N + 1) / 2];
  __shared__ double sn[5][NO];
  __shared__ double sg[6], sgn[5][6];
  __shared__ int snb[5];
  const int t = threadIdx.x;
  const int per = (M.ne + 7) / 8;
  const int e = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (e >= M.ne) return;
  const int typ = M.typ[e];
  const int nf = typ == 0 ? 4 : 5;
  for (int o = t; o < NO; o += 256) sa[o] = a_all[(size_t)e * NO + o];
  for (int k = t; k < N * (N + 1) / 2; k += 256) sS[k] = M.S[(size_t)e * M.spk + k];
  if (t < 6) sg[t] = M.geo[(size_t)e * 6 + t];
  if (t < 5) snb[t] = t < nf ? M.nbr[(size_t)e * 5 + t] : PB_WALL;
  __syncthreads();
  for (int f = 0; f < nf; ++f) {
    const int nb = snb[f];
    if (nb < 0) continue;
    for (int o = t; o < NO; o += 256) sn[f][o] = a_all[(size_t)nb * NO + o];
    if (t < 6) sgn[f][t] = M.geo[(size_t)nb * 6 + t];
  }
  if constexpr (CONC) __syncthreads();  // the face points read sn, sgn next
  using D5 = eg::Dual<PV, double>;
  // ---- volume points: w A_d,vw / L_d and the monomials
  double* sJ = sbuf + VOFF;
  double* sX = sbuf + VOFF + QV * 75;
  // ---- face points: w dF~/dU_own and the monomials
  double* sB = sbuf;
  double* sY = sbuf + NFQ * 25;
  const int nfq = nf * QF;
  auto vol_point = [&](const int t, const int dsel) {
    double Xv[6][3];
    const int nvt = typ == 0 ? 4 : 6;
    for (int k = 0; k < 6; ++k)
      for (int c = 0; c < 3; ++c) Xv[k][c] = k < nvt ? M.xyz[(size_t)M.ev[(size_t)e * 6 + k] * 3 + c] : 0.0;
    double x[3], w, J[3][3];
    if (typ == 0) {
      const double* rq = R.tet + t * 4;
      for (int c = 0; c < 3; ++c) {
        J[0][c] = Xv[1][c] - Xv[0][c];
        J[1][c] = Xv[2][c] - Xv[0][c];
        J[2][c] = Xv[3][c] - Xv[0][c];
        x[c] = Xv[0][c] + rq[0] * J[0][c] + rq[1] * J[1][c] + rq[2] * J[2][c];
      }
      w = rq[3] * fabs(det3(J[0], J[1], J[2]));
    } else {
      const double* rq = R.pri + t * 4;
      const double l1 = rq[0], l2 = rq[1], z = rq[2], l0 = 1.0 - l1 - l2;
      const double lam[3] = {l0, l1, l2};
      for (int c = 0; c < 3; ++c) {
        double xs = 0.0, dz = 0.0;
        for (int k = 0; k < 3; ++k) {
          xs += lam[k] * ((1.0 - z) * Xv[k][c] + z * Xv[k + 3][c]);
          dz += lam[k] * (Xv[k + 3][c] - Xv[k][c]);
        }
        x[c] = xs;
        J[0][c] = (1.0 - z) * (Xv[1][c] - Xv[0][c]) + z * (Xv[4][c] - Xv[3][c]);
        J[1][c] = (1.0 - z) * (Xv[2][c] - Xv[0][c]) + z * (Xv[5][c] - Xv[3][c]);
        J[2][c] = dz;
      }
      w = rq[3] * fabs(det3(J[0], J[1], J[2]));
    }
    double pw[3][P + 1];
    powers<P>(x, sg, pw);
    double U[PV];
    state_at<P>(pw, sa, U);
    D5 Ud[PV];
#pragma unroll
    for (int v = 0; v < PV; ++v) {
      Ud[v] = D5(U[v]);
      Ud[v].d[v] = 1.0;
    }
    if constexpr (VSPLIT) {
      // direction dsel only, the unit normal a run-time value so that the
      // lanes of one wavefront share one code path
      const double nd[3] = {dsel == 0 ? 1.0 : 0.0, dsel == 1 ? 1.0 : 0.0, dsel == 2 ? 1.0 : 0.0};
      D5 F[PV];
      eg::flux_n<3>(Ud, nd, F, gas.g);
      const double sc = w / sg[3 + dsel];
#pragma unroll
      for (int v = 0; v < PV; ++v)
#pragma unroll
        for (int ww = 0; ww < PV; ++ww) sJ[t * 75 + dsel * 25 + v * 5 + ww] = sc * F[v].d[ww];
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double nd[3] = {0.0, 0.0, 0.0};
        nd[d] = 1.0;
        D5 F[PV];
        eg::flux_n<3>(Ud, nd, F, gas.g);
        const double sc = w / sg[3 + d];
#pragma unroll
        for (int v = 0; v < PV; ++v)
#pragma unroll
          for (int ww = 0; ww < PV; ++ww) sJ[t * 75 + d * 25 + v * 5 + ww] = sc * F[v].d[ww];
      }
    }
    if (dsel <= 0) {
      double xv_[N];
      mono_values<P, P>(pw, xv_);
#pragma unroll
      for (int j = 0; j < N; ++j) sX[t * N + j] = xv_[j];
    }
  };
  auto face_point = [&](const int t) {
    const int f = t / QF, q = t % QF;
    const int nb = snb[f];
    const int32_t* cv = M.fcv + ((size_t)e * 5 + f) * 4;
    const double sgnf = (double)M.fsg[(size_t)e * 5 + f];
    const int ncv = cv[3] < 0 ? 3 : 4;
    double C[4][3];
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) C[k][c] = k < ncv ? M.xyz[(size_t)cv[k] * 3 + c] : 0.0;
    double x[3], nv[3], w;
    if (ncv == 3) {
      const double* rq = R.tri + q * 3;
      double e1[3], e2[3];
      for (int c = 0; c < 3; ++c) {
        e1[c] = C[1][c] - C[0][c];
        e2[c] = C[2][c] - C[0][c];
        x[c] = C[0][c] + rq[0] * e1[c] + rq[1] * e2[c];
      }
      nv[0] = e1[1] * e2[2] - e1[2] * e2[1];
      nv[1] = e1[2] * e2[0] - e1[0] * e2[2];
      nv[2] = e1[0] * e2[1] - e1[1] * e2[0];
      w = rq[2];
    } else {
      const double* rq = R.quad + q * 3;
      const double s = rq[0], tt = rq[1];
      double xs[3], xt[3];
      for (int c = 0; c < 3; ++c) {
        x[c] = (1 - s) * (1 - tt) * C[0][c] + s * (1 - tt) * C[1][c] + s * tt * C[2][c] + (1 - s) * tt * C[3][c];
        xs[c] = (1 - tt) * (C[1][c] - C[0][c]) + tt * (C[2][c] - C[3][c]);
        xt[c] = (1 - s) * (C[3][c] - C[0][c]) + s * (C[2][c] - C[1][c]);
      }
      nv[0] = xs[1] * xt[2] - xs[2] * xt[1];
      nv[1] = xs[2] * xt[0] - xs[0] * xt[2];
      nv[2] = xs[0] * xt[1] - xs[1] * xt[0];
      w = rq[2];
    }
    const double area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    double nh[3];
    for (int c = 0; c < 3; ++c) nh[c] = sgnf * (nv[c] / area);
    w *= area;
    double pw[3][P + 1];
    powers<P>(x, sg, pw);
    double UL[PV];
    state_at<P>(pw, sa, UL);
    D5 ULd[PV], Fd[PV];
#pragma unroll
    for (int v = 0; v < PV; ++v) {
      ULd[v] = D5(UL[v]);
      ULd[v].d[v] = 1.0;
    }
    if (nb >= 0) {
      double pn_[3][P + 1], UR[PV];
      powers<P>(x, sgn[f], pn_);
      state_at<P>(pn_, sn[f], UR);
      if (gas.flux == eg::FLUX_ROE) eg::roe<3>(ULd, UR, nh, Fd, gas.g);
      else eg::rusanov<3>(ULd, UR, nh, Fd, gas.g);
    } else {
      D5 UG[PV];
      if (nb == PB_FAR) eg::ghost_far<3>(ULd, nh, UG, gas.Uinf, gas.g);
      else eg::ghost_wall<3>(ULd, nh, UG);
      if (gas.flux == eg::FLUX_ROE) eg::roe<3>(ULd, UG, nh, Fd, gas.g);
      else eg::rusanov<3>(ULd, UG, nh, Fd, gas.g);
    }
#pragma unroll
    for (int v = 0; v < PV; ++v)
#pragma unroll
      for (int ww = 0; ww < PV; ++ww) sB[t * 25 + v * 5 + ww] = w * Fd[v].d[ww];
    double xv_[N];
    mono_values<P, P>(pw, xv_);
#pragma unroll
    for (int j = 0; j < N; ++j) sY[t * N + j] = xv_[j];
  };
  if (t < NVT) {
    if constexpr (VSPLIT) vol_point(t / 3, t % 3);
    else vol_point(t, -1);
  } else if (CONC && t >= FOFF && t - FOFF < nfq) {
    face_point(t - FOFF);
  }
  __syncthreads();
  // each thread owns a mode pair (k, l) and a group of VPT of the 25 (v, w):
  // the two monomial values are read once per point for the whole group, the
  // group's Jacobian entries are contiguous (NG groups keep the 256 threads
  // busy at the low orders)
  double acc[OPT2][VPT];
#pragma unroll
  for (int m = 0; m < OPT2; ++m) {
#pragma unroll
    for (int j = 0; j < VPT; ++j) acc[m][j] = 0.0;
    const int idx = t + 256 * m;
    if (idx < NN * NG) {
      const int kl = idx % NN, vw0 = (idx / NN) * VPT;
      const int k = kl / N, l = kl % N;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int ex = kMono.ex[k][d], lo = kMono.lo[k][d];
        if (ex > 0) {
          for (int q = 0; q < QV; ++q) {
            const double c = (double)ex * sX[q * N + lo] * sX[q * N + l];
            const double* Jq = sJ + q * 75 + d * 25 + vw0;
#pragma unroll
            for (int j = 0; j < VPT; ++j)
              if (vw0 + j < 25) acc[m][j] += Jq[j] * c;
          }
        }
      }
    }
  }
  if constexpr (!CONC) __syncthreads();  // the volume staging is dead from here
  double* sK = sbuf + RF;
#pragma unroll
  for (int m = 0; m < OPT2; ++m) {
    const int idx = t + 256 * m;
    if (idx < NN * NG) {
      const int kl = idx % NN, vw0 = (idx / NN) * VPT;
#pragma unroll
      for (int j = 0; j < VPT; ++j)
        if (vw0 + j < 25) sK[(vw0 + j) * NN + kl] = acc[m][j];
    }
  }
  if constexpr (!CONC) {
    if (t < nfq) face_point(t);
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < OPT2; ++m) {
    const int idx = t + 256 * m;
    if (idx < NN * NG) {
      const int kl = idx % NN, vw0 = (idx / NN) * VPT;
      const int k = kl / N, l = kl % N;
#pragma unroll
      for (int j = 0; j < VPT; ++j) acc[m][j] = 0.0;
      for (int q = 0; q < nfq; ++q) {
        const double c = sY[q * N + k] * sY[q * N + l];
        const double* Bq = sB + q * 25 + vw0;
#pragma unroll
        for (int j = 0; j < VPT; ++j)
          if (vw0 + j < 25) acc[m][j] += Bq[j] * c;
      }
#pragma unroll
      for (int j = 0; j < VPT; ++j)
        if (vw0 + j < 25) sK[(vw0 + j) * NN + kl] -= acc[m][j];
    }
  }
  __syncthreads();
  // ---- T = S K (rows i), then D = T S^T (columns j)
  double acc1[OPT];
#pragma unroll
  for (int m = 0; m < OPT; ++m) {
    const int o = t + 256 * m;
    acc1[m] = 0.0;
    if (o < NK) {
      const int vw = o / (N * N), i = (o / N) % N, l = o % N;
      const double* Si = sS + i * (i + 1) / 2;
      double s = 0.0;
      for (int k = 0; k <= i; ++k) s += Si[k] * sK[vw * N * N + k * N + l];
      acc1[m] = s;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < OPT; ++m) {
    const int o = t + 256 * m;
    if (o < NK) sK[o] = acc1[m];
  }
  __syncthreads();
  for (int o = t; o < NB; o += 256) {
    const int row = o / NO, col = o % NO;
    const int v = row / N, i = row % N, ww = col / N, j = col % N;
    const double* Tr = sK + (v * 5 + ww) * N * N + i * N;
    const double* Sj = sS + j * (j + 1) / 2;
    double s = 0.0;
    for (int l = 0; l <= j; ++l) s += Tr[l] * Sj[l];
    Dout[(size_t)e * NB + o] = s;
  }
}

// LU with partial pivoting of the PRK block P_E = I/dtau_E - D_E
// (Section 2.3, eq. (prk_scalar); the mass matrix is I), one workgroup per
// element with the block in LDS: at step k the largest |a_ik|, i >= k (the
// lowest row on ties) is swapped into row k, the multipliers are stored below
// the diagonal and the trailing block is updated.  In place, row-major;
// piv[k] = the row exchanged with row k at step k.  A zero pivot sets *fail.
template <int P>
__global__ __launch_bounds__(256) void k_poly_lu(int ne, double* __restrict__ D, const double* __restrict__ dtau,
                                                int* __restrict__ piv, int* __restrict__ fail) {
  constexpr int n = PV * pn(P);
  __shared__ double A[n * n];
  __shared__ int s_pr;
  const int e = blockIdx.x, t = threadIdx.x;
  if (e >= ne) return;
  double* De = D + (size_t)e * n * n;
  const double idt = 1.0 / dtau[e];
  for (int k = t; k < n * n; k += 256) A[k] = (k / n == k % n ? idt : 0.0) - De[k];
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot search by the first wavefront: (|a|, lowest row) maximum by
    // butterfly shuffles, so every lane ends with the same winner
    if (t < 64) {
      double best = -1.0;
      int bi = n;
      for (int i = k + t; i < n; i += 64) {
        const double a = fabs(A[i * n + k]);
        if (a > best) { best = a; bi = i; }
      }
      for (int w = 32; w > 0; w >>= 1) {
        const double ob = __shfl_xor(best, w, 64);
        const int oi = __shfl_xor(bi, w, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (t == 0) {
        // no row wins only if the column is all NaN: keep row k (flagged)
        s_pr = bi < n ? bi : k;
        piv[(size_t)e * n + k] = s_pr;
        if (!(best > 0.0) || !isfinite(best)) atomicOr(fail, 1);
      }
    }
    __syncthreads();
    const int pr = s_pr;
    if (pr != k)
      for (int j = t; j < n; j += 256) {
        const double tmp = A[k * n + j];
        A[k * n + j] = A[pr * n + j];
        A[pr * n + j] = tmp;
      }
    __syncthreads();
    const double ip = 1.0 / A[k * n + k];
    for (int i = k + 1 + t; i < n; i += 256) A[i * n + k] *= ip;
    __syncthreads();
    // trailing update on a 16 x 16 grid of threads (rows t / 16, columns
    // t % 16, strided by 16)
    for (int i = k + 1 + (t >> 4); i < n; i += 16) {
      const double l = A[i * n + k];
      for (int j = k + 1 + (t & 15); j < n; j += 16) A[i * n + j] -= l * A[k * n + j];
    }
    __syncthreads();
  }
  for (int k = t; k < n * n; k += 256) De[k] = A[k];
}

// One PRK stage: x = P^{-1} (R + f) by the factors (row exchanges, unit
// lower then upper substitution, each row's dot product split over the lanes
// of one wavefront), then u = u^n + beta x.
template <int P>
__global__ __launch_bounds__(64) void k_poly_stage(int ne, const double* __restrict__ LU, const int* __restrict__ piv,
                                                  const double* __restrict__ R, const double* __restrict__ f,
                                                  const double* __restrict__ un, double beta, double* __restrict__ u) {
  constexpr int n = PV * pn(P);
  __shared__ double x[n];
  const int e = blockIdx.x, t = threadIdx.x;
  if (e >= ne) return;
  const double* A = LU + (size_t)e * n * n;
  for (int i = t; i < n; i += 64) x[i] = R[(size_t)e * n + i] + (f ? f[(size_t)e * n + i] : 0.0);
  __syncthreads();
  if (t == 0)
    for (int k = 0; k < n; ++k) {
      const int pr = piv[(size_t)e * n + k];
      if (pr != k) {
        const double tmp = x[k];
        x[k] = x[pr];
        x[pr] = tmp;
      }
    }
  __syncthreads();
  for (int i = 1; i < n; ++i) {
    double s = 0.0;
    for (int j = t; j < i; j += 64) s += A[(size_t)i * n + j] * x[j];
    for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w, 64);
    if (t == 0) x[i] -= s;
    __syncthreads();
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = 0.0;
    for (int j = i + 1 + t; j < n; j += 64) s += A[(size_t)i * n + j] * x[j];
    for (int w = 32; w > 0; w >>= 1) s += __shfl_xor(s, w, 64);
    if (t == 0) x[i] = (x[i] - s) / A[(size_t)i * n + i];
    __syncthreads();
  }
  for (int i = t; i < n; i += 64) u[(size_t)e * n + i] = un[(size_t)e * n + i] + beta * x[i];
}

__global__ void k_poly_zero_flag(int* flag) { *flag = 0; }

// p = 0 neighbour blocks of J_0 (Section 3.3, eq. (jac2)): for face lf of
// element e with neighbour nb, O[v][w] = -psi0_e psi0_nb sum_q w dF~_v/dU_nb,w
// (the level-0 states are constant, U = a_0 = psi0 u); [E][6][5][5], the
// slots of boundary faces and the sixth slot zero.  One thread per (e, lf).
__global__ __launch_bounds__(256) void k_poly_p0_off(PolyDev M, PolyRule R, eg::Gas gas,
                                                     const double* __restrict__ a0, double* __restrict__ Ao) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)M.ne * 6) return;
  const int e = (int)(idx / 6), lf = (int)(idx % 6);
  double* O = Ao + (size_t)idx * 25;
  const int nf = M.typ[e] == 0 ? 4 : 5;
  const int nb = lf < nf ? M.nbr[(size_t)e * 5 + lf] : PB_WALL;
  double acc[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) acc[k] = 0.0;
  if (nb >= 0) {
    using D5 = eg::Dual<PV, double>;
    const int32_t* cv = M.fcv + ((size_t)e * 5 + lf) * 4;
    const double sgnf = (double)M.fsg[(size_t)e * 5 + lf];
    const int ncv = cv[3] < 0 ? 3 : 4;
    double C[4][3];
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) C[k][c] = k < ncv ? M.xyz[(size_t)cv[k] * 3 + c] : 0.0;
    double UL[PV];
    D5 URd[PV];
#pragma unroll
    for (int v = 0; v < PV; ++v) {
      UL[v] = a0[(size_t)e * PV + v];
      URd[v] = D5(a0[(size_t)nb * PV + v]);
      URd[v].d[v] = 1.0;
    }
    for (int q = 0; q < 4; ++q) {  // the 2 x 2 face rule of p = 0
      double nv[3], w;
      if (ncv == 3) {
        const double* rq = R.tri + q * 3;
        double e1[3], e2[3];
        for (int c = 0; c < 3; ++c) { e1[c] = C[1][c] - C[0][c]; e2[c] = C[2][c] - C[0][c]; }
        nv[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nv[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nv[2] = e1[0] * e2[1] - e1[1] * e2[0];
        w = rq[2];
      } else {
        const double* rq = R.quad + q * 3;
        const double s = rq[0], tt = rq[1];
        double xs[3], xt[3];
        for (int c = 0; c < 3; ++c) {
          xs[c] = (1 - tt) * (C[1][c] - C[0][c]) + tt * (C[2][c] - C[3][c]);
          xt[c] = (1 - s) * (C[3][c] - C[0][c]) + s * (C[2][c] - C[1][c]);
        }
        nv[0] = xs[1] * xt[2] - xs[2] * xt[1];
        nv[1] = xs[2] * xt[0] - xs[0] * xt[2];
        nv[2] = xs[0] * xt[1] - xs[1] * xt[0];
        w = rq[2];
      }
      const double area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      double nh[3];
      for (int c = 0; c < 3; ++c) nh[c] = sgnf * (nv[c] / area);
      w *= area;
      D5 Fd[PV];
      if (gas.flux == eg::FLUX_ROE) eg::roe<3>(UL, URd, nh, Fd, gas.g);
      else eg::rusanov<3>(UL, URd, nh, Fd, gas.g);
#pragma unroll
      for (int v = 0; v < PV; ++v)
#pragma unroll
        for (int ww = 0; ww < PV; ++ww) acc[v * 5 + ww] += w * Fd[v].d[ww];
    }
    const double sc = -M.S[(size_t)e * M.spk] * M.S[(size_t)nb * M.spk];
#pragma unroll
    for (int k = 0; k < 25; ++k) acc[k] *= sc;
  }
#pragma unroll
  for (int k = 0; k < 25; ++k) O[k] = acc[k];
}

// The p = 0 element block of J_0 (Section 3.3, eq. (jac2)): at p = 0 the
// volume term vanishes (grad chi_0 = 0) and the state is the constant
// U = a_0 = psi0 u, so D[v][w] = -psi0^2 sum_faces sum_q w dF~_v/dU_own,w over
// the 2 x 2 face points, ghost states included; [E][25].  Eight lanes per
// element, lane lf taking local face lf (lanes past the element's faces add
// zero), summed over the eight lanes by shuffles in a fixed order.
__global__ __launch_bounds__(256) void k_poly_p0_diag(PolyDev M, PolyRule R, eg::Gas gas,
                                                     const double* __restrict__ a0, double* __restrict__ D0) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int e = (int)(idx >> 3), lf = (int)(idx & 7);
  const bool live = e < M.ne;
  const int nf = live ? (M.typ[e] == 0 ? 4 : 5) : 0;
  double acc[25];
#pragma unroll
  for (int k = 0; k < 25; ++k) acc[k] = 0.0;
  if (lf < nf) {
    using D5 = eg::Dual<PV, double>;
    const int nb = M.nbr[(size_t)e * 5 + lf];
    const int32_t* cv = M.fcv + ((size_t)e * 5 + lf) * 4;
    const double sgnf = (double)M.fsg[(size_t)e * 5 + lf];
    const int ncv = cv[3] < 0 ? 3 : 4;
    double C[4][3];
    for (int k = 0; k < 4; ++k)
      for (int c = 0; c < 3; ++c) C[k][c] = k < ncv ? M.xyz[(size_t)cv[k] * 3 + c] : 0.0;
    D5 ULd[PV];
    double URn[PV];
#pragma unroll
    for (int v = 0; v < PV; ++v) {
      ULd[v] = D5(a0[(size_t)e * PV + v]);
      ULd[v].d[v] = 1.0;
      URn[v] = nb >= 0 ? a0[(size_t)nb * PV + v] : 0.0;
    }
    for (int q = 0; q < 4; ++q) {  // the 2 x 2 face rule of p = 0
      double nv[3], w;
      if (ncv == 3) {
        const double* rq = R.tri + q * 3;
        double e1[3], e2[3];
        for (int c = 0; c < 3; ++c) { e1[c] = C[1][c] - C[0][c]; e2[c] = C[2][c] - C[0][c]; }
        nv[0] = e1[1] * e2[2] - e1[2] * e2[1];
        nv[1] = e1[2] * e2[0] - e1[0] * e2[2];
        nv[2] = e1[0] * e2[1] - e1[1] * e2[0];
        w = rq[2];
      } else {
        const double* rq = R.quad + q * 3;
        const double s = rq[0], tt = rq[1];
        double xs[3], xt[3];
        for (int c = 0; c < 3; ++c) {
          xs[c] = (1 - tt) * (C[1][c] - C[0][c]) + tt * (C[2][c] - C[3][c]);
          xt[c] = (1 - s) * (C[3][c] - C[0][c]) + s * (C[2][c] - C[1][c]);
        }
        nv[0] = xs[1] * xt[2] - xs[2] * xt[1];
        nv[1] = xs[2] * xt[0] - xs[0] * xt[2];
        nv[2] = xs[0] * xt[1] - xs[1] * xt[0];
        w = rq[2];
      }
      const double area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
      double nh[3];
      for (int c = 0; c < 3; ++c) nh[c] = sgnf * (nv[c] / area);
      w *= area;
      D5 UG[PV], Fd[PV];
      if (nb >= 0) {
#pragma unroll
        for (int v = 0; v < PV; ++v) UG[v] = D5(URn[v]);
      } else if (nb == PB_FAR) {
        eg::ghost_far<3>(ULd, nh, UG, gas.Uinf, gas.g);
      } else {
        eg::ghost_wall<3>(ULd, nh, UG);
      }
      if (gas.flux == eg::FLUX_ROE) eg::roe<3>(ULd, UG, nh, Fd, gas.g);
      else eg::rusanov<3>(ULd, UG, nh, Fd, gas.g);
#pragma unroll
      for (int v = 0; v < PV; ++v)
#pragma unroll
        for (int ww = 0; ww < PV; ++ww) acc[v * 5 + ww] += w * Fd[v].d[ww];
    }
  }
#pragma unroll
  for (int k = 0; k < 25; ++k) {
    acc[k] += __shfl_xor(acc[k], 1, 64);
    acc[k] += __shfl_xor(acc[k], 2, 64);
    acc[k] += __shfl_xor(acc[k], 4, 64);
  }
  if (!live) return;
  const double p0 = M.S[(size_t)e * M.spk];
  const double sc = -p0 * p0;
#pragma unroll
  for (int k = 0; k < 25; ++k)
    if ((k & 7) == lf) D0[(size_t)e * 25 + k] = sc * acc[k];
}

// The EXP1 operands (Section 2.1, eq. (EXP1)): dt_E = (p_max+1) dtau_E with
// dtau at p_max from the cell mean, A = T J_0 (Ad = dt D_0, Ao *= dt),
// b = T (R_0 + f); one thread per element.
__global__ void k_poly_p0_scale(int ne, int pmax, double cfl, const double* __restrict__ S, int spk,
                                const double* __restrict__ hE, eg::Gas gas, const double* __restrict__ u0,
                                const double* __restrict__ R0, const double* __restrict__ f0,
                                const double* __restrict__ D0, double* __restrict__ Ad, double* __restrict__ Ao,
                                double* __restrict__ b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double psi0 = S[(size_t)e * spk];
  double U[PV];
#pragma unroll
  for (int v = 0; v < PV; ++v) U[v] = u0[(size_t)e * PV + v] * psi0;
  const double ir = 1.0 / U[0];
  const double q2 = (U[1] * ir) * (U[1] * ir) + (U[2] * ir) * (U[2] * ir) + (U[3] * ir) * (U[3] * ir);
  const double c = sqrt(gas.g * eg::pressure<3>(U, gas.g) * ir);
  const double dt = (pmax + 1.0) * (cfl * hE[e] / ((2.0 * pmax + 1.0) * (sqrt(q2) + c)));
  for (int k = 0; k < 25; ++k) Ad[(size_t)e * 25 + k] = dt * D0[(size_t)e * 25 + k];
  for (int k = 0; k < 150; ++k) Ao[(size_t)e * 150 + k] *= dt;
#pragma unroll
  for (int v = 0; v < PV; ++v)
    b[(size_t)e * PV + v] = dt * (R0[(size_t)e * PV + v] + (f0 ? f0[(size_t)e * PV + v] : 0.0));
}

// u0 += beta V_m y (the Krylov combination of EXP1), one thread per row.
__global__ void k_poly_exp1_update(int K, const double* __restrict__ Vb, const double* __restrict__ y,
                                   const double* __restrict__ info, double* __restrict__ u0) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int mu = (int)info[0];
  const double beta = info[1];
  double t = 0.0;
  for (int j = 0; j < mu; ++j) t += Vb[(size_t)j * K + k] * y[j];
  u0[k] += beta * t;
}

// Element-wise helpers of the V-cycle: z = x + s y (y may be null), and the
// coarse correction x[:Nc] += v - v0 of every [elem][var] row.
__global__ void k_poly_axpy(long long n, const double* __restrict__ x, double s, const double* __restrict__ y,
                            double* __restrict__ z) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = x[i] + (y ? s * y[i] : 0.0);
}
__global__ void k_poly_correct(long long rows, int Nf, int Nc, const double* __restrict__ v,
                               const double* __restrict__ v0, double* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * Nc) return;
  x[(i / Nc) * Nf + (i % Nc)] += v[i] - v0[i];
}

__global__ void k_poly_freestream(int ne, int N, int spk, const double* __restrict__ S, eg::Gas gas,
                                  double* __restrict__ u) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)ne * PV * N) return;
  const int i = (int)(idx % N);
  const long long ev = idx / N;
  const int v = (int)(ev % PV);
  const long long e = ev / PV;
  u[idx] = i == 0 ? gas.Uinf[v] / S[(size_t)e * spk] : 0.0;
}


// Pseudo-time step (Section 4, eq. (x3d)): dtau_E = CFL h_E / ((2p+1)(|v| + c))
// from the cell-mean state u_0 psi_0 (psi_0 = S_00), one thread per element.
__global__ void k_poly_timestep(int ne, int N, int spk, const double* __restrict__ S, const double* __restrict__ hE,
                                eg::Gas gas, double cfl, int p, const double* __restrict__ u,
                                double* __restrict__ dtau) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double psi0 = S[(size_t)e * spk];
  double U[PV];
#pragma unroll
  for (int v = 0; v < PV; ++v) U[v] = u[((size_t)e * PV + v) * N] * psi0;
  const double ir = 1.0 / U[0];
  const double q2 = (U[1] * ir) * (U[1] * ir) + (U[2] * ir) * (U[2] * ir) + (U[3] * ir) * (U[3] * ir);
  const double c = sqrt(gas.g * eg::pressure<3>(U, gas.g) * ir);
  dtau[e] = cfl * hE[e] / ((2.0 * p + 1.0) * (sqrt(q2) + c));
}

// Density-residual norm: per-block partial sums of the squared density
// coefficients (fixed grid, fixed order), then one block sums the partials.
constexpr int NORM_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_poly_norm_partial(long long ne, int N, const double* __restrict__ r,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const long long n = ne * N;
  for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
    const double x = r[(k / N) * PV * N + (k % N)];
    s += x * x;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_poly_norm_final(const double* __restrict__ part, double omega,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  red[threadIdx.x] = threadIdx.x < NORM_BLOCKS ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]) / omega;
}

// Transfers between levels (Section 2.4): with the hierarchical basis the
// level-pc space is the leading Nc modes of every [elem][var] row, so
// restriction is truncation (y = leading slice of x) and prolongation is
// zero padding (x_fine += y_coarse on the leading slice).
__global__ void k_poly_transfer(long long ne, int Nf, int Nc, const double* __restrict__ src, double* __restrict__ dst,
                                int prolong_add) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ne * PV * Nc) return;
  const int i = (int)(idx % Nc);
  const long long ev = idx / Nc;
  if (prolong_add) dst[ev * Nf + i] += src[idx];
  else dst[idx] = src[ev * Nf + i];
}

}  // namespace

struct eg_poly_handle {
  int dev = 0, pmax = 0, ne = 0, nv = 0, nmax = 1;
  hipStream_t st = nullptr;
  eg::Gas gas{};
  std::string err;
  // host copies of the set-up
  std::vector<double> S, geo, vol;
  std::vector<int32_t> nbr_host;  // [E][5]
  // device
  double* d_xyz = nullptr;
  int32_t* d_ev = nullptr;
  int8_t* d_typ = nullptr;
  int32_t* d_nbr = nullptr;
  int32_t* d_fcv = nullptr;
  int8_t* d_fsg = nullptr;
  double* d_geo = nullptr;
  double* d_S = nullptr;
  double* d_a = nullptr;  // [E][5][nmax] monomial coefficients
  double* d_hE = nullptr;    // [E] h_E = 6 |E| / |dE|
  double* d_norm = nullptr;  // [NORM_BLOCKS + 1] norm partials and result
  double omega = 0.0;        // |Omega|
  // PRK work buffers, allocated at the first eg_poly_prk_step for p_max
  double* d_un = nullptr;    // [E][n] u^n
  double* d_R = nullptr;     // [E][n] stage residual
  double* d_P = nullptr;     // [E][n][n] blocks, then their LU factors
  double* d_dtau = nullptr;  // [E]
  int* d_piv = nullptr;      // [E][n]
  int* d_fail = nullptr;     // zero-pivot flag
  // V-cycle: smoother parameters, p = 0 operator, Arnoldi work, level buffers
  int s = 4, m = 30;
  double cfl_max = 100.0;
  int nblk_arn = 0;
  int32_t* d_nbr6 = nullptr;  // [E][6] neighbours for the Arnoldi product (negative: none)
  double *d_D0 = nullptr, *d_Ad = nullptr, *d_Ao = nullptr, *d_b = nullptr, *d_R0 = nullptr;
  double *d_Vb = nullptr, *d_H = nullptr, *d_H2 = nullptr, *d_part1 = nullptr, *d_part2 = nullptr;
  double *d_info = nullptr, *d_wn0 = nullptr, *d_W = nullptr, *d_y = nullptr;
  int *d_arn_st = nullptr, *d_pfail = nullptr;
  double* d_lv[PMAX_POLY + 1][4] = {};  // per level: v, v0, f, r
  double* d_rtop = nullptr;              // R at p_max
  double* d_rule[PMAX_POLY + 1] = {};
  PolyRule rule[PMAX_POLY + 1] = {};
};

namespace {

const int TF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
const int PF[5][4] = {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}};

void host_face(const int8_t typ, const int32_t* ev, int lf, int* vv, int* n) {
  if (typ == 0) {
    *n = 3;
    for (int k = 0; k < 3; ++k) vv[k] = ev[TF[lf][k]];
  } else {
    *n = lf < 2 ? 3 : 4;
    for (int k = 0; k < *n; ++k) vv[k] = ev[PF[lf][k]];
  }
}

// Canonical order: triangle ascending; quad cyclic from its lowest vertex
// towards the lower of that vertex's two neighbours.
void host_canonical(int n, const int* vv, int* cv) {
  if (n == 3) {
    int a = vv[0], b = vv[1], c = vv[2];
    if (a > b) std::swap(a, b);
    if (b > c) std::swap(b, c);
    if (a > b) std::swap(a, b);
    cv[0] = a; cv[1] = b; cv[2] = c; cv[3] = -1;
    return;
  }
  int lo = 0;
  for (int k = 1; k < 4; ++k) if (vv[k] < vv[lo]) lo = k;
  const int step = vv[(lo + 1) & 3] < vv[(lo + 3) & 3] ? 1 : 3;
  for (int k = 0; k < 4; ++k) cv[k] = vv[(lo + step * k) & 3];
}

// Volume points (x, weight) of element e for Q points per direction.
void host_vol_points(int typ, const double (*X)[3], int Q, const double* g01, const double* w01,
                     std::vector<double>& pts, std::vector<double>& wts) {
  pts.clear();
  wts.clear();
  for (int i3 = 0; i3 < Q; ++i3)
    for (int i2 = 0; i2 < Q; ++i2)
      for (int i1 = 0; i1 < Q; ++i1) {
        const double t1 = g01[i1], t2 = g01[i2], t3 = g01[i3];
        double J[3][3], x[3], wf;
        if (typ == 0) {
          const double l1 = t1 * (1 - t2) * (1 - t3), l2 = t2 * (1 - t3), l3 = t3;
          for (int c = 0; c < 3; ++c) {
            J[0][c] = X[1][c] - X[0][c];
            J[1][c] = X[2][c] - X[0][c];
            J[2][c] = X[3][c] - X[0][c];
            x[c] = X[0][c] + l1 * J[0][c] + l2 * J[1][c] + l3 * J[2][c];
          }
          wf = w01[i1] * w01[i2] * w01[i3] * (1 - t2) * (1 - t3) * (1 - t3);
        } else {
          const double l1 = t1 * (1 - t2), l2 = t2, l0 = 1 - l1 - l2, z = t3;
          const double lam[3] = {l0, l1, l2};
          for (int c = 0; c < 3; ++c) {
            double xs = 0, dz = 0;
            for (int k = 0; k < 3; ++k) {
              xs += lam[k] * ((1 - z) * X[k][c] + z * X[k + 3][c]);
              dz += lam[k] * (X[k + 3][c] - X[k][c]);
            }
            x[c] = xs;
            J[0][c] = (1 - z) * (X[1][c] - X[0][c]) + z * (X[4][c] - X[3][c]);
            J[1][c] = (1 - z) * (X[2][c] - X[0][c]) + z * (X[5][c] - X[3][c]);
            J[2][c] = dz;
          }
          wf = w01[i1] * w01[i2] * w01[i3] * (1 - t2);
        }
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[1][0] * (J[0][1] * J[2][2] - J[0][2] * J[2][1]) +
                           J[2][0] * (J[0][1] * J[1][2] - J[0][2] * J[1][1]);
        for (int c = 0; c < 3; ++c) pts.push_back(x[c]);
        wts.push_back(wf * std::fabs(det));
      }
}

template <class T> hipError_t dev_copy(T** d, const T* h, size_t n) {
  hipError_t e = hipMalloc((void**)d, n * sizeof(T) + 16);
  if (e != hipSuccess) return e;
  return hipMemcpy(*d, h, n * sizeof(T), hipMemcpyHostToDevice);
}

eg_status poly_setup(eg_poly_handle* h, const eg_poly_mesh* m) {
  const int ne = m->n_elem, nv = m->n_vert;
  std::vector<int32_t> nbr((size_t)ne * 5, 0), fcv((size_t)ne * 5 * 4, -1);
  std::vector<int8_t> fsg((size_t)ne * 5, 1);
  for (int e = 0; e < ne; ++e) {
    const int typ = m->elem_type[e];
    if (typ != 0 && typ != 1) { h->err = "element type must be 0 (tetrahedron) or 1 (prism)"; return EG_ERR_MESH; }
    for (int k = 0; k < (typ == 0 ? 4 : 6); ++k) {
      const int32_t v = m->elem_vert[(size_t)e * 6 + k];
      if (v < 0 || v >= nv) { h->err = "element vertex index out of range"; return EG_ERR_MESH; }
    }
  }
  // face matching through sorted vertex sets
  std::map<std::array<int, 4>, std::pair<int, int>> open;
  for (int e = 0; e < ne; ++e) {
    const int typ = m->elem_type[e];
    for (int lf = 0; lf < (typ == 0 ? 4 : 5); ++lf) {
      int vv[4], n;
      host_face(typ, &m->elem_vert[(size_t)e * 6], lf, vv, &n);
      host_canonical(n, vv, &fcv[((size_t)e * 5 + lf) * 4]);
      const int tg = m->bface_tag[(size_t)e * 5 + lf];
      if (tg == 1) { nbr[(size_t)e * 5 + lf] = PB_WALL; continue; }
      if (tg == 2) { nbr[(size_t)e * 5 + lf] = PB_FAR; continue; }
      if (tg == 4) { nbr[(size_t)e * 5 + lf] = PB_SYM; continue; }
      if (tg != 0) { h->err = "boundary tag must be 0, 1, 2 or 4"; return EG_ERR_MESH; }
      std::array<int, 4> key{vv[0], vv[1], vv[2], n == 4 ? vv[3] : -1};
      std::sort(key.begin(), key.begin() + n);
      auto it = open.find(key);
      if (it == open.end()) {
        open[key] = {e, lf};
      } else {
        nbr[(size_t)e * 5 + lf] = it->second.first;
        nbr[(size_t)it->second.first * 5 + it->second.second] = e;
        open.erase(it);
      }
    }
  }
  if (!open.empty()) { h->err = "interior face without a matching neighbour"; return EG_ERR_MESH; }
  h->nbr_host = nbr;
  // extents, centroids, outward signs and the MGS basis (volume rule of p_max)
  const int N = pn(h->pmax), Q = h->pmax + 2;
  double g01[8], w01[8];
  eg::gauss_rule01(Q, g01, w01);
  h->geo.assign((size_t)ne * 6, 0.0);
  h->vol.assign(ne, 0.0);
  h->S.assign((size_t)ne * N * N, 0.0);
  std::vector<double> pts, wts, chi, phi;
  for (int e = 0; e < ne; ++e) {
    const int typ = m->elem_type[e], nvt = typ == 0 ? 4 : 6;
    double X[6][3], lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, cE[3] = {0, 0, 0};
    for (int k = 0; k < nvt; ++k)
      for (int c = 0; c < 3; ++c) {
        X[k][c] = m->xyz[(size_t)m->elem_vert[(size_t)e * 6 + k] * 3 + c];
        lo[c] = std::min(lo[c], X[k][c]);
        hi[c] = std::max(hi[c], X[k][c]);
        cE[c] += X[k][c] / nvt;
      }
    {
      double J[3][3];
      for (int c = 0; c < 3; ++c) { J[0][c] = X[1][c] - X[0][c]; J[1][c] = X[2][c] - X[0][c]; J[2][c] = X[3][c] - X[0][c]; }
      const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                         J[1][0] * (J[0][1] * J[2][2] - J[0][2] * J[2][1]) +
                         J[2][0] * (J[0][1] * J[1][2] - J[0][2] * J[1][1]);
      if (!(det > 0.0)) { h->err = "element with non-positive orientation"; return EG_ERR_MESH; }
    }
    host_vol_points(typ, X, Q, g01, w01, pts, wts);
    const int nq = (int)wts.size();
    double vol = 0.0, mx[3] = {0, 0, 0};
    for (int q = 0; q < nq; ++q) {
      vol += wts[q];
      for (int c = 0; c < 3; ++c) mx[c] += wts[q] * pts[q * 3 + c];
    }
    double* g = &h->geo[(size_t)e * 6];
    for (int c = 0; c < 3; ++c) {
      g[c] = mx[c] / vol;
      g[3 + c] = 0.5 * (hi[c] - lo[c]);
    }
    h->vol[e] = vol;
    // monomial values at the points
    chi.assign((size_t)N * nq, 0.0);
    for (int j = 0; j < N; ++j) {
      int ax, ay, az;
      mono_exp(j, ax, ay, az);
      for (int q = 0; q < nq; ++q) {
        double c = 1.0;
        for (int k = 0; k < ax; ++k) c *= (pts[q * 3] - g[0]) / g[3];
        for (int k = 0; k < ay; ++k) c *= (pts[q * 3 + 1] - g[1]) / g[4];
        for (int k = 0; k < az; ++k) c *= (pts[q * 3 + 2] - g[2]) / g[5];
        chi[(size_t)j * nq + q] = c;
      }
    }
    // modified Gram-Schmidt: phi_i starts as chi_i and loses its component
    // along every finished phi_j in turn; S tracks phi in the chi basis
    phi = chi;
    double* Se = &h->S[(size_t)e * N * N];
    for (int i = 0; i < N; ++i) Se[(size_t)i * N + i] = 1.0;
    for (int i = 0; i < N; ++i) {
      double* pi = &phi[(size_t)i * nq];
      for (int j = 0; j < i; ++j) {
        const double* pj = &phi[(size_t)j * nq];
        double hij = 0.0;
        for (int q = 0; q < nq; ++q) hij += wts[q] * pi[q] * pj[q];
        for (int q = 0; q < nq; ++q) pi[q] -= hij * pj[q];
        for (int k = 0; k <= j; ++k) Se[(size_t)i * N + k] -= hij * Se[(size_t)j * N + k];
      }
      double nn = 0.0;
      for (int q = 0; q < nq; ++q) nn += wts[q] * pi[q] * pi[q];
      if (!(nn > 0.0) || !std::isfinite(nn)) { h->err = "degenerate element basis"; return EG_ERR_MESH; }
      const double sc = 1.0 / std::sqrt(nn);
      for (int q = 0; q < nq; ++q) pi[q] *= sc;
      for (int k = 0; k <= i; ++k) Se[(size_t)i * N + k] *= sc;
    }
    // outward sign of each face's canonical normal
    for (int lf = 0; lf < (typ == 0 ? 4 : 5); ++lf) {
      const int32_t* cv = &fcv[((size_t)e * 5 + lf) * 4];
      const int n = cv[3] < 0 ? 3 : 4;
      double C[4][3], cF[3] = {0, 0, 0};
      for (int k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) { C[k][c] = m->xyz[(size_t)cv[k] * 3 + c]; cF[c] += C[k][c] / n; }
      double a[3], b[3], nvv[3];
      for (int c = 0; c < 3; ++c) {
        a[c] = n == 3 ? C[1][c] - C[0][c] : 0.5 * (C[1][c] + C[2][c] - C[0][c] - C[3][c]);
        b[c] = n == 3 ? C[2][c] - C[0][c] : 0.5 * (C[3][c] + C[2][c] - C[0][c] - C[1][c]);
      }
      nvv[0] = a[1] * b[2] - a[2] * b[1];
      nvv[1] = a[2] * b[0] - a[0] * b[2];
      nvv[2] = a[0] * b[1] - a[1] * b[0];
      const double s = nvv[0] * (cF[0] - cE[0]) + nvv[1] * (cF[1] - cE[1]) + nvv[2] * (cF[2] - cE[2]);
      fsg[(size_t)e * 5 + lf] = s < 0.0 ? -1 : 1;
    }
  }
  // |dE| by the face rule of p_max and h_E = 2 d |E| / |dE| (the length
  // scale of the pseudo-time step on the hexahedra)
  std::vector<double> hE(ne, 0.0);
  for (int e = 0; e < ne; ++e) {
    const int typ = m->elem_type[e];
    double surf = 0.0;
    for (int lf = 0; lf < (typ == 0 ? 4 : 5); ++lf) {
      const int32_t* cv = &fcv[((size_t)e * 5 + lf) * 4];
      const int n = cv[3] < 0 ? 3 : 4;
      double C[4][3];
      for (int k = 0; k < n; ++k)
        for (int c = 0; c < 3; ++c) C[k][c] = m->xyz[(size_t)cv[k] * 3 + c];
      for (int i2 = 0; i2 < Q; ++i2)
        for (int i1 = 0; i1 < Q; ++i1) {
          double a[3], b[3], wf;
          if (n == 3) {
            for (int c = 0; c < 3; ++c) { a[c] = C[1][c] - C[0][c]; b[c] = C[2][c] - C[0][c]; }
            wf = w01[i1] * w01[i2] * (1 - g01[i2]);
          } else {
            const double s = g01[i1], t = g01[i2];
            for (int c = 0; c < 3; ++c) {
              a[c] = (1 - t) * (C[1][c] - C[0][c]) + t * (C[2][c] - C[3][c]);
              b[c] = (1 - s) * (C[3][c] - C[0][c]) + s * (C[2][c] - C[1][c]);
            }
            wf = w01[i1] * w01[i2];
          }
          const double nx = a[1] * b[2] - a[2] * b[1], ny = a[2] * b[0] - a[0] * b[2], nz = a[0] * b[1] - a[1] * b[0];
          surf += wf * std::sqrt(nx * nx + ny * ny + nz * nz);
        }
    }
    hE[e] = 6.0 * h->vol[e] / surf;
    h->omega += h->vol[e];
  }
  // reference tables of every order
  std::vector<double> tab;
  for (int p = 0; p <= h->pmax; ++p) {
    const int q = p + 2;
    double x[8], w[8];
    eg::gauss_rule01(q, x, w);
    tab.clear();
    const int nv3 = q * q * q, nv2 = q * q;
    for (int i3 = 0; i3 < q; ++i3)
      for (int i2 = 0; i2 < q; ++i2)
        for (int i1 = 0; i1 < q; ++i1) {
          const double t1 = x[i1], t2 = x[i2], t3 = x[i3];
          tab.insert(tab.end(), {t1 * (1 - t2) * (1 - t3), t2 * (1 - t3), t3,
                                 w[i1] * w[i2] * w[i3] * (1 - t2) * (1 - t3) * (1 - t3)});
        }
    for (int i3 = 0; i3 < q; ++i3)
      for (int i2 = 0; i2 < q; ++i2)
        for (int i1 = 0; i1 < q; ++i1) {
          const double t1 = x[i1], t2 = x[i2], t3 = x[i3];
          tab.insert(tab.end(), {t1 * (1 - t2), t2, t3, w[i1] * w[i2] * w[i3] * (1 - t2)});
        }
    for (int i2 = 0; i2 < q; ++i2)
      for (int i1 = 0; i1 < q; ++i1) tab.insert(tab.end(), {x[i1] * (1 - x[i2]), x[i2], w[i1] * w[i2] * (1 - x[i2])});
    for (int i2 = 0; i2 < q; ++i2)
      for (int i1 = 0; i1 < q; ++i1) tab.insert(tab.end(), {x[i1], x[i2], w[i1] * w[i2]});
    if (dev_copy(&h->d_rule[p], tab.data(), tab.size()) != hipSuccess) { h->err = "rule upload failed"; return EG_ERR_HIP; }
    h->rule[p].tet = h->d_rule[p];
    h->rule[p].pri = h->d_rule[p] + 4 * nv3;
    h->rule[p].tri = h->d_rule[p] + 8 * nv3;
    h->rule[p].quad = h->d_rule[p] + 8 * nv3 + 3 * nv2;
  }
  // S packed row by row (lower triangle): the level-p block is a prefix
  std::vector<double> spk((size_t)ne * (N * (N + 1) / 2));
  for (int e = 0; e < ne; ++e)
    for (int i = 0, k = 0; i < N; ++i)
      for (int j = 0; j <= i; ++j, ++k) spk[(size_t)e * (N * (N + 1) / 2) + k] = h->S[((size_t)e * N + i) * N + j];
  std::vector<int32_t> ev(m->elem_vert, m->elem_vert + (size_t)ne * 6);
  for (int e = 0; e < ne; ++e)
    if (m->elem_type[e] == 0) ev[(size_t)e * 6 + 4] = ev[(size_t)e * 6 + 5] = 0;
  if (dev_copy(&h->d_xyz, m->xyz, (size_t)nv * 3) != hipSuccess || dev_copy(&h->d_ev, ev.data(), ev.size()) != hipSuccess ||
      dev_copy(&h->d_typ, m->elem_type, (size_t)ne) != hipSuccess ||
      dev_copy(&h->d_nbr, nbr.data(), nbr.size()) != hipSuccess ||
      dev_copy(&h->d_fcv, fcv.data(), fcv.size()) != hipSuccess ||
      dev_copy(&h->d_fsg, fsg.data(), fsg.size()) != hipSuccess ||
      dev_copy(&h->d_geo, h->geo.data(), h->geo.size()) != hipSuccess ||
      dev_copy(&h->d_S, spk.data(), spk.size()) != hipSuccess) {
    h->err = "device allocation or upload failed";
    return EG_ERR_ALLOC;
  }
  if (dev_copy(&h->d_hE, hE.data(), hE.size()) != hipSuccess ||
      hipMalloc((void**)&h->d_norm, sizeof(double) * (NORM_BLOCKS + 1)) != hipSuccess) {
    h->err = "device allocation failed";
    return EG_ERR_ALLOC;
  }
  if (hipMalloc((void**)&h->d_a, sizeof(double) * (size_t)ne * PV * N) != hipSuccess) {
    h->err = "device allocation failed";
    return EG_ERR_ALLOC;
  }
  return EG_OK;
}

PolyDev dev_of(const eg_poly_handle* h) {
  PolyDev M;
  M.xyz = h->d_xyz;
  M.ev = h->d_ev;
  M.typ = h->d_typ;
  M.nbr = h->d_nbr;
  M.fcv = h->d_fcv;
  M.fsg = h->d_fsg;
  M.geo = h->d_geo;
  M.S = h->d_S;
  M.ne = h->ne;
  M.spk = h->nmax * (h->nmax + 1) / 2;
  return M;
}

template <int P> hipError_t launch_residual(eg_poly_handle* h, const double* u, double* r) {
  const PolyDev M = dev_of(h);
  hipLaunchKernelGGL(k_poly_mono<P>, dim3((unsigned)h->ne), dim3(64), 0, h->st, M, u, h->d_a);
  const unsigned blocks = 8u * (unsigned)((h->ne + 7) / 8);
  hipLaunchKernelGGL(k_poly_residual<P>, dim3(blocks), dim3(64), 0, h->st, M, h->rule[P], h->gas,
                     (const double*)h->d_a, r);
  return hipGetLastError();
}

template <int P> hipError_t launch_block(eg_poly_handle* h, const double* u, double* D) {
  const PolyDev M = dev_of(h);
  hipLaunchKernelGGL(k_poly_mono<P>, dim3((unsigned)h->ne), dim3(64), 0, h->st, M, u, h->d_a);
  const unsigned blocks = 8u * (unsigned)((h->ne + 7) / 8);
  hipLaunchKernelGGL(k_poly_block<P>, dim3(blocks), dim3(256), 0, h->st, M, h->rule[P], h->gas,
                     (const double*)h->d_a, D);
  return hipGetLastError();
}

template <int P> hipError_t launch_prk(eg_poly_handle* h, int s, double cfl, double* u, const double* f) {
  constexpr int n = PV * pn(P);
  const size_t K = (size_t)h->ne * n;
  hipError_t e = hipMemcpyAsync(h->d_un, u, K * sizeof(double), hipMemcpyDeviceToDevice, h->st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_timestep, dim3((unsigned)((h->ne + 255) / 256)), dim3(256), 0, h->st, h->ne, pn(P),
                     h->nmax * (h->nmax + 1) / 2, (const double*)h->d_S, (const double*)h->d_hE, h->gas, cfl, P,
                     (const double*)u, h->d_dtau);
  e = launch_block<P>(h, u, h->d_P);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_lu<P>, dim3((unsigned)h->ne), dim3(256), 0, h->st, h->ne, h->d_P,
                     (const double*)h->d_dtau, h->d_piv, h->d_fail);
  for (int k = 1; k <= s; ++k) {
    e = launch_residual<P>(h, u, h->d_R);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_poly_stage<P>, dim3((unsigned)h->ne), dim3(64), 0, h->st, h->ne, (const double*)h->d_P,
                       (const int*)h->d_piv, (const double*)h->d_R, f, (const double*)h->d_un, 1.0 / (s - k + 1.0), u);
  }
  return hipGetLastError();
}

eg_status ensure_prk_buffers(eg_poly_handle* h) {
  if (h->d_P) return EG_OK;
  const size_t n = (size_t)PV * h->nmax, E = (size_t)h->ne;
  if (hipMalloc((void**)&h->d_un, sizeof(double) * E * n) != hipSuccess ||
      hipMalloc((void**)&h->d_R, sizeof(double) * E * n) != hipSuccess ||
      hipMalloc((void**)&h->d_P, sizeof(double) * E * n * n) != hipSuccess ||
      hipMalloc((void**)&h->d_dtau, sizeof(double) * E) != hipSuccess ||
      hipMalloc((void**)&h->d_piv, sizeof(int) * E * n) != hipSuccess ||
      hipMalloc((void**)&h->d_fail, sizeof(int)) != hipSuccess) {
    h->err = "device allocation of the PRK buffers failed";
    return EG_ERR_ALLOC;
  }
  return EG_OK;
}

eg_status ensure_vc_buffers(eg_poly_handle* h) {
  eg_status st = ensure_prk_buffers(h);
  if (st != EG_OK || h->d_nbr6) return st;
  const size_t E = (size_t)h->ne, K = E * PV, m = (size_t)h->m;
  h->nblk_arn = eg::arnoldi_blocks((int)K);
  std::vector<int32_t> nb6(E * 6, -1);
  for (size_t e = 0; e < E; ++e)
    for (int lf = 0; lf < 5; ++lf) nb6[e * 6 + lf] = h->nbr_host[e * 5 + lf] >= 0 ? h->nbr_host[e * 5 + lf] : -1;
  bool ok = dev_copy(&h->d_nbr6, nb6.data(), nb6.size()) == hipSuccess;
#define PA(ptr, count) ok = ok && hipMalloc((void**)&(ptr), sizeof(*(ptr)) * (count) + 16) == hipSuccess
  PA(h->d_D0, E * 25);
  PA(h->d_Ad, E * 25);
  PA(h->d_Ao, E * 150);
  PA(h->d_b, K);
  PA(h->d_R0, K);
  PA(h->d_Vb, (m + 1) * K);
  PA(h->d_H, (m + 1) * m);
  PA(h->d_H2, (m + 1) * m);
  PA(h->d_part1, (size_t)h->nblk_arn * (m + 2));
  PA(h->d_part2, (size_t)h->nblk_arn * (m + 2));
  PA(h->d_info, 2);
  PA(h->d_wn0, 2);
  PA(h->d_W, 2 * K);
  PA(h->d_y, m + 1);
  PA(h->d_arn_st, 2);
  PA(h->d_pfail, 1);
  PA(h->d_rtop, E * PV * h->nmax);
  for (int p = 0; p < h->pmax; ++p)
    for (int k = 0; k < 4; ++k) PA(h->d_lv[p][k], E * PV * pn(p));
#undef PA
  if (ok) ok = hipMemset(h->d_info, 0, 2 * sizeof(double)) == hipSuccess &&
               hipMemset(h->d_arn_st, 0, 2 * sizeof(int)) == hipSuccess &&
               hipMemset(h->d_wn0, 0, 2 * sizeof(double)) == hipSuccess &&
               hipMemset(h->d_pfail, 0, sizeof(int)) == hipSuccess;
  if (!ok) {
    h->err = "device allocation of the V-cycle buffers failed";
    return EG_ERR_ALLOC;
  }
  return EG_OK;
}

hipError_t residual_any(eg_poly_handle* h, int p, const double* u, double* r) {
  switch (p) {
    case 0: return launch_residual<0>(h, u, r);
    case 1: return launch_residual<1>(h, u, r);
    case 2: return launch_residual<2>(h, u, r);
    default: return launch_residual<3>(h, u, r);
  }
}

hipError_t prk_any(eg_poly_handle* h, int p, int s, double cfl, double* u, const double* f) {
  switch (p) {
    case 1: return launch_prk<1>(h, s, cfl, u, f);
    case 2: return launch_prk<2>(h, s, cfl, u, f);
    default: return launch_prk<3>(h, s, cfl, u, f);
  }
}

// EXP1 on the level-0 state u0 with forcing f0 (Section 2.1, eq. (EXP1);
// Section 2.2): the operands by k_poly_p0_diag, k_poly_p0_off and
// k_poly_p0_scale, then the library's Arnoldi (two grid-wide kernels per
// step) and phi_1 (Pade on the matrix cores) on the p = 0 operator, then
// u0 += beta V y.
hipError_t poly_exp1_run(eg_poly_handle* h, double cfl, double* u0, const double* f0) {
  const PolyDev M = dev_of(h);
  const int K = h->ne * PV;
  hipError_t e = launch_residual<0>(h, u0, h->d_R0);  // also leaves a = S^T u0 in d_a
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_p0_diag, dim3((unsigned)((h->ne * 8 + 255) / 256)), dim3(256), 0, h->st, M, h->rule[0],
                     h->gas, (const double*)h->d_a, h->d_D0);
  hipLaunchKernelGGL(k_poly_p0_off, dim3((unsigned)((h->ne * 6 + 255) / 256)), dim3(256), 0, h->st, M, h->rule[0],
                     h->gas, (const double*)h->d_a, h->d_Ao);
  hipLaunchKernelGGL(k_poly_p0_scale, dim3((unsigned)((h->ne + 255) / 256)), dim3(256), 0, h->st, h->ne, h->pmax,
                     cfl, (const double*)h->d_S, h->nmax * (h->nmax + 1) / 2, (const double*)h->d_hE, h->gas,
                     (const double*)u0, (const double*)h->d_R0, f0, (const double*)h->d_D0, h->d_Ad, h->d_Ao,
                     h->d_b);
  eg::DevMesh Mv;
  Mv.d = 3;
  Mv.V = PV;
  Mv.ne = h->ne;
  Mv.NF = 6;
  Mv.nbr = h->d_nbr6;
  e = eg::launch_arnoldi(Mv, h->m, h->nblk_arn, h->d_Ad, h->d_Ao, h->d_b, h->d_Vb, h->d_H, h->d_part1, h->d_part2,
                         h->d_info, h->d_arn_st, h->d_wn0, h->d_W, h->d_H2, h->st);
  if (e != hipSuccess) return e;
  e = eg::launch_phi1(h->m, 1, h->d_H, h->d_H2, h->d_info, h->d_y, h->d_pfail, h->st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_exp1_update, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, h->st, K,
                     (const double*)h->d_Vb, (const double*)h->d_y, (const double*)h->d_info, u0);
  return hipGetLastError();
}

// The V-cycle below level p (Section 2.4), as on the hexahedra: PRK, the FAS
// forcing f_{p-1} = Trunc(R_p(u) + f_p) - R_{p-1}(Trunc u), recursion, EXP1
// on p = 0, prolongation of the coarse correction.
hipError_t poly_vc(eg_poly_handle* h, int p, double cfl, double* u, const double* f) {
  if (p == 0) return poly_exp1_run(h, cfl, u, f);
  hipError_t e = prk_any(h, p, h->s, cfl, u, f);
  if (e != hipSuccess) return e;
  const long long rows = (long long)h->ne * PV;
  const int Nf = pn(p), Nc = pn(p - 1);
  double *v = h->d_lv[p - 1][0], *v0 = h->d_lv[p - 1][1], *fc = h->d_lv[p - 1][2], *rc = h->d_lv[p - 1][3];
  double* r = p == h->pmax ? h->d_rtop : h->d_lv[p][3];
  const long long nf = rows * Nf, nc = rows * Nc;
  const unsigned gf = (unsigned)((nf + 255) / 256), gc = (unsigned)((nc + 255) / 256);
  if ((e = residual_any(h, p, u, r)) != hipSuccess) return e;
  if (f) hipLaunchKernelGGL(k_poly_axpy, dim3(gf), dim3(256), 0, h->st, nf, (const double*)r, 1.0, f, r);
  hipLaunchKernelGGL(k_poly_transfer, dim3(gc), dim3(256), 0, h->st, (long long)h->ne, Nf, Nc, (const double*)u, v0, 0);
  hipLaunchKernelGGL(k_poly_transfer, dim3(gc), dim3(256), 0, h->st, (long long)h->ne, Nf, Nc, (const double*)r, rc, 0);
  if ((e = residual_any(h, p - 1, v0, fc)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_axpy, dim3(gc), dim3(256), 0, h->st, nc, (const double*)rc, -1.0, (const double*)fc, fc);
  hipLaunchKernelGGL(k_poly_axpy, dim3(gc), dim3(256), 0, h->st, nc, (const double*)v0, 0.0, (const double*)nullptr, v);
  if ((e = poly_vc(h, p - 1, cfl, v, fc)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_poly_correct, dim3(gc), dim3(256), 0, h->st, rows, Nf, Nc, (const double*)v, (const double*)v0, u);
  return hipGetLastError();
}

double poly_cfl_ramp(double cfl_max, double rn, double rref, int n, int pmax) {
  const double a = rn > 0.0 ? rref / rn : HUGE_VAL;
  const double b = 1.0 + (n - 1.0) / (2.0 * pmax + 1.0);
  return std::min(cfl_max, std::max(a, b));
}

}  // namespace
extern "C" eg_status eg_poly_rnorm(eg_poly_handle* h, int p, const double* r_dev, double* rn_host);
namespace {

// r_n of the state at level p_max (one synchronisation).
eg_status entry_norm(eg_poly_handle* h, const double* u, double* rn) {
  eg_status st = ensure_vc_buffers(h);
  if (st != EG_OK) return st;
  const hipError_t e = residual_any(h, h->pmax, u, h->d_rtop);
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return eg_poly_rnorm(h, h->pmax, h->d_rtop, rn);
}

// One V-cycle at the given CFL; reads the failure flags (one synchronisation).
eg_status run_cycle(eg_poly_handle* h, double* u, double cfl) {
  // the failure flags cover the whole cycle (every level's blocks and phi_1)
  hipLaunchKernelGGL(k_poly_zero_flag, dim3(1), dim3(1), 0, h->st, h->d_fail);
  hipLaunchKernelGGL(k_poly_zero_flag, dim3(1), dim3(1), 0, h->st, h->d_pfail);
  hipError_t e = poly_vc(h, h->pmax, cfl, u, nullptr);
  int fail[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(&fail[0], h->d_fail, sizeof(int), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipMemcpyAsync(&fail[1], h->d_pfail, sizeof(int), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  if (fail[0] || fail[1]) { h->err = "zero pivot or failed phi_1 in the V-cycle"; return EG_ERR_DIVERGED; }
  return EG_OK;
}

}  // namespace

extern "C" {

eg_status eg_poly_prk_step(eg_poly_handle* h, int p, int s, double cfl, double* u_dev, const double* f_dev) {
  if (!h || !u_dev || p < 1 || p > h->pmax || s < 1 || !(cfl > 0.0) || f_dev == (const double*)u_dev)
    return EG_ERR_ARG;
  {
    const eg_status st = ensure_prk_buffers(h);
    if (st != EG_OK) return st;
  }
  hipLaunchKernelGGL(k_poly_zero_flag, dim3(1), dim3(1), 0, h->st, h->d_fail);
  hipError_t e;
  switch (p) {
    case 1: e = launch_prk<1>(h, s, cfl, u_dev, f_dev); break;
    case 2: e = launch_prk<2>(h, s, cfl, u_dev, f_dev); break;
    default: e = launch_prk<3>(h, s, cfl, u_dev, f_dev); break;
  }
  int fail = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&fail, h->d_fail, sizeof(int), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  if (fail) { h->err = "zero or non-finite pivot in a PRK block"; return EG_ERR_DIVERGED; }
  return EG_OK;
}

eg_status eg_poly_exp1_step(eg_poly_handle* h, double cfl, double* u0_dev, const double* f0_dev) {
  if (!h || !u0_dev || !(cfl > 0.0) || f0_dev == (const double*)u0_dev) return EG_ERR_ARG;
  eg_status st = ensure_vc_buffers(h);
  if (st != EG_OK) return st;
  hipLaunchKernelGGL(k_poly_zero_flag, dim3(1), dim3(1), 0, h->st, h->d_pfail);
  hipError_t e = poly_exp1_run(h, cfl, u0_dev, f0_dev);
  int fail = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&fail, h->d_pfail, sizeof(int), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  if (fail) { h->err = "phi_1 evaluation failed (non-finite Hessenberg matrix)"; return EG_ERR_DIVERGED; }
  return EG_OK;
}

eg_status eg_poly_vcycle(eg_poly_handle* h, double* u_dev, int n, double rref, double* rn_host, double* cfl_host) {
  if (!h || !u_dev || n < 1 || h->pmax < 1) return EG_ERR_ARG;
  double rn = 0.0;
  eg_status st = entry_norm(h, u_dev, &rn);
  if (rn_host) *rn_host = rn;
  if (st != EG_OK) return st;
  if (!std::isfinite(rn)) { h->err = "non-finite residual norm"; return EG_ERR_DIVERGED; }
  const double cfl = poly_cfl_ramp(h->cfl_max, rn, rref > 0.0 ? rref : rn, n, h->pmax);
  if (cfl_host) *cfl_host = cfl;
  return run_cycle(h, u_dev, cfl);
}

eg_status eg_poly_solve_steady(eg_poly_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                               int* n_cycles_host) {
  if (!h || !u_dev || !hist_host || !n_cycles_host || max_cycles < 0 || h->pmax < 1) return EG_ERR_ARG;
  double r1 = 0.0;
  for (int n = 1;; ++n) {
    double rn = 0.0;
    const eg_status st = entry_norm(h, u_dev, &rn);
    if (st != EG_OK) return st;
    hist_host[n - 1] = rn;
    if (n == 1) r1 = rn;
    *n_cycles_host = n - 1;
    if (!std::isfinite(rn)) { h->err = "non-finite residual norm"; return EG_ERR_DIVERGED; }
    if (rn <= drop_tol * r1) return EG_OK;
    if (n - 1 == max_cycles) return EG_ERR_NOT_CONVERGED;
    const eg_status sc = run_cycle(h, u_dev, poly_cfl_ramp(h->cfl_max, rn, r1, n, h->pmax));
    if (sc != EG_OK) return sc;
  }
}

eg_status eg_poly_element_block(eg_poly_handle* h, int p, const double* u_dev, double* D_dev) {
  if (!h || !u_dev || !D_dev || p < 0 || p > h->pmax) return EG_ERR_ARG;
  hipError_t e;
  switch (p) {
    case 0: e = launch_block<0>(h, u_dev, D_dev); break;
    case 1: e = launch_block<1>(h, u_dev, D_dev); break;
    case 2: e = launch_block<2>(h, u_dev, D_dev); break;
    default: e = launch_block<3>(h, u_dev, D_dev); break;
  }
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}


eg_status eg_poly_init(const eg_poly_mesh* mesh, const eg_params* prm, void* hip_stream, eg_poly_handle** out) {
  if (!out) return EG_ERR_ARG;
  *out = nullptr;
  if (!mesh || !prm || !mesh->xyz || !mesh->elem_type || !mesh->elem_vert || !mesh->bface_tag) return EG_ERR_ARG;
  if (mesh->n_vert <= 0 || mesh->n_elem <= 0 || mesh->n_elem > (1 << 26)) return EG_ERR_ARG;
  if (prm->p_max < 0 || prm->p_max > PMAX_POLY || !(prm->gamma > 1.0) || !(prm->mach >= 0.0) ||
      prm->rk_stages < 1 || prm->krylov_m < 1 || prm->krylov_m > 48 || !(prm->cfl_max > 0.0) ||
      (prm->flux != EG_FLUX_RUSANOV && prm->flux != EG_FLUX_ROE))
    return EG_ERR_ARG;
  eg_poly_handle* h = new (std::nothrow) eg_poly_handle;
  if (!h) return EG_ERR_ALLOC;
  *out = h;
  hipGetDevice(&h->dev);
  h->st = (hipStream_t)hip_stream;
  h->pmax = prm->p_max;
  h->ne = mesh->n_elem;
  h->nv = mesh->n_vert;
  h->nmax = pn(prm->p_max);
  h->s = prm->rk_stages;
  h->m = prm->krylov_m;
  h->cfl_max = prm->cfl_max;
  const double al = prm->alpha_deg * M_PI / 180.0, be = prm->beta_deg * M_PI / 180.0;
  const double v[3] = {prm->mach * std::cos(al) * std::cos(be), prm->mach * std::sin(al) * std::cos(be),
                       prm->mach * std::sin(be)};
  h->gas.g = prm->gamma;
  h->gas.flux = prm->flux;
  h->gas.Uinf[0] = 1.0;
  double ke = 0.0;
  for (int a = 0; a < 3; ++a) { h->gas.Uinf[1 + a] = v[a]; ke += v[a] * v[a]; }
  h->gas.Uinf[4] = 1.0 / (prm->gamma * (prm->gamma - 1.0)) + 0.5 * ke;
  return poly_setup(h, mesh);
}

void eg_poly_free(eg_poly_handle* h) {
  if (!h) return;
  int cur = 0;
  hipGetDevice(&cur);
  hipSetDevice(h->dev);
  void* bufs[] = {h->d_xyz, h->d_ev, h->d_typ, h->d_nbr, h->d_fcv, h->d_fsg, h->d_geo, h->d_S, h->d_a, h->d_hE, h->d_norm,
                  h->d_un, h->d_R, h->d_P, h->d_dtau, h->d_piv, h->d_fail, h->d_nbr6, h->d_D0, h->d_Ad, h->d_Ao,
                  h->d_b, h->d_R0, h->d_Vb, h->d_H, h->d_H2, h->d_part1, h->d_part2, h->d_info, h->d_wn0, h->d_W,
                  h->d_y, h->d_arn_st, h->d_pfail, h->d_rtop};
  for (void* b : bufs)
    if (b) hipFree(b);
  for (auto* b : h->d_rule)
    if (b) hipFree(b);
  for (auto& lv : h->d_lv)
    for (auto* b : lv)
      if (b) hipFree(b);
  hipSetDevice(cur);
  delete h;
}

const char* eg_poly_last_error(const eg_poly_handle* h) { return h ? h->err.c_str() : "null handle"; }

eg_status eg_poly_freestream(eg_poly_handle* h, int p, double* u_dev) {
  if (!h || !u_dev || p < 0 || p > h->pmax) return EG_ERR_ARG;
  const long long n = (long long)h->ne * PV * pn(p);
  hipLaunchKernelGGL(k_poly_freestream, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->st, h->ne, pn(p),
                     h->nmax * (h->nmax + 1) / 2, (const double*)h->d_S, h->gas, u_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}

eg_status eg_poly_residual(eg_poly_handle* h, int p, const double* u_dev, double* r_dev) {
  if (!h || !u_dev || !r_dev || p < 0 || p > h->pmax || (const double*)r_dev == u_dev) return EG_ERR_ARG;
  hipError_t e;
  switch (p) {
    case 0: e = launch_residual<0>(h, u_dev, r_dev); break;
    case 1: e = launch_residual<1>(h, u_dev, r_dev); break;
    case 2: e = launch_residual<2>(h, u_dev, r_dev); break;
    default: e = launch_residual<3>(h, u_dev, r_dev); break;
  }
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}

eg_status eg_poly_timestep(eg_poly_handle* h, int p, double cfl, const double* u_dev, double* dtau_dev) {
  if (!h || !u_dev || !dtau_dev || p < 0 || p > h->pmax || !(cfl > 0.0)) return EG_ERR_ARG;
  hipLaunchKernelGGL(k_poly_timestep, dim3((unsigned)((h->ne + 255) / 256)), dim3(256), 0, h->st, h->ne, pn(p),
                     h->nmax * (h->nmax + 1) / 2, (const double*)h->d_S, (const double*)h->d_hE, h->gas, cfl, p,
                     u_dev, dtau_dev);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}

eg_status eg_poly_rnorm(eg_poly_handle* h, int p, const double* r_dev, double* rn_host) {
  if (!h || !r_dev || !rn_host || p < 0 || p > h->pmax) return EG_ERR_ARG;
  hipLaunchKernelGGL(k_poly_norm_partial, dim3(NORM_BLOCKS), dim3(256), 0, h->st, (long long)h->ne, pn(p), r_dev,
                     h->d_norm);
  hipLaunchKernelGGL(k_poly_norm_final, dim3(1), dim3(256), 0, h->st, (const double*)h->d_norm, h->omega,
                     h->d_norm + NORM_BLOCKS);
  hipError_t e = hipMemcpyAsync(rn_host, h->d_norm + NORM_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, h->st);
  if (e == hipSuccess) e = hipStreamSynchronize(h->st);
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}

eg_status eg_poly_restrict(eg_poly_handle* h, int pf, int pc, const double* xf_dev, double* yc_dev) {
  if (!h || !xf_dev || !yc_dev || pc < 0 || pc > pf || pf > h->pmax || xf_dev == (const double*)yc_dev)
    return EG_ERR_ARG;
  const long long n = (long long)h->ne * PV * pn(pc);
  hipLaunchKernelGGL(k_poly_transfer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->st, (long long)h->ne,
                     pn(pf), pn(pc), xf_dev, yc_dev, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}

eg_status eg_poly_prolong_add(eg_poly_handle* h, int pc, int pf, const double* yc_dev, double* xf_dev) {
  if (!h || !xf_dev || !yc_dev || pc < 0 || pc > pf || pf > h->pmax || yc_dev == (const double*)xf_dev)
    return EG_ERR_ARG;
  const long long n = (long long)h->ne * PV * pn(pc);
  hipLaunchKernelGGL(k_poly_transfer, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->st, (long long)h->ne,
                     pn(pf), pn(pc), yc_dev, xf_dev, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { h->err = hipGetErrorString(e); return EG_ERR_HIP; }
  return EG_OK;
}

eg_status eg_poly_basis(const eg_poly_handle* h, double* S_host, double* xc_host, double* L_host, double* vol_host) {
  if (!h) return EG_ERR_ARG;
  if (S_host) std::memcpy(S_host, h->S.data(), h->S.size() * sizeof(double));
  for (int e = 0; e < h->ne; ++e) {
    for (int c = 0; c < 3; ++c) {
      if (xc_host) xc_host[e * 3 + c] = h->geo[(size_t)e * 6 + c];
      if (L_host) L_host[e * 3 + c] = h->geo[(size_t)e * 6 + 3 + c];
    }
    if (vol_host) vol_host[e] = h->vol[e];
  }
  return EG_OK;
}

}  // extern "C"
