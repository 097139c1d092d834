// HIP kernels of the eMG hot path for gfx950 (MI355X): FP64, with FP32
// instantiations of the smoother kernels (residual, block assembly + LU, PRK
// stage) for the mixed-precision mode.
//
// State representation.  The paper's basis is psi = T phi per element
// (Section 3.2, eq. (basis)): reference tensor-Legendre phi orthonormalised in
// the physical inner product, T = L^{-1} with G = L L^T the element mass
// matrix of phi.  The kernels keep the state in the phi coordinates
// ut = T^T u (= L^{-T} u), an exact change of variables:
//   residual        Rt(ut) = T^{-1} R(u)            (no T inside the kernel)
//   element block   Pt = T^{-1} P T^{-T} = G/dtau - dRt/dut
//   PRK update      ut^(k) = ut^n + beta_k Pt^{-1} [Rt + ft],  ft = T^{-1} f
// so the smoother never reads T; the restriction of the solution, the norm
// and the conversions at the C ABI use the Cholesky factor L.  The p = 0
// level (EXP1) runs in the paper's psi coordinates, where the Euclidean inner
// product of the Arnoldi process is the L2 inner product.
//
// Layouts (all FP64 unless noted):
//   level-p vector   [E][V][N_p], hierarchical mode order (leading slices)
//   vertices         [E][2^D][D]
//   neighbour        int32 [E][2D]: element index, NB_WALL or NB_FAR
//   face code        uint8 [E][2D]: neighbour face | swap<<3 | flip0<<4 | flip1<<5
//   Cholesky / mass  packed lower triangle [E][NT], NT = N(N+1)/2 of p_max
//   block factors    [E][n][n] column-major LU (unit L), perm int32 [E][n]

#include <hip/hip_runtime.h>

#include <algorithm>

#include "eg_common.h"
#include "eg_launch.h"
#include "eg_physics.h"
#include "eg_device.h"


namespace eg {


// ---------------------------------------------------------------------------
// DG residual (Section 3.1, eq. (euler3)) in the phi coordinates:
//   Rt_{v,i} = sum_q w_q sum_r d_r phi_i(q) [F_v(U_q) . c_r(q)]
//            - sum_faces sum_k w_k |n dsigma| phi_i F~_v(U_own, U_nb; n^)
// A block handles EB elements: (1) stage ut of the tile in LDS, (2) one
// thread per volume point evaluates U, the flux and the contravariant flux,
// (3) one thread per face point evaluates both traces (the neighbour's from
// global memory at its matching Gauss point) and the Rusanov flux, (4) one
// thread per output (element, var, mode) projects onto the test functions.
// Optional: add a forcing vector; or, as the coarse residual of the FAS
// restriction (Section 2.4, steps 2-3, full approximation form), return the
// truncated fine residual t in rt and the forcing t - R in fas.fc instead of
// R (in phi coordinates the truncation of a residual is its leading modes).
// ---------------------------------------------------------------------------
template <int D, int P, class R>
constexpr int res_table_values() {
  using C = Cfg<D, P>;
  return C::QV * C::N * (1 + D) + C::NF * C::QF * C::N;
}

// The basis tables live in LDS when they fit in 32 KiB (every 2D order and
// 3D p = 1); larger 3D orders evaluate the tensor products on the fly.
template <int D, int P, class R>
constexpr bool res_tables() {
  return res_table_values<D, P, R>() * (int)sizeof(R) <= 32 * 1024;
}

template <int D, int P, int EB, class R, bool CQ = false>
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ ut, const double* __restrict__ fadd,
                                                  double* __restrict__ rt, const double* __restrict__ xv, int nc,
                                                  const int* __restrict__ nbr, const uint8_t* __restrict__ ncode,
                                                  int ne, Tab<D, P, R> tab, GasT<R> gas,
                                                  const double* __restrict__ uinf_e, FasOut fas) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, NC = C::NC;
  __shared__ R s_u[EB * V * N];
  __shared__ R s_fc[EB * QV * V * D];
  __shared__ R s_ff[EB * NF * QF * V];
  __shared__ R s_x[EB * NC * D];
  __shared__ Tab<D, P, R> t;
  // basis tables of the block: phi_k and d_r phi_k at the volume points,
  // phi_k at the face points ([q][k], [q][r][k], [lf][kf][k])
  constexpr bool TBL = res_tables<D, P, R>();
  __shared__ R s_phv[TBL ? QV * N : 1];
  __shared__ R s_dphv[TBL ? QV * D * N : 1];
  __shared__ R s_phf[TBL ? NF * QF * N : 1];
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EB;
  copy_tab(t, tab);
  {
    const int nel = min(EB, ne - e0);
    stage<(EB * V * N + 255) / 256>(s_u, ut + (size_t)e0 * V * N, nel * V * N, tid, 256);
    if (!CQ) stage<(EB * NC * D + 255) / 256>(s_x, xv + (size_t)e0 * NC * D, nel * NC * D, tid, 256);
  }
  __syncthreads();
  if constexpr (TBL) {
  for (int it = tid; it < QV * N; it += blockDim.x) {
    const int q = it / N, kk = it % N;
    int iq[D], r0 = q;
#pragma unroll
    for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
    s_phv[it] = phi_vol<D, P, R>(t, kk, iq);
#pragma unroll
    for (int r = 0; r < D; ++r) s_dphv[(q * D + r) * N + kk] = dphi_vol<D, P, R>(t, kk, iq, r);
  }
  for (int it = tid; it < NF * QF * N; it += blockDim.x) {
    const int lf = it / (QF * N), kf = (it / N) % QF, kk = it % N;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = kf;
    face_axes<D>(lf, ta);
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
    s_phf[it] = phi_face<D, P, R>(t, kk, lf, ta, ik);
  }
  __syncthreads();
  }
  // volume points
  for (int it = tid; it < EB * QV; it += blockDim.x) {
    const int el = it / QV, q = it % QV;
    if (e0 + el >= ne) continue;
    int iq[D];
    R xi[D], wq = R(1);
    {
      int r0 = q;
#pragma unroll
      for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; xi[r] = t.x[iq[r]]; wq *= t.w[iq[r]]; }
    }
    R U[V];
#pragma unroll
    for (int v = 0; v < V; ++v) U[v] = R(0);
    const R* su = &s_u[el * V * N];
    for (int k = 0; k < N; ++k) {
      R ph;
      if constexpr (TBL) ph = s_phv[q * N + k];
      else ph = phi_vol<D, P, R>(t, k, iq);
#pragma unroll
      for (int v = 0; v < V; ++v) U[v] += su[v * N + k] * ph;
    }
    R c[D][D], det;
    geom_any<D, CQ>(&s_x[el * NC * D], xv + (size_t)(e0 + el) * nc * D, xi, c, det);
#pragma unroll
    for (int r = 0; r < D; ++r) {
      R F[V];
      flux_n<D>(U, c[r], F, gas.g);
#pragma unroll
      for (int v = 0; v < V; ++v) s_fc[((el * QV + q) * V + v) * D + r] = wq * F[v];
    }
  }
  // face points
  for (int it = tid; it < EB * NF * QF; it += blockDim.x) {
    const int el = it / (NF * QF), lf = (it / QF) % NF, k = it % QF;
    const int e = e0 + el;
    if (e >= ne) continue;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1];
    face_axes<D>(lf, ta);
    R xi[D], wk = R(1);
    xi[lf >> 1] = (lf & 1) ? R(1) : R(-1);
    {
      int r0 = k;
#pragma unroll
      for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; xi[ta[q]] = t.x[ik[q]]; wk *= t.w[ik[q]]; }
    }
    R UL[V], UR[V];
#pragma unroll
    for (int v = 0; v < V; ++v) UL[v] = R(0);
    const R* su = &s_u[el * V * N];
    for (int j = 0; j < N; ++j) {
      R ph;
      if constexpr (TBL) ph = s_phf[(lf * QF + k) * N + j];
      else ph = phi_face<D, P, R>(t, j, lf, ta, ik);
#pragma unroll
      for (int v = 0; v < V; ++v) UL[v] += su[v * N + j] * ph;
    }
    R c[D][D], det;
    geom_any<D, CQ>(&s_x[el * NC * D], xv + (size_t)(e0 + el) * nc * D, xi, c, det);
    R nh[D], a2 = R(0);
    const R sg = (lf & 1) ? R(1) : R(-1);
#pragma unroll
    for (int a = 0; a < D; ++a) { nh[a] = sg * c[lf >> 1][a]; a2 += nh[a] * nh[a]; }
    const R area = dsqrt(a2);
#pragma unroll
    for (int a = 0; a < D; ++a) nh[a] /= area;
    const int nb = nbr[(size_t)e * NF + lf];
    if (nb >= 0) {
      const int code = ncode[(size_t)e * NF + lf];
      const int lf2 = code & 7;
      int ta2[D - 1 > 0 ? D - 1 : 1], jk[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf2, ta2);
      nb_face_index<D, Q>(code, ik, jk);
#pragma unroll
      for (int v = 0; v < V; ++v) UR[v] = R(0);
      const double* un = ut + (size_t)nb * V * N;
      int kf2 = 0;
#pragma unroll
      for (int q = D - 2; q >= 0; --q) kf2 = kf2 * Q + jk[q];
      for (int j = 0; j < N; ++j) {
        R ph;
        if constexpr (TBL) ph = s_phf[(lf2 * QF + kf2) * N + j];
        else ph = phi_face<D, P, R>(t, j, lf2, ta2, jk);
#pragma unroll
        for (int v = 0; v < V; ++v) UR[v] += R(un[v * N + j]) * ph;
      }
    } else if (nb == NB_WALL) {
      ghost_wall<D>(UL, nh, UR);
    } else {
      R Ui[V];
#pragma unroll
      for (int v = 0; v < V; ++v) Ui[v] = uinf_e ? R(uinf_e[(size_t)e * V + v]) : gas.Uinf[v];
      ghost_far<D>(UL, nh, UR, Ui, gas.g);
    }
    R F[V];
    num_flux<D>(UL, UR, nh, F, gas);
#pragma unroll
    for (int v = 0; v < V; ++v) s_ff[((el * NF + lf) * QF + k) * V + v] = wk * area * F[v];
  }
  __syncthreads();
  // projection onto the test functions
  for (int it = tid; it < EB * V * N; it += blockDim.x) {
    const int el = it / (V * N), v = (it / N) % V, i = it % N;
    const int e = e0 + el;
    if (e >= ne) continue;
    R acc = R(0);
    if constexpr (TBL) {
      for (int q = 0; q < QV; ++q) {
        const R* fc = &s_fc[((el * QV + q) * V + v) * D];
#pragma unroll
        for (int r = 0; r < D; ++r) acc += s_dphv[(q * D + r) * N + i] * fc[r];
      }
      for (int fk = 0; fk < NF * QF; ++fk) acc -= s_phf[fk * N + i] * s_ff[(el * NF * QF + fk) * V + v];
    } else {
      for (int q = 0; q < QV; ++q) {
        int iq[D];
        int r0 = q;
#pragma unroll
        for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
        const R* fc = &s_fc[((el * QV + q) * V + v) * D];
#pragma unroll
        for (int r = 0; r < D; ++r) acc += dphi_vol<D, P, R>(t, i, iq, r) * fc[r];
      }
      for (int lf = 0; lf < NF; ++lf) {
        int ta[D - 1 > 0 ? D - 1 : 1];
        face_axes<D>(lf, ta);
        for (int k = 0; k < QF; ++k) {
          int ik[D - 1 > 0 ? D - 1 : 1];
          int r0 = k;
#pragma unroll
          for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
          acc -= phi_face<D, P, R>(t, i, lf, ta, ik) * s_ff[((el * NF + lf) * QF + k) * V + v];
        }
      }
    }
    const size_t o = (size_t)e0 * V * N + it;
    const double r = fadd ? double(acc) + fadd[o] : double(acc);
    if (fas.rhat) {
      const double tr = fas.rhat[((size_t)e * V + v) * fas.Nf + i];
      fas.fc[o] = tr - r;
      rt[o] = tr;
    } else {
      rt[o] = r;
    }
  }
}

// ---------------------------------------------------------------------------
// Element Jacobian block in phi coordinates (Section 3.3, eq. (jac1)):
//   Dt[(v,i),(w,j)] = sum_q w_q sum_r d_r phi_i phi_j [dF_v/dU_w . c_r]
//                   - sum_faces sum_k w_k |n dsigma| phi_i phi_j dF~_v/dU_w,
// with dF~/dU_own including the ghost chain rule on boundary faces, all flux
// derivatives by forward-mode dual numbers.  FACTOR: form
// Pt = G/dtau - Dt (the PRK block) in LDS, LU-factorise it with partial
// pivoting and write the column-major factors and the row permutation; else
// write Dt row-major.  One block per element.
// ---------------------------------------------------------------------------
template <int D, int P>
constexpr int jac_lds_values() {
  using C = Cfg<D, P>;
  constexpr int ph1 = C::V * C::N + C::NC * D + C::QV * D * C::V * C::V + C::NF * C::QF * C::V * C::V;
  constexpr int ph2 = C::NB * C::NB;
  return (ph1 > ph2 ? ph1 : ph2);
}

template <int D, int P, bool FACTOR, class R, bool CQ = false>
__global__ __launch_bounds__(256) void k_jacobian(const double* __restrict__ ut, const double* __restrict__ xv, int nc,
                                                  const int* __restrict__ nbr, const uint8_t* __restrict__ ncode,
                                                  const double* __restrict__ Gpk, int NT, const double* __restrict__ dtau,
                                                  R* __restrict__ out, int* __restrict__ perm, int* __restrict__ fail,
                                                  int ne, Tab<D, P, R> tab, GasT<R> gas,
                                                  const double* __restrict__ uinf_e) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, NC = C::NC, n = C::NB;
  constexpr int NP = N * N;
  constexpr int ROUNDS = (NP + 255) / 256;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* smem = reinterpret_cast<R*>(smem_raw);
  __shared__ Tab<D, P, R> t;
  __shared__ int s_perm[n];
  __shared__ int s_piv;
  R* s_u = smem;
  R* s_x = s_u + V * N;
  R* s_B = s_x + NC * D;
  R* s_C = s_B + QV * D * V * V;
  R* s_A = smem;  // phase 2 reuses the whole region
  const int tid = threadIdx.x;
  const int e = blockIdx.x;
  if (e >= ne) return;
  copy_tab(t, tab);
  for (int i = tid; i < V * N; i += blockDim.x) s_u[i] = ut[(size_t)e * V * N + i];
  if (!CQ)
    for (int i = tid; i < NC * D; i += blockDim.x) s_x[i] = xv[(size_t)e * NC * D + i];
  __syncthreads();
  for (int q = tid; q < QV; q += blockDim.x) {
    int iq[D];
    R xi[D], wq = R(1);
    int r0 = q;
#pragma unroll
    for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; xi[r] = t.x[iq[r]]; wq *= t.w[iq[r]]; }
    Dual<V, R> U[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R s = R(0);
      for (int k = 0; k < N; ++k) s += s_u[v * N + k] * phi_vol<D, P, R>(t, k, iq);
      U[v] = Dual<V, R>(s);
      U[v].d[v] = R(1);
    }
    R c[D][D], det;
    geom_any<D, CQ>(s_x, xv + (size_t)e * nc * D, xi, c, det);
#pragma unroll
    for (int r = 0; r < D; ++r) {
      Dual<V, R> F[V];
      flux_n<D>(U, c[r], F, gas.g);
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int w = 0; w < V; ++w) s_B[((q * D + r) * V + v) * V + w] = wq * F[v].d[w];
    }
  }
  for (int it = tid; it < NF * QF; it += blockDim.x) {
    const int lf = it / QF, k = it % QF;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1];
    face_axes<D>(lf, ta);
    R xi[D], wk = R(1);
    xi[lf >> 1] = (lf & 1) ? R(1) : R(-1);
    int r0 = k;
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; xi[ta[q]] = t.x[ik[q]]; wk *= t.w[ik[q]]; }
    Dual<V, R> UL[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R s = R(0);
      for (int j = 0; j < N; ++j) s += s_u[v * N + j] * phi_face<D, P, R>(t, j, lf, ta, ik);
      UL[v] = Dual<V, R>(s);
      UL[v].d[v] = R(1);
    }
    R c[D][D], det;
    geom_any<D, CQ>(s_x, xv + (size_t)e * nc * D, xi, c, det);
    R nh[D], a2 = R(0);
    const R sg = (lf & 1) ? R(1) : R(-1);
#pragma unroll
    for (int a = 0; a < D; ++a) { nh[a] = sg * c[lf >> 1][a]; a2 += nh[a] * nh[a]; }
    const R area = dsqrt(a2);
#pragma unroll
    for (int a = 0; a < D; ++a) nh[a] /= area;
    Dual<V, R> F[V];
    const int nb = nbr[(size_t)e * NF + lf];
    if (nb >= 0) {
      const int code = ncode[(size_t)e * NF + lf];
      const int lf2 = code & 7;
      int ta2[D - 1 > 0 ? D - 1 : 1], jk[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf2, ta2);
      nb_face_index<D, Q>(code, ik, jk);
      R UR[V];
      const double* un = ut + (size_t)nb * V * N;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        R s = R(0);
        for (int j = 0; j < N; ++j) s += R(un[v * N + j]) * phi_face<D, P, R>(t, j, lf2, ta2, jk);
        UR[v] = s;
      }
      num_flux<D>(UL, UR, nh, F, gas);
    } else {
      Dual<V, R> UG[V];
      if (nb == NB_WALL) ghost_wall<D>(UL, nh, UG);
      else {
        R Ui[V];
#pragma unroll
        for (int v = 0; v < V; ++v) Ui[v] = uinf_e ? R(uinf_e[(size_t)e * V + v]) : gas.Uinf[v];
        ghost_far<D>(UL, nh, UG, Ui, gas.g);
      }
      num_flux<D>(UL, UG, nh, F, gas);
    }
    const R wa = wk * area;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int w = 0; w < V; ++w) s_C[((lf * QF + k) * V + v) * V + w] = wa * F[v].d[w];
  }
  __syncthreads();
  // contraction over quadrature points, one (i, j) mode pair per thread and round
  R acc[ROUNDS][V * V];
#pragma unroll
  for (int rd = 0; rd < ROUNDS; ++rd) {
#pragma unroll
    for (int x = 0; x < V * V; ++x) acc[rd][x] = R(0);
    const int pr = rd * 256 + tid;
    if (pr < NP) {
      const int i = pr / N, j = pr % N;
      for (int q = 0; q < QV; ++q) {
        int iq[D];
        int r0 = q;
#pragma unroll
        for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
        const R pj = phi_vol<D, P, R>(t, j, iq);
#pragma unroll
        for (int r = 0; r < D; ++r) {
          const R a = dphi_vol<D, P, R>(t, i, iq, r) * pj;
          const R* B = &s_B[(q * D + r) * V * V];
#pragma unroll
          for (int x = 0; x < V * V; ++x) acc[rd][x] += a * B[x];
        }
      }
      for (int lf = 0; lf < NF; ++lf) {
        int ta[D - 1 > 0 ? D - 1 : 1];
        face_axes<D>(lf, ta);
        for (int k = 0; k < QF; ++k) {
          int ik[D - 1 > 0 ? D - 1 : 1];
          int r0 = k;
#pragma unroll
          for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
          const R a = phi_face<D, P, R>(t, i, lf, ta, ik) * phi_face<D, P, R>(t, j, lf, ta, ik);
          const R* Cm = &s_C[(lf * QF + k) * V * V];
#pragma unroll
          for (int x = 0; x < V * V; ++x) acc[rd][x] -= a * Cm[x];
        }
      }
    }
  }
  if constexpr (!FACTOR) {
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int pr = rd * 256 + tid;
      if (pr < NP) {
        const int i = pr / N, j = pr % N;
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int w = 0; w < V; ++w) out[(size_t)e * n * n + (size_t)(v * N + i) * n + w * N + j] = acc[rd][v * V + w];
      }
    }
    return;
  } else {
    __syncthreads();  // every thread is done with s_B / s_C
    const R idt = R(1.0 / dtau[e]);
    const double* G = Gpk + (size_t)e * NT;
#pragma unroll
    for (int rd = 0; rd < ROUNDS; ++rd) {
      const int pr = rd * 256 + tid;
      if (pr < NP) {
        const int i = pr / N, j = pr % N;
        const R gij = R((i >= j) ? G[i * (i + 1) / 2 + j] : G[j * (j + 1) / 2 + i]);
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int w = 0; w < V; ++w)
            s_A[(v * N + i) * n + w * N + j] = ((v == w) ? gij * idt : R(0)) - acc[rd][v * V + w];
      }
    }
    for (int i = tid; i < n; i += blockDim.x) s_perm[i] = i;
    __syncthreads();
    // right-looking LU with partial pivoting
    for (int k = 0; k < n; ++k) {
      if (tid < 64) {
        R best = R(-1);
        int bi = k;
        for (int i = k + tid; i < n; i += 64) {
          R a = dabs(s_A[i * n + k]);
          if (a > best) { best = a; bi = i; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          R ob = __shfl_xor(best, o, 64);
          int oi = __shfl_xor(bi, o, 64);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (tid == 0) {
          s_piv = bi;
          if (!(best > R(0))) atomicOr(fail, 1);
        }
      }
      __syncthreads();
      const int pv = s_piv;
      if (pv != k) {
        for (int j = tid; j < n; j += blockDim.x) {
          R tmp = s_A[k * n + j];
          s_A[k * n + j] = s_A[pv * n + j];
          s_A[pv * n + j] = tmp;
        }
        if (tid == 0) { int tp = s_perm[k]; s_perm[k] = s_perm[pv]; s_perm[pv] = tp; }
      }
      __syncthreads();
      const R ipiv = R(1) / s_A[k * n + k];
      for (int i = k + 1 + tid; i < n; i += blockDim.x) s_A[i * n + k] *= ipiv;
      __syncthreads();
      const int mrem = n - k - 1;
      for (int it = tid; it < mrem * mrem; it += blockDim.x) {
        const int i = k + 1 + it / mrem, j = k + 1 + it % mrem;
        s_A[i * n + j] -= s_A[i * n + k] * s_A[k * n + j];
      }
      __syncthreads();
    }
    for (int it = tid; it < n * n; it += blockDim.x) {
      const int j = it / n, i = it % n;
      out[(size_t)e * n * n + it] = s_A[i * n + j];
    }
    for (int i = tid; i < n; i += blockDim.x) perm[(size_t)e * n + i] = s_perm[i];
  }
}

// Pointwise flux Jacobians of every (element, quadrature point), one thread
// each: volume point q writes Bq[r][v][w] = w_q d(F_v . c_r)/dU_w (r < D),
// face point (lf, k) writes Cf[v][w] = w_k |n dsigma| dF~_v/dU_own_w (with the
// ghost chain rule on boundary faces), all by dual numbers.  Layout per
// element: [QV][D][V][V] then [NF*QF][V][V].  The thread index runs over
// all volume points first, then all face points, so that a wavefront takes
// one of the two paths.
template <int D, int P, class R, bool CQ = false>
__global__ __launch_bounds__(256) void k_jac_points(const double* __restrict__ ut, const double* __restrict__ xv, int nc,
                                                    const int* __restrict__ nbr, const uint8_t* __restrict__ ncode,
                                                    R* __restrict__ BC, int ne, Tab<D, P, R> tab, GasT<R> gas,
                                                    const double* __restrict__ uinf_e) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, NC = C::NC;
  constexpr int NPT = QV + NF * QF;
  constexpr int PER = (QV * D + NF * QF) * V * V;
  __shared__ Tab<D, P, R> t;
  copy_tab(t, tab);
  __syncthreads();
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= ne * NPT) return;
  const int nv = ne * QV;
  const int e = it < nv ? it / QV : (it - nv) / (NF * QF);
  const int pt = it < nv ? it % QV : QV + (it - nv) % (NF * QF);
  const double* ue = ut + (size_t)e * V * N;
  R X[NC * D];
#pragma unroll
  for (int a = 0; a < NC * D; ++a) X[a] = R(xv[(size_t)e * nc * D + a]);  // unused when nc == 27
  R* out = BC + (size_t)e * PER;
  if (pt < QV) {
    const int q = pt;
    int iq[D], r0 = q;
    R xi[D], wq = R(1);
#pragma unroll
    for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; xi[r] = t.x[iq[r]]; wq *= t.w[iq[r]]; }
    Dual<V, R> U[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R sacc = R(0);
      for (int k = 0; k < N; ++k) sacc += R(ue[v * N + k]) * phi_vol<D, P, R>(t, k, iq);
      U[v] = Dual<V, R>(sacc);
      U[v].d[v] = R(1);
    }
    R c[D][D], det;
    geom_any<D, CQ>(X, xv + (size_t)e * nc * D, xi, c, det);
#pragma unroll
    for (int r = 0; r < D; ++r) {
      Dual<V, R> F[V];
      flux_n<D>(U, c[r], F, gas.g);
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int w = 0; w < V; ++w) out[((q * D + r) * V + v) * V + w] = wq * F[v].d[w];
    }
  } else {
    const int fi = pt - QV, lf = fi / QF, k = fi % QF;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
    face_axes<D>(lf, ta);
    R xi[D], wk = R(1);
    xi[lf >> 1] = (lf & 1) ? R(1) : R(-1);
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; xi[ta[q]] = t.x[ik[q]]; wk *= t.w[ik[q]]; }
    Dual<V, R> UL[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R sacc = R(0);
      for (int j = 0; j < N; ++j) sacc += R(ue[v * N + j]) * phi_face<D, P, R>(t, j, lf, ta, ik);
      UL[v] = Dual<V, R>(sacc);
      UL[v].d[v] = R(1);
    }
    R c[D][D], det;
    geom_any<D, CQ>(X, xv + (size_t)e * nc * D, xi, c, det);
    R nh[D], a2 = R(0);
    const R sg = (lf & 1) ? R(1) : R(-1);
#pragma unroll
    for (int a = 0; a < D; ++a) { nh[a] = sg * c[lf >> 1][a]; a2 += nh[a] * nh[a]; }
    const R area = dsqrt(a2);
#pragma unroll
    for (int a = 0; a < D; ++a) nh[a] /= area;
    Dual<V, R> F[V];
    const int nb = nbr[(size_t)e * NF + lf];
    if (nb >= 0) {
      const int code = ncode[(size_t)e * NF + lf];
      const int lf2 = code & 7;
      int ta2[D - 1 > 0 ? D - 1 : 1], jk[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf2, ta2);
      nb_face_index<D, Q>(code, ik, jk);
      R UR[V];
      const double* un = ut + (size_t)nb * V * N;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        R sacc = R(0);
        for (int j = 0; j < N; ++j) sacc += R(un[v * N + j]) * phi_face<D, P, R>(t, j, lf2, ta2, jk);
        UR[v] = sacc;
      }
      num_flux<D>(UL, UR, nh, F, gas);
    } else {
      Dual<V, R> UG[V];
      if (nb == NB_WALL) ghost_wall<D>(UL, nh, UG);
      else {
        R Ui[V];
#pragma unroll
        for (int v = 0; v < V; ++v) Ui[v] = uinf_e ? R(uinf_e[(size_t)e * V + v]) : gas.Uinf[v];
        ghost_far<D>(UL, nh, UG, Ui, gas.g);
      }
      num_flux<D>(UL, UG, nh, F, gas);
    }
    const R wa = wk * area;
    R* o = out + QV * D * V * V + fi * V * V;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int w = 0; w < V; ++w) o[v * V + w] = wa * F[v].d[w];
  }
}

// ---------------------------------------------------------------------------
// Table of phi_j at the volume points ([QV][N]) followed by phi_j at the face
// points ([NF QF][N]) of one order, filled once at set-up with the same
// formulas as the LDS tables of the kernels.  The block assembly reads the
// values every lane of a wavefront shares from it (uniform addresses, which
// the compiler turns into scalar loads that the FMAs take as operands).
// ---------------------------------------------------------------------------
template <int D, int P, class R>
__global__ __launch_bounds__(256) void k_fill_phitab(R* __restrict__ out, Tab<D, P, R> tab) {
  using C = Cfg<D, P>;
  constexpr int N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF;
  __shared__ Tab<D, P, R> t;
  copy_tab(t, tab);
  __syncthreads();
  for (int it = threadIdx.x + blockIdx.x * blockDim.x; it < (QV + NF * QF) * N; it += blockDim.x * gridDim.x) {
    if (it < QV * N) {
      const int q = it / N, j = it % N;
      int iq[D], r0 = q;
#pragma unroll
      for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
      out[it] = phi_vol<D, P, R>(t, j, iq);
    } else {
      const int f = it - QV * N;
      const int lf = f / (QF * N), k = (f / N) % QF, j = f % N;
      int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
      face_axes<D>(lf, ta);
#pragma unroll
      for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
      out[it] = phi_face<D, P, R>(t, j, lf, ta, ik);
    }
  }
}

// ---------------------------------------------------------------------------
// PRK block assembly + LU for blocks of size n = V N <= 64, one wavefront per
// element (four elements per block).  Lane r owns row r = (v, i) of
//   Pt = G/dtau - Dt,  Dt = dRt/dut  (Section 3.3, eq. (jac1), phi coordinates)
// in registers: the quadrature contraction of the pointwise flux Jacobians
// (k_jac_points) accumulates directly into the lane's row, then the LU with
// partial pivoting runs in registers (pivot by one 32-bit wave max-reduction
// of |a| keys, pivot row broadcast with readlane; rows are not moved, the
// pivot order is recorded).  Output as k_jacobian: column-major factors (row
// k of the factor = k-th pivot row) and perm.
// ---------------------------------------------------------------------------

template <int D, int P, class R>
__global__ __launch_bounds__(256, 3) void k_jaclu_wave(const R* __restrict__ BC, const double* __restrict__ Gpk,
                                                    int NT, const double* __restrict__ dtau, R* __restrict__ out,
                                                    int* __restrict__ perm, int* __restrict__ fail, int ne,
                                                    Tab<D, P, R> tab, const R* __restrict__ gph) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, n = C::NB;
  static_assert(n <= 64, "one row per lane");
  constexpr int W = 4;  // elements (wavefronts) per block
  constexpr int PER = (QV * D + NF * QF) * V * V;
  __shared__ Tab<D, P, R> t;
  __shared__ R s_dph[QV * D * N];    // d_r phi_i at volume points
  __shared__ R s_phf[NF * QF * N];   // phi_j at face points
  __shared__ R s_BC[W][PER];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e = blockIdx.x * W + wv;
  const bool live = e < ne;
  copy_tab(t, tab);
  if (live) stage<(PER + 63) / 64>(s_BC[wv], BC + (size_t)e * PER, PER, lane, 64);
  __syncthreads();
  for (int it = threadIdx.x; it < QV * N; it += blockDim.x) {
    const int q = it / N, j = it % N;
    int iq[D], r0 = q;
#pragma unroll
    for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
#pragma unroll
    for (int r = 0; r < D; ++r) s_dph[(q * D + r) * N + j] = dphi_vol<D, P, R>(t, j, iq, r);
  }
  for (int it = threadIdx.x; it < NF * QF * N; it += blockDim.x) {
    const int lf = it / (QF * N), k = (it / N) % QF, j = it % N;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
    face_axes<D>(lf, ta);
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
    s_phf[it] = phi_face<D, P, R>(t, j, lf, ta, ik);
  }
  __syncthreads();
  if (!live) return;  // no block barrier below
  const R* sB = s_BC[wv];
  const R* sC = s_BC[wv] + QV * D * V * V;
  // contraction into the lane's row r = (v, i)
  const int rr = lane < n ? lane : 0;
  const int v = rr / N, i = rr % N;
  R acc[n];
#pragma unroll
  for (int c = 0; c < n; ++c) acc[c] = R(0);
  // volume points: the D directions are summed per point before the
  // product with phi_j, so the row update runs once per point
#pragma unroll 1
  for (int q = 0; q < QV; ++q) {
    R bw[V];
#pragma unroll
    for (int w = 0; w < V; ++w) bw[w] = R(0);
#pragma unroll
    for (int r = 0; r < D; ++r) {
      const R a = s_dph[(q * D + r) * N + i];
      const R* B = &sB[((q * D + r) * V + v) * V];
#pragma unroll
      for (int w = 0; w < V; ++w) bw[w] += a * B[w];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const R ph = gph[q * N + j];  // uniform: a scalar load
#pragma unroll
      for (int w = 0; w < V; ++w) acc[w * N + j] += bw[w] * ph;
    }
  }
#pragma unroll 1
  for (int fk = 0; fk < NF * QF; ++fk) {
    const R a = s_phf[fk * N + i];
    const R* Cm = &sC[(fk * V + v) * V];
    R cw[V];
#pragma unroll
    for (int w = 0; w < V; ++w) cw[w] = a * Cm[w];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const R ph = gph[(QV + fk) * N + j];
#pragma unroll
      for (int w = 0; w < V; ++w) acc[w * N + j] -= cw[w] * ph;
    }
  }
  {
    const R idt = R(1.0 / dtau[e]);
    const double* G = Gpk + (size_t)e * NT;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const R gij = R((i >= j) ? G[i * (i + 1) / 2 + j] : G[j * (j + 1) / 2 + i]);
#pragma unroll
      for (int w = 0; w < V; ++w) acc[w * N + j] = ((w == v) ? gij * idt : R(0)) - acc[w * N + j];
    }
  }
  // LU with partial pivoting, rows in registers.  The pivot row is
  // broadcast from its lane with readlane into scalar registers, which the
  // FMAs take as operands (an LDS broadcast of the row would deliver 1 KB
  // per load to the wavefront and bind the factorisation to the LDS
  // bandwidth).  Lanes already used as pivots get a zero multiplier, so the
  // update below leaves their rows unchanged without a branch.
  int mystep = (lane < n) ? -1 : n;
  int bad = 0;  // failure flags of this element, reported once after the elimination
#pragma unroll
  for (int k = 0; k < n; ++k) {
    // key: |a| as float with its 6 low mantissa bits replaced by 63 - lane
    // (largest |a|, ties to the lowest lane); 0 for lanes already used
    unsigned key = 0u;
    if (mystep < 0) key = (__float_as_uint((float)dabs(acc[k])) & ~63u) | (unsigned)(63 - lane);
    const unsigned kmax = wave_max_u32(key);
    const int pl = __builtin_amdgcn_readfirstlane(63 - (int)(kmax & 63u));
    // the winner must be a row not yet used as a pivot
    if (lane == pl && mystep >= 0) bad |= 4;
    mystep = (lane == pl) ? k : mystep;
    const R piv = readlane_d(acc[k], pl);
    if (!(dabs(piv) > R(0))) bad |= 1;
    const R l = (mystep < 0) ? acc[k] * (R(1) / piv) : R(0);
    if (mystep < 0) acc[k] = l;
    // every sixth entry of the pivot row travels through ds_bpermute (the
    // LDS crossbar) instead of readlane, which moves a share of the
    // broadcast off the vector ALU (measured: 3% faster than readlane only)
#pragma unroll
    for (int j = k + 1; j < n; ++j) {
      const R pj = ((j - k) % 6 == 0) ? bperm_d(acc[j], pl * 4) : readlane_d(acc[j], pl);
      acc[j] = fma(-l, pj, acc[j]);
    }
  }
  if (bad & 4) atomicOr(fail, 4);
  if (lane == 0 && (bad & 1)) atomicOr(fail, 1);
  if (lane < n) {
    R* o = out + (size_t)e * n * n;
#pragma unroll
    for (int j = 0; j < n; ++j) o[(size_t)j * n + mystep] = acc[j];
    perm[(size_t)e * n + mystep] = lane;
  }
}

// Maximum of an unsigned key within each 16-lane row of the wavefront (the
// first four DPP steps of wave_max_u32 leave the row maximum in lane 15 of
// the row), broadcast back to the row with the DPP row broadcast.
__device__ __forceinline__ unsigned row_max_u32(unsigned x) {
  int v = (int)x;
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xE, false));  // row_shr:4
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xC, false));  // row_shr:8
  return (unsigned)__builtin_amdgcn_update_dpp(0, v, 0x150 + 15, 0xF, 0xF, false);                 // row_newbcast:15
}

// The block assembly and LU of k_jaclu_wave for 16 x 16 blocks (2D p = 1),
// four elements per wavefront, one per 16-lane row (k_jaclu_wave would
// leave 48 of 64 lanes idle), sixteen per workgroup.  Same contraction,
// pivot keys (largest |a| as float, ties to the lowest row) and elimination
// arithmetic, so the factors are bitwise those of k_jaclu_wave; the pivot
// row, a different lane in each row, travels through ds_bpermute.  Lanes of
// elements past ne work on element ne - 1 and store nothing, so that every
// row takes part in the row-wide DPP steps.
template <int D, int P, class R>
__global__ __launch_bounds__(256) void k_jaclu_g16(const R* __restrict__ BC, const double* __restrict__ Gpk, int NT,
                                                   const double* __restrict__ dtau, R* __restrict__ out,
                                                   int* __restrict__ perm, int* __restrict__ fail, int ne,
                                                   Tab<D, P, R> tab, const R* __restrict__ gph) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, n = C::NB;
  static_assert(n == 16, "one element per 16-lane row");
  constexpr int W = 16;  // elements per block
  constexpr int PER = (QV * D + NF * QF) * V * V;
  __shared__ Tab<D, P, R> t;
  __shared__ R s_dph[QV * D * N];
  __shared__ R s_phf[NF * QF * N];
  __shared__ R s_BC[W * PER];
  const int lane = threadIdx.x & 63, r = lane & 15;
  const int el = 4 * (threadIdx.x >> 6) + (lane >> 4);
  const int e0 = blockIdx.x * W;
  const int e = e0 + el;
  const bool live = e < ne;
  const int elc = live ? el : ne - 1 - e0;  // an element of this block (e0 < ne)
  const int ec = e0 + elc;
  copy_tab(t, tab);
  {
    const int nel = min(W, ne - e0);
    stage<(W * PER + 255) / 256>(s_BC, BC + (size_t)e0 * PER, nel * PER, threadIdx.x, 256);
  }
  __syncthreads();
  for (int it = threadIdx.x; it < QV * N; it += blockDim.x) {
    const int q = it / N, j = it % N;
    int iq[D], r0 = q;
#pragma unroll
    for (int a = 0; a < D; ++a) { iq[a] = r0 % Q; r0 /= Q; }
#pragma unroll
    for (int a = 0; a < D; ++a) s_dph[(q * D + a) * N + j] = dphi_vol<D, P, R>(t, j, iq, a);
  }
  for (int it = threadIdx.x; it < NF * QF * N; it += blockDim.x) {
    const int lf = it / (QF * N), k = (it / N) % QF, j = it % N;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
    face_axes<D>(lf, ta);
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
    s_phf[it] = phi_face<D, P, R>(t, j, lf, ta, ik);
  }
  __syncthreads();
  const R* sB = s_BC + elc * PER;
  const R* sC = sB + QV * D * V * V;
  const int v = r / N, i = r % N;
  R acc[n];
#pragma unroll
  for (int c = 0; c < n; ++c) acc[c] = R(0);
#pragma unroll 1
  for (int q = 0; q < QV; ++q) {
    R bw[V];
#pragma unroll
    for (int w = 0; w < V; ++w) bw[w] = R(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const R ad = s_dph[(q * D + a) * N + i];
      const R* B = &sB[((q * D + a) * V + v) * V];
#pragma unroll
      for (int w = 0; w < V; ++w) bw[w] += ad * B[w];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const R ph = gph[q * N + j];  // uniform: a scalar load
#pragma unroll
      for (int w = 0; w < V; ++w) acc[w * N + j] += bw[w] * ph;
    }
  }
#pragma unroll 1
  for (int fk = 0; fk < NF * QF; ++fk) {
    const R a = s_phf[fk * N + i];
    const R* Cm = &sC[(fk * V + v) * V];
    R cw[V];
#pragma unroll
    for (int w = 0; w < V; ++w) cw[w] = a * Cm[w];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const R ph = gph[(QV + fk) * N + j];
#pragma unroll
      for (int w = 0; w < V; ++w) acc[w * N + j] -= cw[w] * ph;
    }
  }
  {
    const R idt = R(1.0 / dtau[ec]);
    const double* G = Gpk + (size_t)ec * NT;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const R gij = R((i >= j) ? G[i * (i + 1) / 2 + j] : G[j * (j + 1) / 2 + i]);
#pragma unroll
      for (int w = 0; w < V; ++w) acc[w * N + j] = ((w == v) ? gij * idt : R(0)) - acc[w * N + j];
    }
  }
  const int rowbase = lane & ~15;
  int mystep = -1;
  int bad = 0;  // failure flags of this lane's element, reported after the elimination
#pragma unroll
  for (int k = 0; k < n; ++k) {
    unsigned key = 0u;
    if (mystep < 0) key = (__float_as_uint((float)dabs(acc[k])) & ~63u) | (unsigned)(15 - r);
    const unsigned kmax = row_max_u32(key);
    const int pr = 15 - (int)(kmax & 63u);  // pivot row of this lane's element
    const int pa = (rowbase + pr) * 4;       // its lane, as a ds_bpermute address
    if (r == pr && mystep >= 0) bad |= 4;
    mystep = (r == pr) ? k : mystep;
    const R piv = bperm_d(acc[k], pa);
    if (!(dabs(piv) > R(0))) bad |= 1;
    const R l = (mystep < 0) ? acc[k] * (R(1) / piv) : R(0);
    if (mystep < 0) acc[k] = l;
#pragma unroll
    for (int j = k + 1; j < n; ++j) {
      const R pj = bperm_d(acc[j], pa);
      acc[j] = fma(-l, pj, acc[j]);
    }
  }
  if (live && (bad & 4)) atomicOr(fail, 4);
  if (live && r == 0 && (bad & 1)) atomicOr(fail, 1);
  if (live && mystep >= 0) {  // every row is chosen once: an unused row always has the largest key
    R* o = out + (size_t)e * n * n;
#pragma unroll
    for (int j = 0; j < n; ++j) o[(size_t)j * n + mystep] = acc[j];
    perm[(size_t)e * n + mystep] = r;
  }
}

// ---------------------------------------------------------------------------
// PRK stage (Section 2.3, eq. (prk_scalar)) in phi coordinates:
//   ut = un + beta Pt^{-1} (rt [+ ft]),
// one wavefront per element, lane l owning rows l, l+64, ...; forward and
// back substitution on the column-major LU factors.  First stage: un is null,
// the stage starts from ut itself and stores that state in save (the un of
// the later stages).
// ---------------------------------------------------------------------------
template <int NR, class R>
__global__ __launch_bounds__(256) void k_prk_stage(const R* __restrict__ Fm, const int* __restrict__ perm,
                                                   const double* __restrict__ rt, const double* __restrict__ ft,
                                                   const double* __restrict__ un, double* __restrict__ ut,
                                                   double* __restrict__ save, double beta, int n, int ne) {
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (e >= ne) return;
  const R* F = Fm + (size_t)e * n * n;
  const double* r = rt + (size_t)e * n;
  const double* f = ft ? ft + (size_t)e * n : nullptr;
  const int* pm = perm + (size_t)e * n;
  R b[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = lane + 64 * s;
    b[s] = R(0);
    if (i < n) {
      const int o = pm[i];
      b[s] = R(r[o] + (f ? f[o] : 0.0));
    }
  }
  // L y = b (unit diagonal)
  for (int j = 0; j < n; ++j) {
    const int sj = j >> 6;
    R bj = b[0];
#pragma unroll
    for (int s = 1; s < NR; ++s) if (sj == s) bj = b[s];
    const R xj = __shfl(bj, j & 63, 64);
    const R* col = F + (size_t)j * n;
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const int i = lane + 64 * s;
      if (i > j && i < n) b[s] -= col[i] * xj;
    }
  }
  // U x = y
  for (int j = n - 1; j >= 0; --j) {
    const int sj = j >> 6;
    R bj = b[0];
#pragma unroll
    for (int s = 1; s < NR; ++s) if (sj == s) bj = b[s];
    const R* col = F + (size_t)j * n;
    const R xj = __shfl(bj, j & 63, 64) / col[j];
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const int i = lane + 64 * s;
      if (i == j) b[s] = xj;
      else if (i < j) b[s] -= col[i] * xj;
    }
  }
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int i = lane + 64 * s;
    if (i < n) {
      const size_t o = (size_t)e * n + i;
      const double u0 = un ? un[o] : ut[o];
      if (save) save[o] = u0;
      ut[o] = u0 + beta * double(b[s]);
    }
  }
}

// PRK stage for block sizes NB <= 64: lane i first loads its whole factor
// row (column-major storage, so each column load is coalesced over the lanes
// and all NB loads are independent and in flight together; non-temporal,
// as every factor is read once per stage: 2.5 % faster), then runs the
// forward and back substitution in registers, broadcasting x_j with readlane
// at a constant lane.  Same arithmetic and arguments as k_prk_stage.
template <int NB, class R>
__global__ __launch_bounds__(256) void k_prk_stage_t(const R* __restrict__ Fm, const int* __restrict__ perm,
                                                     const double* __restrict__ rt, const double* __restrict__ un,
                                                     double* __restrict__ ut, double* __restrict__ save, double beta,
                                                     int ne) {
  static_assert(NB <= 64, "one row per lane");
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (e >= ne) return;
  const R* F = Fm + (size_t)e * NB * NB;
  const int i = lane < NB ? lane : NB - 1;
  R row[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) row[j] = __builtin_nontemporal_load(&F[(size_t)j * NB + i]);
  R b = R(rt[(size_t)e * NB + perm[(size_t)e * NB + i]]);
  const size_t o = (size_t)e * NB + i;
  const double u0 = un ? un[o] : ut[o];
  // L y = b (unit diagonal): rows below j subtract L(i, j) y_j
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const R xj = readlane_d(b, j);
    b = fma(-((lane > j) ? row[j] : R(0)), xj, b);
  }
  // U x = y
#pragma unroll
  for (int j = NB - 1; j >= 0; --j) {
    const R xj = readlane_d(b, j) / readlane_d(row[j], j);
    b = (lane == j) ? xj : fma(-((lane < j) ? row[j] : R(0)), xj, b);
  }
  if (lane < NB) {
    if (save) save[o] = u0;
    ut[o] = u0 + beta * double(b);
  }
}

// Broadcast of lane J of every 16-lane row to the whole row (the DPP row
// broadcast, row_newbcast), for the 16 x 16 stage below.
template <int J>
__device__ __forceinline__ double row_bcast(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), 0x150 + J, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), 0x150 + J, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int J>
__device__ __forceinline__ float row_bcast(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x150 + J, 0xF, 0xF, false));
}

template <int J, int NB, class R>
__device__ __forceinline__ void g16_forward(const R (&row)[NB], R& b, int i) {
  if constexpr (J < NB) {
    const R xj = row_bcast<J>(b);
    b = fma(-((i > J) ? row[J] : R(0)), xj, b);
    g16_forward<J + 1, NB, R>(row, b, i);
  }
}
template <int J, int NB, class R>
__device__ __forceinline__ void g16_backward(const R (&row)[NB], R& b, int i) {
  if constexpr (J >= 0) {
    const R xj = row_bcast<J>(b) / row_bcast<J>(row[J]);
    b = (i == J) ? xj : fma(-((i < J) ? row[J] : R(0)), xj, b);
    g16_backward<J - 1, NB, R>(row, b, i);
  }
}

// PRK stage for 16 x 16 blocks (2D p = 1): four elements per wavefront, one
// per 16-lane row, so that every lane holds a factor row (k_prk_stage_t
// would leave 48 of 64 lanes idle); x_j goes to the lanes of its element by
// the DPP row broadcast of lane j.  Lanes of elements past ne work on
// element ne - 1 and store nothing, so that every row of the wavefront takes
// part in the broadcasts.  Same arithmetic and arguments as k_prk_stage_t.
template <class R>
__global__ __launch_bounds__(256) void k_prk_stage_g16(const R* __restrict__ Fm, const int* __restrict__ perm,
                                                       const double* __restrict__ rt, const double* __restrict__ un,
                                                       double* __restrict__ ut, double* __restrict__ save,
                                                       double beta, int ne) {
  constexpr int NB = 16;
  const int lane = threadIdx.x & 63, i = lane & 15;
  const int e = 4 * (blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) + (lane >> 4);
  const bool act = e < ne;
  const int ec = act ? e : ne - 1;
  const R* F = Fm + (size_t)ec * NB * NB;
  R row[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) row[j] = __builtin_nontemporal_load(&F[(size_t)j * NB + i]);
  const size_t o = (size_t)ec * NB + i;
  R b = R(rt[(size_t)ec * NB + perm[o]]);
  const double u0 = un ? un[o] : ut[o];
  g16_forward<0, NB, R>(row, b, i);
  g16_backward<NB - 1, NB, R>(row, b, i);
  if (act) {
    if (save) save[o] = u0;
    ut[o] = u0 + beta * double(b);
  }
}

// PRK stage for block sizes 64 < NB <= 320: one wavefront per element with
// RPL rows per lane (lane, lane + 64, ...); the factor columns stream
// through registers in chunks of eight whose loads are all issued before
// the chunk is used (a loop over single columns would wait for each load in
// turn), x_j broadcast with readlane.  A column j in row slot sl is read
// only in the slots the substitution touches (rows >= 64 sl forward,
// rows < 64 sl + 64 backward).  The chunk loop is not unrolled, which
// keeps few registers live and many wavefronts per SIMD to cover the load
// latency.  Same arithmetic and arguments as k_prk_stage.
template <int NB, class R>
__global__ __launch_bounds__(256) void k_prk_stage_c(const R* __restrict__ Fm, const int* __restrict__ perm,
                                                     const double* __restrict__ rt, const double* __restrict__ un,
                                                     double* __restrict__ ut, double* __restrict__ save, double beta,
                                                     int ne) {
  constexpr int RPL = (NB + 63) / 64, CH = 8;
  static_assert(NB > 64 && NB <= 320, "rows per lane");
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (e >= ne) return;
  const R* F = Fm + (size_t)e * NB * NB;
  int ic[RPL];  // clamped rows: every load in bounds
  R b[RPL];
  double u0[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int i = lane + 64 * s;
    ic[s] = i < NB ? i : NB - 1;
    const size_t o = (size_t)e * NB + ic[s];
    b[s] = (i < NB) ? R(rt[(size_t)e * NB + perm[o]]) : R(0);
    u0[s] = un ? un[o] : ut[o];
  }
  // L y = b (unit diagonal); the columns j of row slot sl (64 sl <= j <
  // 64 sl + 64) take x_j from b[sl], chunks never straddle two slots
#pragma unroll
  for (int sl = 0; sl < RPL; ++sl) {
#pragma unroll 1
    for (int j0 = 64 * sl; j0 < NB && j0 < 64 * sl + 64; j0 += CH) {
      R cf[CH][RPL];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = j0 + c < NB ? j0 + c : NB - 1;
#pragma unroll
        for (int s = sl; s < RPL; ++s) cf[c][s] = F[(size_t)j * NB + ic[s]];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = j0 + c;
        if (j < NB) {
          const R xj = readlane_d(b[sl], j & 63);
#pragma unroll
          for (int s = sl; s < RPL; ++s) b[s] = fma(-((lane + 64 * s > j) ? cf[c][s] : R(0)), xj, b[s]);
        }
      }
    }
  }
  // U x = y
#pragma unroll
  for (int sl = RPL - 1; sl >= 0; --sl) {
    const int jlast = (NB < 64 * sl + 64 ? NB : 64 * sl + 64) - 1;
#pragma unroll 1
    for (int j0 = (jlast / CH) * CH; j0 >= 64 * sl; j0 -= CH) {
      R cf[CH][RPL];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int j = j0 + c < NB ? j0 + c : NB - 1;
#pragma unroll
        for (int s = 0; s <= sl; ++s) cf[c][s] = F[(size_t)j * NB + ic[s]];
      }
#pragma unroll
      for (int c = CH - 1; c >= 0; --c) {
        const int j = j0 + c;
        if (j < NB) {
          const R xj = readlane_d(b[sl], j & 63) / readlane_d(cf[c][sl], j & 63);
#pragma unroll
          for (int s = 0; s <= sl; ++s) {
            const int i = lane + 64 * s;
            b[s] = (i == j) ? xj : fma(-((i < j) ? cf[c][s] : R(0)), xj, b[s]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int i = lane + 64 * s;
    if (i < NB) {
      const size_t o = (size_t)e * NB + i;
      if (save) save[o] = u0[s];
      ut[o] = u0[s] + beta * double(b[s]);
    }
  }
}

// ---------------------------------------------------------------------------
// Basis changes with the packed Cholesky factor L (leading N x N block of the
// p_max factor), one thread per (element, variable):
//   mode 0: ut = L^{-T} u     (psi -> phi coordinates of a state)
//   mode 1: u  = L^T ut       (phi -> psi of a state)
//   mode 2: r  = L^{-1} rt    (phi -> psi of a residual / forcing)
//   mode 3: rt = L r          (psi -> phi of a residual / forcing)
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(256) void k_basis(const double* __restrict__ x, double* __restrict__ y,
                                               const double* __restrict__ Lpk, int NT, int V, int ne, int mode) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * V) return;
  const int e = id / V;
  const double* L = Lpk + (size_t)e * NT;
  const double* a = x + (size_t)id * N;
  double* o = y + (size_t)id * N;
  double r[N];
  if (mode == 0) {
    for (int i = N - 1; i >= 0; --i) {
      double s = a[i];
      for (int j = i + 1; j < N; ++j) s -= L[j * (j + 1) / 2 + i] * r[j];
      r[i] = s / L[i * (i + 1) / 2 + i];
    }
  } else if (mode == 1) {
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int j = i; j < N; ++j) s += L[j * (j + 1) / 2 + i] * a[j];
      r[i] = s;
    }
  } else if (mode == 2) {
    for (int i = 0; i < N; ++i) {
      double s = a[i];
      for (int j = 0; j < i; ++j) s -= L[i * (i + 1) / 2 + j] * r[j];
      r[i] = s / L[i * (i + 1) / 2 + i];
    }
  } else {
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int j = 0; j <= i; ++j) s += L[i * (i + 1) / 2 + j] * a[j];
      r[i] = s;
    }
  }
  for (int i = 0; i < N; ++i) o[i] = r[i];
}

// Lanes per element row of N modes in the lane-group kernels: N rounded up
// to a power of two, so that a group never straddles a wavefront.
template <int N>
constexpr int norm_group() {
  return N <= 1 ? 1 : N <= 4 ? 4 : N <= 8 ? 8 : N <= 16 ? 16 : N <= 32 ? 32 : 64;
}

// Restriction of the solution from order p (N modes) to p-1 (Nc modes): the
// L2 projection, which in psi coordinates is truncation: u = L^T ut, keep
// the leading Nc entries, ut_c = L_c^{-T} u_c.  The composed operator
// R = L_c^{-T} [I 0] L^T of each element is formed at set-up, stored by
// columns ([N][Nc]: the Nc threads of a row read consecutive entries); one
// thread per coarse coefficient applies its row of R.
template <int N, int Nc>
__global__ __launch_bounds__(256) void k_restrict(const double* __restrict__ ut, double* __restrict__ uc,
                                                  double* __restrict__ uc0, const double* __restrict__ Rop, int V,
                                                  int ne) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * V * Nc) return;
  const int k = id % Nc, row = id / Nc, e = row / V;
  const double* a = ut + (size_t)row * N;
  const double* r = Rop + (size_t)e * Nc * N + k;  // R[k][j] at r[j * Nc]
  double s = 0.0;
  // sixteen loads of each operand in flight, then their products in order
  for (int j0 = 0; j0 < N; j0 += 16) {
    double av[16], rv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + u < N ? j0 + u : N - 1;
      av[u] = a[j];
      rv[u] = r[(size_t)j * Nc];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (j0 + u < N) s += rv[u] * av[u];
  }
  uc[id] = s;
  uc0[id] = s;
}

// ---------------------------------------------------------------------------
// Pseudo-time step (Section 4, eq. (x3d)) from the element mean
//   Ubar = u_0 psi_0,  u_0 = (L^T ut)_0,  psi_0 = phi_0 / L_00,
// dtau = cfl h / ((2p+1)(|v| + c)).  mult scales the result (EXP1 uses
// (p_max + 1) dtau).
// ---------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(256) void k_timestep(const double* __restrict__ ut, int N, const double* __restrict__ Lpk,
                                                  int NT, const double* __restrict__ hE, int p, double cfl, double mult,
                                                  double* __restrict__ dtau, int ne, double g,
                                                  const double* __restrict__ cfl_e, int cfl_stride) {
  // G lanes per element: lane t sums the entries t, t + G, ... of the
  // element's [V][N] block (coalesced loads), then the G partial sums of
  // every variable are combined by shuffles within the group
  constexpr int V = D + 2, G = 16;
  const int e = blockIdx.x * (256 / G) + (int)threadIdx.x / G, t = (int)threadIdx.x % G;
  const bool act = e < ne;
  double U[V];
#pragma unroll
  for (int v = 0; v < V; ++v) U[v] = 0.0;
  if (act) {
    const double* L = Lpk + (size_t)e * NT;
    const double* a = ut + (size_t)e * V * N;
    for (int idx = t; idx < V * N; idx += G) {
      const int v = idx / N, j = idx % N;
      const double x = L[j * (j + 1) / 2] * a[idx];
#pragma unroll
      for (int w = 0; w < V; ++w) U[w] += (w == v) ? x : 0.0;
    }
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1)
#pragma unroll
    for (int v = 0; v < V; ++v) U[v] += __shfl_xor(U[v], o, 64);
  if (!act || t != 0) return;
  const double psi0 = (D == 2 ? 0.5 : 0.35355339059327373) / Lpk[(size_t)e * NT];
#pragma unroll
  for (int v = 0; v < V; ++v) U[v] *= psi0;
  double q2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) q2 += (U[1 + a] / U[0]) * (U[1 + a] / U[0]);
  const double c = sqrt(g * pressure<D>(U, g) / U[0]);
  dtau[e] = mult * (cfl_e ? cfl_e[(size_t)cfl_stride * e] : cfl) * hE[e] / ((2.0 * p + 1.0) * (sqrt(q2) + c));
}

// ---------------------------------------------------------------------------
// Density-residual norm (Section 4): sum over elements of |L^{-1} rt_rho|^2,
// block partial sums then one deterministic final sum.
// ---------------------------------------------------------------------------
// G lanes per element (G = N rounded up to a power of two, so a group never
// straddles a wavefront): lane i holds r_i and row i of L and the forward
// substitution runs by columns, x_j broadcast from lane j, which performs
// the same operations per row as a sequential solve.
template <int D, int N>
__global__ __launch_bounds__(256) void k_norm_partial(const double* __restrict__ rt, const double* __restrict__ Lpk,
                                                      int NT, int ne, double* __restrict__ part) {
  constexpr int V = D + 2, G = norm_group<N>(), EPB = 256 / G;
  __shared__ double s_w[4];
  const int e = blockIdx.x * EPB + (int)threadIdx.x / G, i = (int)threadIdx.x % G;
  const int base = (int)(threadIdx.x & 63) - i;  // first lane of the group
  const bool act = e < ne && i < N;
  double r = 0.0, l[N];
#pragma unroll
  for (int j = 0; j < N; ++j) l[j] = 0.0;
  if (act) {
    const double* L = Lpk + (size_t)e * NT + i * (i + 1) / 2;
    r = rt[(size_t)e * V * N + i];
#pragma unroll
    for (int j = 0; j < N; ++j) l[j] = (j <= i) ? L[j] : 0.0;
  }
  double x = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double xj = __shfl(r, base + j, 64) / __shfl(l[j], base + j, 64);
    if (i == j) x = xj;
    else if (i > j) r -= l[j] * xj;
  }
  double acc = act ? x * x : 0.0;
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ part, int nblk, double omega,
                                                    double* __restrict__ out) {
  __shared__ double s_w[4];
  double acc = 0.0;
  // fixed assignment of partials to threads, fixed reduction tree
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += part[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = sqrt(s_w[0] + s_w[1] + s_w[2] + s_w[3]) / omega;
}

// Density-residual norm of every solve of a batch: the squared norm of
// every element (lanes per element as in k_norm_partial), then one block per
// solve sums its element range [seg_e0[s], seg_e0[s + 1]) in a fixed order.
template <int D, int N>
__global__ __launch_bounds__(256) void k_norm_elem(const double* __restrict__ rt, const double* __restrict__ Lpk,
                                                   int NT, int ne, double* __restrict__ enorm) {
  constexpr int V = D + 2, G = norm_group<N>(), EPB = 256 / G;
  const int e = blockIdx.x * EPB + (int)threadIdx.x / G, i = (int)threadIdx.x % G;
  const int base = (int)(threadIdx.x & 63) - i;
  const bool act = e < ne && i < N;
  double r = 0.0, l[N];
#pragma unroll
  for (int j = 0; j < N; ++j) l[j] = 0.0;
  if (act) {
    const double* L = Lpk + (size_t)e * NT + i * (i + 1) / 2;
    r = rt[(size_t)e * V * N + i];
#pragma unroll
    for (int j = 0; j < N; ++j) l[j] = (j <= i) ? L[j] : 0.0;
  }
  double x = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double xj = __shfl(r, base + j, 64) / __shfl(l[j], base + j, 64);
    if (i == j) x = xj;
    else if (i > j) r -= l[j] * xj;
  }
  double acc = act ? x * x : 0.0;
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (e < ne && i == 0) enorm[e] = acc;
}

__global__ __launch_bounds__(256) void k_norm_segsum(const double* __restrict__ enorm, const int* __restrict__ seg_e0,
                                                     const double* __restrict__ seg_omega, double* __restrict__ out) {
  __shared__ double s_w[4];
  const int sg = blockIdx.x;
  const int e0 = seg_e0[sg], e1 = seg_e0[sg + 1];
  double acc = 0.0;
  for (int e = e0 + threadIdx.x; e < e1; e += blockDim.x) acc += enorm[e];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[sg] = sqrt(s_w[0] + s_w[1] + s_w[2] + s_w[3]) / seg_omega[sg];
}

// ---------------------------------------------------------------------------
// p = 0 level set-up for EXP1 (Sections 2.1 and 3.3 at p = 0), psi
// coordinates, one thread per element:
//   u0 = L_00 ut0,  R0 = -sum_faces sum_k w |n dsigma| psi_0 F~,
//   J0 diagonal / neighbour blocks from dual-number flux derivatives,
//   dt = (p_max+1) dtau(p_max),  b = dt (R0 + f0),  A = dt J0 (row scaling).
// scale = false: dt = 1 (plain J0 and R0 + f0).
// ---------------------------------------------------------------------------
template <int D, bool CQ = false>
__global__ __launch_bounds__(256) void k_p0_setup(const double* __restrict__ ut0, const double* __restrict__ ft0,
                                                  const double* __restrict__ xv, int nc, const int* __restrict__ nbr,
                                                  const double* __restrict__ Lpk, int NT, const double* __restrict__ hE,
                                                  int pmax, double cfl, int scale, double* __restrict__ u0,
                                                  double* __restrict__ bvec, double* __restrict__ Ad,
                                                  double* __restrict__ Ao, double* __restrict__ dtout, int ne, Gas gas,
                                                  const double* __restrict__ gx, const double* __restrict__ gw,
                                                  const double* __restrict__ uinf_e, const double* __restrict__ cfl_e,
                                                  int cfl_stride) {
  // one lane per (face, face point) of an element, G lanes per element
  // (padded to a power of two); the contributions are summed over the points
  // of a face (neighbour block) and over all faces (R0, diagonal block) by
  // butterfly shuffles, a fixed order
  constexpr int V = D + 2, NF = 2 * D, NC = geo_nodes(D), QF = 1 << (D - 1);
  constexpr int G = (D == 2) ? 8 : 32, EPB = 256 / G;
  const int e = blockIdx.x * EPB + (int)threadIdx.x / G, t = (int)threadIdx.x % G;
  const int lf = t / QF, k = t % QF;
  const bool act = e < ne && lf < NF;
  const double phi0 = (D == 2 ? 0.5 : 0.35355339059327373);
  const int ec = e < ne ? e : ne - 1;  // clamped element: every lane loads in bounds
  const double L00 = Lpk[(size_t)ec * NT];
  double U[V];
#pragma unroll
  for (int v = 0; v < V; ++v) U[v] = ut0[(size_t)ec * V + v] * phi0;
  double dt = 1.0;
  if (scale) {
    double q2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) q2 += (U[1 + a] / U[0]) * (U[1 + a] / U[0]);
    const double c = sqrt(gas.g * pressure<D>(U, gas.g) / U[0]);
    const double ce = cfl_e ? cfl_e[(size_t)cfl_stride * ec] : cfl;
    dt = (pmax + 1.0) * ce * hE[ec] / ((2.0 * pmax + 1.0) * (sqrt(q2) + c));
  }
  double R[V], Jd[V * V], Jo[V * V];
#pragma unroll
  for (int v = 0; v < V; ++v) R[v] = 0.0;
#pragma unroll
  for (int x = 0; x < V * V; ++x) { Jd[x] = 0.0; Jo[x] = 0.0; }
  int nb = -1;
  double L00n = 1.0;
  if (act) {
    double X[NC * D];
#pragma unroll
    for (int i = 0; i < NC * D; ++i) X[i] = xv[(size_t)e * nc * D + i];  // unused when nc == 27
    nb = nbr[(size_t)e * NF + lf];
    double UN[V];
    if (nb >= 0) {
      L00n = Lpk[(size_t)nb * NT];
#pragma unroll
      for (int v = 0; v < V; ++v) UN[v] = ut0[(size_t)nb * V + v] * phi0;
    }
    int ta[D - 1];
    face_axes<D>(lf, ta);
    double xi[D], wk = 1.0;
    xi[lf >> 1] = (lf & 1) ? 1.0 : -1.0;
    int r0 = k;
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { xi[ta[q]] = gx[r0 & 1]; wk *= gw[r0 & 1]; r0 >>= 1; }
    double c[D][D], det;
    geom_any<D, CQ>(X, xv + (size_t)e * nc * D, xi, c, det);
    double nh[D], a2 = 0.0;
    const double sg = (lf & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) { nh[a] = sg * c[lf >> 1][a]; a2 += nh[a] * nh[a]; }
    const double area = sqrt(a2);
#pragma unroll
    for (int a = 0; a < D; ++a) nh[a] /= area;
    const double wa = wk * area * phi0;
    Dual<V> UL[V], F[V];
#pragma unroll
    for (int v = 0; v < V; ++v) { UL[v] = Dual<V>(U[v]); UL[v].d[v] = 1.0; }
    if (nb >= 0) {
      num_flux<D>(UL, UN, nh, F, gas);
      Dual<V> UR[V], F2[V];
#pragma unroll
      for (int v = 0; v < V; ++v) { UR[v] = Dual<V>(UN[v]); UR[v].d[v] = 1.0; }
      num_flux<D>(U, UR, nh, F2, gas);
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int w = 0; w < V; ++w) Jo[v * V + w] = -(wa * phi0 * F2[v].d[w]);
    } else {
      Dual<V> UG[V];
      if (nb == NB_WALL) ghost_wall<D>(UL, nh, UG);
      else {
        double Ui[V];
#pragma unroll
        for (int v = 0; v < V; ++v) Ui[v] = uinf_e ? uinf_e[(size_t)e * V + v] : gas.Uinf[v];
        ghost_far<D>(UL, nh, UG, Ui, gas.g);
      }
      num_flux<D>(UL, UG, nh, F, gas);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R[v] = -(wa * F[v].v);
#pragma unroll
      for (int w = 0; w < V; ++w) Jd[v * V + w] = -(wa * phi0 * F[v].d[w]);
    }
  }
#pragma unroll
  for (int o = 1; o < QF; o <<= 1)
#pragma unroll
    for (int x = 0; x < V * V; ++x) Jo[x] += __shfl_xor(Jo[x], o, 64);
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
#pragma unroll
    for (int v = 0; v < V; ++v) R[v] += __shfl_xor(R[v], o, 64);
#pragma unroll
    for (int x = 0; x < V * V; ++x) Jd[x] += __shfl_xor(Jd[x], o, 64);
  }
  if (!act) return;
  if (k == 0) {
    // psi coordinates: dR0_E/du0_F = Jt / (L00_E L00_F)
    const double so = dt / (L00 * L00n);
#pragma unroll
    for (int x = 0; x < V * V; ++x) Ao[((size_t)e * NF + lf) * V * V + x] = (nb >= 0) ? so * Jo[x] : 0.0;
  }
  if (t != 0) return;
  const double sd = dt / (L00 * L00);
#pragma unroll
  for (int x = 0; x < V * V; ++x) Ad[(size_t)e * V * V + x] = sd * Jd[x];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const double f = ft0 ? ft0[(size_t)e * V + v] / L00 : 0.0;
    bvec[(size_t)e * V + v] = dt * (R[v] / L00 + f);
    u0[(size_t)e * V + v] = L00 * ut0[(size_t)e * V + v];
  }
  dtout[e] = dt;
}

// ---------------------------------------------------------------------------
// Arnoldi process of EXP1 (Section 2.2, eqs. (vm)-(vm2)): classical
// Gram-Schmidt with one re-orthogonalisation (CGS2), the block sparse
// product y = A x with A = T J0, and deterministic reductions (every block
// sums the per-block partials in the same order, so all blocks take
// identical decisions).  Output: basis Vb[j][K], Hessenberg H[(m+1) x m]
// row-major, info[0] = Krylov dimension used, info[1] = beta = ||b||.
// Helpers first: one row of the block-sparse product, block partial dots.
// ---------------------------------------------------------------------------
template <int V, int NF>
__device__ __forceinline__ double spmv_row(int row, const int* __restrict__ nbr, const double* __restrict__ Ad,
                                           const double* __restrict__ Ao, const double* __restrict__ x) {
  const int e = row / V, v = row % V;
  int nb[NF];
#pragma unroll
  for (int lf = 0; lf < NF; ++lf) nb[lf] = nbr[(size_t)e * NF + lf];
  double s = 0.0;
  const double* a = Ad + (size_t)e * V * V + v * V;
#pragma unroll
  for (int w = 0; w < V; ++w) s += a[w] * x[(size_t)e * V + w];
  // boundary faces (nb < 0) read the element's own row and drop the term, so
  // that every load is issued without a branch
#pragma unroll
  for (int lf = 0; lf < NF; ++lf) {
    const int src = nb[lf] >= 0 ? nb[lf] : e;
    const double* o = Ao + ((size_t)e * NF + lf) * V * V + v * V;
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < V; ++w) t += o[w] * x[(size_t)src * V + w];
    s += nb[lf] >= 0 ? t : 0.0;
  }
  return s;
}

// Sum over the 64 lanes of a wavefront with DPP moves of the two 32-bit
// halves (the pattern of wave_max_u32: quad permutations, row shifts by 4
// and 8, row broadcasts of lanes 15 and 31); lanes whose DPP source is
// disabled contribute zero.  Lane 63 holds the total, returned uniformly.
template <int CTRL, int RM, int BM>
__device__ __forceinline__ double dpp_move_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, RM, BM, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, RM, BM, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum_d(double x) {
  x += dpp_move_d<0xB1, 0xF, 0xF>(x);
  x += dpp_move_d<0x4E, 0xF, 0xF>(x);
  x += dpp_move_d<0x114, 0xF, 0xE>(x);
  x += dpp_move_d<0x118, 0xF, 0xC>(x);
  x += dpp_move_d<0x142, 0xA, 0xF>(x);
  x += dpp_move_d<0x143, 0xC, 0xF>(x);
  return readlane_d(x, 63);
}

// Block sums s_out[i] = sum over the block's threads of f(i), i < cnt <= NV
// (cnt uniform): wave sums by DPP, then the four waves in a fixed order.
// Every thread of the block must call it (DPP needs the full wavefront).
template <int NV, class F>
__device__ __forceinline__ void block_sums(int cnt, F f, double* s_wave /*[4][64]*/, double* s_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i)
    if (i < cnt) {
      const double t = wave_sum_d(f(i));
      if (lane == 0) s_wave[wv * 64 + i] = t;
    }
  __syncthreads();
  if (threadIdx.x < cnt) {
    const int i = threadIdx.x;
    s_out[i] = (s_wave[i] + s_wave[64 + i]) + (s_wave[128 + i] + s_wave[192 + i]);
  }
  __syncthreads();
}

// Wave reduce-scatter of NV (a power of two, <= 64) values per lane: at each
// halving step a lane keeps one half of its values and adds the partner's
// copy of that half (lane ^ o); after log2(NV) steps a lane holds one value,
// and the remaining xor steps complete the 64-lane sum.  Lane l ends with the
// total of value index l >> (6 - log2 NV); p is overwritten.
template <int H, int NV>
__device__ __forceinline__ void rs_level(double (&p)[NV], int lane) {
  if constexpr (H >= 1) {
    constexpr int O = 64 * H / NV;  // partner offset of this halving step
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double send = up ? p[i] : p[i + H];
      const double keep = up ? p[i + H] : p[i];
      p[i] = keep + __shfl_xor(send, O, 64);
    }
    rs_level<H / 2, NV>(p, lane);
  }
}

template <int NV>
__device__ __forceinline__ double wave_reduce_scatter(double (&p)[NV]) {
  static_assert(NV >= 1 && NV <= 64 && (NV & (NV - 1)) == 0, "NV must be a power of two <= 64");
  const int lane = threadIdx.x & 63;
  rs_level<NV / 2, NV>(p, lane);
  double r = p[0];
#pragma unroll
  for (int o = 32 / NV; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
  return r;
}

// Block sums of NV per-thread values p[i] (i < cnt <= NV) plus one more
// value x, written to s_out[0..cnt) and s_out[cnt]: wave reduce-scatter,
// then the four waves in a fixed order.  Every thread must call it.
template <int NV>
__device__ __forceinline__ void block_sums_rs(double (&p)[NV], double x, int cnt, double* s_wave /*[4][64]*/,
                                              double* s_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int SH = (NV == 64) ? 0 : (NV == 32) ? 1 : (NV == 16) ? 2 : (NV == 8) ? 3 : (NV == 4) ? 4 : (NV == 2) ? 5 : 6;
  const double r = wave_reduce_scatter<NV>(p);
  const double xs = wave_sum_d(x);
  const int idx = lane >> SH;
  if ((lane & ((1 << SH) - 1)) == 0 && idx < cnt) s_wave[wv * 64 + idx] = r;
  if (lane == 0) s_wave[wv * 64 + cnt] = xs;
  __syncthreads();
  if (threadIdx.x <= cnt) {
    const int i = threadIdx.x;
    s_out[i] = (s_wave[i] + s_wave[64 + i]) + (s_wave[128 + i] + s_wave[192 + i]);
  }
  __syncthreads();
}

// Deterministic sum over the blocks [b0, b1) of cnt per-block partials
// (part[q * P + i]) into s_out[i]: group g of threads sums q = b0 + g,
// b0 + g + G, ... with its loads issued sixteen at a time, then the G group
// sums are added in order.  Every block of the range computes bitwise the
// same totals.
__device__ __forceinline__ void grid_partials_sum(const double* __restrict__ part, int b0, int b1, int P, int cnt,
                                                  double* s_tmp /*[256]*/, double* s_out) {
  const int G = blockDim.x / cnt;
  const int t = threadIdx.x;
  if (t < G * cnt) {
    const int g = t / cnt, i = t % cnt;
    double s = 0.0;
    for (int q0 = b0 + g; q0 < b1; q0 += 16 * G) {
      double a[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int q = q0 + u * G;
        a[u] = q < b1 ? part[(size_t)q * P + i] : 0.0;
      }
#pragma unroll
      for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
        for (int u = 0; u < w; ++u) a[u] += a[u + w];
      s += a[0];
    }
    s_tmp[g * cnt + i] = s;
  }
  __syncthreads();
  if (t < cnt) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += s_tmp[g * cnt + t];
    s_out[t] = s;
  }
  __syncthreads();
}

// Solve segments of a batched Arnoldi (all null for a single solve): block b
// covers rows [brow0[b], brow1[b]) of solve bseg[b]; solve s owns blocks
// [sblk0[s], sblk0[s + 1]).  Each solve has its own Hessenberg matrix, beta,
// Krylov dimension and breakdown flag, so batched solves stay independent.
struct ArnSeg {
  const int* brow0;
  const int* brow1;
  const int* bseg;
  const int* sblk0;
};

struct SegPos {
  int sg, b0, b1, k, kend;
};

__device__ __forceinline__ SegPos seg_pos(const ArnSeg& S, int K) {
  SegPos r;
  r.sg = S.bseg ? S.bseg[blockIdx.x] : 0;
  r.b0 = S.sblk0 ? S.sblk0[r.sg] : 0;
  r.b1 = S.sblk0 ? S.sblk0[r.sg + 1] : (int)gridDim.x;
  r.k = (S.brow0 ? S.brow0[blockIdx.x] : (int)(blockIdx.x * blockDim.x)) + (int)threadIdx.x;
  r.kend = S.brow1 ? S.brow1[blockIdx.x] : K;
  return r;
}

// Arnoldi process of EXP1 as a sequence of full-grid kernels (a kernel
// boundary is the global barrier; on this GPU it is several times cheaper
// than a cooperative grid barrier).  One thread per row of the K-vectors
// (the grid is ceil(K / 256) blocks of 256), which keeps its row of the
// basis V_j in registers (NVM >= the number of basis vectors the kernel
// touches), so every global load of a kernel is issued before the first
// wait.  The product w = A v_j lives in scratch vector W[j % 2]; v_{j+1}
// goes to Vb[j + 1].  Kernels:
//   a  (j = 0 only): W0 = A v_0, partials of <W0, v_0>, ||W0||^2, ||v_0||^2
//   b  (step j): h1 = sum of partials, W -= V_j h1 (first Gram-Schmidt
//      pass), partials of the second pass; first it normalises v_j by the
//      norm the previous kernel measured (below)
//   ca (step j, then j + 1): h2 and hn = sqrt(||W||^2 - ||h2||^2) finish
//      column j of H; v_{j+1} = (W - V_j h2)/hn; and, fused, the next
//      product A v_{j+1} = (A W - V_{j+1} (H~_j h2)) / hn (Arnoldi relation
//      A V_j = V_{j+1} H~_j), which needs W only at neighbour rows, all final
//      since the previous kernel; partials of the next first pass and of
//      ||v_{j+1}||^2.  On the last step only v_{j+1} is formed.
// hn from Pythagoras resolves the true norm only down to ~1e-8 ||W||, so
// the next b kernel measures s = ||v_{j+1}|| of the vector actually formed
// and rescales: v_{j+1} /= s, A v_{j+1} /= s, h_{j+2,j+1} = s hn (exact:
// the Arnoldi relation holds for any scaling of v_{j+1}), and the breakdown
// test is repeated on s hn.  Happy breakdown (h <= 1e-12 ||A v_j||) sets
// st[0], so every later kernel returns; info[0] = Krylov dimension used,
// info[1] = beta.  ||A v_j|| is kept in two slots per solve (step j writes
// slot j % 2), so no kernel reads a slot one of its own blocks writes.
__global__ __launch_bounds__(256) void k_arn_beta(int K, const double* __restrict__ b, double* __restrict__ part,
                                                  int P, int* __restrict__ st, ArnSeg S) {
  __shared__ double s_wave[4 * 64];
  __shared__ double s_h[64];
  const SegPos sp = seg_pos(S, K);
  const double x = sp.k < sp.kend ? b[sp.k] : 0.0;
  block_sums<1>(1, [&](int) { return x * x; }, s_wave, s_h);
  if (threadIdx.x == 0) part[blockIdx.x * P] = s_h[0];
  if (blockIdx.x == sp.b0 && threadIdx.x == 0) { st[2 * sp.sg] = 0; st[2 * sp.sg + 1] = 0; }
}

__global__ __launch_bounds__(256) void k_arn_start(int K, int m, const double* __restrict__ b,
                                                   const double* __restrict__ part, int P, double* __restrict__ Vb,
                                                   double* __restrict__ info, int* __restrict__ st, ArnSeg S) {
  __shared__ double s_tmp[256];
  __shared__ double s_g[64];
  const SegPos sp = seg_pos(S, K);
  grid_partials_sum(part, sp.b0, sp.b1, P, 1, s_tmp, s_g);
  const double beta = sqrt(s_g[0]);
  if (blockIdx.x == sp.b0 && threadIdx.x == 0) {
    info[2 * sp.sg + 1] = beta;
    info[2 * sp.sg] = (beta == 0.0) ? 0.0 : (double)m;
    if (beta == 0.0) st[2 * sp.sg] = 1;
  }
  if (beta == 0.0) return;
  if (sp.k < sp.kend) Vb[sp.k] = b[sp.k] / beta;
}

template <int V, int NF>
__global__ __launch_bounds__(256) void k_arn_a(int K, const int* __restrict__ nbr, const double* __restrict__ Ad,
                                               const double* __restrict__ Ao, const double* __restrict__ Vb,
                                               double* __restrict__ W, double* __restrict__ part, int P,
                                               const int* __restrict__ st, ArnSeg S) {
  const SegPos sp = seg_pos(S, K);
  if (st[2 * sp.sg]) return;
  __shared__ double s_wave[4 * 64];
  __shared__ double s_h[64];
  const int k = sp.k;
  const bool act = k < sp.kend;
  const double v0 = act ? Vb[k] : 0.0;
  const double w = act ? spmv_row<V, NF>(k, nbr, Ad, Ao, Vb) : 0.0;
  if (act) W[k] = w;
  block_sums<3>(3, [&](int i) { return i == 0 ? w * v0 : i == 1 ? w * w : v0 * v0; }, s_wave, s_h);
  if (threadIdx.x < 3) part[blockIdx.x * P + threadIdx.x] = s_h[threadIdx.x];
}

template <int NVM>
__global__ __launch_bounds__(256) void k_arn_b(int K, int m, int j, double* __restrict__ Vb,
                                               double* __restrict__ W, const double* __restrict__ part1,
                                               double* __restrict__ part2, int P, double* __restrict__ H,
                                               double* __restrict__ H2, double* __restrict__ wn0,
                                               double* __restrict__ info, int* __restrict__ st, ArnSeg S) {
  const SegPos sp = seg_pos(S, K);
  if (st[2 * sp.sg]) return;
  __shared__ double s_wave[4 * 64];
  __shared__ double s_h[64];
  __shared__ double s_g[64];
  __shared__ double s_tmp[256];
  H += (size_t)sp.sg * (m + 1) * m;
  H2 += (size_t)sp.sg * (m + 1) * m;
  wn0 += 2 * sp.sg;
  const int k = sp.k;
  const bool act = k < sp.kend;
  const int kc = act ? k : sp.kend - 1;  // clamped row: loads need no divergent branch
  double vr[NVM];
#pragma unroll
  for (int i = 0; i < NVM; ++i) vr[i] = (i <= j) ? Vb[(size_t)i * K + kc] : 0.0;
  double w = act ? W[kc] : 0.0;
#pragma unroll
  for (int i = 0; i < NVM; ++i) vr[i] = act ? vr[i] : 0.0;
  // h_{j,j-1} from the previous step (H is not written by this kernel, so
  // every block reads the same value)
  const double hprev = j > 0 ? H[j * m + j - 1] : 0.0;
  const double wprev = wn0[(j + 1) & 1];  // ||A v_{j-1}||, written by the previous step
  grid_partials_sum(part1, sp.b0, sp.b1, P, j + 3, s_tmp, s_g);
  // normalise v_j by its measured norm s (every block computes the same s);
  // the subdiagonal's correction s hn - hn goes to H2 (the Hessenberg
  // matrix is H + H2)
  const double sn = sqrt(s_g[j + 2]);
  if (j > 0 && blockIdx.x == sp.b0 && threadIdx.x == 0) H2[j * m + j - 1] = hprev * sn - hprev;
  if (j > 0 && !(hprev * sn > 1e-12 * wprev)) {
    // the true subdiagonal is at the breakdown level: dimension j
    if (blockIdx.x == sp.b0 && threadIdx.x == 0) {
      st[2 * sp.sg] = 1;
      info[2 * sp.sg] = (double)j;
    }
    return;
  }
  const double isc = 1.0 / sn;
  __syncthreads();  // every thread has read s_g[j + 2] before it is rescaled
  if (threadIdx.x <= j + 1) s_g[threadIdx.x] *= (threadIdx.x < j) ? isc : isc * isc;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NVM; ++i)
    if (i == j) {
      vr[i] *= isc;
      if (act) Vb[(size_t)i * K + k] = vr[i];
    }
  w *= isc;
  double a0 = 0.0, a1 = 0.0;
#pragma unroll
  for (int i = 0; i < NVM; i += 2) {
    if (i <= j) a0 += s_g[i] * vr[i];
    if (i + 1 <= j) a1 += s_g[i + 1] * vr[i + 1];
  }
  const double w1 = w - (a0 + a1);
  if (act) W[k] = w1;
  if (blockIdx.x == sp.b0 && threadIdx.x <= j) H[threadIdx.x * m + j] = s_g[threadIdx.x];
  if (blockIdx.x == sp.b0 && threadIdx.x == 0) wn0[j & 1] = sqrt(s_g[j + 1]);
  constexpr int NP = NVM > 32 ? 64 : NVM > 16 ? 32 : NVM;  // a power of two
  double pp[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) pp[i] = (i < NVM) ? w1 * vr[i < NVM ? i : 0] : 0.0;
  block_sums_rs<NP>(pp, w1 * w1, j + 1, s_wave, s_h);
  if (threadIdx.x < j + 2) part2[blockIdx.x * P + threadIdx.x] = s_h[threadIdx.x];
}

// Finishes step j (and, when NEXT, starts step j + 1 with the fused product).
// H holds the first-pass coefficients h1 and the subdiagonal hn; the second
// pass coefficients h2 go to H2 (the Hessenberg matrix is H + H2), so no
// kernel reads an entry another block of the same kernel writes.
template <int V, int NF, bool NEXT, int NVM>
__global__ __launch_bounds__(256) void k_arn_ca(int K, int m, int j, const int* __restrict__ nbr,
                                                const double* __restrict__ Ad, const double* __restrict__ Ao,
                                                double* __restrict__ Vb, const double* __restrict__ W,
                                                double* __restrict__ Wn, const double* __restrict__ part2,
                                                double* __restrict__ part1, int P, double* __restrict__ H,
                                                double* __restrict__ H2, const double* __restrict__ wn0,
                                                double* __restrict__ info, int* __restrict__ st, ArnSeg S) {
  const SegPos sp = seg_pos(S, K);
  if (st[2 * sp.sg]) return;
  H += (size_t)sp.sg * (m + 1) * m;
  H2 += (size_t)sp.sg * (m + 1) * m;
  wn0 += 2 * sp.sg;
  info += 2 * sp.sg;
  st += 2 * sp.sg;
  __shared__ double s_wave[4 * 64];
  __shared__ double s_h[64];
  __shared__ double s_c[64];
  __shared__ double s_p[64];
  __shared__ double s_tmp[256];
  __shared__ double s_Hf[NEXT ? NVM * NVM : 1];
  const int k = sp.k;
  const bool act = k < sp.kend;
  const int kc = act ? k : sp.kend - 1;  // clamped row: loads need no divergent branch
  // every global load first: the basis row, w, the product A w and the
  // finished columns of the Hessenberg matrix
  double vr[NVM];
#pragma unroll
  for (int i = 0; i < NVM; ++i) vr[i] = (i <= j) ? Vb[(size_t)i * K + kc] : 0.0;
  const double w1 = act ? W[kc] : 0.0;
  double aw = 0.0;
  if (NEXT) aw = act ? spmv_row<V, NF>(kc, nbr, Ad, Ao, W) : 0.0;
#pragma unroll
  for (int i = 0; i < NVM; ++i) vr[i] = act ? vr[i] : 0.0;
  if (NEXT) {
    // all loads of the staging issued together: (j + 2)(j + 1) <= NVM^2
    constexpr int IT = (NVM * NVM + 255) / 256;
    const int nH = (j + 2) * (j + 1);
    double h1v[IT], h2v[IT];
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int t = threadIdx.x + u * 256;
      const int kk = t / (j + 1), i = t % (j + 1);
      const bool in = t < nH && kk <= i + 1;
      h1v[u] = in ? H[kk * m + i] : 0.0;
      h2v[u] = (in && i < j && kk <= i + 1) ? H2[kk * m + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < IT; ++u) {
      const int t = threadIdx.x + u * 256;
      const int kk = t / (j + 1), i = t % (j + 1);
      // columns < j: final values; column j: h1 only (h2 added below)
      if (t < nH) s_Hf[kk * NVM + i] = h1v[u] + h2v[u];
    }
  }
  grid_partials_sum(part2, sp.b0, sp.b1, P, j + 2, s_tmp, s_h);
  double h2sq = 0.0;
  for (int i = 0; i <= j; ++i) h2sq += s_h[i] * s_h[i];
  const double hn = sqrt(fmax(s_h[j + 1] - h2sq, 0.0));
  const bool brk = !(hn > 1e-12 * wn0[j & 1]);
  if (NEXT && !brk) {
    // c = H~_j h2: columns < j split over the four waves (s_tmp is free
    // again), column j from this kernel's own values
    const int kk = threadIdx.x & 63, q = threadIdx.x >> 6;
    double sacc = 0.0;
    if (kk <= j + 1)
      for (int i = (kk > 0 ? kk - 1 : 0) + q; i < j; i += 4) sacc += s_Hf[kk * NVM + i] * s_h[i];
    s_tmp[q * 64 + kk] = sacc;
    __syncthreads();
    if (threadIdx.x <= j + 1) {
      const double hkj = (kk <= j) ? s_Hf[kk * NVM + j] + s_h[kk] : hn;
      s_c[kk] = ((s_tmp[kk] + s_tmp[64 + kk]) + (s_tmp[128 + kk] + s_tmp[192 + kk])) + hkj * s_h[j];
    }
  }
  __syncthreads();
  if (blockIdx.x == sp.b0 && threadIdx.x <= j) H2[threadIdx.x * m + j] = s_h[threadIdx.x];
  if (blockIdx.x == sp.b0 && threadIdx.x == 0) {
    H[(j + 1) * m + j] = hn;
    if (brk) { st[0] = 1; info[0] = (double)(j + 1); }
  }
  if (brk) return;  // uniform: every block computed the same hn
  const double ihn = 1.0 / hn;
  double a0 = 0.0, a1 = 0.0, c0 = 0.0, c1 = 0.0;
#pragma unroll
  for (int i = 0; i < NVM; i += 2) {
    if (i <= j) { a0 += s_h[i] * vr[i]; c0 += s_c[i] * vr[i]; }
    if (i + 1 <= j) { a1 += s_h[i + 1] * vr[i + 1]; c1 += s_c[i + 1] * vr[i + 1]; }
  }
  const double v = (w1 - (a0 + a1)) * ihn;
  if (act) Vb[(size_t)(j + 1) * K + k] = v;
  if constexpr (NEXT) {
    const double wn = (aw - ((c0 + c1) + s_c[j + 1] * v)) * ihn;
    if (act) Wn[k] = wn;
    constexpr int NP = NVM > 32 ? 64 : NVM > 16 ? 32 : NVM;  // a power of two
    double pp[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) pp[i] = (i <= j) ? wn * vr[i < NVM ? i : 0] : (i == j + 1 ? wn * v : 0.0);
    block_sums_rs<NP>(pp, wn * wn, j + 2, s_wave, s_p);
    block_sums<1>(1, [&](int) { return v * v; }, s_wave, s_p + j + 3);
    if (threadIdx.x < j + 4) part1[blockIdx.x * P + threadIdx.x] = s_p[threadIdx.x];
  }
}

// ---------------------------------------------------------------------------
// phi_1(H_m) e_1 on one block: exponential of the augmented matrix
// [[H, e_1], [0, 0]] by the degree-13 diagonal Pade approximant with scaling
// and squaring (Higham 2005); stands in for the paper's rational
// approximation of exp(dt H_m) (end of Section 2.2).  y[i] = E[i][m].
// ---------------------------------------------------------------------------
// Cm = A B for n x n row-major matrices in LDS, by a block of 256 threads.
// For n <= 32 on the FP64 matrix cores: the product is padded to 32 x 32
// and wavefront w computes the 16 x 16 output tile (w / 2, w % 2) with eight
// 16 x 16 x 4 steps (lane l holds A[i][k] and B[k][j] for i, j = l % 16 and
// k = l / 16 of the step, and receives rows l / 16 + 4 r, r = 0 .. 3, of
// column l % 16 of the tile); every fragment is read from LDS before the
// first step.  Larger n takes one output per thread and pass.

__device__ void lds_matmul(int n, const double* A, const double* B, double* Cm) {
  if (n <= 32) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int ia = 16 * (w >> 1) + li, jb = 16 * (w & 1) + li;
    double a[8], b[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const int k = 4 * st + lk;
      a[st] = (ia < n && k < n) ? A[ia * n + k] : 0.0;
      b[st] = (k < n && jb < n) ? B[k * n + jb] : 0.0;
    }
    dbl4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 8; ++st) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st], b[st], c, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * (w >> 1) + lk + 4 * r;
      if (i < n && jb < n) Cm[i * n + jb] = c[r];
    }
  } else {
    for (int it = threadIdx.x; it < n * n; it += blockDim.x) {
      const int i = it / n, j = it % n;
      double s = 0.0;
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      Cm[it] = s;
    }
  }
  __syncthreads();
}

// (V - U) E = V + U for n <= 32 by the four wavefronts of the block, with no
// block barrier inside the elimination: every wave holds the coefficient
// matrix, one row per lane and zero-padded to order 32 by an identity block,
// plus eight of the right-hand-side columns.  The waves make the same pivot
// choices (largest |a| of the unused rows, compared as float keys with ties
// to the lowest lane), eliminate with the pivot row broadcast by readlane
// and back-substitute in pivot order.  E overwrites X.
__device__ void phi1_solve_wave(int n, const double* Pm, double* X, int* fail) {
  constexpr int NM = 32, NC = 8;
  const int lane = threadIdx.x & 63, c0 = (threadIdx.x >> 6) * NC;
  double a[NM], x[NC];
#pragma unroll
  for (int j = 0; j < NM; ++j) a[j] = (lane < n && j < n) ? Pm[lane * n + j] : (lane == j ? 1.0 : 0.0);
#pragma unroll
  for (int c = 0; c < NC; ++c) x[c] = (lane < n && c0 + c < n) ? X[lane * n + c0 + c] : (lane == c0 + c ? 1.0 : 0.0);
  __syncthreads();  // X is overwritten below
  int mystep = (lane < NM) ? -1 : 64;
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    unsigned key = 0u;
    if (mystep < 0) key = (__float_as_uint((float)fabs(a[k])) & ~63u) | (unsigned)(63 - lane);
    const unsigned kmax = wave_max_u32(key);
    const int pl = __builtin_amdgcn_readfirstlane(63 - (int)(kmax & 63u));
    mystep = (lane == pl) ? k : mystep;
    const double piv = readlane_d(a[k], pl);
    if (threadIdx.x == 0 && !(fabs(piv) > 0.0)) atomicOr(fail, 2);
    const double l = (mystep < 0) ? a[k] * (1.0 / piv) : 0.0;
#pragma unroll
    for (int j = k + 1; j < NM; ++j) a[j] = fma(-l, readlane_d(a[j], pl), a[j]);
#pragma unroll
    for (int c = 0; c < NC; ++c) x[c] = fma(-l, readlane_d(x[c], pl), x[c]);
  }
  // back substitution: the row of step k is final once the rows of later
  // steps are; it is scaled by 1/u_kk and removed from the rows of earlier
  // steps (u_sk = a[k] of the lane of step s < k)
#pragma unroll
  for (int k = NM - 1; k >= 0; --k) {
    const int q = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(mystep == k)));
    const double inv = 1.0 / readlane_d(a[k], q);
    const double coef = (mystep < k) ? a[k] : 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double xq = readlane_d(x[c], q) * inv;
      x[c] = (lane == q) ? xq : fma(-coef, xq, x[c]);
    }
  }
  if (mystep < n) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c0 + c < n) X[mystep * n + c0 + c] = x[c];
  }
  __syncthreads();
}

template <bool WAVE>
__global__ __launch_bounds__(256) void k_phi1(const double* __restrict__ H, const double* __restrict__ H2, int mstride,
                                              const double* __restrict__ info, double* __restrict__ y,
                                              int* __restrict__ fail) {
  extern __shared__ double sm[];
  __shared__ int s_sq, s_piv;
  __shared__ double s_red[256];
  // one block per solve of a batch
  H += (size_t)blockIdx.x * (mstride + 1) * mstride;
  H2 += (size_t)blockIdx.x * (mstride + 1) * mstride;
  info += 2 * blockIdx.x;
  y += (size_t)blockIdx.x * (mstride + 1);
  const int mu = (int)info[0];
  if (mu <= 0) return;
  const int n = mu + 1, nn = n * n;
  double* B = sm;
  double* B2 = B + nn;
  double* B4 = B2 + nn;
  double* B6 = B4 + nn;
  double* W = B6 + nn;
  double* T = W + nn;
  double* U = T + nn;
  double* Vm = U + nn;
  const double b[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0, 1187353796428800.0,
                        129060195264000.0,   10559470521600.0,    670442572800.0,     33522128640.0,
                        1323241920.0,        40840800.0,          960960.0,           16380.0,
                        182.0,               1.0};
  for (int it = threadIdx.x; it < nn; it += blockDim.x) {
    const int i = it / n, j = it % n;
    double v = 0.0;
    // only the Hessenberg part (i <= j + 1) is written by the Arnoldi kernel
    if (i < mu && j < mu && i <= j + 1) v = H[i * mstride + j] + H2[i * mstride + j];
    if (i == 0 && j == mu) v = 1.0;
    B[it] = v;
  }
  __syncthreads();
  // 1-norm
  double cs = 0.0;
  if (threadIdx.x < n) for (int i = 0; i < n; ++i) cs += fabs(B[i * n + threadIdx.x]);
  s_red[threadIdx.x] = cs;
  __syncthreads();
  if (threadIdx.x == 0) {
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) nrm = fmax(nrm, s_red[i]);
    const double theta13 = 5.371920351148152;
    int sq = 0;
    // a non-finite H (a diverged solve) takes no squarings: its result is
    // non-finite either way, and the exponent must stay bounded
    if (nrm > theta13 && nrm <= 1.0e300) sq = min(1000, (int)ceil(log2(nrm / theta13)));
    s_sq = sq;
  }
  __syncthreads();
  const int sq = s_sq;
  const double sc = ldexp(1.0, -sq);
  for (int it = threadIdx.x; it < nn; it += blockDim.x) B[it] *= sc;
  __syncthreads();
  lds_matmul(n, B, B, B2);
  lds_matmul(n, B2, B2, B4);
  lds_matmul(n, B4, B2, B6);
  for (int it = threadIdx.x; it < nn; it += blockDim.x) W[it] = b[13] * B6[it] + b[11] * B4[it] + b[9] * B2[it];
  __syncthreads();
  lds_matmul(n, B6, W, T);
  for (int it = threadIdx.x; it < nn; it += blockDim.x) {
    T[it] += b[7] * B6[it] + b[5] * B4[it] + b[3] * B2[it] + ((it / n == it % n) ? b[1] : 0.0);
  }
  __syncthreads();
  lds_matmul(n, B, T, U);
  for (int it = threadIdx.x; it < nn; it += blockDim.x) W[it] = b[12] * B6[it] + b[10] * B4[it] + b[8] * B2[it];
  __syncthreads();
  lds_matmul(n, B6, W, Vm);
  for (int it = threadIdx.x; it < nn; it += blockDim.x) {
    Vm[it] += b[6] * B6[it] + b[4] * B4[it] + b[2] * B2[it] + ((it / n == it % n) ? b[0] : 0.0);
  }
  __syncthreads();
  // (V - U) E = (V + U): Gaussian elimination with partial pivoting
  double* Pm = B2;
  double* X = B4;
  for (int it = threadIdx.x; it < nn; it += blockDim.x) { Pm[it] = Vm[it] - U[it]; X[it] = Vm[it] + U[it]; }
  __syncthreads();
  if constexpr (WAVE) {
    phi1_solve_wave(n, Pm, X, fail);
  } else {
    __shared__ double s_l[64];
    for (int k = 0; k < n; ++k) {
      // pivot: wave 0 finds the first row of largest |Pm[i][k]|, i >= k
      // (n <= 49 rows, one per lane)
      if (threadIdx.x < 64) {
        const int i = threadIdx.x;
        double a = (i >= k && i < n) ? fabs(Pm[i * n + k]) : -1.0;
        int idx = i;
  #pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
          const double a2 = __shfl_xor(a, o, 64);
          const int i2 = __shfl_xor(idx, o, 64);
          if (a2 > a || (a2 == a && i2 < idx)) { a = a2; idx = i2; }
        }
        if (threadIdx.x == 0) {
          if (!(a > 0.0)) atomicOr(fail, 2);
          s_piv = idx;
        }
      }
      __syncthreads();
      const int pv = s_piv;
      if (pv != k) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
          double t1 = Pm[k * n + j]; Pm[k * n + j] = Pm[pv * n + j]; Pm[pv * n + j] = t1;
          double t2 = X[k * n + j]; X[k * n + j] = X[pv * n + j]; X[pv * n + j] = t2;
        }
        __syncthreads();
      }
      // row multipliers once per row, then the rank-1 update
      if (threadIdx.x > k && threadIdx.x < n) s_l[threadIdx.x] = Pm[threadIdx.x * n + k] / Pm[k * n + k];
      __syncthreads();
      for (int it = threadIdx.x; it < (n - k - 1) * n; it += blockDim.x) {
        const int i = k + 1 + it / n, j = it % n;
        const double l = s_l[i];
        X[i * n + j] -= l * X[k * n + j];
        if (j > k) Pm[i * n + j] -= l * Pm[k * n + j];
        else if (j == k) Pm[i * n + j] = 0.0;
      }
      __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {
      for (int j = threadIdx.x; j < n; j += blockDim.x) X[k * n + j] /= Pm[k * n + k];
      __syncthreads();
      for (int it = threadIdx.x; it < k * n; it += blockDim.x) {
        const int i = it / n, j = it % n;
        X[i * n + j] -= Pm[i * n + k] * X[k * n + j];
      }
      __syncthreads();
    }
  }
  double* E = X;
  double* Tm = B6;
  for (int s = 0; s < sq; ++s) {
    lds_matmul(n, E, E, Tm);
    for (int it = threadIdx.x; it < nn; it += blockDim.x) E[it] = Tm[it];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < mu; i += blockDim.x) y[i] = E[i * n + mu];
}

// sum_{i < mu} Vb[i][k] y[i] in order of i, the loads issued sixteen at a
// time (a loop of single loads would wait for each of them in turn).
__device__ __forceinline__ double basis_dot(const double* __restrict__ Vb, size_t K, int k,
                                            const double* __restrict__ ys, int mu) {
  double s = 0.0;
  for (int i0 = 0; i0 < mu; i0 += 16) {
    double a[16], b[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int i = i0 + u < mu ? i0 + u : i0;
      a[u] = Vb[(size_t)i * K + k];
      b[u] = ys[i];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (i0 + u < mu) s += a[u] * b[u];
  }
  return s;
}

// u0 += beta V_m y ; then back to phi coordinates: ut0 = u0 / L00 (y and
// beta of the row's solve).
__global__ __launch_bounds__(256) void k_exp1_update(int K, int V, const double* __restrict__ Vb,
                                                     const double* __restrict__ y, const double* __restrict__ info,
                                                     const double* __restrict__ u0, const double* __restrict__ Lpk,
                                                     int NT, double* __restrict__ ut0, const int* __restrict__ sid,
                                                     int ystride) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const int sg = sid ? sid[k / V] : 0;
  const int mu = (int)info[2 * sg];
  const double beta = info[2 * sg + 1];
  const double* ys = y + (size_t)sg * ystride;
  const double s = basis_dot(Vb, K, k, ys, mu);
  const double u = u0[k] + beta * s;
  ut0[k] = u / Lpk[(size_t)(k / V) * NT];
}

// The EXP1 update of the p = 0 state followed by the whole prolongation
// chain of the V-cycle (Section 2.4, steps 5-6, from level 1 up to p_max):
//   ut0 as k_exp1_update computes it, then for l = 1..p_max
//   ut_l[:N_{l-1}] += ut_{l-1} - uc0_{l-1}.
// Modes are independent along the chain, so one thread takes one (row, mode)
// pair, j < N_{p_max - 1}, and carries its corrected value of ut_{l-1} from
// level to level.  The threads of mode 0, which also form ut0 (a dot
// product over the Krylov basis), come first, one per row, so that they
// fill whole wavefronts; the other modes follow.  Same operations in the
// same order as k_exp1_update followed by the prolongations one level at a
// time.
__global__ __launch_bounds__(256) void k_exp1_prolong(int K, int V, const double* __restrict__ Vb,
                                                      const double* __restrict__ y, const double* __restrict__ info,
                                                      const double* __restrict__ u0, const double* __restrict__ Lpk,
                                                      int NT, const int* __restrict__ sid, int ystride, UpChain c) {
  const int NJ = c.N[c.pmax - 1];
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= K * NJ) return;
  const int k = id < K ? id : (id - K) / (NJ - 1), j = id < K ? 0 : 1 + (id - K) % (NJ - 1);
  // every load of the chain first: ut_l and uc0_{l-1} at (k, j), and
  // ut_{l-1} where the level below leaves mode j as it is (no thread writes
  // such an entry, so it can be read ahead of the corrections)
  double a_ut[4], a_uc0[4], a_prev[4];
#pragma unroll
  for (int l = 1; l <= 4; ++l) {
    const bool on = l <= c.pmax && j < c.N[l - 1];
    const int Nc = c.N[l - 1];
    a_ut[l - 1] = on ? c.ut[l][(size_t)k * c.N[l] + j] : 0.0;
    a_uc0[l - 1] = on ? c.uc0[l - 1][(size_t)k * Nc + j] : 0.0;
    a_prev[l - 1] = (on && l >= 2 && j >= c.N[l - 2]) ? c.ut[l - 1][(size_t)k * Nc + j] : 0.0;
  }
  double cur = 0.0;  // this thread's value of ut_{l-1}[k][j]
  if (j == 0) {
    const int sg = sid ? sid[k / V] : 0;
    const int mu = (int)info[2 * sg];
    const double beta = info[2 * sg + 1];
    const double s = basis_dot(Vb, K, k, y + (size_t)sg * ystride, mu);
    const double u = u0[k] + beta * s;
    cur = u / Lpk[(size_t)(k / V) * NT];
    c.ut[0][k] = cur;
  }
#pragma unroll
  for (int l = 1; l <= 4; ++l) {
    if (l > c.pmax || j >= c.N[l - 1]) continue;  // mode j joins the chain at a higher level
    // a mode the level below did not correct enters as it stands
    if (l >= 2 && j >= c.N[l - 2]) cur = a_prev[l - 1];
    cur = a_ut[l - 1] + (cur - a_uc0[l - 1]);
    c.ut[l][(size_t)k * c.N[l] + j] = cur;
  }
}

// Neighbour table for export: element index, or -1 on any boundary face.
__global__ void k_nbr_export(const int* __restrict__ nbr, int* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = nbr[i] >= 0 ? nbr[i] : -1;
}

// out = a - b (the defect of the FP32 residual against the FP64 one)
__global__ void k_sub(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// Uniform free stream as level-p coefficients in psi coordinates:
// u_{E,v,0} = U_v / psi_0 = U_v L_00 / phi_0.
__global__ void k_freestream(double* __restrict__ u, int V, int N, const double* __restrict__ Lpk, int NT, double phi0,
                             Gas gas, int ne, const double* __restrict__ uinf_e) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * V * N) return;
  const int e = id / (V * N), v = (id / N) % V, i = id % N;
  u[id] = (i == 0) ? (uinf_e ? uinf_e[(size_t)e * V + v] : gas.Uinf[v]) * Lpk[(size_t)e * NT] / phi0 : 0.0;
}

// D = L^{-1} Dt L^{-T} per (v, w) block (tests of the Jacobian in psi
// coordinates), one thread per (element, v, w).
template <int N>
__global__ __launch_bounds__(128) void k_jac_to_psi(double* __restrict__ Dm, const double* __restrict__ Lpk, int NT,
                                                    int V, int ne) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * V * V) return;
  const int e = id / (V * V), v = (id / V) % V, w = id % V;
  const int n = V * N;
  double* Db = Dm + (size_t)e * n * n;
  const double* L = Lpk + (size_t)e * NT;
  // columns: X = L^{-1} Dt_vw (forward substitution on each column j)
  for (int j = 0; j < N; ++j) {
    for (int i = 0; i < N; ++i) {
      double s = Db[(size_t)(v * N + i) * n + w * N + j];
      for (int k = 0; k < i; ++k) s -= L[i * (i + 1) / 2 + k] * Db[(size_t)(v * N + k) * n + w * N + j];
      Db[(size_t)(v * N + i) * n + w * N + j] = s / L[i * (i + 1) / 2 + i];
    }
  }
  // rows: Y = X L^{-T}, i.e. solve L Y^T = X^T row by row
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      double s = Db[(size_t)(v * N + i) * n + w * N + j];
      for (int k = 0; k < j; ++k) s -= L[j * (j + 1) / 2 + k] * Db[(size_t)(v * N + i) * n + w * N + k];
      Db[(size_t)(v * N + i) * n + w * N + j] = s / L[j * (j + 1) / 2 + j];
    }
  }
}

// ===========================================================================
// Adjoint (drag sensitivity): the pressure drag functional and its gradient,
// the transposed-Jacobian residual, the transposed PRK stage and the
// transposed p = 0 operator of the adjoint V-cycle.
// ===========================================================================

// Pressure drag on the slip walls (the functional of the adjoint study):
//   C_D = scale * sum_{wall faces} sum_k w_k |n dsigma| p(U(x_k)) (n^ . dir),
// scale = -1 / (q_inf S_ref), n^ the element's outward unit normal (into the
// body).  One thread per element: part[e] = its contribution, gt[e] = dC_D/dut
// (phi coordinates; zero off the wall), the pressure derivative by dual
// numbers.
struct Dir3 {
  double v[3];
};

template <int D, int P, bool CQ = false>
__global__ __launch_bounds__(128) void k_drag(const double* __restrict__ ut, const double* __restrict__ xv, int nc,
                                              const int* __restrict__ nbr, const uint8_t* __restrict__ ncode,
                                              int ne, Tab<D, P> tab, Gas gas, Dir3 dir,
                                              double scale, double* __restrict__ part, double* __restrict__ gt) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QF = C::QF, NF = C::NF, NC = C::NC;
  __shared__ Tab<D, P> t;
  copy_tab(t, tab);
  __syncthreads();
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double* g = gt + (size_t)e * V * N;  // owned by this thread
  for (int x = 0; x < V * N; ++x) g[x] = 0.0;
  double acc = 0.0;
  const double* ue = ut + (size_t)e * V * N;
  for (int lf = 0; lf < NF; ++lf) {
    if (nbr[(size_t)e * NF + lf] != NB_WALL || ncode[(size_t)e * NF + lf] == NCODE_SYMMETRY) continue;
    double X[NC * D];
#pragma unroll
    for (int a = 0; a < NC * D; ++a) X[a] = xv[(size_t)e * nc * D + a];  // unused when nc == 27
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1];
    face_axes<D>(lf, ta);
    for (int k = 0; k < QF; ++k) {
      double xi[D], wk = 1.0;
      xi[lf >> 1] = (lf & 1) ? 1.0 : -1.0;
      int r0 = k;
#pragma unroll
      for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; xi[ta[q]] = t.x[ik[q]]; wk *= t.w[ik[q]]; }
      double c[D][D], det;
      geom_any<D, CQ>(X, xv + (size_t)e * nc * D, xi, c, det);
      double nh[D], a2 = 0.0;
      const double sg = (lf & 1) ? 1.0 : -1.0;
#pragma unroll
      for (int a = 0; a < D; ++a) { nh[a] = sg * c[lf >> 1][a]; a2 += nh[a] * nh[a]; }
      const double area = sqrt(a2);
      double nd = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) nd += nh[a] / area * dir.v[a];
      Dual<V> U[V];
#pragma unroll
      for (int v = 0; v < V; ++v) U[v] = Dual<V>(0.0);
      for (int j = 0; j < N; ++j) {
        const double ph = phi_face<D, P>(t, j, lf, ta, ik);
#pragma unroll
        for (int v = 0; v < V; ++v) U[v].v += ue[v * N + j] * ph;
      }
#pragma unroll
      for (int v = 0; v < V; ++v) U[v].d[v] = 1.0;
      const Dual<V> pr = pressure<D>(U, gas.g);
      const double wt = scale * wk * area * nd;
      acc += wt * pr.v;
      for (int j = 0; j < N; ++j) {
        const double ph = phi_face<D, P>(t, j, lf, ta, ik);
#pragma unroll
        for (int v = 0; v < V; ++v) g[v * N + j] += wt * pr.d[v] * ph;
      }
    }
  }
  part[e] = acc;
}

// Deterministic sum of n values: per-block partial sums, then one block adds
// them in a fixed order.
__global__ __launch_bounds__(256) void k_sum_partial(const double* __restrict__ x, const double* __restrict__ y, size_t n,
                                                     double* __restrict__ part) {
  __shared__ double s[256];
  double a = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a += y ? x[i] * y[i] : x[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, int nblk, int take_sqrt,
                                                   double* __restrict__ out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = take_sqrt ? sqrt(s[0]) : s[0];
}

// ---------------------------------------------------------------------------
// Transposed-Jacobian residual (the adjoint residual) in phi coordinates:
//   out = Dt^T w (+ g),  Dt = dRt/dut at the linearisation state,
// matrix free from the pointwise flux Jacobians of k_jac_points at that
// state (per element [QV][D][V][V] volume, [NF*QF][V][V] faces):
//   out_{(w,j)} = sum_q phi_j(q) sum_r sum_v B_{q,r}[v][w] G_{v,r}(q)
//               - sum_faces sum_k phi_j(x_k) sum_v C_k[v][w] (W_v(x_k) - W^nb_v(x_k)),
// G_{v,r}(q) = sum_i w_{v,i} d_r phi_i(q) the reference gradient and W, W^nb
// the traces of w on the element and on the neighbour (zero on boundary
// faces).  The neighbour term is the transposed off-diagonal block: the
// Rusanov flux is antisymmetric under exchanging the sides and flipping the
// normal, so dF~_nb/dU_own = -dF~_own/dU_own, and the neighbour's residual
// couples to this element through this element's own face Jacobian C_k.
// ---------------------------------------------------------------------------
template <int D, int P, int EB>
__global__ __launch_bounds__(256) void k_adj_residual(const double* __restrict__ wt, const double* __restrict__ gadd,
                                                      const double* __restrict__ BC, const int* __restrict__ nbr,
                                                      const uint8_t* __restrict__ ncode, int ne, Tab<D, P> tab,
                                                      double* __restrict__ out) {
  using C = Cfg<D, P>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF;
  constexpr int PER = (QV * D + NF * QF) * V * V;
  __shared__ double s_w[EB * V * N];
  __shared__ double s_hv[EB * QV * V];
  __shared__ double s_hf[EB * NF * QF * V];
  __shared__ Tab<D, P> t;
  const int tid = threadIdx.x;
  const int e0 = blockIdx.x * EB;
  copy_tab(t, tab);
  {
    const int nel = min(EB, ne - e0);
    stage<(EB * V * N + 255) / 256>(s_w, wt + (size_t)e0 * V * N, nel * V * N, tid, 256);
  }
  __syncthreads();
  for (int it = tid; it < EB * QV; it += blockDim.x) {
    const int el = it / QV, q = it % QV;
    const int e = e0 + el;
    if (e >= ne) continue;
    int iq[D];
    {
      int r0 = q;
#pragma unroll
      for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
    }
    double G[V][D];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int r = 0; r < D; ++r) G[v][r] = 0.0;
    const double* sw = &s_w[el * V * N];
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int r = 0; r < D; ++r) {
        const double dp = dphi_vol<D, P>(t, i, iq, r);
#pragma unroll
        for (int v = 0; v < V; ++v) G[v][r] += sw[v * N + i] * dp;
      }
    }
    const double* B = BC + (size_t)e * PER + (size_t)q * D * V * V;
    double H[V];
#pragma unroll
    for (int w = 0; w < V; ++w) H[w] = 0.0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int w = 0; w < V; ++w) H[w] += B[(r * V + v) * V + w] * G[v][r];
#pragma unroll
    for (int w = 0; w < V; ++w) s_hv[(el * QV + q) * V + w] = H[w];
  }
  for (int it = tid; it < EB * NF * QF; it += blockDim.x) {
    const int el = it / (NF * QF), lf = (it / QF) % NF, k = it % QF;
    const int e = e0 + el;
    if (e >= ne) continue;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1];
    face_axes<D>(lf, ta);
    {
      int r0 = k;
#pragma unroll
      for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
    }
    double W[V];
#pragma unroll
    for (int v = 0; v < V; ++v) W[v] = 0.0;
    const double* sw = &s_w[el * V * N];
    for (int j = 0; j < N; ++j) {
      const double ph = phi_face<D, P>(t, j, lf, ta, ik);
#pragma unroll
      for (int v = 0; v < V; ++v) W[v] += sw[v * N + j] * ph;
    }
    const int nb = nbr[(size_t)e * NF + lf];
    if (nb >= 0) {
      const int code = ncode[(size_t)e * NF + lf];
      const int lf2 = code & 7;
      int ta2[D - 1 > 0 ? D - 1 : 1], jk[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf2, ta2);
      nb_face_index<D, Q>(code, ik, jk);
      const double* wn = wt + (size_t)nb * V * N;
      for (int j = 0; j < N; ++j) {
        const double ph = phi_face<D, P>(t, j, lf2, ta2, jk);
#pragma unroll
        for (int v = 0; v < V; ++v) W[v] -= wn[v * N + j] * ph;
      }
    }
    const double* Cm = BC + (size_t)e * PER + (size_t)QV * D * V * V + (size_t)(lf * QF + k) * V * V;
    double H[V];
#pragma unroll
    for (int w = 0; w < V; ++w) H[w] = 0.0;
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int w = 0; w < V; ++w) H[w] += Cm[v * V + w] * W[v];
#pragma unroll
    for (int w = 0; w < V; ++w) s_hf[((el * NF + lf) * QF + k) * V + w] = H[w];
  }
  __syncthreads();
  for (int it = tid; it < EB * V * N; it += blockDim.x) {
    const int el = it / (V * N), w = (it / N) % V, j = it % N;
    const int e = e0 + el;
    if (e >= ne) continue;
    double acc = 0.0;
    for (int q = 0; q < QV; ++q) {
      int iq[D];
      int r0 = q;
#pragma unroll
      for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
      acc += phi_vol<D, P>(t, j, iq) * s_hv[(el * QV + q) * V + w];
    }
    for (int lf = 0; lf < NF; ++lf) {
      int ta[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf, ta);
      for (int k = 0; k < QF; ++k) {
        int ik[D - 1 > 0 ? D - 1 : 1];
        int r0 = k;
#pragma unroll
        for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
        acc -= phi_face<D, P>(t, j, lf, ta, ik) * s_hf[((el * NF + lf) * QF + k) * V + w];
      }
    }
    const size_t o = (size_t)e0 * V * N + it;
    out[o] = gadd ? acc + gadd[o] : acc;
  }
}

// Transposed PRK stage: lam = lam_n + beta Pt^{-T} r with the LU factors of
// Pt (Pi Pt = L U, column-major, row k = k-th pivot row): solve U^T z = r,
// L^T y = z, x[perm[k]] = y_k.  One wavefront per element, lane l holding
// column l of the factor (U(k, l) for k <= l, L(k, l) for k > l).
template <int NB>
__global__ __launch_bounds__(256) void k_prk_stage_tr(const double* __restrict__ Fm, const int* __restrict__ perm,
                                                      const double* __restrict__ rt, const double* __restrict__ un,
                                                      double* __restrict__ ut, double beta, int ne) {
  static_assert(NB <= 64, "one column per lane");
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (e >= ne) return;
  const double* F = Fm + (size_t)e * NB * NB;
  const int l = lane < NB ? lane : NB - 1;
  double col[NB];
#pragma unroll
  for (int m = 0; m < NB; ++m) col[m] = F[(size_t)l * NB + m];
  double b = rt[(size_t)e * NB + l];
  // U^T z = r (forward): z_k = b_k / U(k, k); lanes l > k subtract U(k, l) z_k
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double zk = readlane_d(b, k) / readlane_d(col[k], k);
    b = (lane == k) ? zk : fma(-((lane > k) ? col[k] : 0.0), zk, b);
  }
  // L^T y = z (backward, unit diagonal): lanes l < k subtract L(k, l) y_k
#pragma unroll
  for (int k = NB - 1; k >= 0; --k) {
    const double yk = readlane_d(b, k);
    b = fma(-((lane < k) ? col[k] : 0.0), yk, b);
  }
  if (lane < NB) {
    const int o = perm[(size_t)e * NB + lane];
    ut[(size_t)e * NB + o] = un[(size_t)e * NB + o] + beta * b;
  }
}

// Transposed PRK stage for 64 < NB <= 320: lanes hold columns lane, lane +
// 64, ... of the factor, whose elements stream through registers in chunks
// of eight (loads of a chunk issued together; only the column slots the
// substitution touches); x_k broadcast by readlane from the lane of column
// k.  Same arithmetic as k_prk_stage_tr.
template <int NB>
__global__ __launch_bounds__(256) void k_prk_stage_trc(const double* __restrict__ Fm, const int* __restrict__ perm,
                                                       const double* __restrict__ rt, const double* __restrict__ un,
                                                       double* __restrict__ ut, double beta, int ne) {
  constexpr int RPL = (NB + 63) / 64, CH = 8;
  static_assert(NB > 64 && NB <= 320, "columns per lane");
  const int lane = threadIdx.x & 63;
  const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (e >= ne) return;
  const double* F = Fm + (size_t)e * NB * NB;
  int lc[RPL];  // clamped columns: every load in bounds
  double b[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int l = lane + 64 * s;
    lc[s] = l < NB ? l : NB - 1;
    b[s] = (l < NB) ? rt[(size_t)e * NB + lc[s]] : 0.0;
  }
  // U^T z = r (forward): z_k = b_k / U(k, k); columns l > k subtract U(k, l) z_k
#pragma unroll
  for (int sl = 0; sl < RPL; ++sl) {
#pragma unroll 1
    for (int k0 = 64 * sl; k0 < NB && k0 < 64 * sl + 64; k0 += CH) {
      double cf[CH][RPL];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = k0 + c < NB ? k0 + c : NB - 1;
#pragma unroll
        for (int s = sl; s < RPL; ++s) cf[c][s] = F[(size_t)lc[s] * NB + k];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = k0 + c;
        if (k < NB) {
          const double zk = readlane_d(b[sl], k & 63) / readlane_d(cf[c][sl], k & 63);
#pragma unroll
          for (int s = sl; s < RPL; ++s) {
            const int l = lane + 64 * s;
            b[s] = (l == k) ? zk : fma(-((l > k) ? cf[c][s] : 0.0), zk, b[s]);
          }
        }
      }
    }
  }
  // L^T y = z (backward, unit diagonal): columns l < k subtract L(k, l) y_k
#pragma unroll
  for (int sl = RPL - 1; sl >= 0; --sl) {
    const int klast = (NB < 64 * sl + 64 ? NB : 64 * sl + 64) - 1;
#pragma unroll 1
    for (int k0 = (klast / CH) * CH; k0 >= 64 * sl; k0 -= CH) {
      double cf[CH][RPL];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int k = k0 + c < NB ? k0 + c : NB - 1;
#pragma unroll
        for (int s = 0; s <= sl; ++s) cf[c][s] = F[(size_t)lc[s] * NB + k];
      }
#pragma unroll
      for (int c = CH - 1; c >= 0; --c) {
        const int k = k0 + c;
        if (k < NB) {
          const double yk = readlane_d(b[sl], k & 63);
#pragma unroll
          for (int s = 0; s <= sl; ++s) b[s] = fma(-((lane + 64 * s < k) ? cf[c][s] : 0.0), yk, b[s]);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int l = lane + 64 * s;
    if (l < NB) {
      const int o = perm[(size_t)e * NB + l];
      ut[(size_t)e * NB + o] = un[(size_t)e * NB + o] + beta * b[s];
    }
  }
}

// Transposed p = 0 operator for the adjoint EXP1: A^T-side blocks
// (T J0^T)_{F,E} = dt_F (J0_{E,F})^T from the forward blocks Ad = T J0 (diag)
// and Ao[E][lf2] = dt_E J0_{E,F} (lf2: the face of E that touches F).
template <int V, int NF>
__global__ __launch_bounds__(256) void k_p0_transpose(const double* __restrict__ Ad, const double* __restrict__ Ao,
                                                      const double* __restrict__ dt, const int* __restrict__ nbr,
                                                      const uint8_t* __restrict__ ncode, double* __restrict__ AdT,
                                                      double* __restrict__ AoT, int ne) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * (1 + NF)) return;
  const int e = id / (1 + NF), slot = id % (1 + NF);
  if (slot == 0) {
#pragma unroll
    for (int w = 0; w < V; ++w)
#pragma unroll
      for (int v = 0; v < V; ++v) AdT[(size_t)e * V * V + w * V + v] = Ad[(size_t)e * V * V + v * V + w];
    return;
  }
  const int lf = slot - 1;
  const int nb = nbr[(size_t)e * NF + lf];
  double* o = AoT + ((size_t)e * NF + lf) * V * V;
  if (nb < 0) {
#pragma unroll
    for (int x = 0; x < V * V; ++x) o[x] = 0.0;
    return;
  }
  const int lf2 = ncode[(size_t)e * NF + lf] & 7;
  const double* a = Ao + ((size_t)nb * NF + lf2) * V * V;
  const double sc = dt[e] / dt[nb];
#pragma unroll
  for (int w = 0; w < V; ++w)
#pragma unroll
    for (int v = 0; v < V; ++v) o[w * V + v] = sc * a[v * V + w];
}

// Adjoint p = 0 right-hand side in psi coordinates: b = dt * gt0 / L00.
__global__ __launch_bounds__(256) void k_adj_p0_rhs(const double* __restrict__ gt0, const double* __restrict__ Lpk,
                                                    int NT, const double* __restrict__ dt, int V, int ne,
                                                    double* __restrict__ b) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ne * V) return;
  const int e = id / V;
  b[id] = dt[e] * gt0[id] / Lpk[(size_t)e * NT];
}

// Leading-slice truncation y = Trunc(x) (N -> Nc modes per row) and the
// padded correction x += Pad(y); zero fill.
__global__ void k_trunc(const double* __restrict__ x, double* __restrict__ y, int N, int Nc, int rows) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= rows * Nc) return;
  const int r = id / Nc, i = id % Nc;
  y[id] = x[(size_t)r * N + i];
}

__global__ void k_pad_add(double* __restrict__ x, const double* __restrict__ y, int N, int Nc, int rows) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= rows * Nc) return;
  const int r = id / Nc, i = id % Nc;
  x[(size_t)r * N + i] += y[id];
}

// Per-element CFL of a batch from the per-solve values.
__global__ void k_expand_cfl(const double* __restrict__ cfl_s, const int* __restrict__ sid, double* __restrict__ cfl_e,
                             int ne) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) cfl_e[e] = cfl_s[sid[e]];
}

__global__ void k_fill0(double* __restrict__ x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// ===========================================================================
// launchers
// ===========================================================================
namespace {

template <int D, int P, class R>
constexpr int res_tile() {
  using C = Cfg<D, P>;
  constexpr int per = (C::V * C::N + C::QV * C::V * D + C::NF * C::QF * C::V + C::NC * D) * (int)sizeof(R);
  constexpr int tables = res_tables<D, P, R>() ? res_table_values<D, P, R>() * (int)sizeof(R) : 0;
  constexpr int budget = 48 * 1024 - tables;
  constexpr int eb0 = budget / per < 1 ? 1 : (budget / per > 32 ? 32 : budget / per);
  // with the tables in LDS, at most one pass of the block over the volume
  // points: smaller tiles put more blocks on every compute unit, which hides
  // the latency of the three dependent phases better than a larger share of
  // the table set-up
  constexpr int eb1 = !res_tables<D, P, R>() ? eb0 : (256 / C::QV < 1 ? 1 : 256 / C::QV);
  return eb0 < eb1 ? eb0 : eb1;
}

template <class R>
GasT<R> gas_as(const Gas& g) {
  GasT<R> o;
  o.g = R(g.g);
  o.flux = g.flux;
  for (int v = 0; v < 5; ++v) o.Uinf[v] = R(g.Uinf[v]);
  return o;
}

// Residual tiles (elements per workgroup) the autotuner chooses among: half,
// the default and one and a half times the default (res_tile).
template <int D, int P, class R, int C>
constexpr int res_tile_cand() {
  constexpr int def = res_tile<D, P, R>();
  constexpr int half = def / 2 < 1 ? 1 : def / 2, more = (3 * def) / 2 > 32 ? 32 : (3 * def) / 2;
  return C == 0 ? half : C == 2 ? (more < 1 ? 1 : more) : def;
}

template <int D, int P, int EB, class R, bool CQ = false>
hipError_t residual_launch(const DevMesh& M, const Tab<D, P, R>& t, const double* ut, const double* fadd, double* rt,
                           const FasOut& fas, hipStream_t st) {
  const int grid = (M.ne + EB - 1) / EB;
  hipLaunchKernelGGL((k_residual<D, P, EB, R, CQ>), dim3(grid), dim3(256), 0, st, ut, fadd, rt, M.xv, M.NC, M.nbr,
                     M.ncode, M.ne, t, gas_as<R>(M.gas), M.uinf_e, fas);
  return hipGetLastError();
}

template <int D, int P, class R>
hipError_t residual_t(const DevMesh& M, const TabData& td, const double* ut, const double* fadd, double* rt,
                      const FasOut& fas, int choice, hipStream_t st) {
  Tab<D, P, R> t;
  fill_tab(t, td);
  if constexpr (D == 3) {
    // curved hexes: the triquadratic instantiations, same tile candidates
    if (M.NC == 27) {
      switch (choice) {
        case 0: return residual_launch<D, P, res_tile_cand<D, P, R, 0>(), R, true>(M, t, ut, fadd, rt, fas, st);
        case 2: return residual_launch<D, P, res_tile_cand<D, P, R, 2>(), R, true>(M, t, ut, fadd, rt, fas, st);
        default: return residual_launch<D, P, res_tile_cand<D, P, R, 1>(), R, true>(M, t, ut, fadd, rt, fas, st);
      }
    }
  }
  switch (choice) {
    case 0: return residual_launch<D, P, res_tile_cand<D, P, R, 0>(), R>(M, t, ut, fadd, rt, fas, st);
    case 2: return residual_launch<D, P, res_tile_cand<D, P, R, 2>(), R>(M, t, ut, fadd, rt, fas, st);
    default: return residual_launch<D, P, res_tile_cand<D, P, R, 1>(), R>(M, t, ut, fadd, rt, fas, st);
  }
}

template <int D, int P, class R>
int res_tile_of(int choice) {
  return choice == 0 ? res_tile_cand<D, P, R, 0>() : choice == 2 ? res_tile_cand<D, P, R, 2>() : res_tile_cand<D, P, R, 1>();
}

// Point Jacobians of every element (k_jac_points, the triquadratic
// instantiation on curved hexes).
template <int D, int P, class R>
void launch_jac_points_t(const DevMesh& M, const Tab<D, P, R>& t, const GasT<R>& gas, const double* ut, R* bc,
                         hipStream_t st) {
  using C = Cfg<D, P>;
  constexpr int NPT = C::QV + C::NF * C::QF;
  const int items = M.ne * NPT;
  if constexpr (D == 3) {
    if (M.NC == 27) {
      hipLaunchKernelGGL((k_jac_points<D, P, R, true>), dim3((items + 255) / 256), dim3(256), 0, st, ut, M.xv, M.NC,
                         M.nbr, M.ncode, bc, M.ne, t, gas, M.uinf_e);
      return;
    }
  }
  hipLaunchKernelGGL((k_jac_points<D, P, R>), dim3((items + 255) / 256), dim3(256), 0, st, ut, M.xv, M.NC, M.nbr,
                     M.ncode, bc, M.ne, t, gas, M.uinf_e);
}

// The generic one-workgroup-per-element assembly (and LU), straight or curved.
template <int D, int P, bool FACTOR, class R, bool CQ>
hipError_t launch_jacobian_generic(const DevMesh& M, const Tab<D, P, R>& t, const GasT<R>& gas, const double* ut,
                                   const double* dtau, R* out, int* perm, int* fail, hipStream_t st) {
  const size_t lds = (size_t)jac_lds_values<D, P>() * sizeof(R);
  auto kf = k_jacobian<D, P, FACTOR, R, CQ>;
  static bool attr = false;  // set once: not a stream operation, so also fine while capturing
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(kf, dim3(M.ne), dim3(256), lds, st, ut, M.xv, M.NC, M.nbr, M.ncode, M.Gpk, M.NT, dtau, out, perm,
                     fail, M.ne, t, gas, M.uinf_e);
  return hipGetLastError();
}

template <int D, int P, class R>
hipError_t jacobian_t(const DevMesh& M, const TabData& td, const double* ut, const double* dtau, void* outv,
                      int* perm, int* fail, bool factor, hipStream_t st) {
  Tab<D, P, R> t;
  fill_tab(t, td);
  R* out = static_cast<R*>(outv);
  const GasT<R> gas = gas_as<R>(M.gas);
  if constexpr (Cfg<D, P>::NB < 256) {
    if (factor && M.bc) {
      R* bc = static_cast<R*>(M.bc);
      launch_jac_points_t<D, P, R>(M, t, gas, ut, bc, st);
      if constexpr (Cfg<D, P>::NB == 16) {
        const R* gph = static_cast<const R*>(M.phitab[P][sizeof(R) == 4 ? PREC_FP32 : PREC_FP64]);
        if (!gph) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_jaclu_g16<D, P, R>), dim3((M.ne + 15) / 16), dim3(256), 0, st, bc, M.Gpk, M.NT, dtau,
                           out, perm, fail, M.ne, t, gph);
      } else if constexpr (Cfg<D, P>::NB <= 64) {
        const R* gph = static_cast<const R*>(M.phitab[P][sizeof(R) == 4 ? PREC_FP32 : PREC_FP64]);
        if (!gph) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_jaclu_wave<D, P, R>), dim3((M.ne + 3) / 4), dim3(256), 0, st, bc, M.Gpk, M.NT, dtau,
                           out, perm, fail, M.ne, t, gph);
      } else {
        // 64 < n < 256: the LDS-resident kernel (every such block size that
        // the residual supports)
        if (!jaclu_lds_supported(D, P)) return hipErrorInvalidValue;
        return launch_jaclu_lds(M, td, P, sizeof(R) == 4 ? PREC_FP32 : PREC_FP64, bc, dtau, out, perm, fail, st);
      }
      return hipGetLastError();
    }
  } else {
    // n >= 256 (3D p = 3): point Jacobians, then assembly (and LU) with the
    // block in global memory, factored or not
    if (!M.bc || !jaclu_big_supported(D, P)) return hipErrorInvalidValue;
    R* bc = static_cast<R*>(M.bc);
    launch_jac_points_t<D, P, R>(M, t, gas, ut, bc, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_jaclu_big(M, P, sizeof(R) == 4 ? PREC_FP32 : PREC_FP64, bc,
                            M.phitab[P][sizeof(R) == 4 ? PREC_FP32 : PREC_FP64], dtau, out, perm, fail, factor, st);
  }
  if constexpr (Cfg<D, P>::NB < 256) {
    if constexpr (D == 3) {
      if (M.NC == 27)
        return factor ? launch_jacobian_generic<D, P, true, R, true>(M, t, gas, ut, dtau, out, perm, fail, st)
                      : launch_jacobian_generic<D, P, false, R, true>(M, t, gas, ut, dtau, out, perm, fail, st);
    }
    return factor ? launch_jacobian_generic<D, P, true, R, false>(M, t, gas, ut, dtau, out, perm, fail, st)
                  : launch_jacobian_generic<D, P, false, R, false>(M, t, gas, ut, dtau, out, perm, fail, st);
  }
}

template <int N>
hipError_t basis_t(const DevMesh& M, const double* x, double* y, int mode, hipStream_t st) {
  const int rows = M.ne * M.V;
  hipLaunchKernelGGL((k_basis<N>), dim3((rows + 255) / 256), dim3(256), 0, st, x, y, M.Lpk, M.NT, M.V, M.ne, mode);
  return hipGetLastError();
}

template <int N, int Nc>
hipError_t restrict_t(const DevMesh& M, const double* R, const double* ut, double* uc, double* uc0, hipStream_t st) {
  if (!R) return hipErrorInvalidValue;
  const int cnt = M.ne * M.V * Nc;
  hipLaunchKernelGGL((k_restrict<N, Nc>), dim3((cnt + 255) / 256), dim3(256), 0, st, ut, uc, uc0, R, M.V, M.ne);
  return hipGetLastError();
}

template <int D, int N>
hipError_t norm_t(const DevMesh& M, const double* rt, double* part, double* out, hipStream_t st) {
  constexpr int EPB = 256 / norm_group<N>();  // elements per block
  if (M.seg_e0) {
    // part holds >= ne values here: the squared norm of every element
    hipLaunchKernelGGL((k_norm_elem<D, N>), dim3((M.ne + EPB - 1) / EPB), dim3(256), 0, st, rt, M.Lpk, M.NT, M.ne,
                       part);
    hipLaunchKernelGGL(k_norm_segsum, dim3(M.nseg), dim3(256), 0, st, part, M.seg_e0, M.seg_omega, out);
    return hipGetLastError();
  }
  const int nblk = (M.ne + EPB - 1) / EPB;  // part holds >= ne / 4 + 1 values
  hipLaunchKernelGGL((k_norm_partial<D, N>), dim3(nblk), dim3(256), 0, st, rt, M.Lpk, M.NT, M.ne, part);
  hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(256), 0, st, part, nblk, M.omega, out);
  return hipGetLastError();
}

template <int N>
hipError_t jac_to_psi_t(const DevMesh& M, double* Dm, hipStream_t st) {
  const int cnt = M.ne * M.V * M.V;
  hipLaunchKernelGGL((k_jac_to_psi<N>), dim3((cnt + 127) / 128), dim3(128), 0, st, Dm, M.Lpk, M.NT, M.V, M.ne);
  return hipGetLastError();
}

}  // namespace

#define EG_DISPATCH_P(D, p, CALL)                            \
  switch (p) {                                               \
    case 0: return CALL(D, 0);                               \
    case 1: return CALL(D, 1);                               \
    case 2: return CALL(D, 2);                               \
    case 3: return CALL(D, 3);                               \
    case 4: if (D == 2) return CALL(2, 4); break;            \
    default: break;                                          \
  }

hipError_t launch_residual(const DevMesh& M, const TabData& td, int p, const double* ut, const double* fadd,
                           double* rt, int prec, hipStream_t st, const FasOut& fas) {
  const int choice = (p >= 0 && p < 5) ? M.res_tile_choice[p][prec == PREC_FP32 ? 1 : 0] : 1;
  if (prec == PREC_FP32) {
#define CALL_RES(DD, PP) residual_t<DD, PP, float>(M, td, ut, fadd, rt, fas, choice, st)
    if (M.d == 2) { EG_DISPATCH_P(2, p, CALL_RES) }
    else { EG_DISPATCH_P(3, p, CALL_RES) }
#undef CALL_RES
  } else {
#define CALL_RES(DD, PP) residual_t<DD, PP, double>(M, td, ut, fadd, rt, fas, choice, st)
    if (M.d == 2) { EG_DISPATCH_P(2, p, CALL_RES) }
    else { EG_DISPATCH_P(3, p, CALL_RES) }
#undef CALL_RES
  }
  return hipErrorInvalidValue;
}

size_t jac_points_per_elem(int d, int p, bool fp32) {
  const int V = d + 2, Q = p + 2, N = (d == 2) ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1);
  // blocks that take the point-Jacobian kernels (k_jaclu_g16, k_jaclu_wave,
  // k_jaclu_lds, k_jaclu_big)
  (void)fp32;
  if (p < 1 || V * N > 320) return 0;
  const int QV = (d == 2) ? Q * Q : Q * Q * Q, QF = (d == 2) ? Q : Q * Q;
  return (size_t)(QV * d + 2 * d * QF) * V * V;
}

bool jacobian_supported(int d, int p) {
  if (p < 1) return false;
  if (d == 2) return p <= 4;
  return p <= 3;
}

template <class R>
static hipError_t launch_jacobian_r(const DevMesh& M, const TabData& td, int p, const double* ut, const double* dtau,
                                   void* out, int* perm, int* fail, bool factor, hipStream_t st) {
#define CALL_JAC(DD, PP) jacobian_t<DD, PP, R>(M, td, ut, dtau, out, perm, fail, factor, st)
  if (M.d == 2) {
    switch (p) {
      case 1: return CALL_JAC(2, 1);
      case 2: return CALL_JAC(2, 2);
      case 3: return CALL_JAC(2, 3);
      case 4: return CALL_JAC(2, 4);
      default: break;
    }
  } else {
    switch (p) {
      case 1: return CALL_JAC(3, 1);
      case 2: return CALL_JAC(3, 2);
      case 3: return CALL_JAC(3, 3);
      default: break;
    }
  }
#undef CALL_JAC
  return hipErrorInvalidValue;
}

hipError_t launch_jacobian(const DevMesh& M, const TabData& td, int p, const double* ut, const double* dtau,
                           void* out, int* perm, int* fail, bool factor, int prec, hipStream_t st) {
  if (!jacobian_supported(M.d, p)) return hipErrorInvalidValue;
  if (prec == PREC_FP32) return launch_jacobian_r<float>(M, td, p, ut, dtau, out, perm, fail, factor, st);
  return launch_jacobian_r<double>(M, td, p, ut, dtau, out, perm, fail, factor, st);
}

template <class R>
static hipError_t launch_prk_stage_r(const DevMesh& M, int n, const R* F, const int* perm, const double* rt,
                                     const double* ft, const double* un, double* ut, double* save, double beta,
                                     hipStream_t st) {
  const int grid = (M.ne + 3) / 4;
  if (!ft) {
    switch (n) {
      case 16: hipLaunchKernelGGL((k_prk_stage_g16<R>), dim3((M.ne + 15) / 16), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      case 36: hipLaunchKernelGGL((k_prk_stage_t<36, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      case 64: hipLaunchKernelGGL((k_prk_stage_t<64, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      case 40: hipLaunchKernelGGL((k_prk_stage_t<40, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      case 100: hipLaunchKernelGGL((k_prk_stage_c<100, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      case 135: hipLaunchKernelGGL((k_prk_stage_c<135, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      case 320: hipLaunchKernelGGL((k_prk_stage_c<320, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, save, beta, M.ne); return hipGetLastError();
      default: break;
    }
  }
  if (n <= 64) hipLaunchKernelGGL((k_prk_stage<1, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, ft, un, ut, save, beta, n, M.ne);
  else if (n <= 128) hipLaunchKernelGGL((k_prk_stage<2, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, ft, un, ut, save, beta, n, M.ne);
  else if (n <= 192) hipLaunchKernelGGL((k_prk_stage<3, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, ft, un, ut, save, beta, n, M.ne);
  else if (n <= 320) hipLaunchKernelGGL((k_prk_stage<5, R>), dim3(grid), dim3(256), 0, st, F, perm, rt, ft, un, ut, save, beta, n, M.ne);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_prk_stage(const DevMesh& M, int n, const void* F, const int* perm, const double* rt,
                            const double* ft, const double* un, double* ut, double beta, int prec, hipStream_t st,
                            double* save) {
  if (prec == PREC_FP32)
    return launch_prk_stage_r<float>(M, n, static_cast<const float*>(F), perm, rt, ft, un, ut, save, beta, st);
  return launch_prk_stage_r<double>(M, n, static_cast<const double*>(F), perm, rt, ft, un, ut, save, beta, st);
}

hipError_t launch_basis(const DevMesh& M, int N, const double* x, double* y, int mode, hipStream_t st) {
  switch (N) {
    case 1: return basis_t<1>(M, x, y, mode, st);
    case 4: return basis_t<4>(M, x, y, mode, st);
    case 8: return basis_t<8>(M, x, y, mode, st);
    case 9: return basis_t<9>(M, x, y, mode, st);
    case 16: return basis_t<16>(M, x, y, mode, st);
    case 25: return basis_t<25>(M, x, y, mode, st);
    case 27: return basis_t<27>(M, x, y, mode, st);
    case 64: return basis_t<64>(M, x, y, mode, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_restrict(const DevMesh& M, int p, const double* ut, double* uc, double* uc0, hipStream_t st) {
  if (M.d == 2) {
    switch (p) {
      case 1: return restrict_t<4, 1>(M, M.Rop[p], ut, uc, uc0, st);
      case 2: return restrict_t<9, 4>(M, M.Rop[p], ut, uc, uc0, st);
      case 3: return restrict_t<16, 9>(M, M.Rop[p], ut, uc, uc0, st);
      case 4: return restrict_t<25, 16>(M, M.Rop[p], ut, uc, uc0, st);
      default: break;
    }
  } else {
    switch (p) {
      case 1: return restrict_t<8, 1>(M, M.Rop[p], ut, uc, uc0, st);
      case 2: return restrict_t<27, 8>(M, M.Rop[p], ut, uc, uc0, st);
      case 3: return restrict_t<64, 27>(M, M.Rop[p], ut, uc, uc0, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

// CFL source of the time-step kernels: a per-element array (batch), a
// device scalar (captured V-cycles), or the host value passed by argument.
static const double* cfl_ptr(const DevMesh& M) { return M.cfl_e ? M.cfl_e : M.cfl_one; }
static int cfl_stride(const DevMesh& M) { return M.cfl_e ? 1 : 0; }

hipError_t launch_timestep(const DevMesh& M, int p, int N, double cfl, double mult, const double* ut, double* dtau,
                           hipStream_t st) {
  const int grid = (M.ne + 15) / 16;  // 16 lanes per element
  if (M.d == 2)
    hipLaunchKernelGGL((k_timestep<2>), dim3(grid), dim3(256), 0, st, ut, N, M.Lpk, M.NT, M.hE, p, cfl, mult, dtau,
                       M.ne, M.gas.g, cfl_ptr(M), cfl_stride(M));
  else
    hipLaunchKernelGGL((k_timestep<3>), dim3(grid), dim3(256), 0, st, ut, N, M.Lpk, M.NT, M.hE, p, cfl, mult, dtau,
                       M.ne, M.gas.g, cfl_ptr(M), cfl_stride(M));
  return hipGetLastError();
}

hipError_t launch_norm(const DevMesh& M, int N, const double* rt, double* part, double* out, hipStream_t st) {
  if (M.d == 2) {
    switch (N) {
      case 1: return norm_t<2, 1>(M, rt, part, out, st);
      case 4: return norm_t<2, 4>(M, rt, part, out, st);
      case 9: return norm_t<2, 9>(M, rt, part, out, st);
      case 16: return norm_t<2, 16>(M, rt, part, out, st);
      case 25: return norm_t<2, 25>(M, rt, part, out, st);
      default: break;
    }
  } else {
    switch (N) {
      case 1: return norm_t<3, 1>(M, rt, part, out, st);
      case 8: return norm_t<3, 8>(M, rt, part, out, st);
      case 27: return norm_t<3, 27>(M, rt, part, out, st);
      case 64: return norm_t<3, 64>(M, rt, part, out, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_p0_setup(const DevMesh& M, const double* ut0, const double* ft0, int pmax, double cfl, int scale,
                           double* u0, double* b, double* Ad, double* Ao, double* dt, hipStream_t st) {
  // 8 (2D) or 32 (3D) lanes per element
  const int grid = M.d == 2 ? (M.ne + 31) / 32 : (M.ne + 7) / 8;
  if (M.d == 2)
    hipLaunchKernelGGL((k_p0_setup<2>), dim3(grid), dim3(256), 0, st, ut0, ft0, M.xv, M.NC, M.nbr, M.Lpk, M.NT, M.hE, pmax,
                       cfl, scale, u0, b, Ad, Ao, dt, M.ne, M.gas, M.g2x, M.g2w, M.uinf_e, cfl_ptr(M), cfl_stride(M));
  else if (M.NC == 27)
    hipLaunchKernelGGL((k_p0_setup<3, true>), dim3(grid), dim3(256), 0, st, ut0, ft0, M.xv, M.NC, M.nbr, M.Lpk, M.NT,
                       M.hE, pmax, cfl, scale, u0, b, Ad, Ao, dt, M.ne, M.gas, M.g2x, M.g2w, M.uinf_e, cfl_ptr(M),
                       cfl_stride(M));
  else
    hipLaunchKernelGGL((k_p0_setup<3>), dim3(grid), dim3(256), 0, st, ut0, ft0, M.xv, M.NC, M.nbr, M.Lpk, M.NT, M.hE, pmax,
                       cfl, scale, u0, b, Ad, Ao, dt, M.ne, M.gas, M.g2x, M.g2w, M.uinf_e, cfl_ptr(M), cfl_stride(M));
  return hipGetLastError();
}

int arnoldi_blocks(int K) { return (K + 255) / 256; }

// Smallest register-resident basis size covering `need` vectors: 8, 16, 24,
// 32, then 48 (a kernel issues the loads of its whole size).
static int arn_nvm(int need) { return need <= 32 ? 8 * ((need + 7) / 8) : 48; }

template <int NVM>
static void launch_arn_b(int nblk, hipStream_t s, int K, int m, int j, double* Vb, double* W,
                         const double* part1, double* part2, int P, double* H, double* H2, double* wn0,
                         double* info, int* st, ArnSeg S) {
  hipLaunchKernelGGL(k_arn_b<NVM>, dim3(nblk), dim3(256), 0, s, K, m, j, Vb, W, part1, part2, P, H, H2, wn0, info,
                     st, S);
}

template <int V, int NF, bool NEXT, int NVM>
static void launch_arn_ca(int nblk, hipStream_t s, int K, int m, int j, const int* nbr, const double* Ad,
                          const double* Ao, double* Vb, const double* W, double* Wn, const double* part2,
                          double* part1, int P, double* H, double* H2, const double* wn0, double* info, int* st,
                          ArnSeg S) {
  hipLaunchKernelGGL((k_arn_ca<V, NF, NEXT, NVM>), dim3(nblk), dim3(256), 0, s, K, m, j, nbr, Ad, Ao, Vb, W, Wn,
                     part2, part1, P, H, H2, wn0, info, st, S);
}

template <int V, int NF, bool NEXT>
static void dispatch_arn_ca(int nvm, int nblk, hipStream_t s, int K, int m, int j, const int* nbr,
                            const double* Ad, const double* Ao, double* Vb, const double* W, double* Wn,
                            const double* part2, double* part1, int P, double* H, double* H2, const double* wn0,
                            double* info, int* st, ArnSeg S) {
  switch (nvm) {
    case 8: launch_arn_ca<V, NF, NEXT, 8>(nblk, s, K, m, j, nbr, Ad, Ao, Vb, W, Wn, part2, part1, P, H, H2, wn0, info, st, S); break;
    case 16: launch_arn_ca<V, NF, NEXT, 16>(nblk, s, K, m, j, nbr, Ad, Ao, Vb, W, Wn, part2, part1, P, H, H2, wn0, info, st, S); break;
    case 24: launch_arn_ca<V, NF, NEXT, 24>(nblk, s, K, m, j, nbr, Ad, Ao, Vb, W, Wn, part2, part1, P, H, H2, wn0, info, st, S); break;
    case 32: launch_arn_ca<V, NF, NEXT, 32>(nblk, s, K, m, j, nbr, Ad, Ao, Vb, W, Wn, part2, part1, P, H, H2, wn0, info, st, S); break;
    default: launch_arn_ca<V, NF, NEXT, 48>(nblk, s, K, m, j, nbr, Ad, Ao, Vb, W, Wn, part2, part1, P, H, H2, wn0, info, st, S); break;
  }
}

hipError_t launch_arnoldi(const DevMesh& M, int m, int nblk, const double* Ad, const double* Ao, const double* b,
                          double* Vb, double* H, double* part1, double* part2, double* info, int* st,
                          double* wn0, double* W2, double* H2, hipStream_t stream) {
  const int K = M.ne * M.V;
  const int P = m + 2;
  // one thread per row, at most 48 basis vectors held in registers; a batch
  // brings its own block tables (every block inside one solve's rows)
  if ((!M.brow0 && nblk != arnoldi_blocks(K)) || m < 1 || m > 48) return hipErrorInvalidValue;
  const ArnSeg S{M.brow0, M.brow1, M.bseg, M.sblk0};
  double* W[2] = {W2, W2 + K};
  hipLaunchKernelGGL(k_arn_beta, dim3(nblk), dim3(256), 0, stream, K, b, part1, P, st, S);
  hipLaunchKernelGGL(k_arn_start, dim3(nblk), dim3(256), 0, stream, K, m, b, part1, P, Vb, info, st, S);
  if (M.d == 2) hipLaunchKernelGGL((k_arn_a<4, 4>), dim3(nblk), dim3(256), 0, stream, K, M.nbr, Ad, Ao, Vb, W[0], part1, P, st, S);
  else hipLaunchKernelGGL((k_arn_a<5, 6>), dim3(nblk), dim3(256), 0, stream, K, M.nbr, Ad, Ao, Vb, W[0], part1, P, st, S);
  for (int j = 0; j < m; ++j) {
    double* Wc = W[j & 1];
    double* Wn = W[(j + 1) & 1];
    switch (arn_nvm(j + 1)) {
      case 8: launch_arn_b<8>(nblk, stream, K, m, j, Vb, Wc, part1, part2, P, H, H2, wn0, info, st, S); break;
      case 16: launch_arn_b<16>(nblk, stream, K, m, j, Vb, Wc, part1, part2, P, H, H2, wn0, info, st, S); break;
      case 24: launch_arn_b<24>(nblk, stream, K, m, j, Vb, Wc, part1, part2, P, H, H2, wn0, info, st, S); break;
      case 32: launch_arn_b<32>(nblk, stream, K, m, j, Vb, Wc, part1, part2, P, H, H2, wn0, info, st, S); break;
      default: launch_arn_b<48>(nblk, stream, K, m, j, Vb, Wc, part1, part2, P, H, H2, wn0, info, st, S); break;
    }
    const bool next = (j + 1 < m);
    const int nvm = arn_nvm(next ? j + 2 : j + 1);
    if (M.d == 2) {
      if (next) dispatch_arn_ca<4, 4, true>(nvm, nblk, stream, K, m, j, M.nbr, Ad, Ao, Vb, Wc, Wn, part2, part1, P, H, H2, wn0, info, st, S);
      else dispatch_arn_ca<4, 4, false>(nvm, nblk, stream, K, m, j, M.nbr, Ad, Ao, Vb, Wc, Wn, part2, part1, P, H, H2, wn0, info, st, S);
    } else {
      if (next) dispatch_arn_ca<5, 6, true>(nvm, nblk, stream, K, m, j, M.nbr, Ad, Ao, Vb, Wc, Wn, part2, part1, P, H, H2, wn0, info, st, S);
      else dispatch_arn_ca<5, 6, false>(nvm, nblk, stream, K, m, j, M.nbr, Ad, Ao, Vb, Wc, Wn, part2, part1, P, H, H2, wn0, info, st, S);
    }
  }
  return hipGetLastError();
}

hipError_t launch_phi1(int m, int nseg, const double* H, const double* H2, const double* info, double* y, int* fail,
                       hipStream_t st) {
  const size_t lds = (size_t)8 * (m + 1) * (m + 1) * 8;
  if (m + 1 <= 32) {
    // 8 matrices of order <= 32: 64 KiB, within the default limit
    hipLaunchKernelGGL(k_phi1<true>, dim3(nseg), dim3(256), lds, st, H, H2, m, info, y, fail);
    return hipGetLastError();
  }
  static size_t attr_lds = 0;  // largest size set so far
  if (lds > attr_lds) {
    hipError_t e = hipFuncSetAttribute((const void*)k_phi1<false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr_lds = lds;
  }
  hipLaunchKernelGGL(k_phi1<false>, dim3(nseg), dim3(256), lds, st, H, H2, m, info, y, fail);
  return hipGetLastError();
}

hipError_t launch_exp1_update(const DevMesh& M, int m, const double* Vb, const double* y, const double* info,
                              const double* u0, double* ut0, hipStream_t st) {
  const int K = M.ne * M.V;
  hipLaunchKernelGGL(k_exp1_update, dim3((K + 255) / 256), dim3(256), 0, st, K, M.V, Vb, y, info, u0, M.Lpk, M.NT,
                     ut0, M.sid, m + 1);
  return hipGetLastError();
}

hipError_t launch_exp1_prolong(const DevMesh& M, int m, const double* Vb, const double* y, const double* info,
                               const double* u0, const UpChain& c, hipStream_t st) {
  if (c.pmax < 1 || c.pmax > 4) return hipErrorInvalidValue;
  const int K = M.ne * M.V;
  const size_t T = (size_t)K * c.N[c.pmax - 1];
  hipLaunchKernelGGL(k_exp1_prolong, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, K, M.V, Vb, y, info, u0,
                     M.Lpk, M.NT, M.sid, m + 1, c);
  return hipGetLastError();
}

hipError_t launch_nbr_export(const DevMesh& M, int* out, hipStream_t st) {
  const int n = M.ne * M.NF;
  hipLaunchKernelGGL(k_nbr_export, dim3((n + 255) / 256), dim3(256), 0, st, M.nbr, out, n);
  return hipGetLastError();
}

hipError_t launch_sub(const double* a, const double* b, double* out, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, out, n);
  return hipGetLastError();
}

hipError_t launch_copy(const double* a, double* b, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

hipError_t launch_freestream(const DevMesh& M, int N, double* u, hipStream_t st) {
  const int cnt = M.ne * M.V * N;
  const double phi0 = (M.d == 2) ? 0.5 : 0.35355339059327373;
  hipLaunchKernelGGL(k_freestream, dim3((cnt + 255) / 256), dim3(256), 0, st, u, M.V, N, M.Lpk, M.NT, phi0, M.gas,
                     M.ne, M.uinf_e);
  return hipGetLastError();
}

hipError_t launch_jac_to_psi(const DevMesh& M, int N, double* Dm, hipStream_t st) {
  switch (N) {
    case 4: return jac_to_psi_t<4>(M, Dm, st);
    case 8: return jac_to_psi_t<8>(M, Dm, st);
    case 9: return jac_to_psi_t<9>(M, Dm, st);
    case 16: return jac_to_psi_t<16>(M, Dm, st);
    case 25: return jac_to_psi_t<25>(M, Dm, st);
    case 27: return jac_to_psi_t<27>(M, Dm, st);
    case 64: return jac_to_psi_t<64>(M, Dm, st);
    default: return hipErrorInvalidValue;
  }
}


// ---------------------------------------------------------------------------
// adjoint launchers
// ---------------------------------------------------------------------------
int residual_tile(int d, int p, int prec, int choice) {
#define TILE_OF(DD, PP) (prec == PREC_FP32 ? res_tile_of<DD, PP, float>(choice) : res_tile_of<DD, PP, double>(choice))
  if (d == 2) {
    switch (p) {
      case 0: return TILE_OF(2, 0);
      case 1: return TILE_OF(2, 1);
      case 2: return TILE_OF(2, 2);
      case 3: return TILE_OF(2, 3);
      case 4: return TILE_OF(2, 4);
      default: break;
    }
  } else {
    switch (p) {
      case 0: return TILE_OF(3, 0);
      case 1: return TILE_OF(3, 1);
      case 2: return TILE_OF(3, 2);
      case 3: return TILE_OF(3, 3);
      default: break;
    }
  }
#undef TILE_OF
  return 0;
}

size_t phitab_values(int d, int p) {
  const int Q = p + 2, N = (d == 2) ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1);
  const int QV = (d == 2) ? Q * Q : Q * Q * Q, QF = (d == 2) ? Q : Q * Q;
  return (size_t)(QV + 2 * d * QF) * N;
}

template <int D, int P, class R>
static hipError_t fill_phitab_t(const TabData& td, void* dst, hipStream_t st) {
  Tab<D, P, R> t;
  fill_tab(t, td);
  hipLaunchKernelGGL((k_fill_phitab<D, P, R>), dim3(8), dim3(256), 0, st, static_cast<R*>(dst), t);
  return hipGetLastError();
}

hipError_t launch_fill_phitab(const DevMesh& M, const TabData& td, int p, int prec, void* dst, hipStream_t st) {
#define CALL_FT(DD, PP) \
  (prec == PREC_FP32 ? fill_phitab_t<DD, PP, float>(td, dst, st) : fill_phitab_t<DD, PP, double>(td, dst, st))
  if (M.d == 2) {
    switch (p) {
      case 1: return CALL_FT(2, 1);
      case 2: return CALL_FT(2, 2);
      case 3: return CALL_FT(2, 3);
      case 4: return CALL_FT(2, 4);
      default: break;
    }
  } else {
    switch (p) {
      case 1: return CALL_FT(3, 1);
      case 2: return CALL_FT(3, 2);
      default: break;
    }
  }
#undef CALL_FT
  return hipErrorInvalidValue;
}

size_t jac_points_size(int d, int p) {
  const int V = d + 2, Q = p + 2;
  const int QV = (d == 2) ? Q * Q : Q * Q * Q, QF = (d == 2) ? Q : Q * Q;
  return (size_t)(QV * d + 2 * d * QF) * V * V;
}

namespace {
template <int D, int P>
hipError_t jac_points_only_t(const DevMesh& M, const TabData& td, const double* ut, double* bc, hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  launch_jac_points_t<D, P, double>(M, t, M.gas, ut, bc, st);
  return hipGetLastError();
}

template <int D, int P>
constexpr int adj_tile() {
  using C = Cfg<D, P>;
  constexpr int per = (C::V * C::N + C::QV * C::V + C::NF * C::QF * C::V) * 8;
  constexpr int eb = 40 * 1024 / per;
  return eb < 1 ? 1 : (eb > 32 ? 32 : eb);
}

template <int D, int P>
hipError_t adj_residual_t(const DevMesh& M, const TabData& td, const double* wt, const double* gadd,
                          const double* bc, double* out, hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  constexpr int EB = adj_tile<D, P>();
  const int grid = (M.ne + EB - 1) / EB;
  hipLaunchKernelGGL((k_adj_residual<D, P, EB>), dim3(grid), dim3(256), 0, st, wt, gadd, bc, M.nbr, M.ncode, M.ne, t,
                     out);
  return hipGetLastError();
}

template <int D, int P>
hipError_t drag_t(const DevMesh& M, const TabData& td, const double* ut, const double* dir, double scale,
                  double* part, double* gt, hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  Dir3 dv{{dir[0], dir[1], dir[2]}};
  if (D == 3 && M.NC == 27)
    hipLaunchKernelGGL((k_drag<D, P, true>), dim3((M.ne + 127) / 128), dim3(128), 0, st, ut, M.xv, M.NC, M.nbr,
                       M.ncode, M.ne, t, M.gas, dv, scale, part, gt);
  else
    hipLaunchKernelGGL((k_drag<D, P>), dim3((M.ne + 127) / 128), dim3(128), 0, st, ut, M.xv, M.NC, M.nbr, M.ncode,
                       M.ne, t, M.gas, dv, scale, part, gt);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_jac_points(const DevMesh& M, const TabData& td, int p, const double* ut, double* bc,
                             hipStream_t st) {
#define CALL_JP(DD, PP) jac_points_only_t<DD, PP>(M, td, ut, bc, st)
  if (M.d == 2) {
    switch (p) {
      case 1: return CALL_JP(2, 1);
      case 2: return CALL_JP(2, 2);
      case 3: return CALL_JP(2, 3);
      case 4: return CALL_JP(2, 4);
      default: break;
    }
  } else {
    switch (p) {
      case 1: return CALL_JP(3, 1);
      case 2: return CALL_JP(3, 2);
      case 3: return CALL_JP(3, 3);
      default: break;
    }
  }
#undef CALL_JP
  return hipErrorInvalidValue;
}

hipError_t launch_adj_residual(const DevMesh& M, const TabData& td, int p, const double* wt, const double* gadd,
                               const double* bc, double* out, hipStream_t st) {
#define CALL_AR(DD, PP) adj_residual_t<DD, PP>(M, td, wt, gadd, bc, out, st)
  if (M.d == 2) {
    switch (p) {
      case 1: return CALL_AR(2, 1);
      case 2: return CALL_AR(2, 2);
      case 3: return CALL_AR(2, 3);
      case 4: return CALL_AR(2, 4);
      default: break;
    }
  } else {
    switch (p) {
      case 1: return CALL_AR(3, 1);
      case 2: return CALL_AR(3, 2);
      case 3: return CALL_AR(3, 3);
      default: break;
    }
  }
#undef CALL_AR
  return hipErrorInvalidValue;
}

hipError_t launch_drag(const DevMesh& M, const TabData& td, int p, const double* ut, const double* dir, double scale,
                       double* part, double* gt, hipStream_t st) {
#define CALL_DR(DD, PP) drag_t<DD, PP>(M, td, ut, dir, scale, part, gt, st)
  if (M.d == 2) { EG_DISPATCH_P(2, p, CALL_DR) }
  else { EG_DISPATCH_P(3, p, CALL_DR) }
#undef CALL_DR
  return hipErrorInvalidValue;
}

// n = 100 (2D p = 4) is left out: its adjoint V-cycle diverged on every
// state tried, with the transposed kernel checked by a CPU emulation of its
// loops and (dR/du)^T w equal to the oracle's at every level; the cause is
// not established.
bool prk_tr_supported(int n) {
  return n == 16 || n == 36 || n == 64 || n == 100 || n == 40 || n == 135 || n == 320;
}

hipError_t launch_prk_stage_tr(const DevMesh& M, int n, const double* F, const int* perm, const double* rt,
                               const double* un, double* ut, double beta, hipStream_t st) {
  const int grid = (M.ne + 3) / 4;
  switch (n) {
    case 16: hipLaunchKernelGGL((k_prk_stage_tr<16>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    case 36: hipLaunchKernelGGL((k_prk_stage_tr<36>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    case 40: hipLaunchKernelGGL((k_prk_stage_tr<40>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    case 100: hipLaunchKernelGGL((k_prk_stage_trc<100>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    case 135: hipLaunchKernelGGL((k_prk_stage_trc<135>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    case 320: hipLaunchKernelGGL((k_prk_stage_trc<320>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    case 64: hipLaunchKernelGGL((k_prk_stage_tr<64>), dim3(grid), dim3(256), 0, st, F, perm, rt, un, ut, beta, M.ne); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_p0_transpose(const DevMesh& M, const double* Ad, const double* Ao, const double* dt, double* AdT,
                               double* AoT, hipStream_t st) {
  const int cnt = M.ne * (1 + M.NF);
  if (M.d == 2)
    hipLaunchKernelGGL((k_p0_transpose<4, 4>), dim3((cnt + 255) / 256), dim3(256), 0, st, Ad, Ao, dt, M.nbr, M.ncode,
                       AdT, AoT, M.ne);
  else
    hipLaunchKernelGGL((k_p0_transpose<5, 6>), dim3((cnt + 255) / 256), dim3(256), 0, st, Ad, Ao, dt, M.nbr, M.ncode,
                       AdT, AoT, M.ne);
  return hipGetLastError();
}

hipError_t launch_adj_p0_rhs(const DevMesh& M, const double* gt0, const double* dt, double* b, hipStream_t st) {
  const int cnt = M.ne * M.V;
  hipLaunchKernelGGL(k_adj_p0_rhs, dim3((cnt + 255) / 256), dim3(256), 0, st, gt0, M.Lpk, M.NT, dt, M.V, M.ne, b);
  return hipGetLastError();
}

hipError_t launch_trunc(const double* x, double* y, int N, int Nc, int rows, hipStream_t st) {
  const int cnt = rows * Nc;
  hipLaunchKernelGGL(k_trunc, dim3((cnt + 255) / 256), dim3(256), 0, st, x, y, N, Nc, rows);
  return hipGetLastError();
}

hipError_t launch_pad_add(double* x, const double* y, int N, int Nc, int rows, hipStream_t st) {
  const int cnt = rows * Nc;
  hipLaunchKernelGGL(k_pad_add, dim3((cnt + 255) / 256), dim3(256), 0, st, x, y, N, Nc, rows);
  return hipGetLastError();
}

hipError_t launch_expand_cfl(const DevMesh& M, const double* cfl_s, hipStream_t st) {
  hipLaunchKernelGGL(k_expand_cfl, dim3((M.ne + 255) / 256), dim3(256), 0, st, cfl_s, M.sid, M.cfl_e, M.ne);
  return hipGetLastError();
}

hipError_t launch_fill0(double* x, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill0, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n);
  return hipGetLastError();
}

int sum_blocks(size_t n) { return (int)std::min<size_t>(256, (n + 255) / 256); }

hipError_t launch_sum(const double* x, const double* y, size_t n, double* part, int take_sqrt, double* out,
                      hipStream_t st) {
  const int nb = sum_blocks(n);
  hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(256), 0, st, x, y, n, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, part, nb, take_sqrt, out);
  return hipGetLastError();
}

}  // namespace eg
