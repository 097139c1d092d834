// Matrix-free Jacobian-vector product of the DG residual (Section 3.3,
// eqs. (jac1) and (jac2): the element-diagonal and neighbour blocks applied
// together), (dR_p/du)(u) v, by forward-mode differentiation of the residual
// of Section 3.1, eq. (euler3): every quadrature point evaluates the state
// and the flux as dual numbers with one tangent component (value from u,
// tangent from v), so the tangent of the volume flux, of the numerical flux
// (Rusanov or Roe; both traces perturbed on interior faces) and of the
// ghost states on
// boundary faces is exact, with the same tie rules for |x| and max as
// the block Jacobians.  The projection onto the test functions is the
// residual's.  Phi coordinates (ut = T^T u, vt = T^T v, output T^{-1} J v),
// as every smoother kernel.
//
// One workgroup per element; the basis values come from the 1D tables in
// LDS.  Not on the V-cycle path (the smoother uses the assembled element
// blocks), so it favours simplicity: any order the residual supports.

#include <hip/hip_runtime.h>

#include "eg_common.h"
#include "eg_device.h"
#include "eg_launch.h"
#include "eg_physics.h"

namespace eg {

namespace {

template <int D, int P, bool CQ = false>
__global__ __launch_bounds__(256) void k_tangent(const double* __restrict__ ut, const double* __restrict__ vt,
                                                 double* __restrict__ jv, const double* __restrict__ xv, int nc,
                                                 const int* __restrict__ nbr, const uint8_t* __restrict__ ncode,
                                                 int ne, Tab<D, P, double> tab, Gas gas,
                                                 const double* __restrict__ uinf_e) {
  using C = Cfg<D, P>;
  using T1 = Dual<1, double>;
  constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, NC = C::NC;
  __shared__ Tab<D, P, double> t;
  __shared__ double s_u[V * N], s_v[V * N], s_x[NC * D];
  __shared__ double s_fc[QV * V * D];      // w_q d(F_v . c_r)
  __shared__ double s_ff[NF * QF * V];     // w_k |n dsigma| dF~_v
  const int e = blockIdx.x, tid = threadIdx.x;
  if (e >= ne) return;
  copy_tab(t, tab);
  for (int i = tid; i < V * N; i += blockDim.x) {
    s_u[i] = ut[(size_t)e * V * N + i];
    s_v[i] = vt[(size_t)e * V * N + i];
  }
  if (!CQ)
    for (int i = tid; i < NC * D; i += blockDim.x) s_x[i] = xv[(size_t)e * NC * D + i];
  __syncthreads();
  // volume points
  for (int q = tid; q < QV; q += blockDim.x) {
    int iq[D], r0 = q;
    double xi[D], wq = 1.0;
#pragma unroll
    for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; xi[r] = t.x[iq[r]]; wq *= t.w[iq[r]]; }
    T1 U[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double a = 0.0, b = 0.0;
      for (int k = 0; k < N; ++k) {
        const double ph = phi_vol<D, P, double>(t, k, iq);
        a += s_u[v * N + k] * ph;
        b += s_v[v * N + k] * ph;
      }
      U[v] = T1(a);
      U[v].d[0] = b;
    }
    double c[D][D], det;
    geom_any<D, CQ>(s_x, xv + (size_t)e * nc * D, xi, c, det);
#pragma unroll
    for (int r = 0; r < D; ++r) {
      T1 F[V];
      flux_n<D>(U, c[r], F, gas.g);
#pragma unroll
      for (int v = 0; v < V; ++v) s_fc[(q * V + v) * D + r] = wq * F[v].d[0];
    }
  }
  // face points
  for (int it = tid; it < NF * QF; it += blockDim.x) {
    const int lf = it / QF, k = it % QF;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
    face_axes<D>(lf, ta);
    double xi[D], wk = 1.0;
    xi[lf >> 1] = (lf & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; xi[ta[q]] = t.x[ik[q]]; wk *= t.w[ik[q]]; }
    T1 UL[V], UR[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double a = 0.0, b = 0.0;
      for (int j = 0; j < N; ++j) {
        const double ph = phi_face<D, P, double>(t, j, lf, ta, ik);
        a += s_u[v * N + j] * ph;
        b += s_v[v * N + j] * ph;
      }
      UL[v] = T1(a);
      UL[v].d[0] = b;
    }
    double c[D][D], det;
    geom_any<D, CQ>(s_x, xv + (size_t)e * nc * D, xi, c, det);
    double nh[D], a2 = 0.0;
    const double sg = (lf & 1) ? 1.0 : -1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) { nh[a] = sg * c[lf >> 1][a]; a2 += nh[a] * nh[a]; }
    const double area = sqrt(a2);
#pragma unroll
    for (int a = 0; a < D; ++a) nh[a] /= area;
    const int nb = nbr[(size_t)e * NF + lf];
    if (nb >= 0) {
      const int code = ncode[(size_t)e * NF + lf];
      const int lf2 = code & 7;
      int ta2[D - 1 > 0 ? D - 1 : 1], jk[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf2, ta2);
      nb_face_index<D, Q>(code, ik, jk);
      const double* un = ut + (size_t)nb * V * N;
      const double* vn = vt + (size_t)nb * V * N;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < N; ++j) {
          const double ph = phi_face<D, P, double>(t, j, lf2, ta2, jk);
          a += un[v * N + j] * ph;
          b += vn[v * N + j] * ph;
        }
        UR[v] = T1(a);
        UR[v].d[0] = b;
      }
    } else if (nb == NB_WALL) {
      ghost_wall<D>(UL, nh, UR);
    } else {
      double Ui[V];
#pragma unroll
      for (int v = 0; v < V; ++v) Ui[v] = uinf_e ? uinf_e[(size_t)e * V + v] : gas.Uinf[v];
      ghost_far<D>(UL, nh, UR, Ui, gas.g);
    }
    T1 F[V];
    num_flux<D>(UL, UR, nh, F, gas);
#pragma unroll
    for (int v = 0; v < V; ++v) s_ff[(lf * QF + k) * V + v] = wk * area * F[v].d[0];
  }
  __syncthreads();
  // projection onto the test functions
  for (int it = tid; it < V * N; it += blockDim.x) {
    const int v = it / N, i = it % N;
    double acc = 0.0;
    for (int q = 0; q < QV; ++q) {
      int iq[D], r0 = q;
#pragma unroll
      for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
#pragma unroll
      for (int r = 0; r < D; ++r) acc += dphi_vol<D, P, double>(t, i, iq, r) * s_fc[(q * V + v) * D + r];
    }
    for (int lf = 0; lf < NF; ++lf) {
      int ta[D - 1 > 0 ? D - 1 : 1];
      face_axes<D>(lf, ta);
      for (int k = 0; k < QF; ++k) {
        int ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
#pragma unroll
        for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
        acc -= phi_face<D, P, double>(t, i, lf, ta, ik) * s_ff[(lf * QF + k) * V + v];
      }
    }
    jv[(size_t)e * V * N + it] = acc;
  }
}

template <int D, int P>
hipError_t tangent_t(const DevMesh& M, const TabData& td, const double* ut, const double* vt, double* jv,
                     hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  if (D == 3 && M.NC == 27)
    hipLaunchKernelGGL((k_tangent<D, P, true>), dim3(M.ne), dim3(128), 0, st, ut, vt, jv, M.xv, M.NC, M.nbr, M.ncode,
                       M.ne, t, M.gas, M.uinf_e);
  else
    hipLaunchKernelGGL((k_tangent<D, P>), dim3(M.ne), dim3(128), 0, st, ut, vt, jv, M.xv, M.NC, M.nbr, M.ncode, M.ne,
                       t, M.gas, M.uinf_e);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tangent(const DevMesh& M, const TabData& td, int p, const double* ut, const double* vt, double* jv,
                          hipStream_t st) {
  if (M.d == 2) {
    switch (p) {
      case 0: return tangent_t<2, 0>(M, td, ut, vt, jv, st);
      case 1: return tangent_t<2, 1>(M, td, ut, vt, jv, st);
      case 2: return tangent_t<2, 2>(M, td, ut, vt, jv, st);
      case 3: return tangent_t<2, 3>(M, td, ut, vt, jv, st);
      case 4: return tangent_t<2, 4>(M, td, ut, vt, jv, st);
      default: break;
    }
  } else {
    switch (p) {
      case 0: return tangent_t<3, 0>(M, td, ut, vt, jv, st);
      case 1: return tangent_t<3, 1>(M, td, ut, vt, jv, st);
      case 2: return tangent_t<3, 2>(M, td, ut, vt, jv, st);
      case 3: return tangent_t<3, 3>(M, td, ut, vt, jv, st);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace eg
