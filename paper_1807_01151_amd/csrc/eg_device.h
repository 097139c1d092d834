// Device helpers shared by the kernel translation units of the HIP path:
// the multilinear element map, face-point index maps, basis values from the
// 1D tables, LDS staging, and wavefront reductions and broadcasts.
#pragma once

#include <hip/hip_runtime.h>

#include "eg_common.h"
#include "eg_launch.h"
#include "eg_physics.h"

namespace eg {

// Orders LDS accesses between the lanes of one wavefront: a store by one
// lane before the call is seen by a load of another lane after it.  Without
// it the per-thread memory model lets the compiler hoist a load above
// another lane's (conditional) store to the same address.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The same for data that may live in global memory: workgroup-scope fences
// (every earlier store of the wavefront complete before its later loads).
__device__ __forceinline__ void wave_mem_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The numerical flux selected for the handle (uniform over a launch).
template <int D, class SL, class SR, class S, class R>
__device__ __forceinline__ void num_flux(const SL* UL, const SR* UR, const real_t<S>* nh, S* F,
                                         const GasT<R>& gas) {
  if (gas.flux == FLUX_ROE) roe<D>(UL, UR, nh, F, real_t<S>(gas.g));
  else rusanov<D>(UL, UR, nh, F, real_t<S>(gas.g));
}

// Four FP64 accumulators of a 16 x 16 x 4 FP64 matrix-core product (lane l
// holds rows (l >> 4) + 4 r, r = 0..3, of column l & 15).
typedef double dbl4_t __attribute__((ext_vector_type(4)));

// Kernel-argument copy of the 1D tables of one order (host side).
template <int D, int P, class R>
inline void fill_tab(Tab<D, P, R>& t, const TabData& td) {
  for (int i = 0; i < P + 2; ++i) { t.x[i] = R(td.x[i]); t.w[i] = R(td.w[i]); }
  for (int a = 0; a <= P; ++a) {
    for (int i = 0; i < P + 2; ++i) { t.L[a][i] = R(td.L[a][i]); t.dL[a][i] = R(td.dL[a][i]); }
    t.Lb[a][0] = R(td.Lb[a][0]);
    t.Lb[a][1] = R(td.Lb[a][1]);
  }
  for (int k = 0; k < Cfg<D, P>::N; ++k)
    for (int r = 0; r < 3; ++r) t.m[k][r] = (int8_t)td.m[k][r];
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Element map (biquadratic through nine nodes in 2D, trilinear in 3D): the
// vectors c[r] with c[r] . (dx/dxi_r') = det delta_rr', i.e.
// det * grad_x = sum_r c[r] d/dxi_r; (2s-1) c[r] is the scaled outward
// normal of face (r, s).
template <int D, class R>
__device__ __forceinline__ void geom(const R* X, const R* xi, R c[D][D], R& det) {
  R t[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int a = 0; a < D; ++a) t[r][a] = R(0);
  if constexpr (D == 2) {
    // quadratic Lagrange factors through -1, 0, 1 and their derivatives
    const R x = xi[0], y = xi[1];
    const R lx[3] = {R(0.5) * x * (x - R(1)), R(1) - x * x, R(0.5) * x * (x + R(1))};
    const R dx[3] = {x - R(0.5), R(-2) * x, x + R(0.5)};
    const R ly[3] = {R(0.5) * y * (y - R(1)), R(1) - y * y, R(0.5) * y * (y + R(1))};
    const R dy[3] = {y - R(0.5), R(-2) * y, y + R(0.5)};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      R s0[2] = {R(0), R(0)}, s1[2] = {R(0), R(0)};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          s0[q] += dx[a] * X[(a + 3 * b) * 2 + q];
          s1[q] += lx[a] * X[(a + 3 * b) * 2 + q];
        }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        t[0][q] += ly[b] * s0[q];
        t[1][q] += dy[b] * s1[q];
      }
    }
    c[0][0] = t[1][1]; c[0][1] = -t[1][0];
    c[1][0] = -t[0][1]; c[1][1] = t[0][0];
    det = t[0][0] * t[1][1] - t[0][1] * t[1][0];
  } else {
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
      R g[D];
#pragma unroll
      for (int r = 0; r < D; ++r) {
        R v = R(1);
#pragma unroll
        for (int q = 0; q < D; ++q) {
          R s = ((k >> q) & 1) ? R(1) : R(-1);
          v *= (q == r) ? R(0.5) * s : R(0.5) * (R(1) + s * xi[q]);
        }
        g[r] = v;
      }
#pragma unroll
      for (int r = 0; r < D; ++r)
#pragma unroll
        for (int a = 0; a < D; ++a) t[r][a] += g[r] * X[k * D + a];
    }
    c[0][0] = t[1][1] * t[2][2] - t[1][2] * t[2][1];
    c[0][1] = t[1][2] * t[2][0] - t[1][0] * t[2][2];
    c[0][2] = t[1][0] * t[2][1] - t[1][1] * t[2][0];
    c[1][0] = t[2][1] * t[0][2] - t[2][2] * t[0][1];
    c[1][1] = t[2][2] * t[0][0] - t[2][0] * t[0][2];
    c[1][2] = t[2][0] * t[0][1] - t[2][1] * t[0][0];
    c[2][0] = t[0][1] * t[1][2] - t[0][2] * t[1][1];
    c[2][1] = t[0][2] * t[1][0] - t[0][0] * t[1][2];
    c[2][2] = t[0][0] * t[1][1] - t[0][1] * t[1][0];
    det = t[0][0] * c[0][0] + t[0][1] * c[0][1] + t[0][2] * c[0][2];
  }
}

// Triquadratic map through 27 nodes (node a + 3b + 9c at reference point
// (a-1, b-1, c-1); curved hexes, read from global memory): the same c[r] and
// det as geom<3>.  X holds the element's 81 FP64 node coordinates.
template <class R>
__device__ __forceinline__ void geom_q3(const double* __restrict__ X, const R* xi, R c[3][3], R& det) {
  R l[3][3], dl[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const R z = xi[r];
    l[r][0] = R(0.5) * z * (z - R(1));
    l[r][1] = R(1) - z * z;
    l[r][2] = R(0.5) * z * (z + R(1));
    dl[r][0] = z - R(0.5);
    dl[r][1] = R(-2) * z;
    dl[r][2] = z + R(0.5);
  }
  R t[3][3];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int a = 0; a < 3; ++a) t[r][a] = R(0);
  for (int cc = 0; cc < 3; ++cc)
    for (int b = 0; b < 3; ++b) {
      // nodes (0..2, b, cc): partial sums over a of l and dl
      R sl[3] = {R(0), R(0), R(0)}, sd[3] = {R(0), R(0), R(0)};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double* x = X + (a + 3 * b + 9 * cc) * 3;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const R v = R(x[q]);
          sl[q] += l[0][a] * v;
          sd[q] += dl[0][a] * v;
        }
      }
      const R w0 = l[1][b] * l[2][cc], w1 = dl[1][b] * l[2][cc], w2 = l[1][b] * dl[2][cc];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        t[0][q] += w0 * sd[q];
        t[1][q] += w1 * sl[q];
        t[2][q] += w2 * sl[q];
      }
    }
  c[0][0] = t[1][1] * t[2][2] - t[1][2] * t[2][1];
  c[0][1] = t[1][2] * t[2][0] - t[1][0] * t[2][2];
  c[0][2] = t[1][0] * t[2][1] - t[1][1] * t[2][0];
  c[1][0] = t[2][1] * t[0][2] - t[2][2] * t[0][1];
  c[1][1] = t[2][2] * t[0][0] - t[2][0] * t[0][2];
  c[1][2] = t[2][0] * t[0][1] - t[2][1] * t[0][0];
  c[2][0] = t[0][1] * t[1][2] - t[0][2] * t[1][1];
  c[2][1] = t[0][2] * t[1][0] - t[0][0] * t[1][2];
  c[2][2] = t[0][0] * t[1][1] - t[0][1] * t[1][0];
  det = t[0][0] * c[0][0] + t[0][1] * c[0][1] + t[0][2] * c[0][2];
}

// Element map at xi: the nine-node quad map or the trilinear hex map from the
// staged nodes Xs, or, in the instantiations for curved hexes (CQ), the
// triquadratic map from the element's 27 nodes Xg in global memory.  A
// compile-time choice: a run-time branch would give the straight-hex kernels
// the register footprint of both paths.
template <int D, bool CQ, class R>
__device__ __forceinline__ void geom_any(const R* Xs, const double* __restrict__ Xg, const R* xi, R c[D][D],
                                         R& det) {
  if constexpr (D == 3 && CQ) geom_q3<R>(Xg, xi, c, det);
  else geom<D>(Xs, xi, c, det);
}

// Tangential axes of face lf (ascending, skipping the normal axis lf / 2);
// every index is static, so the caller's array stays in registers.
template <int D>
__device__ __forceinline__ void face_axes(int lf, int* ta) {
  const int r = lf >> 1;
#pragma unroll
  for (int q = 0; q < D - 1; ++q) ta[q] = q + (q >= r ? 1 : 0);
}

// Point index on the neighbour's face seen from this element's face point
// with tangential Gauss indices ik.
template <int D, int Q>
__device__ __forceinline__ void nb_face_index(int code, const int* ik, int* jk) {
  if constexpr (D == 2) {
    jk[0] = ((code >> 4) & 1) ? Q - 1 - ik[0] : ik[0];
  } else {
    int a = ((code >> 3) & 1) ? ik[1] : ik[0];
    int b = ((code >> 3) & 1) ? ik[0] : ik[1];
    jk[0] = ((code >> 4) & 1) ? Q - 1 - a : a;
    jk[1] = ((code >> 5) & 1) ? Q - 1 - b : b;
  }
}

// phi_k at face lf, tangential Gauss indices ik.
template <int D, int P, class R>
__device__ __forceinline__ R phi_face(const Tab<D, P, R>& t, int k, int lf, const int* ta, const int* ik) {
  R v = t.Lb[t.m[k][lf >> 1]][lf & 1];
#pragma unroll
  for (int q = 0; q < D - 1; ++q) v *= t.L[t.m[k][ta[q]]][ik[q]];
  return v;
}

template <int D, int P, class R>
__device__ __forceinline__ R phi_vol(const Tab<D, P, R>& t, int k, const int* iq) {
  R v = t.L[t.m[k][0]][iq[0]];
#pragma unroll
  for (int r = 1; r < D; ++r) v *= t.L[t.m[k][r]][iq[r]];
  return v;
}

template <int D, int P, class R>
__device__ __forceinline__ R dphi_vol(const Tab<D, P, R>& t, int k, const int* iq, int r) {
  R v = R(1);
#pragma unroll
  for (int q = 0; q < D; ++q) v *= (q == r) ? t.dL[t.m[k][q]][iq[q]] : t.L[t.m[k][q]][iq[q]];
  return v;
}

template <int D, int P, class R>
__device__ __forceinline__ void copy_tab(Tab<D, P, R>& dst, const Tab<D, P, R>& src) {
  const int n = sizeof(Tab<D, P, R>) / 4;
  const uint32_t* s = reinterpret_cast<const uint32_t*>(&src);
  uint32_t* d = reinterpret_cast<uint32_t*>(&dst);
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

// Copies cnt values from global memory into LDS (converting to the LDS
// type); each thread issues all of its (at most ITEMS) loads before its
// stores, so the global latency is paid once instead of once per element.
template <int ITEMS, class DT, class ST>
__device__ __forceinline__ void stage(DT* dst, const ST* __restrict__ src, int cnt, int tid, int nthr) {
  ST r[ITEMS];
#pragma unroll
  for (int u = 0; u < ITEMS; ++u) {
    const int i = tid + u * nthr;
    r[u] = (i < cnt) ? src[i] : ST(0);
  }
#pragma unroll
  for (int u = 0; u < ITEMS; ++u) {
    const int i = tid + u * nthr;
    if (i < cnt) dst[i] = DT(r[u]);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave-wide maximum of an unsigned key with DPP moves (no LDS round trip):
// quad permutations, row shifts by 4 and 8, then the row broadcasts of lanes
// 15 and 31; lane 63 ends up with the maximum, which is returned uniformly.
// Lanes whose DPP source is disabled keep their own value (max is idempotent).
__device__ __forceinline__ unsigned wave_max_u32(unsigned x) {
  int v = (int)x;
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xE, false));  // row_shr:4
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xC, false));  // row_shr:8
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false));  // row_bcast:15
  v = (int)max((unsigned)v, (unsigned)__builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ double readlane_d(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane_d(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
// Value of x in the lane at byte address addr (lane * 4) through the LDS
// crossbar (no LDS storage is used).
__device__ __forceinline__ double bperm_d(double x, int addr) {
  const int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(x));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(x));
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float bperm_d(float x, int addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}

}  // namespace eg
