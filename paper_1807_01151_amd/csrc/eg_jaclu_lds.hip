// PRK element block assembly and LU for 64 < n = V N < 256 (2D p = 4:
// n = 100; 3D p = 2: n = 135) in FP64 on the matrix cores.
//
// The block (Section 2.3, end; Section 3.3, eq. (jac1), phi coordinates) is
//   Pt[(v,i),(w,j)] = delta_vw G_ij / dtau - Dt[(v,i),(w,j)],
//   Dt[(v,i),(w,j)] = sum_q X_vw[i][q] phi_j(q) - sum_k phi_i(k) C_k[v][w] phi_j(k),
//   X_vw[i][q] = sum_r d_r phi_i(q) B_q,r[v][w],
// with B and C the pointwise flux Jacobians (quadrature weights and metric
// included) that k_jac_points writes.  Dt is a product of an element
// matrix X (N x points) with the basis table phi (points x N): a dense
// contraction, which runs here on the 16 x 16 x 4 FP64 matrix-core
// instruction.  Its A operand is formed in registers from the LDS copies of
// d_r phi and B (the D directions summed per point), its B operand is read
// from the LDS basis table, and the accumulators of every (v, w, 16-row
// tile) job stay in registers until the whole block is done.
//
// One workgroup (eight wavefronts) per element.  LDS first holds the basis
// tables and the element's pointwise Jacobians (phase 1: 134 KB for 3D
// p = 2), then the assembled block, column-major (phase 2: 146 KB), on
// which the LU with partial pivoting runs in panels of 16 columns:
//   (a) wavefront 0 factorises the panel in registers (rows in lanes,
//       largest |a| as the pivot, ties to the lowest row slot), writes it
//       back and records the new logical row order: pivot rows first, in
//       pivot order, then the others;
//   (b) U12 = L11^{-1} A12 by forward substitution, one column per thread;
//   (c) A22 -= L21 U12 on the matrix cores, one 16 x 16 tile per
//       wavefront at a time.
// Rows are never moved: the logical order lives in s_prow and the factors
// are written out in it, column-major with perm[k] = the block row of the
// k-th pivot, the format of the other factorisation kernels (read by the
// PRK stage kernels).

#include <hip/hip_runtime.h>

#include "eg_common.h"
#include "eg_device.h"
#include "eg_launch.h"

namespace eg {

namespace {

template <int D, int P>
struct LdsLu {
  using C = Cfg<D, P>;
  static constexpr int V = C::V, N = C::N, Q = C::Q, QV = C::QV, QF = C::QF, NF = C::NF, n = C::NB;
  static constexpr int NPF = NF * QF;                 // face points
  static constexpr int KSV = QV / 4, KSF = NPF / 4;   // k-steps of four points
  static constexpr int NT16 = (N + 15) / 16;          // 16-row (or column) tiles of one variable's modes
  static constexpr int NW = 8;                        // wavefronts per element
  static constexpr int JOBS = V * V * NT16;           // (v, w, row tile) jobs of the assembly
  static constexpr int JPW = (JOBS + NW - 1) / NW;    // jobs per wavefront
  static constexpr int RPL = (n + 63) / 64;           // panel rows per lane
  static constexpr int LDA = n;                       // column stride of the block in LDS
  static constexpr int PER = (QV * D + NPF) * V * V;  // pointwise Jacobian values per element
  static constexpr int OFF_PH = QV * D * N;           // phase-1 LDS layout: d phi, phi, B | C
  static constexpr int OFF_B = OFF_PH + (QV + NPF) * N;
  static constexpr int PH1 = OFF_B + PER;
  static constexpr int PH2 = n * LDA;
  static constexpr int VALUES = PH1 > PH2 ? PH1 : PH2;
  static_assert(QV % 4 == 0 && NPF % 4 == 0, "k-steps of four points");
  static_assert(n > 64 && n < 192 && RPL <= 3, "block size");
};

template <int D, int P>
constexpr size_t jaclu_lds_bytes() {
  return (size_t)LdsLu<D, P>::VALUES * sizeof(double);
}

template <int D, int P>
__global__ __launch_bounds__(512, 1) void k_jaclu_lds(const double* __restrict__ BC, const double* __restrict__ Gpk,
                                                      int NT, const double* __restrict__ dtau, double* __restrict__ out,
                                                      int* __restrict__ perm, int* __restrict__ fail, int ne,
                                                      Tab<D, P, double> tab) {
  using L = LdsLu<D, P>;
  constexpr int V = L::V, N = L::N, Q = L::Q, QV = L::QV, QF = L::QF, NF = L::NF, n = L::n, NW = L::NW;
  constexpr int NPF = L::NPF, NT16 = L::NT16, JPW = L::JPW, JOBS = L::JOBS, RPL = L::RPL, LDA = L::LDA;
  extern __shared__ double s_mem[];
  __shared__ Tab<D, P, double> t;
  __shared__ int s_prow[n];
  const int e = blockIdx.x;
  if (e >= ne) return;  // whole workgroup
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int il = lane & 15, kq = lane >> 4;
  double* s_dph = s_mem;               // [QV][D][N]
  double* s_ph = s_mem + L::OFF_PH;    // [QV + NPF][N]: phi at the volume, then the face points
  double* s_B = s_mem + L::OFF_B;      // [QV][D][V][V] then [NPF][V][V]
  const double* s_C = s_B + QV * D * V * V;

  // ---- phase 1: tables and the element's pointwise Jacobians into LDS
  copy_tab(t, tab);
  stage<(L::PER + 511) / 512>(s_B, BC + (size_t)e * L::PER, L::PER, tid, 512);
  __syncthreads();
  for (int it = tid; it < QV * N; it += 512) {
    const int q = it / N, j = it % N;
    int iq[D], r0 = q;
#pragma unroll
    for (int r = 0; r < D; ++r) { iq[r] = r0 % Q; r0 /= Q; }
#pragma unroll
    for (int r = 0; r < D; ++r) s_dph[(q * D + r) * N + j] = dphi_vol<D, P, double>(t, j, iq, r);
    s_ph[q * N + j] = phi_vol<D, P, double>(t, j, iq);
  }
  for (int it = tid; it < NPF * N; it += 512) {
    const int lf = it / (QF * N), k = (it / N) % QF, j = it % N;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
    face_axes<D>(lf, ta);
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
    s_ph[(QV + lf * QF + k) * N + j] = phi_face<D, P, double>(t, j, lf, ta, ik);
  }
  for (int k = tid; k < n; k += 512) s_prow[k] = k;
  __syncthreads();

  // ---- assembly: job = (v, w, row tile it), two column tiles each
  int jv[JPW], jw[JPW], jt[JPW];
#pragma unroll
  for (int jj = 0; jj < JPW; ++jj) {
    const int job = wv + NW * jj;
    const int jb = job < JOBS ? job : 0;
    jt[jj] = jb % NT16;
    jv[jj] = (jb / NT16) / V;
    jw[jj] = (jb / NT16) % V;
  }
  dbl4_t acc[JPW][NT16];
#pragma unroll
  for (int jj = 0; jj < JPW; ++jj)
#pragma unroll
    for (int c = 0; c < NT16; ++c) acc[jj][c] = dbl4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
  for (int ks = 0; ks < L::KSV; ++ks) {
    const int q = 4 * ks + kq;
    double bf[NT16], dp[NT16][D];
#pragma unroll
    for (int c = 0; c < NT16; ++c) {
      const int j = 16 * c + il;
      bf[c] = j < N ? s_ph[q * N + j] : 0.0;
#pragma unroll
      for (int r = 0; r < D; ++r) dp[c][r] = j < N ? s_dph[(q * D + r) * N + j] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
      if (wv + NW * jj < JOBS) {
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < D; ++r) {
          const double d = NT16 == 1 ? dp[0][r] : (jt[jj] == 0 ? dp[0][r] : dp[NT16 - 1][r]);
          a = fma(d, s_B[((q * D + r) * V + jv[jj]) * V + jw[jj]], a);
        }
#pragma unroll
        for (int c = 0; c < NT16; ++c) acc[jj][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[c], acc[jj][c], 0, 0, 0);
      }
    }
  }
#pragma unroll 1
  for (int ks = 0; ks < L::KSF; ++ks) {
    const int fk = 4 * ks + kq;
    double bf[NT16];
#pragma unroll
    for (int c = 0; c < NT16; ++c) {
      const int j = 16 * c + il;
      bf[c] = j < N ? s_ph[(QV + fk) * N + j] : 0.0;
    }
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
      if (wv + NW * jj < JOBS) {
        const double fa = NT16 == 1 ? bf[0] : (jt[jj] == 0 ? bf[0] : bf[NT16 - 1]);
        const double a = -fa * s_C[(fk * V + jv[jj]) * V + jw[jj]];
#pragma unroll
        for (int c = 0; c < NT16; ++c) acc[jj][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[c], acc[jj][c], 0, 0, 0);
      }
    }
  }
  __syncthreads();  // phase-1 LDS is overwritten by the block below

  // ---- the block Pt = G/dtau - Dt, column-major in LDS
  double* A = s_mem;
  {
    const double idt = 1.0 / dtau[e];
    const double* G = Gpk + (size_t)e * NT;
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
      if (wv + NW * jj >= JOBS) continue;
#pragma unroll
      for (int c = 0; c < NT16; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * jt[jj] + kq + 4 * r, j = 16 * c + il;
          if (i < N && j < N) {
            double g = 0.0;
            if (jv[jj] == jw[jj]) g = ((i >= j) ? G[i * (i + 1) / 2 + j] : G[j * (j + 1) / 2 + i]) * idt;
            A[(jw[jj] * N + j) * LDA + jv[jj] * N + i] = g - acc[jj][c][r];
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- LU with partial pivoting, panels of 16 columns
#pragma unroll 1
  for (int kb = 0; kb < n; kb += 16) {
    const int nbk = min(16, n - kb);
    // (a) panel factorisation by wavefront 0
    if (wv == 0) {
      double pv[RPL][16];
      int prw[RPL], used[RPL];
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int lr = kb + lane + 64 * s;
        prw[s] = lr < n ? s_prow[lr] : 0;
        used[s] = lr < n ? -1 : 16;
#pragma unroll
        for (int c = 0; c < 16; ++c) pv[s][c] = (lr < n && c < nbk) ? A[(kb + c) * LDA + prw[s]] : 0.0;
      }
#pragma unroll
      for (int tt = 0; tt < 16; ++tt) {
        if (tt < nbk) {
          unsigned key = 0u;
#pragma unroll
          for (int s = 0; s < RPL; ++s)
            if (used[s] < 0)
              key = max(key, (__float_as_uint((float)fabs(pv[s][tt])) & ~255u) | (unsigned)(255 - (lane + 64 * s)));
          const unsigned kmax = wave_max_u32(key);
          const int ws = __builtin_amdgcn_readfirstlane(255 - (int)(kmax & 255u));
          const int wl = ws & 63, wsl = ws >> 6;
          double pr[16];
#pragma unroll
          for (int c = 0; c < 16; ++c) {
            double x = pv[0][c];
#pragma unroll
            for (int s = 1; s < RPL; ++s) x = (wsl == s) ? pv[s][c] : x;
            pr[c] = readlane_d(x, wl);
          }
          if (lane == 0 && !(fabs(pr[tt]) > 0.0)) atomicOr(fail, 1);
          const double ip = 1.0 / pr[tt];
#pragma unroll
          for (int s = 0; s < RPL; ++s) {
            if (lane + 64 * s == ws) {
              if (used[s] >= 0) atomicOr(fail, 4);  // the winner must be an unused row
              used[s] = tt;
            } else if (used[s] < 0) {
              const double l = pv[s][tt] * ip;
              pv[s][tt] = l;
              // fixed trip count (the bound is constant only once the step
              // loop is unrolled), so that pv stays in registers
#pragma unroll
              for (int c = 0; c < 16; ++c)
                if (c > tt) pv[s][c] = fma(-l, pr[c], pv[s][c]);
            }
          }
        }
      }
      // write the panel back and the new logical order of rows kb..n-1
      int before = 0;  // unused rows in the slots before this one
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int lr = kb + lane + 64 * s;
        const bool live = lr < n;
        const bool rest = live && used[s] < 0;
        const unsigned long long bal = __ballot(rest);
        const int below = __popcll(bal & ((1ull << lane) - 1ull));
        if (live) {
#pragma unroll
          for (int c = 0; c < 16; ++c)
            if (c < nbk) A[(kb + c) * LDA + prw[s]] = pv[s][c];
          const int pos = rest ? kb + nbk + before + below : kb + used[s];
          s_prow[pos] = prw[s];
        }
        before += __popcll(bal);
      }
    }
    __syncthreads();
    const int k1 = kb + nbk, m = n - k1;
    if (m <= 0) break;
    // (b) U12 = L11^{-1} A12, one column per thread
    if (tid < m) {
      const int col = k1 + tid;
      double y[16];
#pragma unroll
      for (int tt = 0; tt < 16; ++tt) y[tt] = tt < nbk ? A[col * LDA + s_prow[kb + tt]] : 0.0;
#pragma unroll
      for (int tt = 1; tt < 16; ++tt) {
        if (tt < nbk) {
          const int pr = s_prow[kb + tt];
#pragma unroll
          for (int t2 = 0; t2 < 16; ++t2)
            if (t2 < tt) y[tt] = fma(-A[(kb + t2) * LDA + pr], y[t2], y[tt]);
        }
      }
#pragma unroll
      for (int tt = 1; tt < 16; ++tt)
        if (tt < nbk) A[col * LDA + s_prow[kb + tt]] = y[tt];
    }
    __syncthreads();
    // (c) A22 -= L21 U12 on the matrix cores
    const int T = (m + 15) / 16;
#pragma unroll 1
    for (int tile = wv; tile < T * T; tile += NW) {
      const int ti = tile / T, tj = tile % T;
      const int cc = k1 + 16 * tj + il;
      const bool cok = cc < n;
      int crow[4];
      dbl4_t c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = k1 + 16 * ti + kq + 4 * r;
        crow[r] = lr < n ? s_prow[lr] : -1;
        c[r] = (crow[r] >= 0 && cok) ? A[cc * LDA + crow[r]] : 0.0;
      }
      const int alr = k1 + 16 * ti + il;
      const int arow = alr < n ? s_prow[alr] : -1;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + kq;
        const bool kok = k < nbk;
        const double a = (arow >= 0 && kok) ? -A[(kb + k) * LDA + arow] : 0.0;
        const double b = (kok && cok) ? A[cc * LDA + s_prow[kb + k]] : 0.0;
        c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (crow[r] >= 0 && cok) A[cc * LDA + crow[r]] = c[r];
    }
    __syncthreads();
  }

  // ---- factors in pivot order, column-major, and the permutation
  double* o = out + (size_t)e * n * n;
  for (int it = tid; it < n * n; it += 512) {
    const int col = it / n, k = it % n;
    o[it] = A[col * LDA + s_prow[k]];
  }
  for (int k = tid; k < n; k += 512) perm[(size_t)e * n + k] = s_prow[k];
}

template <int D, int P>
hipError_t jaclu_lds_t(const DevMesh& M, const TabData& td, const double* bc, const double* dtau, double* out,
                       int* perm, int* fail, hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  const size_t lds = jaclu_lds_bytes<D, P>();
  static bool attr = false;  // set once: not a stream operation, so also fine while capturing
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jaclu_lds<D, P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_jaclu_lds<D, P>), dim3(M.ne), dim3(512), lds, st, bc, M.Gpk, M.NT, dtau, out, perm, fail,
                     M.ne, t);
  return hipGetLastError();
}

}  // namespace

bool jaclu_lds_supported(int d, int p) { return (d == 2 && p == 4) || (d == 3 && p == 2); }

hipError_t launch_jaclu_lds(const DevMesh& M, const TabData& td, int p, const double* bc, const double* dtau,
                            double* out, int* perm, int* fail, hipStream_t st) {
  if (M.d == 2 && p == 4) return jaclu_lds_t<2, 4>(M, td, bc, dtau, out, perm, fail, st);
  if (M.d == 3 && p == 2) return jaclu_lds_t<3, 2>(M, td, bc, dtau, out, perm, fail, st);
  return hipErrorInvalidValue;
}

}  // namespace eg
