// PRK element block assembly and LU for 64 < n = V N < 256 (2D p = 4:
// n = 100; 3D p = 2: n = 135) on the matrix cores: FP64 for the FP64
// smoother, FP32 with FP32 accumulation for the mixed-precision one.
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
//       largest |a| as the pivot, ties to the lowest row slot, the pivot
//       row broadcast by lane reads), writes it back, records the new logical
//       row order (pivot rows first, in pivot order, then the others) and
//       forms L11^{-1};
//   (b, c) every wavefront takes a 16-column tile of the trailing part:
//       U12 = L11^{-1} A12 on the matrix cores, whose accumulators are in
//       the B-operand layout of the next product, then A22 -= L21 U12 tile
//       by tile (waves sharing a column tile split its row tiles).
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

template <int D, int P, class R>
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

template <int D, int P, class R>
constexpr size_t jaclu_lds_bytes() {
  return (size_t)LdsLu<D, P, R>::VALUES * sizeof(R);
}

// The 16 x 16 x 4 matrix-core product of the arithmetic type: FP64 for the
// FP64 smoother, FP32 (FP32 accumulation) for the mixed-precision one.  The
// accumulator layouts differ: lane l holds rows (l >> 4) + 4 r (FP64) or
// 4 (l >> 4) + r (FP32) of column l & 15; the A operand is A[l & 15][l >> 4]
// and the B operand B[l >> 4][l & 15] in both (checked on the GPU by
// in-bounds probes).
typedef float flt4_t __attribute__((ext_vector_type(4)));
template <class R> struct Mfma;
template <> struct Mfma<double> {
  using acc = dbl4_t;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
};
template <> struct Mfma<float> {
  using acc = flt4_t;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
};

// Panel factorisation of columns kb .. kb + nbk - 1 of the LDS block by one
// wavefront: the rows of logical positions kb .. n - 1 in its lanes (NS
// slots of 64, as many as rows remain), the panel in registers.  A holds
// the columns from cb on (column c at A + (c - cb) LDA).  Pivot: the largest |a| among the unused rows
// (float keys with the row slot in the low bits, ties to the lowest slot);
// the pivot row is read out of the winning lane's registers into
// scalar registers (the slot index is uniform: a scalar branch).  Then the
// panel is written back, the new logical row order recorded (pivot rows
// first, in pivot order, then the others in their previous order) and
// L11^{-1} formed in s_linv (row-major, unit lower triangular, identity past
// nbk).
// Pointers into LDS, typed as such so that a called function addresses
// them with LDS instructions (a generic pointer would take flat accesses).
template <class T>
using lds_p = __attribute__((address_space(3))) T*;

template <int NS, int n, int LDA, class R>
__device__ __forceinline__ void panel_body(lds_p<R> A, int cb, lds_p<const int> s_in, lds_p<int> s_prow,
                                           lds_p<R> s_linv, int* fail, int kb, int nbk, int lane) {
  // the row slot index in the low bits of the key: 8 bits up to n = 256, 9 up to 512
  constexpr unsigned KM = n <= 256 ? 255u : 511u;
  static_assert(n <= 512, "row index bits of the pivot key");
  R pv[NS][16];
  int prw[NS], used[NS];
  int bad = 0;  // a zero or non-finite pivot, reported once per panel
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int lr = kb + lane + 64 * s;
    prw[s] = lr < n ? s_in[lr] : 0;
    used[s] = lr < n ? -1 : 16;
#pragma unroll
    for (int c = 0; c < 16; ++c) pv[s][c] = (lr < n && c < nbk) ? A[(kb + c - cb) * LDA + prw[s]] : R(0);
  }
#pragma unroll
  for (int tt = 0; tt < 16; ++tt) {
    if (tt < nbk) {
      unsigned key = 0u;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const unsigned ks = (__float_as_uint((float)fabs(pv[s][tt])) & ~KM) | (KM - (unsigned)(lane + 64 * s));
        key = max(key, used[s] < 0 ? ks : 0u);
      }
      const unsigned kmax = wave_max_u32(key);
      const int ws = __builtin_amdgcn_readfirstlane((int)(KM - (kmax & KM)));
      const int wl = ws & 63, wsl = ws >> 6;
      R pr[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) pr[c] = R(0);
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (wsl == s) {
#pragma unroll
          for (int c = 0; c < 16; ++c)
            if (c >= tt) pr[c] = readlane_d(pv[s][c], wl);
        }
      if (!(fabs(pr[tt]) > R(0))) bad = 1;
      const R ip = R(1) / pr[tt];
      // rows not used as pivots take multiplier l, the others l = 0 (their
      // values are then left unchanged by the update)
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (lane + 64 * s == ws) used[s] = tt;
        const bool act = used[s] < 0;
        const R l = act ? pv[s][tt] * ip : R(0);
        pv[s][tt] = act ? l : pv[s][tt];
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c > tt) pv[s][c] = fma(-l, pr[c], pv[s][c]);
      }
    }
  }
  if (lane == 0 && bad) atomicOr(fail, 1);
  if (s_in != s_prow)
    for (int i = lane; i < kb; i += 64) s_prow[i] = s_in[i];  // the rows already pivoted keep their places
  int before = 0;  // unused rows in the slots before this one
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int lr = kb + lane + 64 * s;
    const bool live = lr < n;
    const bool rest = live && used[s] < 0;
    const unsigned long long bal = __ballot(rest);
    const int below = __popcll(bal & ((1ull << lane) - 1ull));
    if (live) {
#pragma unroll
      for (int c = 0; c < 16; ++c)
        if (c < nbk) A[(kb + c - cb) * LDA + prw[s]] = pv[s][c];
      const int pos = rest ? kb + nbk + before + below : kb + used[s];
      s_prow[pos] = prw[s];
    }
    before += __popcll(bal);
  }
  // lane j < 16 forms column j of L11^{-1} by forward substitution from the
  // panel and the row order the other lanes have just written
  wave_mem_sync();
  if (lane < 16) {
    R x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      R v = (t == lane) ? R(1) : R(0);
      if (t < nbk) {
        const int pr = s_prow[kb + t];
#pragma unroll
        for (int t2 = 0; t2 < 16; ++t2)
          if (t2 < t) v = fma(-A[(kb + t2 - cb) * LDA + pr], x[t2], v);
      }
      x[t] = v;
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) s_linv[t * 16 + lane] = x[t];
  }
}

// The panel as a called function (one copy per slot count, so that the
// kernel holds only the live variant's registers).
template <int NS, int n, int LDA, class R>
__device__ __noinline__ void panel_wave(lds_p<R> A, int cb, lds_p<const int> s_in, lds_p<int> s_prow,
                                        lds_p<R> s_linv, int* fail, int kb, int nbk, int lane) {
  panel_body<NS, n, LDA, R>(A, cb, s_in, s_prow, s_linv, fail, kb, nbk, lane);
}

// The same with the kernels' LDS arrays (generic pointers into LDS).
template <int NS, int n, int LDA, class R>
__device__ __forceinline__ void panel_lds(R* A, int cb, const int* s_in, int* s_prow, R* s_linv, int* fail, int kb,
                                          int nbk, int lane) {
  panel_wave<NS, n, LDA, R>((lds_p<R>)A, cb, (lds_p<const int>)s_in, (lds_p<int>)s_prow, (lds_p<R>)s_linv, fail, kb,
                            nbk, lane);
}

// FP32 blocks take half the LDS, so two workgroups share a compute unit
// (the serial panel steps of one overlap the other's matrix-core work):
// four waves per SIMD, 128 registers per lane; FP64: two waves per SIMD.
template <int D, int P, class R>
__global__ __launch_bounds__(512, sizeof(R) == 4 ? 4 : 2) void k_jaclu_lds(const R* __restrict__ BC, const double* __restrict__ Gpk,
                                                      int NT, const double* __restrict__ dtau, R* __restrict__ out,
                                                      int* __restrict__ perm, int* __restrict__ fail, int ne,
                                                      Tab<D, P, double> tab) {
  using L = LdsLu<D, P, R>;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc;
  constexpr int V = L::V, N = L::N, Q = L::Q, QV = L::QV, QF = L::QF, NF = L::NF, n = L::n, NW = L::NW;
  constexpr int NPF = L::NPF, NT16 = L::NT16, JPW = L::JPW, JOBS = L::JOBS, RPL = L::RPL, LDA = L::LDA;
  extern __shared__ __align__(16) unsigned char s_raw[];
  R* s_mem = reinterpret_cast<R*>(s_raw);
  __shared__ Tab<D, P, double> t;
  __shared__ int s_prow2[2][n];   // logical row order (two buffers: look-ahead)
  __shared__ R s_linv2[2][16 * 16];  // L11^{-1} of the current panel, row-major (two buffers: look-ahead)
  const int e = blockIdx.x;
  if (e >= ne) return;  // whole workgroup
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int il = lane & 15, kq = lane >> 4;
  R* s_dph = s_mem;               // [QV][D][N]
  R* s_ph = s_mem + L::OFF_PH;    // [QV + NPF][N]: phi at the volume, then the face points
  R* s_B = s_mem + L::OFF_B;      // [QV][D][V][V] then [NPF][V][V]
  const R* s_C = s_B + QV * D * V * V;

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
    for (int r = 0; r < D; ++r) s_dph[(q * D + r) * N + j] = R(dphi_vol<D, P, double>(t, j, iq, r));
    s_ph[q * N + j] = R(phi_vol<D, P, double>(t, j, iq));
  }
  for (int it = tid; it < NPF * N; it += 512) {
    const int lf = it / (QF * N), k = (it / N) % QF, j = it % N;
    int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
    face_axes<D>(lf, ta);
#pragma unroll
    for (int q = 0; q < D - 1; ++q) { ik[q] = r0 % Q; r0 /= Q; }
    s_ph[(QV + lf * QF + k) * N + j] = R(phi_face<D, P, double>(t, j, lf, ta, ik));
  }
  for (int k = tid; k < n; k += 512) s_prow2[0][k] = k;
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
  acc_t acc[JPW][NT16];
#pragma unroll
  for (int jj = 0; jj < JPW; ++jj)
#pragma unroll
    for (int c = 0; c < NT16; ++c) acc[jj][c] = acc_t{R(0), R(0), R(0), R(0)};
#pragma unroll 1
  for (int ks = 0; ks < L::KSV; ++ks) {
    const int q = 4 * ks + kq;
    R bf[NT16], dp[NT16][D];
#pragma unroll
    for (int c = 0; c < NT16; ++c) {
      const int j = 16 * c + il;
      bf[c] = j < N ? s_ph[q * N + j] : R(0);
#pragma unroll
      for (int r = 0; r < D; ++r) dp[c][r] = j < N ? s_dph[(q * D + r) * N + j] : R(0);
    }
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
      if (wv + NW * jj < JOBS) {
        R a = R(0);
#pragma unroll
        for (int r = 0; r < D; ++r) {
          const R d = NT16 == 1 ? dp[0][r] : (jt[jj] == 0 ? dp[0][r] : dp[NT16 - 1][r]);
          a = fma(d, s_B[((q * D + r) * V + jv[jj]) * V + jw[jj]], a);
        }
#pragma unroll
        for (int c = 0; c < NT16; ++c) acc[jj][c] = MF::run(a, bf[c], acc[jj][c]);
      }
    }
  }
#pragma unroll 1
  for (int ks = 0; ks < L::KSF; ++ks) {
    const int fk = 4 * ks + kq;
    R bf[NT16];
#pragma unroll
    for (int c = 0; c < NT16; ++c) {
      const int j = 16 * c + il;
      bf[c] = j < N ? s_ph[(QV + fk) * N + j] : R(0);
    }
#pragma unroll
    for (int jj = 0; jj < JPW; ++jj) {
      if (wv + NW * jj < JOBS) {
        const R fa = NT16 == 1 ? bf[0] : (jt[jj] == 0 ? bf[0] : bf[NT16 - 1]);
        const R a = -fa * s_C[(fk * V + jv[jj]) * V + jw[jj]];
#pragma unroll
        for (int c = 0; c < NT16; ++c) acc[jj][c] = MF::run(a, bf[c], acc[jj][c]);
      }
    }
  }
  __syncthreads();  // phase-1 LDS is overwritten by the block below

  // ---- the block Pt = G/dtau - Dt, column-major in LDS
  R* A = s_mem;
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
          const int i = 16 * jt[jj] + MF::row(kq, r), j = 16 * c + il;
          if (i < N && j < N) {
            R g = R(0);
            if (jv[jj] == jw[jj]) g = R(((i >= j) ? G[i * (i + 1) / 2 + j] : G[j * (j + 1) / 2 + i]) * idt);
            A[(jw[jj] * N + j) * LDA + jv[jj] * N + i] = g - acc[jj][c][r];
          }
        }
      }
    }
  }
  __syncthreads();

  // ---- LU with partial pivoting, panels of 16 columns, with look-ahead:
  // while wavefront 0 factorises panel k + 1, the others apply panel k's
  // update to the columns beyond it.  The row order is double-buffered: the
  // panel writes the new order into the other buffer while the update still
  // reads the old one (the set of rows below the panel is the same in both).
  auto panel = [&](int kb, int nbk, const int* pin, int* pout, R* s_linv) {
    const int rows = n - kb;
    if constexpr (RPL >= 3) {
      if (rows > 128) panel_lds<3, n, LDA>(A, 0, pin, pout, s_linv, fail, kb, nbk, lane);
      else if (rows > 64) panel_lds<2, n, LDA>(A, 0, pin, pout, s_linv, fail, kb, nbk, lane);
      else panel_lds<1, n, LDA>(A, 0, pin, pout, s_linv, fail, kb, nbk, lane);
    } else {
      if (rows > 64) panel_lds<2, n, LDA>(A, 0, pin, pout, s_linv, fail, kb, nbk, lane);
      else panel_lds<1, n, LDA>(A, 0, pin, pout, s_linv, fail, kb, nbk, lane);
    }
  };
  // A22 tile (ti, tj) below and right of panel kb (nbk columns) -= L21 U12,
  // rows in the order ord; one wavefront, every load issued before the products
  auto tile = [&](const int* ord, int kb, int nbk, int k1, int ti, int tj) {
    const int cc = k1 + 16 * tj + il;
    const bool cok = cc < n;
    int crow[4];
    acc_t c;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = k1 + 16 * ti + MF::row(kq, r);
      crow[r] = lr < n ? ord[lr] : -1;
      c[r] = (crow[r] >= 0 && cok) ? A[cc * LDA + crow[r]] : R(0);
    }
    const int alr = k1 + 16 * ti + il;
    const int arow = alr < n ? ord[alr] : -1;
    R a[4], b[4];
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int k = 4 * s4 + kq;
      a[s4] = (arow >= 0 && k < nbk) ? -A[(kb + k) * LDA + arow] : R(0);
      b[s4] = (k < nbk && cok) ? A[cc * LDA + ord[kb + k]] : R(0);
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) c = MF::run(a[s4], b[s4], c);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (crow[r] >= 0 && cok) A[cc * LDA + crow[r]] = c[r];
  };
  int cur = 1;
  if constexpr (sizeof(R) == 4) {
    // FP32: two workgroups share a compute unit, so the other one's work
    // overlaps a panel; no look-ahead (its extra phases cost more than
    // they hide here), one row-order buffer
    cur = 0;
#pragma unroll 1
    for (int kb = 0; kb < n; kb += 16) {
      const int nbk = min(16, n - kb);
      if (wv == 0) panel(kb, nbk, s_prow2[0], s_prow2[0], s_linv2[0]);
      __syncthreads();
      const int k1 = kb + nbk, m = n - k1;
      if (m <= 0) break;
      const int* ord = s_prow2[0];
      const R* s_linv = s_linv2[0];
      const int T = (m + 15) / 16;
#pragma unroll 1
      for (int tj = wv; tj < T; tj += NW) {
        const int cc = k1 + 16 * tj + il;
        const bool cok = cc < n;
        acc_t u = acc_t{R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + kq;
          u = MF::run(s_linv[il * 16 + k], (k < nbk && cok) ? A[cc * LDA + ord[kb + k]] : R(0), u);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = MF::row(kq, r);
          if (k < nbk && cok) A[cc * LDA + ord[kb + k]] = u[r];
        }
      }
      __syncthreads();
#pragma unroll 2
      for (int it = wv; it < T * T; it += NW) tile(ord, kb, nbk, k1, it % T, it / T);
      __syncthreads();
    }
  } else {
    if (wv == 0) panel(0, min(16, n), s_prow2[0], s_prow2[1], s_linv2[1]);
    __syncthreads();
    // FP64 (one workgroup per compute unit): per panel kb
    //   phase 1: U12 of the column tiles beyond the next panel (in place),
    //            and the next panel's columns (tile 0) updated with their
    //            U12 tile formed in registers (the FP64 accumulator layout
    //            is the B-operand layout), A12 of tile 0 left unchanged;
    //   phase 2: wavefront 0 factorises the next panel (its L11^{-1} into
    //            the other buffer); wavefront 1 stores U12 of tile 0 (pivot
    //            rows, which the panel does not touch);
    //            the wavefronts of the other SIMDs update the tiles beyond.
#pragma unroll 1
    for (int kb = 0;;) {
      const int nbk = min(16, n - kb), k1 = kb + nbk, m = n - k1;
      if (m <= 0) break;
      const int* ord = s_prow2[cur];
      const R* s_linv = s_linv2[cur];
      const int T = (m + 15) / 16;
      auto u12 = [&](int tj) {
        const int cc = k1 + 16 * tj + il;
        const bool cok = cc < n;
        acc_t u = acc_t{R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + kq;
          u = MF::run(s_linv[il * 16 + k], (k < nbk && cok) ? A[cc * LDA + ord[kb + k]] : R(0), u);
        }
        return u;
      };
#pragma unroll 1
      for (int it = wv; it < 2 * T - 1; it += NW) {
        if (it < T - 1) {
          const int tj = 1 + it;
          const acc_t u = u12(tj);
          const int cc = k1 + 16 * tj + il;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int k = MF::row(kq, r);
            if (k < nbk && cc < n) A[cc * LDA + ord[kb + k]] = u[r];
          }
        } else {
          const int ti = it - (T - 1);
          const acc_t u = u12(0);
          const int cc = k1 + il;
          const bool cok = cc < n;
          int crow[4];
          acc_t c;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int lr = k1 + 16 * ti + MF::row(kq, r);
            crow[r] = lr < n ? ord[lr] : -1;
            c[r] = (crow[r] >= 0 && cok) ? A[cc * LDA + crow[r]] : R(0);
          }
          const int alr = k1 + 16 * ti + il;
          const int arow = alr < n ? ord[alr] : -1;
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int k = 4 * s4 + kq;
            const R a = (arow >= 0 && k < nbk) ? -A[(kb + k) * LDA + arow] : R(0);
            c = MF::run(a, u[s4], c);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (crow[r] >= 0 && cok) A[cc * LDA + crow[r]] = c[r];
        }
      }
      __syncthreads();
      if (wv == 0) {
        panel(k1, min(16, n - k1), ord, s_prow2[cur ^ 1], s_linv2[cur ^ 1]);
      } else if (wv == 1) {
        const acc_t u = u12(0);
        const int cc = k1 + il;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = MF::row(kq, r);
          if (k < nbk && cc < n) A[cc * LDA + ord[kb + k]] = u[r];
        }
      }
      if (wv % 4 != 0) {
        // the SIMDs other than wavefront 0's (wavefront w runs on SIMD w mod 4)
        const int slot = wv - 1 - wv / 4;  // 0 .. NW - NW / 4 - 1
#pragma unroll 1
        for (int it = slot; it < T * (T - 1); it += NW - NW / 4) tile(ord, kb, nbk, k1, it % T, 1 + it / T);
      }
      __syncthreads();
      cur ^= 1;
      kb = k1;
    }
  }
  const int* s_prow = s_prow2[cur];

  // ---- factors in pivot order, column-major, and the permutation
  R* o = out + (size_t)e * n * n;
  for (int it = tid; it < n * n; it += 512) {
    const int col = it / n, k = it % n;
    o[it] = A[col * LDA + s_prow[k]];
  }
  for (int k = tid; k < n; k += 512) perm[(size_t)e * n + k] = s_prow[k];
}

template <int D, int P, class R>
hipError_t jaclu_lds_t(const DevMesh& M, const TabData& td, const void* bc, const double* dtau, void* out,
                       int* perm, int* fail, hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  const size_t lds = jaclu_lds_bytes<D, P, R>();
  static bool attr = false;  // set once: not a stream operation, so also fine while capturing
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jaclu_lds<D, P, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_jaclu_lds<D, P, R>), dim3(M.ne), dim3(512), lds, st, static_cast<const R*>(bc), M.Gpk, M.NT,
                     dtau, static_cast<R*>(out), perm, fail, M.ne, t);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Element blocks too large for LDS (3D p = 3: n = 320, 819 KB in FP64): the
// same assembly and LU with the block in global memory (the factor output
// buffer itself, column-major, rows in their original order until the end).
//
// Basis tables of the order (one copy per device, read through the caches
// by every workgroup; filled once at set-up by k_fill_bigtab with the
// kernels' own basis formulas):
//   [QV][D][N] d_r phi_j at the volume points, [QV][N] phi_j there,
//   [NF QF][N] phi_j at the face points.
// ---------------------------------------------------------------------------
template <int D, int P>
struct BigLu {
  using C = Cfg<D, P>;
  static constexpr int V = C::V, N = C::N, QV = C::QV, QF = C::QF, NF = C::NF, n = C::NB;
  static constexpr int NPF = NF * QF;
  static constexpr int KSV = (QV + 3) / 4, KSF = (NPF + 3) / 4;  // k-steps of four points (last one padded)
  static constexpr int NT16 = N / 16;
  static constexpr int NW = 8, JR = 2;                            // wavefronts; jobs per wavefront and round
  static constexpr int JOBS = V * V * NT16;
  static constexpr int ROUNDS = (JOBS + NW * JR - 1) / (NW * JR);
  static constexpr int PER = (QV * D + NPF) * V * V;              // pointwise Jacobian values per element
  static constexpr int TAB_D = 0, TAB_V = QV * D * N, TAB_F = TAB_V + QV * N, TAB = TAB_F + NPF * N;
  static constexpr int RPL = (n + 63) / 64;
  static_assert(N % 16 == 0 && n % 16 == 0 && n <= 320, "tiles of 16; at most five row slots");
};

template <int D, int P, class R>
constexpr size_t jaclu_big_lds_values() {
  using L = BigLu<D, P>;
  return (size_t)(L::PER > L::NW * L::n ? L::PER : L::NW * L::n);
}

template <int D, int P, class R>
__global__ __launch_bounds__(256) void k_fill_bigtab(R* __restrict__ out, Tab<D, P, double> tab) {
  using L = BigLu<D, P>;
  constexpr int N = L::N, Q = Cfg<D, P>::Q, QV = L::QV, QF = L::QF;
  __shared__ Tab<D, P, double> t;
  copy_tab(t, tab);
  __syncthreads();
  for (int it = threadIdx.x + blockIdx.x * blockDim.x; it < L::TAB; it += blockDim.x * gridDim.x) {
    if (it < L::TAB_V) {
      const int q = it / (D * N), r = (it / N) % D, j = it % N;
      int iq[D], r0 = q;
#pragma unroll
      for (int a = 0; a < D; ++a) { iq[a] = r0 % Q; r0 /= Q; }
      out[it] = R(dphi_vol<D, P, double>(t, j, iq, r));
    } else if (it < L::TAB_F) {
      const int q = (it - L::TAB_V) / N, j = it % N;
      int iq[D], r0 = q;
#pragma unroll
      for (int a = 0; a < D; ++a) { iq[a] = r0 % Q; r0 /= Q; }
      out[it] = R(phi_vol<D, P, double>(t, j, iq));
    } else {
      const int f = it - L::TAB_F;
      const int lf = f / (QF * N), k = (f / N) % QF, j = f % N;
      int ta[D - 1 > 0 ? D - 1 : 1], ik[D - 1 > 0 ? D - 1 : 1], r0 = k;
      face_axes<D>(lf, ta);
#pragma unroll
      for (int a = 0; a < D - 1; ++a) { ik[a] = r0 % Q; r0 /= Q; }
      out[it] = R(phi_face<D, P, double>(t, j, lf, ta, ik));
    }
  }
}

template <int NT, class R>
__device__ __forceinline__ R sel_tile(const R (&x)[NT], int i) {
  R v = x[0];
#pragma unroll
  for (int c = 1; c < NT; ++c) v = (i == c) ? x[c] : v;
  return v;
}

// One workgroup (eight wavefronts) per element.
// Assembly: the element's pointwise Jacobians in LDS; jobs (v, w, 16-row
// tile) in rounds of two per wavefront, each accumulating its N/16 output
// tiles over the volume and face points on the 16 x 16 x 4 matrix-core
// instruction (operands as in k_jaclu_lds, basis values from the device
// table), then written to global memory: Pt = G/dtau - Dt (factor) or Dt
// itself (row-major, the unfactored element block).
// LU with partial pivoting in panels of 16 columns, as k_jaclu_lds: (a) the
// panel is copied to LDS, wavefront 0 factorises it there (panel_wave) and
// it is copied back, (b) U12 = L11^{-1} A12 per 16-column tile on the
// matrix cores, (c) A22 -= L21 U12 per 16 x 16 tile (L21 from the LDS
// panel), the tiles spread over the wavefronts.  Finally every column is permuted
// into pivot order through LDS.
template <int D, int P, class R>
__global__ __launch_bounds__(512, sizeof(R) == 4 ? 4 : 2) void k_jaclu_big(
    const R* __restrict__ BC, const R* __restrict__ gtab, const double* __restrict__ Gpk, int NT,
    const double* __restrict__ dtau, R* __restrict__ out, int* __restrict__ perm, int* __restrict__ fail, int ne,
    int factor) {
  using L = BigLu<D, P>;
  using MF = Mfma<R>;
  using acc_t = typename MF::acc;
  constexpr int V = L::V, N = L::N, QV = L::QV, NPF = L::NPF, n = L::n, NW = L::NW, JR = L::JR, NT16 = L::NT16;
  extern __shared__ __align__(16) unsigned char s_raw[];
  R* s_mem = reinterpret_cast<R*>(s_raw);
  __shared__ int s_prow[n];
  __shared__ R s_linv[16 * 16];
  const int e = blockIdx.x;
  if (e >= ne) return;  // whole workgroup
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int il = lane & 15, kq = lane >> 4;
  R* A = out + (size_t)e * n * n;
  const R* s_B = s_mem;                       // [QV][D][V][V]
  const R* s_C = s_mem + QV * D * V * V;      // [NPF][V][V]
  const R* tdp = gtab + L::TAB_D;
  const R* tph = gtab + L::TAB_V;
  const R* tpf = gtab + L::TAB_F;

  stage<(L::PER + 511) / 512>(s_mem, BC + (size_t)e * L::PER, L::PER, tid, 512);
  for (int k = tid; k < n; k += 512) s_prow[k] = k;
  __syncthreads();

  // ---- assembly
  const double idt = 1.0 / dtau[e];
  const double* G = Gpk + (size_t)e * NT;
#pragma unroll 1
  for (int rd = 0; rd < L::ROUNDS; ++rd) {
    int jv[JR], jw[JR], jt[JR];
    bool jon[JR];
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
      const int job = (rd * NW + wv) * JR + jj;
      jon[jj] = job < L::JOBS;
      const int jb = jon[jj] ? job : 0;
      jt[jj] = jb % NT16;
      jv[jj] = (jb / NT16) / V;
      jw[jj] = (jb / NT16) % V;
    }
    if (!jon[0]) continue;  // uniform over the wavefront
    acc_t acc[JR][NT16];
#pragma unroll
    for (int jj = 0; jj < JR; ++jj)
#pragma unroll
      for (int c = 0; c < NT16; ++c) acc[jj][c] = acc_t{R(0), R(0), R(0), R(0)};
#pragma unroll 2
    for (int ks = 0; ks < L::KSV; ++ks) {
      const int q = 4 * ks + kq;
      const bool qv = q < QV;
      const int qc = qv ? q : QV - 1;
      R bf[NT16];
#pragma unroll
      for (int c = 0; c < NT16; ++c) bf[c] = qv ? tph[qc * N + 16 * c + il] : R(0);
#pragma unroll
      for (int jj = 0; jj < JR; ++jj) {
        if (jon[jj]) {
          R a = R(0);
#pragma unroll
          for (int r = 0; r < D; ++r)
            a = fma(tdp[(qc * D + r) * N + 16 * jt[jj] + il], s_B[((qc * D + r) * V + jv[jj]) * V + jw[jj]], a);
          a = qv ? a : R(0);
#pragma unroll
          for (int c = 0; c < NT16; ++c) acc[jj][c] = MF::run(a, bf[c], acc[jj][c]);
        }
      }
    }
#pragma unroll 2
    for (int ks = 0; ks < L::KSF; ++ks) {
      const int fk = 4 * ks + kq;
      const bool fv = fk < NPF;
      const int fc = fv ? fk : NPF - 1;
      R bf[NT16];
#pragma unroll
      for (int c = 0; c < NT16; ++c) bf[c] = fv ? tpf[fc * N + 16 * c + il] : R(0);
#pragma unroll
      for (int jj = 0; jj < JR; ++jj) {
        if (jon[jj]) {
          const R a = -sel_tile(bf, jt[jj]) * s_C[(fc * V + jv[jj]) * V + jw[jj]];
#pragma unroll
          for (int c = 0; c < NT16; ++c) acc[jj][c] = MF::run(a, bf[c], acc[jj][c]);
        }
      }
    }
#pragma unroll
    for (int jj = 0; jj < JR; ++jj) {
      if (!jon[jj]) continue;
#pragma unroll
      for (int c = 0; c < NT16; ++c) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * jt[jj] + MF::row(kq, r), j = 16 * c + il;
          if (factor) {
            R g = R(0);
            if (jv[jj] == jw[jj]) g = R(((i >= j) ? G[i * (i + 1) / 2 + j] : G[j * (j + 1) / 2 + i]) * idt);
            A[(size_t)(jw[jj] * N + j) * n + jv[jj] * N + i] = g - acc[jj][c][r];
          } else {
            A[(size_t)(jv[jj] * N + i) * n + jw[jj] * N + j] = acc[jj][c][r];
          }
        }
      }
    }
  }
  if (!factor) return;  // uniform
  __syncthreads();  // the block is complete (global memory, one workgroup)

  // ---- LU with partial pivoting, panels of 16 columns
  R* s_pan = s_mem;  // the current panel, [16][n] (rows in their original order)
#pragma unroll 1
  for (int kb = 0; kb < n; kb += 16) {
    for (int it = tid; it < 16 * n; it += 512) s_pan[it] = A[(size_t)kb * n + it];
    __syncthreads();
    if (wv == 0) {
      const int rows = n - kb;
      if (rows > 256) panel_lds<5, n, n>(s_pan, kb, s_prow, s_prow, s_linv, fail, kb, 16, lane);
      else if (rows > 192) panel_lds<4, n, n>(s_pan, kb, s_prow, s_prow, s_linv, fail, kb, 16, lane);
      else if (rows > 128) panel_lds<3, n, n>(s_pan, kb, s_prow, s_prow, s_linv, fail, kb, 16, lane);
      else if (rows > 64) panel_lds<2, n, n>(s_pan, kb, s_prow, s_prow, s_linv, fail, kb, 16, lane);
      else panel_lds<1, n, n>(s_pan, kb, s_prow, s_prow, s_linv, fail, kb, 16, lane);
    }
    __syncthreads();
    for (int it = tid; it < 16 * n; it += 512) A[(size_t)kb * n + it] = s_pan[it];
    const int k1 = kb + 16, m = n - k1;
    if (m <= 0) break;
    const int T = m / 16;
    // (b) U12 = L11^{-1} A12, one 16-column tile per wavefront at a time
#pragma unroll 1
    for (int tj = wv; tj < T; tj += NW) {
      const int cc = k1 + 16 * tj + il;
      acc_t u = acc_t{R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int k = 4 * s4 + kq;
        u = MF::run(s_linv[il * 16 + k], A[(size_t)cc * n + s_prow[kb + k]], u);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) A[(size_t)cc * n + s_prow[kb + MF::row(kq, r)]] = u[r];
    }
    __syncthreads();
    // (c) A22 -= L21 U12 over the T x T tiles, two per wavefront at a time
    // with every load issued before the products
#pragma unroll 1
    for (int it0 = 2 * wv; it0 < T * T; it0 += 2 * NW) {
      acc_t c2[2];
      R a2[2][4], b2[2][4];
      int crow[2][4], ccol[2];
      bool on[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int it = it0 + h;
        on[h] = it < T * T;
        const int ti = on[h] ? it / T : 0, tj = on[h] ? it % T : 0;
        ccol[h] = k1 + 16 * tj + il;
        const int arow = s_prow[k1 + 16 * ti + il];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          crow[h][r] = s_prow[k1 + 16 * ti + MF::row(kq, r)];
          c2[h][r] = A[(size_t)ccol[h] * n + crow[h][r]];
        }
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + kq;
          a2[h][s4] = -s_pan[k * n + arow];
          b2[h][s4] = A[(size_t)ccol[h] * n + s_prow[kb + k]];
        }
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) c2[h] = MF::run(a2[h][s4], b2[h][s4], c2[h]);
        if (on[h]) {
#pragma unroll
          for (int r = 0; r < 4; ++r) A[(size_t)ccol[h] * n + crow[h][r]] = c2[h][r];
        }
      }
    }
    __syncthreads();
  }

  __syncthreads();  // the last panel's copy-back is complete; LDS is reused below

  // ---- factors in pivot order: each column through LDS (one wavefront per
  // column; its reads of the column complete before its writes)
  R* s_col = s_mem + wv * n;
#pragma unroll 1
  for (int col = wv; col < n; col += NW) {
    R* cp = A + (size_t)col * n;
#pragma unroll
    for (int s = 0; s < L::RPL; ++s)
      if (lane + 64 * s < n) s_col[lane + 64 * s] = cp[lane + 64 * s];
    wave_lds_sync();
#pragma unroll
    for (int s = 0; s < L::RPL; ++s)
      if (lane + 64 * s < n) cp[lane + 64 * s] = s_col[s_prow[lane + 64 * s]];
    wave_lds_sync();
  }
  for (int k = tid; k < n; k += 512) perm[(size_t)e * n + k] = s_prow[k];
}

template <int D, int P, class R>
hipError_t jaclu_big_t(const DevMesh& M, const void* bc, const void* tab, const double* dtau, void* out, int* perm,
                       int* fail, bool factor, hipStream_t st) {
  const size_t lds = jaclu_big_lds_values<D, P, R>() * sizeof(R);
  static bool attr = false;  // set once: not a stream operation, so also fine while capturing
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_jaclu_big<D, P, R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_jaclu_big<D, P, R>), dim3(M.ne), dim3(512), lds, st, static_cast<const R*>(bc),
                     static_cast<const R*>(tab), M.Gpk, M.NT, dtau, static_cast<R*>(out), perm, fail, M.ne,
                     factor ? 1 : 0);
  return hipGetLastError();
}

template <int D, int P, class R>
hipError_t fill_bigtab_t(const TabData& td, void* dst, hipStream_t st) {
  Tab<D, P, double> t;
  fill_tab(t, td);
  hipLaunchKernelGGL((k_fill_bigtab<D, P, R>), dim3(64), dim3(256), 0, st, static_cast<R*>(dst), t);
  return hipGetLastError();
}

}  // namespace

bool jaclu_lds_supported(int d, int p) { return (d == 2 && p == 4) || (d == 3 && p == 2); }

hipError_t launch_jaclu_lds(const DevMesh& M, const TabData& td, int p, int prec, const void* bc, const double* dtau,
                            void* out, int* perm, int* fail, hipStream_t st) {
  const bool f32 = prec == PREC_FP32;
  if (M.d == 2 && p == 4)
    return f32 ? jaclu_lds_t<2, 4, float>(M, td, bc, dtau, out, perm, fail, st)
               : jaclu_lds_t<2, 4, double>(M, td, bc, dtau, out, perm, fail, st);
  if (M.d == 3 && p == 2)
    return f32 ? jaclu_lds_t<3, 2, float>(M, td, bc, dtau, out, perm, fail, st)
               : jaclu_lds_t<3, 2, double>(M, td, bc, dtau, out, perm, fail, st);
  return hipErrorInvalidValue;
}

bool jaclu_big_supported(int d, int p) { return d == 3 && p == 3; }

size_t bigtab_values(int d, int p) {
  if (d == 3 && p == 3) return (size_t)BigLu<3, 3>::TAB;
  return 0;
}

hipError_t launch_fill_bigtab(const DevMesh& M, const TabData& td, int p, int prec, void* dst, hipStream_t st) {
  if (M.d == 3 && p == 3)
    return prec == PREC_FP32 ? fill_bigtab_t<3, 3, float>(td, dst, st) : fill_bigtab_t<3, 3, double>(td, dst, st);
  return hipErrorInvalidValue;
}

hipError_t launch_jaclu_big(const DevMesh& M, int p, int prec, const void* bc, const void* tab, const double* dtau,
                            void* out, int* perm, int* fail, bool factor, hipStream_t st) {
  if (!tab) return hipErrorInvalidValue;
  if (M.d == 3 && p == 3)
    return prec == PREC_FP32 ? jaclu_big_t<3, 3, float>(M, bc, tab, dtau, out, perm, fail, factor, st)
                             : jaclu_big_t<3, 3, double>(M, bc, tab, dtau, out, perm, fail, factor, st);
  return hipErrorInvalidValue;
}

}  // namespace eg
