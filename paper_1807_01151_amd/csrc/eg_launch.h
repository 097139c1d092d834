// Internal interface between the host driver and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "eg_common.h"

namespace eg {

// Device-resident mesh data and constants (owned by the handle).
struct DevMesh {
  int d = 2, V = 4, ne = 0, NF = 4, NC = 9;
  int NT = 0;              // packed triangle size of the p_max basis
  double omega = 0.0;      // |Omega|
  Gas gas{};
  double* xv = nullptr;    // [E][NC][d] geometry nodes (9 per quad, 8 per hex)
  int* nbr = nullptr;      // [E][2d]
  uint8_t* ncode = nullptr;
  double* Lpk = nullptr;   // [E][NT] Cholesky factor of the phi mass matrix
  // restriction p -> p - 1 per element, R = L_c^{-T} [I 0] L^T by columns: [E][N(p)][N(p-1)]
  double* Rop[5] = {};
  double* Gpk = nullptr;   // [E][NT] phi mass matrix
  double* hE = nullptr;    // [E] 2 d |E| / |dE|
  double* g2x = nullptr;   // 2-point Gauss rule (p = 0 faces)
  double* g2w = nullptr;
  void* bc = nullptr;      // pointwise flux-Jacobian scratch of the block assembly (FP64 or FP32)
  // per order and precision: phi at the volume points [QV][N], then at the
  // face points [NF QF][N] (the shared operands of the block assembly); for
  // 3D p = 3 the global-memory kernel's table (bigtab_values(3, 3) values:
  // d phi and phi at the volume points, phi at the face points)
  const void* phitab[5][2] = {};
  // residual tile per order and precision (FP64, FP32): index of the
  // candidate (0: half, 1: default, 2: 1.5 x the default), set by eg_autotune
  int res_tile_choice[5][2] = {{1, 1}, {1, 1}, {1, 1}, {1, 1}, {1, 1}};
  // batched solves (null for a single solve): per-element free stream [E][V]
  // and CFL [E]; solve segments (element ranges) and Arnoldi block tables
  double* uinf_e = nullptr;
  double* cfl_e = nullptr;
  double* cfl_one = nullptr;  // device scalar CFL (bound while a V-cycle is captured)
  int nseg = 1;
  int* sid = nullptr;        // [E] solve of each element
  int* seg_e0 = nullptr;     // [nseg + 1] first element of each solve
  double* seg_omega = nullptr;  // [nseg] |Omega| of each solve
  int* brow0 = nullptr;      // [nblk] first row of each Arnoldi block
  int* brow1 = nullptr;      // [nblk] end row of each Arnoldi block
  int* bseg = nullptr;       // [nblk] solve of each Arnoldi block
  int* sblk0 = nullptr;      // [nseg + 1] first Arnoldi block of each solve
};

// arithmetic precision of a smoother kernel
constexpr int PREC_FP64 = 0;
constexpr int PREC_FP32 = 1;

// values per element of the pointwise flux-Jacobian scratch at order p for
// FP64 or FP32 blocks (0 if that order uses the single-kernel assembly)
size_t jac_points_per_elem(int d, int p, bool fp32);
size_t phitab_values(int d, int p);
// elements per workgroup of the residual at (d, p, precision) for a tile choice
int residual_tile(int d, int p, int prec, int choice);

// Host copy of the 1D tables of one order (filled by the set-up code).
struct TabData {
  double x[8], w[8];
  double L[8][8], dL[8][8], Lb[8][2];
  int m[128][3];
};

// FAS form of the residual output: with rhat set, rt receives the fine
// residual rhat (Nf modes per row) truncated to the level's modes and fc the
// forcing rt - R (fc = fine - coarse); fadd must then be null.
struct FasOut {
  const double* rhat = nullptr;
  int Nf = 0;
  double* fc = nullptr;
};
hipError_t launch_residual(const DevMesh& M, const TabData& td, int p, const double* ut, const double* fadd,
                           double* rt, int prec, hipStream_t st, const FasOut& fas = FasOut{});
bool jacobian_supported(int d, int p);
// Block assembly on the matrix cores and LDS-resident blocked LU
// (eg_jaclu_lds.hip) for 2D p = 4 and 3D p = 2, FP64 or FP32 (prec); bc
// from k_jac_points in the same precision, out FP64 or FP32 factors.
bool jaclu_lds_supported(int d, int p);
// Block assembly and LU with the block in global memory (eg_jaclu_lds.hip)
// for 3D p = 3 (n = 320), FP64 or FP32 (prec); bc the point Jacobians of
// k_jac_points, tab the order's basis table (launch_fill_bigtab); factor =
// false writes the unfactored element block Dt row-major instead.
bool jaclu_big_supported(int d, int p);
size_t bigtab_values(int d, int p);
hipError_t launch_fill_bigtab(const DevMesh& M, const TabData& td, int p, int prec, void* dst, hipStream_t st);
hipError_t launch_jaclu_big(const DevMesh& M, int p, int prec, const void* bc, const void* tab, const double* dtau,
                            void* out, int* perm, int* fail, bool factor, hipStream_t st);
hipError_t launch_jaclu_lds(const DevMesh& M, const TabData& td, int p, int prec, const void* bc, const double* dtau,
                            void* out, int* perm, int* fail, hipStream_t st);
hipError_t launch_jacobian(const DevMesh& M, const TabData& td, int p, const double* ut, const double* dtau,
                           void* out, int* perm, int* fail, bool factor, int prec, hipStream_t st);
// un null: the stage starts from ut and, if save is set, stores it there
hipError_t launch_prk_stage(const DevMesh& M, int n, const void* F, const int* perm, const double* rt,
                            const double* ft, const double* un, double* ut, double beta, int prec, hipStream_t st,
                            double* save = nullptr);
hipError_t launch_sub(const double* a, const double* b, double* out, size_t n, hipStream_t st);
hipError_t launch_basis(const DevMesh& M, int N, const double* x, double* y, int mode, hipStream_t st);
hipError_t launch_restrict(const DevMesh& M, int p, const double* ut, double* uc, double* uc0, hipStream_t st);
hipError_t launch_timestep(const DevMesh& M, int p, int N, double cfl, double mult, const double* ut, double* dtau,
                           hipStream_t st);
hipError_t launch_norm(const DevMesh& M, int N, const double* rt, double* part, double* out, hipStream_t st);
hipError_t launch_p0_setup(const DevMesh& M, const double* ut0, const double* ft0, int pmax, double cfl, int scale,
                           double* u0, double* b, double* Ad, double* Ao, double* dt, hipStream_t st);
int arnoldi_blocks(int K);
// wn0: two slots per solve (the norm of A v_j of the last two steps).
hipError_t launch_arnoldi(const DevMesh& M, int m, int nblk, const double* Ad, const double* Ao, const double* b,
                          double* Vb, double* H, double* part1, double* part2, double* info, int* st, double* wn0,
                          double* W2, double* H2, hipStream_t stream);
hipError_t launch_phi1(int m, int nseg, const double* H, const double* H2, const double* info, double* y, int* fail,
                       hipStream_t st);
hipError_t launch_exp1_update(const DevMesh& M, int m, const double* Vb, const double* y, const double* info,
                              const double* u0, double* ut0, hipStream_t st);
// Levels 0..pmax of the V-cycle state: ut[l] and the restricted copies
// uc0[l] (N[l] modes per row); pmax <= 4.
struct UpChain {
  double* ut[5];
  const double* uc0[5];
  int N[5];
  int pmax;
};
// EXP1 update of ut[0] followed by the prolongations to levels 1..pmax.
hipError_t launch_exp1_prolong(const DevMesh& M, int m, const double* Vb, const double* y, const double* info,
                               const double* u0, const UpChain& c, hipStream_t st);
hipError_t launch_nbr_export(const DevMesh& M, int* out, hipStream_t st);
hipError_t launch_copy(const double* a, double* b, size_t n, hipStream_t st);
hipError_t launch_freestream(const DevMesh& M, int N, double* u, hipStream_t st);
hipError_t launch_jac_to_psi(const DevMesh& M, int N, double* Dm, hipStream_t st);

// (dRt_p/dut)(ut) vt by forward-mode dual numbers (eg_tangent.hip), p >= 0
hipError_t launch_tangent(const DevMesh& M, const TabData& td, int p, const double* ut, const double* vt, double* jv,
                          hipStream_t st);

// adjoint (drag sensitivity)
size_t jac_points_size(int d, int p);  // values per element of the pointwise flux Jacobians
hipError_t launch_jac_points(const DevMesh& M, const TabData& td, int p, const double* ut, double* bc, hipStream_t st);
// fills M.phitab[p][prec] (phitab_values(d, p) values of that precision)
hipError_t launch_fill_phitab(const DevMesh& M, const TabData& td, int p, int prec, void* dst, hipStream_t st);
hipError_t launch_adj_residual(const DevMesh& M, const TabData& td, int p, const double* wt, const double* gadd,
                               const double* bc, double* out, hipStream_t st);
hipError_t launch_drag(const DevMesh& M, const TabData& td, int p, const double* ut, const double* dir, double scale,
                       double* part, double* gt, hipStream_t st);
bool prk_tr_supported(int n);
hipError_t launch_prk_stage_tr(const DevMesh& M, int n, const double* F, const int* perm, const double* rt,
                               const double* un, double* ut, double beta, hipStream_t st);
hipError_t launch_p0_transpose(const DevMesh& M, const double* Ad, const double* Ao, const double* dt, double* AdT,
                               double* AoT, hipStream_t st);
hipError_t launch_adj_p0_rhs(const DevMesh& M, const double* gt0, const double* dt, double* b, hipStream_t st);
hipError_t launch_trunc(const double* x, double* y, int N, int Nc, int rows, hipStream_t st);
hipError_t launch_pad_add(double* x, const double* y, int N, int Nc, int rows, hipStream_t st);
hipError_t launch_fill0(double* x, size_t n, hipStream_t st);
hipError_t launch_expand_cfl(const DevMesh& M, const double* cfl_s, hipStream_t st);
// No-allocation density norm (eg_noalloc.hip): the file-scope workspace's
// address on `device` is resolved once, with that device current; the launch
// then needs no allocation.  ne <= noalloc_max_elems().
int noalloc_max_elems();
hipError_t noalloc_resolve(int device);
hipError_t launch_dnorm_noalloc(int device, int ne, int V, int N, double omega, const double* r, double* out,
                                hipStream_t st);
// Achievable peaks (eg_peak.hip): kind 0 HBM copy GB/s, 1 FP64 matrix-core
// TFLOP/s, 2 FP64 vector FMA TFLOP/s; allocates its own buffers.
hipError_t measure_peak(int kind, hipStream_t st, double* value);
int sum_blocks(size_t n);
hipError_t launch_sum(const double* x, const double* y, size_t n, double* part, int take_sqrt, double* out,
                      hipStream_t st);

}  // namespace eg
