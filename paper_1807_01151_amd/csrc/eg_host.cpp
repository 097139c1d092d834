// Host side of the MI355X eMG library: mesh set-up, device workspaces, the
// C ABI declared in include/eg.h and the V-cycle driver (arXiv:1807.01151,
// Section 2.4).  Every floating-point step of the hot path runs in the HIP
// kernels of eg_kernels.hip; the host only prepares mesh data once, launches
// kernels and reads back the residual norm.

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
#include "eg_launch.h"

using eg::DevMesh;
using eg::TabData;

struct eg_handle {
  DevMesh M;
  int dev = 0;  // device current at eg_init_mesh / eg_init_batch
  int pmax = 1, s = 4, m = 30, relr = 1;
  int mixed = 0;  // EG_MIXED: FP32 smoother on p >= 1 (phase A), then FP64 residuals (phase B)
  int phase_b = 0;  // mixed mode: the current V-cycle is a defect-correction (phase B) cycle
  double cfl_max = 100.0;
  hipStream_t st = nullptr;
  std::string err;
  std::vector<TabData> tabs;
  std::vector<std::array<int, 3>> modes;  // p_max modes
  double* ut[5] = {};
  double* un[5] = {};
  double* rt[5] = {};
  double* ft[5] = {};
  double* uc0[5] = {};
  void* F[5] = {};  // block LU factors, FP64 or (mixed) FP32
  int* perm[5] = {};
  double* dtau = nullptr;
  double* tmp = nullptr;
  double* tmp2 = nullptr;
  double* u0 = nullptr;
  double* b0 = nullptr;
  double* Ad = nullptr;
  double* Ao = nullptr;
  double* dt0 = nullptr;
  double* Vb = nullptr;
  double* H = nullptr;
  double* part1 = nullptr;
  double* part2 = nullptr;
  double* info = nullptr;
  int* arn_st = nullptr;
  double* arn_wn0 = nullptr;
  double* arn_W = nullptr;   // two scratch vectors of the Arnoldi products
  double* H2 = nullptr;      // second Gram-Schmidt pass coefficients
  double* y = nullptr;
  double* npart = nullptr;
  double* nout = nullptr;
  int* dfail = nullptr;
  double* hpin = nullptr;
  int nblk_arn = 0;
  std::vector<void*> allocs;
  // per-kernel-class event timing (eg_profile)
  struct ProfRec { int cls, p; hipEvent_t a, b; };
  bool prof = false;
  // state of the last steady solve (eg_solve_resume continues it)
  int sv_next = 0;
  double sv_r1 = 0.0;
  int sv_phase_b = 0, sv_nmin = 0;  // mixed mode: phase B reached; cycle of the smallest norm
  double sv_rmin = 0.0;
  double sv_ring[64] = {};  // mixed mode: entry norms of the last cycles (index n mod 64)
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<ProfRec> recs;
  double mach = 0.3;
  // drag functional
  double* dpart = nullptr;  // [E] per-element contributions
  double* spart = nullptr;  // partial sums of the deterministic reductions
  double* sout = nullptr;
  // adjoint workspaces (allocated by the first adjoint call), phi coordinates
  bool adj_ready = false;
  double* adj_bc[5] = {};    // pointwise flux Jacobians at the linearisation state, per level p >= 1
  double* adj_F[5] = {};     // FP64 LU factors of the PRK blocks at that state
  int* adj_perm[5] = {};
  double* adj_u[5] = {};     // linearisation state restricted to each level
  double* lam[5] = {};       // adjoint iterate (p_max) and coarse corrections
  double* lamn[5] = {};
  double* gq[5] = {};        // adjoint forcing per level
  double* rho[5] = {};       // adjoint residual per level
  double* AdT = nullptr;     // transposed p = 0 operator
  double* AoT = nullptr;
  double* zero0 = nullptr;   // K0 zeros
  // batched solves (eg_init_batch): per-solve CFL staging and norms
  bool batch = false;
  std::vector<int> seg_e0;   // host copy of the element ranges
  double* dcfl = nullptr;    // [nseg] device CFL per solve
  double* bsave = nullptr;   // [K at p_max] states of converged solves, saved at their last norm
  double* cfl_e_buf = nullptr;  // [E] per-element CFL (bound to M.cfl_e only inside eg_solve_batch)
  // graph replay of the V-cycle below the entry norm (eg_set_graphs)
  bool graphs = false;
  hipStream_t gst = nullptr;          // internal capture stream (non-default, default priority)
  hipEvent_t gev = nullptr;
  hipGraph_t ggraph[2] = {};          // per mixed-precision phase
  hipGraphExec_t gexec[2] = {};
  double* dcfl1 = nullptr;            // device CFL scalar read by the captured kernels
  double* hcfl1 = nullptr;            // pinned
  double* hcfl = nullptr;    // [nseg] pinned
  double* hnorm = nullptr;   // [nseg] pinned
};

namespace {

int nmodes_of(int d, int p) { return d == 2 ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1); }

// Gauss-Legendre nodes (ascending) and weights: Newton on P_Q started from
// the asymptotic root estimate; the rule is symmetrised exactly.
void gauss_rule(int Q, double* x, double* w) {
  for (int k = 0; k < (Q + 1) / 2; ++k) {
    double z = std::cos(M_PI * (4.0 * k + 3.0) / (4.0 * Q + 2.0));
    double dP = 1.0;
    for (int it = 0; it < 50; ++it) {
      double pm = 1.0, p = z;
      for (int j = 1; j < Q; ++j) {
        double pn = ((2 * j + 1) * z * p - j * pm) / (j + 1);
        pm = p;
        p = pn;
      }
      if (Q == 1) { p = z; pm = 1.0; }
      dP = Q * (pm - z * p) / (1.0 - z * z);
      double dz = p / dP;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * std::max(1.0, std::fabs(z))) break;
    }
    double pm = 1.0, p = z;
    for (int j = 1; j < Q; ++j) {
      double pn = ((2 * j + 1) * z * p - j * pm) / (j + 1);
      pm = p;
      p = pn;
    }
    if (Q == 1) { p = z; pm = 1.0; }
    dP = Q * (pm - z * p) / (1.0 - z * z);
    double wk = 2.0 / ((1.0 - z * z) * dP * dP);
    x[Q - 1 - k] = z;
    x[k] = -z;
    w[Q - 1 - k] = wk;
    w[k] = wk;
  }
  if (Q % 2 == 1) x[Q / 2] = 0.0;
}

// Orthonormal Legendre sqrt((2a+1)/2) P_a(t) and derivative, a = 0..pm.
void legendre_values(int pm, double t, double* L, double* dL) {
  double P[10], dP[10];
  P[0] = 1.0;
  dP[0] = 0.0;
  P[1] = t;
  dP[1] = 1.0;
  for (int a = 1; a < pm; ++a) {
    P[a + 1] = ((2 * a + 1) * t * P[a] - a * P[a - 1]) / (a + 1);
    dP[a + 1] = dP[a - 1] + (2 * a + 1) * P[a];
  }
  for (int a = 0; a <= pm; ++a) {
    double s = std::sqrt(a + 0.5);
    L[a] = s * P[a];
    dL[a] = s * dP[a];
  }
}

std::vector<std::array<int, 3>> hier_modes(int d, int p) {
  std::vector<std::array<int, 3>> v;
  for (int c = 0; c <= (d == 3 ? p : 0); ++c)
    for (int b = 0; b <= p; ++b)
      for (int a = 0; a <= p; ++a) v.push_back({a, b, c});
  std::stable_sort(v.begin(), v.end(), [](const std::array<int, 3>& l, const std::array<int, 3>& r) {
    int ml = std::max(l[0], std::max(l[1], l[2])), mr = std::max(r[0], std::max(r[1], r[2]));
    if (ml != mr) return ml < mr;
    if (l[0] != r[0]) return l[0] < r[0];
    if (l[1] != r[1]) return l[1] < r[1];
    return l[2] < r[2];
  });
  return v;
}

void fill_tabdata(TabData& t, int d, int p, const std::vector<std::array<int, 3>>& modes) {
  std::memset(&t, 0, sizeof t);
  const int Q = p + 2;
  gauss_rule(Q, t.x, t.w);
  for (int i = 0; i < Q; ++i) {
    double L[10], dL[10];
    legendre_values(std::max(p, 1), t.x[i], L, dL);
    for (int a = 0; a <= p; ++a) { t.L[a][i] = L[a]; t.dL[a][i] = dL[a]; }
  }
  for (int s = 0; s < 2; ++s) {
    double L[10], dL[10];
    legendre_values(std::max(p, 1), s ? 1.0 : -1.0, L, dL);
    for (int a = 0; a <= p; ++a) t.Lb[a][s] = L[a];
  }
  const int N = nmodes_of(d, p);
  for (int k = 0; k < N; ++k)
    for (int r = 0; r < 3; ++r) t.m[k][r] = modes[k][r];
}

// Tangents of the element map at xi (biquadratic through nine nodes in 2D,
// trilinear, or triquadratic through 27 nodes, in 3D); returns det and c[r]
// (see geom in the kernels).
double host_geom(int d, int ng, const double* X, const double* xi, double c[3][3]) {
  double t[3][3] = {};
  auto lq = [](int a, double z) { return a == 0 ? 0.5 * z * (z - 1.0) : a == 1 ? 1.0 - z * z : 0.5 * z * (z + 1.0); };
  auto dlq = [](int a, double z) { return a == 0 ? z - 0.5 : a == 1 ? -2.0 * z : z + 0.5; };
  if (d == 3 && ng == 27) {
    for (int k = 0; k < 27; ++k) {
      const int a[3] = {k % 3, (k / 3) % 3, k / 9};
      for (int r = 0; r < 3; ++r) {
        double g = 1.0;
        for (int q = 0; q < 3; ++q) g *= (q == r) ? dlq(a[q], xi[q]) : lq(a[q], xi[q]);
        for (int b = 0; b < 3; ++b) t[r][b] += g * X[k * 3 + b];
      }
    }
  } else if (d == 2) {
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 2; ++q) {
          t[0][q] += dlq(a, xi[0]) * lq(b, xi[1]) * X[(a + 3 * b) * 2 + q];
          t[1][q] += lq(a, xi[0]) * dlq(b, xi[1]) * X[(a + 3 * b) * 2 + q];
        }
    c[0][0] = t[1][1]; c[0][1] = -t[1][0];
    c[1][0] = -t[0][1]; c[1][1] = t[0][0];
    return t[0][0] * t[1][1] - t[0][1] * t[1][0];
  }
  for (int k = 0; k < (ng == 27 ? 0 : 1 << d); ++k)
    for (int r = 0; r < d; ++r) {
      double g = 1.0;
      for (int q = 0; q < d; ++q) {
        double s = ((k >> q) & 1) ? 1.0 : -1.0;
        g *= (q == r) ? 0.5 * s : 0.5 * (1.0 + s * xi[q]);
      }
      for (int a = 0; a < d; ++a) t[r][a] += g * X[k * d + a];
    }
  if (d == 2) {
    c[0][0] = t[1][1]; c[0][1] = -t[1][0];
    c[1][0] = -t[0][1]; c[1][1] = t[0][0];
    return t[0][0] * t[1][1] - t[0][1] * t[1][0];
  }
  for (int r = 0; r < 3; ++r) {
    const double* a = t[(r + 1) % 3];
    const double* b = t[(r + 2) % 3];
    c[r][0] = a[1] * b[2] - a[2] * b[1];
    c[r][1] = a[2] * b[0] - a[0] * b[2];
    c[r][2] = a[0] * b[1] - a[1] * b[0];
  }
  return t[0][0] * c[0][0] + t[0][1] * c[0][1] + t[0][2] * c[0][2];
}

eg_status fail(eg_handle* h, eg_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

eg_status hipfail(eg_handle* h, hipError_t e, const char* where) {
  return fail(h, EG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hipfail((h), e_, #call); \
  } while (0)

template <class T>
eg_status dalloc(eg_handle* h, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return EG_OK;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(h, EG_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
  h->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return EG_OK;
}

hipEvent_t next_event(eg_handle* h) {
  if (h->evused == h->evpool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->evpool.push_back(e);
  }
  return h->evpool[h->evused++];
}

// Launch with optional event timing of kernel class cls at level p.
#define PCALL(h, cls, p, call)                                          \
  do {                                                                  \
    hipEvent_t a_ = nullptr;                                            \
    if ((h)->prof && (a_ = next_event(h))) (void)hipEventRecord(a_, (h)->st); \
    HIPCHK(h, call);                                                    \
    if (a_) {                                                           \
      hipEvent_t b_ = next_event(h);                                    \
      if (b_) {                                                         \
        (void)hipEventRecord(b_, (h)->st);                              \
        (h)->recs.push_back({(cls), (p), a_, b_});                      \
      }                                                                 \
    }                                                                   \
  } while (0)

#define ECHK(call)                 \
  do {                             \
    eg_status s_ = (call);         \
    if (s_ != EG_OK) return s_;    \
  } while (0)

// Mesh set-up: faces matched through their vertex sets, orientation codes of
// the neighbour's face points, element geometry (|E|, |dE|, h_E) and the
// Cholesky factor of the phi mass matrix, all with the (p_max+2)-point rule
// (exact for the mass matrix of multilinear elements).
// The nine nodes of a straight-sided quad (corners Xc[a + 2b]): the bilinear
// map written as a biquadratic one.
void straight_nodes9(const double Xc[][3], double* X) {
  for (int b = 0; b < 3; ++b)
    for (int a = 0; a < 3; ++a)
      for (int q = 0; q < 2; ++q) {
        const double wa[2] = {1.0 - 0.5 * a, 0.5 * a}, wb[2] = {1.0 - 0.5 * b, 0.5 * b};
        double v = 0.0;
        for (int j = 0; j < 2; ++j)
          for (int i = 0; i < 2; ++i) v += wa[i] * wb[j] * Xc[i + 2 * j][q];
        X[(a + 3 * b) * 2 + q] = v;
      }
}

// The 27 nodes of a straight-sided hex (corners Xc[a + 2b + 4c]): the
// trilinear map written as a triquadratic one.
void straight_nodes27(const double Xc[][3], double* X) {
  for (int k = 0; k < 27; ++k) {
    const int n[3] = {k % 3, (k / 3) % 3, k / 9};
    for (int q = 0; q < 3; ++q) {
      double v = 0.0;
      for (int j = 0; j < 8; ++j) {
        double w = 1.0;
        for (int r = 0; r < 3; ++r) w *= ((j >> r) & 1) ? 0.5 * n[r] : 1.0 - 0.5 * n[r];
        v += w * Xc[j][q];
      }
      X[k * 3 + q] = v;
    }
  }
}

eg_status setup_mesh(eg_handle* h, const eg_mesh* mesh, std::vector<double>& xv, std::vector<int>& nbr,
                     std::vector<uint8_t>& ncode, std::vector<double>& Lpk, std::vector<double>& Gpk,
                     std::vector<double>& hE, double& omega, std::vector<double>& vol) {
  const int d = mesh->dim, ne = mesh->n_elem, nf = 2 * d, nc = 1 << d, ncf = 1 << (d - 1);
  // geometry nodes per element: 9 per quad, 8 per straight hex, 27 per curved hex
  const int ng = (mesh->elem_geo && d == 3) ? 27 : eg::geo_nodes(d);
  auto near = [](double a, double b) { return std::fabs(a - b) <= 1e-12 * std::max(1.0, std::fabs(a)); };
  xv.assign((size_t)ne * ng * d, 0.0);
  for (int e = 0; e < ne; ++e) {
    double Xc[8][3];
    for (int k = 0; k < nc; ++k) {
      int vid = mesh->elem_vert[(size_t)e * nc + k];
      if (vid < 0 || vid >= mesh->n_vert) return fail(h, EG_ERR_MESH, "vertex index out of range");
      for (int a = 0; a < d; ++a) Xc[k][a] = mesh->xyz[(size_t)vid * d + a];
    }
    double* X = &xv[(size_t)e * ng * d];
    if (mesh->elem_geo) {
      const double* G = &mesh->elem_geo[(size_t)e * ng * d];
      for (int k = 0; k < ng * d; ++k) X[k] = G[k];
      for (int k = 0; k < nc; ++k) {
        int node = 0;  // the node at vertex k: digits 2 * bit_r in base 3
        for (int r = 0, p3 = 1; r < d; ++r, p3 *= 3) node += 2 * ((k >> r) & 1) * p3;
        for (int a = 0; a < d; ++a)
          if (!near(Xc[k][a], X[node * d + a]))
            return fail(h, EG_ERR_MESH, "curved element node at a corner differs from its vertex");
      }
    } else if (d == 3) {
      for (int k = 0; k < nc; ++k)
        for (int a = 0; a < d; ++a) X[k * d + a] = Xc[k][a];
    } else {
      straight_nodes9(Xc, X);
    }
  }
  nbr.assign((size_t)ne * nf, 0);
  ncode.assign((size_t)ne * nf, 0);
  auto face_corners = [&](int e, int lf, int* vv) {
    int r = lf / 2, s = lf % 2, ta[2], k = 0;
    for (int a = 0; a < d; ++a) if (a != r) ta[k++] = a;
    for (int c = 0; c < ncf; ++c) {
      int loc = s << r;
      for (int q = 0; q < d - 1; ++q) if ((c >> q) & 1) loc |= 1 << ta[q];
      vv[c] = mesh->elem_vert[(size_t)e * nc + loc];
    }
  };
  std::map<std::array<int, 4>, std::pair<int, int>> pending;
  std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> pairs;
  for (int e = 0; e < ne; ++e)
    for (int lf = 0; lf < nf; ++lf) {
      int tag = mesh->bface_tag[(size_t)e * nf + lf];
      if (tag == EG_FACE_WALL) { nbr[(size_t)e * nf + lf] = eg::NB_WALL; continue; }
      if (tag == EG_FACE_SYMMETRY) {
        nbr[(size_t)e * nf + lf] = eg::NB_WALL;
        ncode[(size_t)e * nf + lf] = eg::NCODE_SYMMETRY;
        continue;
      }
      if (tag == EG_FACE_FARFIELD) { nbr[(size_t)e * nf + lf] = eg::NB_FAR; continue; }
      if (tag != EG_FACE_INTERIOR) return fail(h, EG_ERR_MESH, "unknown boundary tag");
      int vv[4] = {-1, -1, -1, -1};
      face_corners(e, lf, vv);
      std::array<int, 4> key{vv[0], vv[1], vv[2], vv[3]};
      std::sort(key.begin(), key.begin() + ncf);
      auto it = pending.find(key);
      if (it == pending.end()) pending.emplace(key, std::make_pair(e, lf));
      else { pairs.push_back({it->second, {e, lf}}); pending.erase(it); }
    }
  if (!pending.empty()) return fail(h, EG_ERR_MESH, "interior face without a matching neighbour face");
  // orientation code of the map from one side's face coordinates to the other's
  auto code_of = [&](int e, int lf, int e2, int lf2, uint8_t& code) -> bool {
    int va[4], vb[4];
    face_corners(e, lf, va);
    face_corners(e2, lf2, vb);
    auto pos = [&](int vid, double* sc) {
      for (int c = 0; c < ncf; ++c) if (vb[c] == vid) {
        for (int q = 0; q < d - 1; ++q) sc[q] = ((c >> q) & 1) ? 1.0 : -1.0;
        return true;
      }
      return false;
    };
    double s0[2] = {0, 0}, s1[2] = {0, 0}, s2[2] = {0, 0};
    if (!pos(va[0], s0) || !pos(va[1], s1)) return false;
    if (d == 3 && !pos(va[2], s2)) return false;
    int Mx[2][2] = {{0, 0}, {0, 0}};
    for (int k = 0; k < d - 1; ++k) {
      Mx[k][0] = (int)std::lround(0.5 * (s1[k] - s0[k]));
      if (d == 3) Mx[k][1] = (int)std::lround(0.5 * (s2[k] - s0[k]));
    }
    // every corner must map through M with zero offset
    for (int c = 0; c < ncf; ++c) {
      double sl[2], sr[2] = {0, 0};
      for (int q = 0; q < d - 1; ++q) sl[q] = ((c >> q) & 1) ? 1.0 : -1.0;
      if (!pos(va[c], sr)) return false;
      for (int k = 0; k < d - 1; ++k) {
        double sm = 0.0;
        for (int q = 0; q < d - 1; ++q) sm += Mx[k][q] * sl[q];
        if (sm != sr[k]) return false;
      }
    }
    int swap = 0, f0 = 0, f1 = 0;
    if (d == 2) {
      f0 = Mx[0][0] < 0;
    } else if (Mx[0][0] != 0) {
      f0 = Mx[0][0] < 0;
      f1 = Mx[1][1] < 0;
    } else {
      swap = 1;
      f0 = Mx[0][1] < 0;
      f1 = Mx[1][0] < 0;
    }
    code = (uint8_t)(lf2 | (swap << 3) | (f0 << 4) | (f1 << 5));
    return true;
  };
  for (auto& pr : pairs) {
    int e1 = pr.first.first, l1 = pr.first.second, e2 = pr.second.first, l2 = pr.second.second;
    uint8_t c12, c21;
    if (!code_of(e1, l1, e2, l2, c12) || !code_of(e2, l2, e1, l1, c21))
      return fail(h, EG_ERR_MESH, "non-conforming face");
    if (mesh->elem_geo) {
      // a curved face is shared only if both sides put its nodes (3 per
      // edge, 9 per quadrilateral face) at the same points
      auto face_nodes = [&](int e, int lf, std::vector<const double*>& out) {
        const int r = lf / 2, s2 = 2 * (lf % 2);
        out.clear();
        for (int k = 0; k < ng; ++k) {
          int dig = k;
          for (int q = 0; q < r; ++q) dig /= 3;
          if (dig % 3 == s2) out.push_back(&xv[((size_t)e * ng + k) * d]);
        }
      };
      std::vector<const double*> f1, f2;
      face_nodes(e1, l1, f1);
      face_nodes(e2, l2, f2);
      for (const double* a : f1) {
        bool found = false;
        for (const double* b : f2) {
          bool same = true;
          for (int q = 0; q < d; ++q) same = same && near(a[q], b[q]);
          found = found || same;
        }
        if (!found) return fail(h, EG_ERR_MESH, "non-conforming curved face");
      }
    }
    nbr[(size_t)e1 * nf + l1] = e2;
    ncode[(size_t)e1 * nf + l1] = c12;
    nbr[(size_t)e2 * nf + l2] = e1;
    ncode[(size_t)e2 * nf + l2] = c21;
  }
  // geometry and basis
  const int pm = h->pmax, Q = pm + 2, N = nmodes_of(d, pm), NT = N * (N + 1) / 2;
  double gx[8], gw[8];
  gauss_rule(Q, gx, gw);
  Lpk.assign((size_t)ne * NT, 0.0);
  Gpk.assign((size_t)ne * NT, 0.0);
  hE.assign(ne, 0.0);
  vol.assign(ne, 0.0);
  int nq = 1;
  for (int r = 0; r < d; ++r) nq *= Q;
  // phi at the volume points (element independent)
  std::vector<double> phi((size_t)nq * N);
  for (int q = 0; q < nq; ++q) {
    int iq[3] = {0, 0, 0}, t = q;
    for (int r = 0; r < d; ++r) { iq[r] = t % Q; t /= Q; }
    for (int k = 0; k < N; ++k) {
      double v = 1.0;
      for (int r = 0; r < d; ++r) {
        double L[10], dL[10];
        legendre_values(std::max(pm, 1), gx[iq[r]], L, dL);
        v *= L[h->modes[k][r]];
      }
      phi[(size_t)q * N + k] = v;
    }
  }
  int bad = 0;
  for (int e = 0; e < ne; ++e) {
    const double* X = &xv[(size_t)e * ng * d];
    std::vector<double> G((size_t)N * N, 0.0), L((size_t)N * N, 0.0);
    double V = 0.0, S = 0.0;
    for (int q = 0; q < nq; ++q) {
      int iq[3] = {0, 0, 0}, t = q;
      double xi[3], wq = 1.0;
      for (int r = 0; r < d; ++r) { iq[r] = t % Q; t /= Q; xi[r] = gx[iq[r]]; wq *= gw[iq[r]]; }
      double c[3][3];
      double det = host_geom(d, ng, X, xi, c);
      if (!(det > 0.0)) bad++;
      V += wq * det;
      const double* ph = &phi[(size_t)q * N];
      for (int i = 0; i < N; ++i)
        for (int j = 0; j <= i; ++j) G[(size_t)i * N + j] += wq * det * ph[i] * ph[j];
    }
    for (int k = 0; k < nc; ++k) {  // corners
      double xi[3];
      for (int r = 0; r < d; ++r) xi[r] = ((k >> r) & 1) ? 1.0 : -1.0;
      double c[3][3];
      if (!(host_geom(d, ng, X, xi, c) > 0.0)) bad++;
    }
    for (int lf = 0; lf < nf; ++lf) {
      int r = lf / 2, ta[2], kk = 0;
      for (int a = 0; a < d; ++a) if (a != r) ta[kk++] = a;
      int nqf = nq / Q;
      for (int k = 0; k < nqf; ++k) {
        double xi[3], wk = 1.0;
        xi[r] = (lf & 1) ? 1.0 : -1.0;
        int t = k;
        for (int q2 = 0; q2 < d - 1; ++q2) { xi[ta[q2]] = gx[t % Q]; wk *= gw[t % Q]; t /= Q; }
        double c[3][3];
        host_geom(d, ng, X, xi, c);
        double a2 = 0.0;
        for (int a = 0; a < d; ++a) a2 += c[r][a] * c[r][a];
        S += wk * std::sqrt(a2);
      }
    }
    vol[e] = V;
    hE[e] = 2.0 * d * V / S;
    // Cholesky G = L L^T
    for (int j = 0; j < N; ++j) {
      double sjj = G[(size_t)j * N + j];
      for (int k = 0; k < j; ++k) sjj -= L[(size_t)j * N + k] * L[(size_t)j * N + k];
      if (!(sjj > 0.0)) { bad++; sjj = 1.0; }
      L[(size_t)j * N + j] = std::sqrt(sjj);
      for (int i = j + 1; i < N; ++i) {
        double sij = G[(size_t)i * N + j];
        for (int k = 0; k < j; ++k) sij -= L[(size_t)i * N + k] * L[(size_t)j * N + k];
        L[(size_t)i * N + j] = sij / L[(size_t)j * N + j];
      }
    }
    for (int i = 0; i < N; ++i)
      for (int j = 0; j <= i; ++j) {
        Lpk[(size_t)e * NT + i * (i + 1) / 2 + j] = L[(size_t)i * N + j];
        Gpk[(size_t)e * NT + i * (i + 1) / 2 + j] = G[(size_t)i * N + j];
      }
  }
  if (bad) return fail(h, EG_ERR_MESH, "inverted element or singular mass matrix");
  omega = 0.0;
  for (int e = 0; e < ne; ++e) omega += vol[e];
  return EG_OK;
}

eg_status sync_status(eg_handle* h) {
  HIPCHK(h, hipStreamSynchronize(h->st));
  return EG_OK;
}

int NB(const eg_handle* h, int p) { return h->M.V * nmodes_of(h->M.d, p); }

// Arithmetic of the kernels at level p.  Mixed mode, phase A: residuals,
// blocks, LU and stage solves in FP32 on p >= 1.  Phase B: every residual in
// FP64 and only the blocks, their LU and the stage solves in FP32, so that
// the nonlinear evaluations that drive the state carry no FP32 noise.
int blk_prec(const eg_handle* h, int p) { return (h->mixed && p >= 1) ? eg::PREC_FP32 : eg::PREC_FP64; }
int res_prec(const eg_handle* h, int p) {
  return (h->mixed && !h->phase_b && p >= 1) ? eg::PREC_FP32 : eg::PREC_FP64;
}

// Mixed mode switches to phase B for good once the FP64 residual norm has
// dropped below this fraction of r_1, has not reached a new minimum for
// EG_STALL_CYCLES cycles, or has fallen by less than 10% over the last
// EG_SLOW_CYCLES cycles (the FP32 noise floor of phase A is ~1e-5 r_1 in
// 2D; in 3D the norm creeps along a plateau near 1e-4 r_1 instead).
constexpr double EG_PHASE_B_DROP = 1e-4;
constexpr int EG_STALL_CYCLES = 100;
constexpr int EG_SLOW_CYCLES = 50;
constexpr double EG_SLOW_FACTOR = 0.9;
static_assert(EG_SLOW_CYCLES < 64, "ring of past norms");

bool phase_a_over(double rn, double r1, int n, int nmin, const double* ring) {
  if (rn <= EG_PHASE_B_DROP * r1 || n - nmin >= EG_STALL_CYCLES) return true;
  return n > EG_SLOW_CYCLES && rn > EG_SLOW_FACTOR * ring[(n - EG_SLOW_CYCLES) % 64];
}

double cfl_ramp(double cfl_max, double rn, double rref, int n, int pmax) {
  double a = (rn > 0.0) ? rref / rn : HUGE_VAL;
  double b = 1.0 + (n - 1.0) / (2.0 * pmax + 1.0);
  return std::min(cfl_max, std::max(a, b));
}

// EXP1 on the phi-coordinate p = 0 state ut0 with optional forcing ft0; with
// update = false the final update of ut0 is left to the caller.
eg_status run_exp1(eg_handle* h, double cfl, double* ut0, const double* ft0, bool update = true) {
  const DevMesh& M = h->M;
  PCALL(h, EG_K_P0_SETUP, 0, eg::launch_p0_setup(M, ut0, ft0, h->pmax, cfl, 1, h->u0, h->b0, h->Ad, h->Ao, h->dt0, h->st));
  PCALL(h, EG_K_ARNOLDI, 0, eg::launch_arnoldi(M, h->m, h->nblk_arn, h->Ad, h->Ao, h->b0, h->Vb, h->H, h->part1,
                                                h->part2, h->info, h->arn_st, h->arn_wn0, h->arn_W, h->H2, h->st));
  PCALL(h, EG_K_PHI1, 0, eg::launch_phi1(h->m, h->M.nseg, h->H, h->H2, h->info, h->y, h->dfail, h->st));
  if (update) PCALL(h, EG_K_EXP1_UPDATE, 0, eg::launch_exp1_update(M, h->m, h->Vb, h->y, h->info, h->u0, ut0, h->st));
  return EG_OK;
}

// One PRK step at level p on ut[p] with forcing ft (may be null); rt[p] must
// hold the stage-1 residual R_p(ut) + ft.
eg_status run_prk(eg_handle* h, int p, double cfl, const double* ft) {
  const DevMesh& M = h->M;
  const int N = nmodes_of(M.d, p), n = NB(h, p);
  PCALL(h, EG_K_TIMESTEP, p, eg::launch_timestep(M, p, N, cfl, 1.0, h->ut[p], h->dtau, h->st));
  const int pb = blk_prec(h, p), pr = res_prec(h, p);
  PCALL(h, EG_K_JACOBIAN_LU, p,
        eg::launch_jacobian(M, h->tabs[p], p, h->ut[p], h->dtau, h->F[p], h->perm[p], h->dfail, true, pb, h->st));
  for (int k = 1; k <= h->s; ++k) {
    if (k > 1)
      PCALL(h, EG_K_RESIDUAL, p, eg::launch_residual(M, h->tabs[p], p, h->ut[p], ft, h->rt[p], pr, h->st));
    const double beta = 1.0 / (h->s - k + 1.0);
    // the first stage starts from ut and keeps it in un for the later stages
    PCALL(h, EG_K_PRK_STAGE, p,
          eg::launch_prk_stage(M, n, h->F[p], h->perm[p], h->rt[p], nullptr, k == 1 ? nullptr : h->un[p], h->ut[p],
                               beta, pb, h->st, k == 1 ? h->un[p] : nullptr));
  }
  return EG_OK;
}

// Descending half of the V-cycle below level p >= 1 (Section 2.4): PRK,
// restriction with FAS forcing, recursion, down to the EXP1 step on p = 0
// without its final update.  Requires rt[p] = R_p + f_p.
eg_status vc_down(eg_handle* h, int p, double cfl) {
  const DevMesh& M = h->M;
  const double* fp = (p == h->pmax) ? nullptr : h->ft[p];
  if (p == 0) return run_exp1(h, cfl, h->ut[0], fp, false);
  const int pr = res_prec(h, p);
  if (p == h->pmax && pr == eg::PREC_FP32) {
    // phase A: rt holds R64(u^n) (the entry norm's residual); the top level
    // takes d = R64(u^n) - R32(u^n) as its forcing for this cycle, so that the
    // first stage sees the FP64 residual and the later ones R32 + d
    const size_t K = (size_t)M.ne * NB(h, p);
    PCALL(h, EG_K_RESIDUAL, p, eg::launch_residual(M, h->tabs[p], p, h->ut[p], nullptr, h->tmp2, pr, h->st));
    PCALL(h, EG_K_TRANSFER, p, eg::launch_sub(h->rt[p], h->tmp2, h->ft[p], K, h->st));
    fp = h->ft[p];
  }
  ECHK(run_prk(h, p, cfl, fp));
  const int N = nmodes_of(M.d, p);
  PCALL(h, EG_K_RESIDUAL, p, eg::launch_residual(M, h->tabs[p], p, h->ut[p], fp, h->rt[p], pr, h->st));
  PCALL(h, EG_K_TRANSFER, p, eg::launch_restrict(M, p, h->ut[p], h->ut[p - 1], h->uc0[p - 1], h->st));
  {
    // FAS forcing of level p - 1 with that level's own residual R_{p-1}(v0)
    // (FP32 on p - 1 >= 1 in mixed mode, FP64 on p = 0), fused with the
    // forcing f = trunc(r_p) - R_{p-1} and rt[p - 1] = trunc(r_p)
    const int pc = res_prec(h, p - 1);
    eg::FasOut fas;
    fas.rhat = h->rt[p];
    fas.Nf = N;
    fas.fc = h->ft[p - 1];
    PCALL(h, EG_K_RESIDUAL, p - 1,
          eg::launch_residual(M, h->tabs[p - 1], p - 1, h->ut[p - 1], nullptr, h->rt[p - 1], pc, h->st, fas));
  }
  return vc_down(h, p - 1, cfl);
}

// One V-cycle (Section 2.4): the descent, then the EXP1 update on p = 0 and
// the prolongation of the coarse corrections up to p_max in one kernel (the
// cycle has no post-smoothing, so nothing runs between them).
eg_status vc_rec(eg_handle* h, int p, double cfl) {
  if (p == 0) return run_exp1(h, cfl, h->ut[0], nullptr);
  ECHK(vc_down(h, p, cfl));
  eg::UpChain c{};
  for (int l = 0; l <= p; ++l) {
    c.ut[l] = h->ut[l];
    c.uc0[l] = h->uc0[l];
    c.N[l] = nmodes_of(h->M.d, l);
  }
  c.pmax = p;
  PCALL(h, EG_K_EXP1_UPDATE, 0, eg::launch_exp1_prolong(h->M, h->m, h->Vb, h->y, h->info, h->u0, c, h->st));
  return EG_OK;
}

// Residual and norm of the phi-coordinate state ut[pmax] -> host value.
eg_status entry_norm(eg_handle* h, double* rn) {
  const DevMesh& M = h->M;
  const int p = h->pmax, N = nmodes_of(M.d, p);
  // the norm is always of the FP64 residual
  PCALL(h, EG_K_RESIDUAL, p,
        eg::launch_residual(M, h->tabs[p], p, h->ut[p], nullptr, h->rt[p], eg::PREC_FP64, h->st));
  PCALL(h, EG_K_NORM, p, eg::launch_norm(M, N, h->rt[p], h->npart, h->nout, h->st));
  HIPCHK(h, hipMemcpyAsync(h->hpin, h->nout, sizeof(double), hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipMemcpyAsync(h->hpin + 1, h->dfail, sizeof(int), hipMemcpyDeviceToHost, h->st));
  ECHK(sync_status(h));
  *rn = h->hpin[0];
  int fl = 0;
  std::memcpy(&fl, h->hpin + 1, sizeof(int));
  if (fl) return fail(h, EG_ERR_DIVERGED, "singular pivot in a block factorisation or in phi_1");
  return EG_OK;
}

// ---------------------------------------------------------------------------
// Adjoint of the steady problem (drag sensitivity): (dR/du)^T lambda + g = 0
// solved by the transposed linear V-cycle: on p >= 1 the PRK smoother with the
// transposed blocks Pt^T = G/dtau - Dt^T (same LU factors, transposed
// solves), the adjoint residual restricted by truncation and the correction
// prolongated by padding (the transposes of the forward transfers), and on
// p = 0 one EXP1 step of the linear adjoint problem with the transposed
// p = 0 operator.  The blocks, dtau (at CFL_max) and the pointwise flux
// Jacobians are evaluated once at the linearisation state.
// ---------------------------------------------------------------------------
eg_status adj_alloc(eg_handle* h) {
  if (h->adj_ready) return EG_OK;
  const DevMesh& M = h->M;
  const int d = M.d, ne = M.ne, V = M.V;
  for (int p = 0; p <= h->pmax; ++p) {
    const size_t K = (size_t)ne * V * nmodes_of(d, p);
    ECHK(dalloc(h, &h->adj_u[p], K));
    ECHK(dalloc(h, &h->lam[p], K));
    ECHK(dalloc(h, &h->lamn[p], K));
    ECHK(dalloc(h, &h->gq[p], K));
    ECHK(dalloc(h, &h->rho[p], K));
    if (p >= 1) {
      const size_t n = (size_t)V * nmodes_of(d, p);
      ECHK(dalloc(h, &h->adj_bc[p], (size_t)ne * eg::jac_points_size(d, p)));
      ECHK(dalloc(h, &h->adj_F[p], (size_t)ne * n * n));
      ECHK(dalloc(h, &h->adj_perm[p], (size_t)ne * n));
    }
  }
  ECHK(dalloc(h, &h->AdT, (size_t)ne * V * V));
  ECHK(dalloc(h, &h->AoT, (size_t)ne * M.NF * V * V));
  ECHK(dalloc(h, &h->zero0, (size_t)ne * V));
  HIPCHK(h, eg::launch_fill0(h->zero0, (size_t)ne * V, h->st));
  h->adj_ready = true;
  return EG_OK;
}

eg_status adj_supported(eg_handle* h) {
  for (int p = 1; p <= h->pmax; ++p)
    if (!eg::prk_tr_supported(NB(h, p)))
      return fail(h, EG_ERR_UNSUPPORTED, "adjoint: no transposed block solve for this order (2D p <= 4, 3D p <= 3)");
  return EG_OK;
}

// Linearisation state u (psi coordinates, level p_max) on every level, the
// pointwise Jacobians and FP64 block factors for p >= 1, the transposed p = 0
// operator.
eg_status adj_setup(eg_handle* h, const double* u_dev) {
  const DevMesh& M = h->M;
  const int pm = h->pmax;
  HIPCHK(h, eg::launch_basis(M, nmodes_of(M.d, pm), u_dev, h->adj_u[pm], 0, h->st));
  for (int p = pm; p >= 1; --p) HIPCHK(h, eg::launch_restrict(M, p, h->adj_u[p], h->adj_u[p - 1], h->uc0[p - 1], h->st));
  for (int p = 1; p <= pm; ++p) {
    DevMesh M2 = M;
    M2.bc = h->adj_bc[p];
    HIPCHK(h, eg::launch_timestep(M, p, nmodes_of(M.d, p), h->cfl_max, 1.0, h->adj_u[p], h->dtau, h->st));
    HIPCHK(h, eg::launch_jac_points(M, h->tabs[p], p, h->adj_u[p], h->adj_bc[p], h->st));
    HIPCHK(h, eg::launch_jacobian(M2, h->tabs[p], p, h->adj_u[p], h->dtau, h->adj_F[p], h->adj_perm[p], h->dfail,
                                  true, eg::PREC_FP64, h->st));
  }
  HIPCHK(h, eg::launch_p0_setup(M, h->adj_u[0], nullptr, pm, h->cfl_max, 1, h->u0, h->b0, h->Ad, h->Ao, h->dt0, h->st));
  HIPCHK(h, eg::launch_p0_transpose(M, h->Ad, h->Ao, h->dt0, h->AdT, h->AoT, h->st));
  return EG_OK;
}

// One transposed V-cycle below level p on lam[p] with forcing gq[p].
eg_status adj_vc(eg_handle* h, int p) {
  const DevMesh& M = h->M;
  if (p == 0) {
    HIPCHK(h, eg::launch_adj_p0_rhs(M, h->gq[0], h->dt0, h->b0, h->st));
    HIPCHK(h, eg::launch_arnoldi(M, h->m, h->nblk_arn, h->AdT, h->AoT, h->b0, h->Vb, h->H, h->part1, h->part2,
                                 h->info, h->arn_st, h->arn_wn0, h->arn_W, h->H2, h->st));
    HIPCHK(h, eg::launch_phi1(h->m, h->M.nseg, h->H, h->H2, h->info, h->y, h->dfail, h->st));
    HIPCHK(h, eg::launch_exp1_update(M, h->m, h->Vb, h->y, h->info, h->zero0, h->lam[0], h->st));
    return EG_OK;
  }
  const int n = NB(h, p), N = nmodes_of(M.d, p), Nc = nmodes_of(M.d, p - 1), rows = M.ne * M.V;
  const size_t K = (size_t)M.ne * n;
  HIPCHK(h, eg::launch_copy(h->lam[p], h->lamn[p], K, h->st));
  for (int k = 1; k <= h->s; ++k) {
    HIPCHK(h, eg::launch_adj_residual(M, h->tabs[p], p, h->lam[p], h->gq[p], h->adj_bc[p], h->rho[p], h->st));
    const double beta = 1.0 / (h->s - k + 1.0);
    HIPCHK(h, eg::launch_prk_stage_tr(M, n, h->adj_F[p], h->adj_perm[p], h->rho[p], h->lamn[p], h->lam[p], beta,
                                      h->st));
  }
  HIPCHK(h, eg::launch_adj_residual(M, h->tabs[p], p, h->lam[p], h->gq[p], h->adj_bc[p], h->rho[p], h->st));
  HIPCHK(h, eg::launch_trunc(h->rho[p], h->gq[p - 1], N, Nc, rows, h->st));
  HIPCHK(h, eg::launch_fill0(h->lam[p - 1], (size_t)rows * Nc, h->st));
  ECHK(adj_vc(h, p - 1));
  HIPCHK(h, eg::launch_pad_add(h->lam[p], h->lam[p - 1], N, Nc, rows, h->st));
  return EG_OK;
}

// ||psi-coordinate adjoint residual at p_max||_2 -> host.
eg_status adj_norm(eg_handle* h, double* out) {
  const DevMesh& M = h->M;
  const int pm = h->pmax, N = nmodes_of(M.d, pm);
  const size_t K = (size_t)M.ne * M.V * N;
  HIPCHK(h, eg::launch_adj_residual(M, h->tabs[pm], pm, h->lam[pm], h->gq[pm], h->adj_bc[pm], h->rho[pm], h->st));
  HIPCHK(h, eg::launch_basis(M, N, h->rho[pm], h->tmp2, 2, h->st));
  HIPCHK(h, eg::launch_sum(h->tmp2, h->tmp2, K, h->spart, 1, h->sout, h->st));
  HIPCHK(h, hipMemcpyAsync(h->hpin, h->sout, sizeof(double), hipMemcpyDeviceToHost, h->st));
  HIPCHK(h, hipMemcpyAsync(h->hpin + 1, h->dfail, sizeof(int), hipMemcpyDeviceToHost, h->st));
  ECHK(sync_status(h));
  *out = h->hpin[0];
  int fl = 0;
  std::memcpy(&fl, h->hpin + 1, sizeof(int));
  if (fl) return fail(h, EG_ERR_DIVERGED, "singular pivot in a block factorisation or in phi_1");
  return EG_OK;
}

}  // namespace

namespace eg {
// The Gauss-Legendre rule mapped to [0, 1] (points ascending, weights summing
// to 1), for the tetrahedron / prism set-up.
void gauss_rule01(int Q, double* x, double* w) {
  gauss_rule(Q, x, w);
  for (int k = 0; k < Q; ++k) {
    x[k] = 0.5 * (1.0 + x[k]);
    w[k] *= 0.5;
  }
}
}  // namespace eg

namespace {

// Free-stream conserved state of a parameter set (rho = 1, p = 1/gamma).
void freestream_of(const eg_params* prm, int d, double* U) {
  const double al = prm->alpha_deg * M_PI / 180.0, be = prm->beta_deg * M_PI / 180.0;
  double v[3] = {prm->mach * std::cos(al) * std::cos(be), prm->mach * std::sin(al) * std::cos(be),
                 prm->mach * std::sin(be)};
  double ke = 0.0;
  for (int x = 0; x < 5; ++x) U[x] = 0.0;
  U[0] = 1.0;
  for (int a = 0; a < d; ++a) { U[1 + a] = v[a]; ke += v[a] * v[a]; }
  U[d + 1] = 1.0 / (prm->gamma * (prm->gamma - 1.0)) + 0.5 * ke;
}

// Batch definition: element ranges of the solves in the union mesh and
// their free-stream states.
struct BatchDef {
  int n = 0;
  std::vector<int> e0;                     // [n + 1]
  std::vector<std::array<double, 5>> uinf;  // [n]
};

eg_status init_common(eg_handle* h, const eg_mesh* mesh, const eg_params* prm, void* hip_stream,
                      const BatchDef* bd) {
  const int d = mesh->dim;
  const int pmax_lim = (d == 2) ? 4 : 3;
  if (prm->p_max < 0 || prm->p_max > pmax_lim || prm->rk_stages < 1 || prm->krylov_m < 1 || prm->krylov_m > 48 ||
      !(prm->cfl_max > 0.0) || !(prm->gamma > 1.0) || !(prm->mach >= 0.0) ||
      (prm->precision != EG_FP64 && prm->precision != EG_MIXED) ||
      (prm->flux != EG_FLUX_RUSANOV && prm->flux != EG_FLUX_ROE)) {
    h->err = "invalid parameters (p_max, rk_stages, krylov_m 1..48, cfl_max, gamma, mach, precision or flux)";
    return EG_ERR_ARG;
  }
  h->pmax = prm->p_max;
  h->s = prm->rk_stages;
  h->m = prm->krylov_m;
  h->relr = prm->relative_ramp;
  h->mach = prm->mach;
  h->mixed = prm->precision == EG_MIXED;
  h->cfl_max = prm->cfl_max;
  h->st = static_cast<hipStream_t>(hip_stream);
  h->modes = hier_modes(d, h->pmax);
  {
    // the handle's device; the no-allocation norm's static workspace is
    // resolved here, once per device, with that device current
    hipError_t e = hipGetDevice(&h->dev);
    if (e == hipSuccess) e = eg::noalloc_resolve(h->dev);
    if (e != hipSuccess) return hipfail(h, e, "device set-up");
  }
  DevMesh& M = h->M;
  M.d = d;
  M.V = d + 2;
  M.ne = mesh->n_elem;
  M.NF = 2 * d;
  M.NC = (mesh->elem_geo && d == 3) ? 27 : eg::geo_nodes(d);
  const int N = nmodes_of(d, h->pmax);
  M.NT = N * (N + 1) / 2;
  M.gas.g = prm->gamma;
  M.gas.flux = prm->flux == EG_FLUX_ROE ? eg::FLUX_ROE : eg::FLUX_RUSANOV;
  {
    const double al = prm->alpha_deg * M_PI / 180.0, be = prm->beta_deg * M_PI / 180.0;
    double v[3] = {prm->mach * std::cos(al) * std::cos(be), prm->mach * std::sin(al) * std::cos(be),
                   prm->mach * std::sin(be)};
    double ke = 0.0;
    M.gas.Uinf[0] = 1.0;
    for (int a = 0; a < d; ++a) { M.gas.Uinf[1 + a] = v[a]; ke += v[a] * v[a]; }
    M.gas.Uinf[d + 1] = 1.0 / (prm->gamma * (prm->gamma - 1.0)) + 0.5 * ke;
  }
  std::vector<double> xv, Lpk, Gpk, hE, vol;
  std::vector<int> nbr;
  std::vector<uint8_t> ncode;
  double omega = 0.0;
  eg_status s = setup_mesh(h, mesh, xv, nbr, ncode, Lpk, Gpk, hE, omega, vol);
  if (s != EG_OK) return s;
  M.omega = omega;
  h->tabs.resize(h->pmax + 1);
  for (int p = 0; p <= h->pmax; ++p) fill_tabdata(h->tabs[p], d, p, h->modes);
  // device allocations
  const int ne = M.ne, V = M.V;
#define AL(ptr, cnt)                                  \
  do {                                                \
    eg_status a_ = dalloc(h, &(ptr), (size_t)(cnt));  \
    if (a_ != EG_OK) return a_;                       \
  } while (0)
  AL(M.xv, xv.size());
  AL(M.nbr, nbr.size());
  AL(M.ncode, ncode.size());
  AL(M.Lpk, Lpk.size());
  AL(M.Gpk, Gpk.size());
  AL(M.hE, hE.size());
  AL(M.g2x, 2);
  AL(M.g2w, 2);
  {
    size_t per = 0;
    for (int p = 1; p <= h->pmax; ++p)
      per = std::max(per, eg::jac_points_per_elem(d, p, h->mixed && blk_prec(h, p) == eg::PREC_FP32));
    if (per) {
      double* bc = nullptr;  // sized for FP64 values; the FP32 assembly uses the front half
      AL(bc, (size_t)ne * per);
      M.bc = bc;
    }
  }
  // basis tables of the block assembly, both precisions
  for (int p = 1; p <= h->pmax; ++p) {
    if (!eg::jacobian_supported(d, p)) continue;
    const bool big = eg::jaclu_big_supported(d, p);  // the global-memory kernel's table
    const size_t cnt = big ? eg::bigtab_values(d, p) : eg::phitab_values(d, p);
    double* t64 = nullptr;
    float* t32 = nullptr;
    AL(t64, cnt);
    AL(t32, cnt);
    if (big) {
      HIPCHK(h, eg::launch_fill_bigtab(M, h->tabs[p], p, eg::PREC_FP64, t64, h->st));
      HIPCHK(h, eg::launch_fill_bigtab(M, h->tabs[p], p, eg::PREC_FP32, t32, h->st));
    } else {
      HIPCHK(h, eg::launch_fill_phitab(M, h->tabs[p], p, eg::PREC_FP64, t64, h->st));
      HIPCHK(h, eg::launch_fill_phitab(M, h->tabs[p], p, eg::PREC_FP32, t32, h->st));
    }
    M.phitab[p][eg::PREC_FP64] = t64;
    M.phitab[p][eg::PREC_FP32] = t32;
  }
  // restriction operators p -> p - 1 of every element, R = L_c^{-T} [I 0] L^T
  // (stored by columns, [N][Nc]; L the Cholesky factor of the phi mass
  // matrix, L_c its leading Nc x Nc block): column j of R solves
  // L_c^T x = (row j of L)_c
  for (int p = 1; p <= h->pmax; ++p) {
    const int N = nmodes_of(d, p), Nc = nmodes_of(d, p - 1), NT = M.NT;
    std::vector<double> R((size_t)ne * Nc * N), y(Nc);
    for (int e = 0; e < ne; ++e) {
      const double* L = &Lpk[(size_t)e * NT];
      double* Re = &R[(size_t)e * Nc * N];
      for (int j = 0; j < N; ++j) {
        for (int m = 0; m < Nc; ++m) y[m] = (m <= j) ? L[j * (j + 1) / 2 + m] : 0.0;
        for (int k = Nc - 1; k >= 0; --k) {
          double sk = y[k];
          for (int m = k + 1; m < Nc; ++m) sk -= L[m * (m + 1) / 2 + k] * y[m];
          y[k] = sk / L[k * (k + 1) / 2 + k];
        }
        for (int k = 0; k < Nc; ++k) Re[(size_t)j * Nc + k] = y[k];
      }
    }
    AL(M.Rop[p], R.size());
    HIPCHK(h, hipMemcpy(M.Rop[p], R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  for (int p = 0; p <= h->pmax; ++p) {
    const size_t K = (size_t)ne * V * nmodes_of(d, p);
    AL(h->ut[p], K);
    AL(h->un[p], K);
    AL(h->rt[p], K);
    AL(h->ft[p], K);
    AL(h->uc0[p], K);
    if (p >= 1) {
      const size_t n = (size_t)V * nmodes_of(d, p);
      if (eg::jacobian_supported(d, p)) {
        if (h->mixed) {
          float* f = nullptr;
          AL(f, (size_t)ne * n * n);
          h->F[p] = f;
        } else {
          double* f = nullptr;
          AL(f, (size_t)ne * n * n);
          h->F[p] = f;
        }
        AL(h->perm[p], (size_t)ne * n);
      }
    }
  }
  const size_t Kmax = (size_t)ne * V * N;
  AL(h->dtau, ne);
  AL(h->tmp, Kmax);
  AL(h->tmp2, Kmax);
  const size_t K0 = (size_t)ne * V;
  AL(h->u0, K0);
  AL(h->b0, K0);
  AL(h->Ad, (size_t)ne * V * V);
  AL(h->Ao, (size_t)ne * M.NF * V * V);
  AL(h->dt0, ne);
  // batch tables: solve of each element, element ranges, |Omega| per solve,
  // per-element free stream, and Arnoldi blocks that never straddle solves
  const int nseg = bd ? bd->n : 1;
  std::vector<int> brow0, brow1, bseg, sblk0;
  std::vector<int> sid;
  std::vector<double> seg_omega, uinf_e;
  if (bd) {
    M.nseg = nseg;
    h->batch = true;
    h->seg_e0 = bd->e0;
    sid.assign(ne, 0);
    seg_omega.assign(nseg, 0.0);
    uinf_e.assign((size_t)ne * V, 0.0);
    sblk0.push_back(0);
    for (int sg = 0; sg < nseg; ++sg) {
      for (int e = bd->e0[sg]; e < bd->e0[sg + 1]; ++e) {
        sid[e] = sg;
        seg_omega[sg] += vol[e];
        for (int v = 0; v < V; ++v) uinf_e[(size_t)e * V + v] = bd->uinf[sg][v];
      }
      const int r0 = bd->e0[sg] * V, r1 = bd->e0[sg + 1] * V;
      for (int r = r0; r < r1; r += 256) {
        brow0.push_back(r);
        brow1.push_back(std::min(r + 256, r1));
        bseg.push_back(sg);
      }
      sblk0.push_back((int)brow0.size());
    }
    h->nblk_arn = (int)brow0.size();
    AL(M.sid, ne);
    AL(M.seg_e0, nseg + 1);
    AL(M.seg_omega, nseg);
    AL(M.uinf_e, (size_t)ne * V);
    AL(h->cfl_e_buf, ne);
    AL(M.brow0, brow0.size());
    AL(M.brow1, brow1.size());
    AL(M.bseg, bseg.size());
    AL(M.sblk0, sblk0.size());
    AL(h->dcfl, nseg);
  } else {
    h->nblk_arn = eg::arnoldi_blocks((int)K0);
  }
  AL(h->Vb, (size_t)(h->m + 1) * K0);
  AL(h->H, (size_t)nseg * (h->m + 1) * h->m);
  AL(h->part1, (size_t)h->nblk_arn * (h->m + 2));
  AL(h->part2, (size_t)h->nblk_arn * (h->m + 2));
  AL(h->info, 2 * nseg);
  AL(h->arn_st, 2 * nseg);
  AL(h->arn_wn0, 2 * nseg);  // ||A v_j|| in two slots per solve
  AL(h->arn_W, 2 * K0);
  AL(h->H2, (size_t)nseg * (h->m + 1) * h->m);
  AL(h->y, (size_t)nseg * (h->m + 1));
  AL(h->npart, (size_t)ne + 2);  // block partials, or one value per element (batch norms)
  AL(h->nout, nseg);
  AL(h->dfail, 1);
  AL(h->dpart, ne);
  AL(h->spart, 256);
  AL(h->sout, 1);
  AL(h->dcfl1, 1);
#undef AL
  {
    hipError_t e = hipHostMalloc((void**)&h->hpin, 64, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&h->hcfl1, sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess && bd) e = hipHostMalloc((void**)&h->hcfl, sizeof(double) * nseg, hipHostMallocDefault);
    if (e == hipSuccess && bd) e = hipHostMalloc((void**)&h->hnorm, sizeof(double) * nseg, hipHostMallocDefault);
    if (e != hipSuccess) { h->err = "hipHostMalloc failed"; return EG_ERR_ALLOC; }
  }
  // the p = 0 face rule is the 2-point rule of the order-0 tables
  double g2x[2] = {h->tabs[0].x[0], h->tabs[0].x[1]}, g2w[2] = {h->tabs[0].w[0], h->tabs[0].w[1]};
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(M.xv, xv.data(), xv.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.ncode, ncode.data(), ncode.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.Lpk, Lpk.data(), Lpk.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.Gpk, Gpk.data(), Gpk.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.hE, hE.data(), hE.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.g2x, g2x, 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M.g2w, g2w, 16, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(h->dfail, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(h->info, 0, 2 * nseg * sizeof(double));
  if (bd) {
    if (e == hipSuccess) e = hipMemcpy(M.sid, sid.data(), sid.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.seg_e0, bd->e0.data(), bd->e0.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.seg_omega, seg_omega.data(), seg_omega.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.uinf_e, uinf_e.data(), uinf_e.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.brow0, brow0.data(), brow0.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.brow1, brow1.data(), brow1.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.bseg, bseg.data(), bseg.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(M.sblk0, sblk0.data(), sblk0.size() * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hipfail(h, e, "upload");
  return EG_OK;
}

// One V-cycle below the entry norm (rt[p_max] holds the entry residual):
// eagerly, or by replaying a captured graph of it.  The graph reads the CFL
// from device memory (per element in a batch, else the scalar dcfl1), so one
// capture per mixed-precision phase serves every cycle; everything else it
// touches is handle-owned and fixed.
// Captures (once per mixed-precision phase) the V-cycle below the entry
// norm on the handle's stream into h->ggraph[g] / h->gexec[g].
eg_status ensure_graph(eg_handle* h, double cfl) {
  const int g = h->mixed && h->phase_b ? 1 : 0;
  if (h->gexec[g]) return EG_OK;
  if (!h->batch) h->M.cfl_one = h->dcfl1;
  HIPCHK(h, hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
  eg_status st = vc_rec(h, h->pmax, cfl);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(h->st, &graph);
  h->M.cfl_one = nullptr;
  if (st != EG_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hipfail(h, e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hipfail(h, e, "hipGraphInstantiate");
  }
  h->ggraph[g] = graph;
  h->gexec[g] = ex;
  return EG_OK;
}

eg_status vcycle_run(eg_handle* h, double cfl) {
  if (!h->graphs || h->prof) return vc_rec(h, h->pmax, cfl);
  if (!h->batch) {
    h->hcfl1[0] = cfl;
    HIPCHK(h, hipMemcpyAsync(h->dcfl1, h->hcfl1, sizeof(double), hipMemcpyHostToDevice, h->st));
  }
  ECHK(ensure_graph(h, cfl));
  HIPCHK(h, hipGraphLaunch(h->gexec[h->mixed && h->phase_b ? 1 : 0], h->st));
  return EG_OK;
}

// Solve loops in graph mode run on the handle's internal stream, ordered
// after the caller's stream on entry and before it on exit.
struct StreamSwap {
  eg_handle* h;
  hipStream_t caller;
  bool on = false;
  eg_status begin() {
    caller = h->st;
    if (!h->graphs || h->prof) return EG_OK;
    if (!h->gst) {
      HIPCHK(h, hipStreamCreateWithFlags(&h->gst, hipStreamNonBlocking));
      HIPCHK(h, hipEventCreateWithFlags(&h->gev, hipEventDisableTiming));
    }
    HIPCHK(h, hipEventRecord(h->gev, caller));
    HIPCHK(h, hipStreamWaitEvent(h->gst, h->gev, 0));
    h->st = h->gst;
    on = true;
    return EG_OK;
  }
  void end() {
    if (!on) return;
    (void)hipEventRecord(h->gev, h->gst);
    (void)hipStreamWaitEvent(caller, h->gev, 0);
    h->st = caller;
    on = false;
  }
  ~StreamSwap() { end(); }
};

// Binds the batch's per-element CFL array for the duration of a batch solve.
struct CflBind {
  eg_handle* h;
  explicit CflBind(eg_handle* hh) : h(hh) { h->M.cfl_e = h->cfl_e_buf; }
  ~CflBind() { h->M.cfl_e = nullptr; }
};

// The bookkeeping of one batch handle's steady solve across V-cycles (shared
// by eg_solve_batch and eg_solve_multi): per-solve first norms, minima,
// convergence and divergence flags, the norm ring of the mixed-precision
// switch.  A solve whose norm is not finite has diverged: it is recorded
// and left alone (its values stay inside its own elements and Krylov
// segment) while the others go on; a converged solve's state is saved at
// the norm that reached the drop (later cycles of the batch still run over
// its elements) and restored at the end.
struct BatchRun {
  eg_handle* h = nullptr;
  double* u_dev = nullptr;
  double drop_tol = 0.0;
  int max_cycles = 0;
  double* hist = nullptr;
  int* ncyc = nullptr;
  int nseg = 0, pm = 0, N = 0;
  size_t per_elem = 0;
  std::vector<double> r1, rmin, ring;
  std::vector<int> done, nmin;
  int phase_b = 0;
  bool over = false;  // the solve has ended; its status is `result`
  eg_status result = EG_OK;

  eg_status begin() {
    const DevMesh& M = h->M;
    nseg = M.nseg;
    pm = h->pmax;
    N = nmodes_of(M.d, pm);
    per_elem = (size_t)M.V * N;
    if (!h->bsave) ECHK(dalloc(h, &h->bsave, (size_t)M.ne * per_elem));
    r1.assign(nseg, -1.0);
    rmin.assign(nseg, HUGE_VAL);
    ring.assign((size_t)nseg * 64, 0.0);
    done.assign(nseg, 0);
    nmin.assign(nseg, 1);
    for (int sg = 0; sg < nseg; ++sg) ncyc[sg] = 0;
    HIPCHK(h, eg::launch_basis(M, N, u_dev, h->ut[pm], 0, h->st));
    return EG_OK;
  }
  // FP64 entry norms of every solve and the pivot-failure flag, copied to
  // the host (asynchronous; read after the stream's synchronisation)
  eg_status launch_entry() {
    const DevMesh& M = h->M;
    PCALL(h, EG_K_RESIDUAL, pm,
          eg::launch_residual(M, h->tabs[pm], pm, h->ut[pm], nullptr, h->rt[pm], eg::PREC_FP64, h->st));
    PCALL(h, EG_K_NORM, pm, eg::launch_norm(M, N, h->rt[pm], h->npart, h->nout, h->st));
    HIPCHK(h, hipMemcpyAsync(h->hnorm, h->nout, sizeof(double) * nseg, hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipMemcpyAsync(h->hpin + 1, h->dfail, sizeof(int), hipMemcpyDeviceToHost, h->st));
    return EG_OK;
  }
  // Cycle n's entry norms (after the synchronisation): records them, and
  // either ends the solve (over, result) or sets the next cycle's CFL
  // numbers and arithmetic phase.
  eg_status update(int n) {
    bool all = true;
    double worst = 0.0;
    for (int sg = 0; sg < nseg; ++sg) {
      const double rn = h->hnorm[sg];
      if (r1[sg] < 0.0) r1[sg] = rn;
      if (!done[sg]) {
        hist[(size_t)sg * (max_cycles + 1) + (n - 1)] = rn;
        ncyc[sg] = n - 1;
        if (!std::isfinite(rn)) done[sg] = 2;
        else if (rn <= drop_tol * r1[sg]) {
          done[sg] = 1;
          const size_t o = (size_t)h->seg_e0[sg] * per_elem;
          const size_t cnt = (size_t)(h->seg_e0[sg + 1] - h->seg_e0[sg]) * per_elem;
          HIPCHK(h, hipMemcpyAsync(h->bsave + o, h->ut[pm] + o, cnt * sizeof(double), hipMemcpyDeviceToDevice,
                                   h->st));
        }
      }
      all = all && done[sg];
      if (done[sg] != 2) {
        worst = std::max(worst, rn / r1[sg]);
        if (!(rn >= rmin[sg])) { rmin[sg] = rn; nmin[sg] = n; }
      }
      h->hcfl[sg] = std::isfinite(rn) ? cfl_ramp(h->cfl_max, rn, h->relr ? r1[sg] : 1.0, n, pm) : 1.0;
    }
    if (all) {
      over = true;
      for (int sg = 0; sg < nseg; ++sg)
        if (done[sg] == 2) result = fail(h, EG_ERR_DIVERGED, "a solve of the batch diverged (non-finite norm)");
      return EG_OK;
    }
    if (n - 1 == max_cycles) {
      bool div = false;
      for (int sg = 0; sg < nseg; ++sg) div = div || done[sg] == 2;
      over = true;
      result = fail(h, div ? EG_ERR_DIVERGED : EG_ERR_NOT_CONVERGED,
                    div ? "a solve of the batch diverged (non-finite norm)" : "max_cycles reached");
      return EG_OK;
    }
    if (h->mixed && !phase_b) {
      bool stall = false;
      for (int sg = 0; sg < nseg; ++sg)
        stall = stall || (done[sg] == 0 && phase_a_over(h->hnorm[sg], 0.0, n, nmin[sg], &ring[(size_t)sg * 64]));
      if (worst <= EG_PHASE_B_DROP || stall) phase_b = 1;
    }
    for (int sg = 0; sg < nseg; ++sg) ring[(size_t)sg * 64 + n % 64] = h->hnorm[sg];
    h->phase_b = phase_b;
    return EG_OK;
  }
  // the next cycle's per-solve CFL numbers to the device, per element
  eg_status launch_cfl() {
    HIPCHK(h, hipMemcpyAsync(h->dcfl, h->hcfl, sizeof(double) * nseg, hipMemcpyHostToDevice, h->st));
    HIPCHK(h, eg::launch_expand_cfl(h->M, h->dcfl, h->st));
    return EG_OK;
  }
  // converged solves back to their saved states; the state to u_dev
  eg_status finish() {
    eg_status st = EG_OK;
    for (int sg = 0; sg < nseg; ++sg) {
      if (done[sg] != 1) continue;
      const size_t o = (size_t)h->seg_e0[sg] * per_elem;
      const size_t cnt = (size_t)(h->seg_e0[sg + 1] - h->seg_e0[sg]) * per_elem;
      hipError_t ec =
          hipMemcpyAsync(h->ut[pm] + o, h->bsave + o, cnt * sizeof(double), hipMemcpyDeviceToDevice, h->st);
      if (ec != hipSuccess && st == EG_OK) st = hipfail(h, ec, "restore converged states");
    }
    hipError_t e = eg::launch_basis(h->M, N, h->ut[pm], u_dev, 1, h->st);
    if (e != hipSuccess && st == EG_OK) st = hipfail(h, e, "basis");
    return st;
  }
};

}  // namespace

extern "C" {

eg_status eg_set_graphs(eg_handle* h, int enable) {
  if (!h) return EG_ERR_ARG;
  h->graphs = enable != 0;
  return EG_OK;
}

eg_status eg_autotune(eg_handle* h, int reps, int* tiles_host) {
  if (!h || reps < 1) return EG_ERR_ARG;
  eg::DevMesh& M = h->M;
  for (int i = 0; i < 2; ++i) {  // captured graphs hold the old launches
    if (h->gexec[i]) (void)hipGraphExecDestroy(h->gexec[i]);
    if (h->ggraph[i]) (void)hipGraphDestroy(h->ggraph[i]);
    h->gexec[i] = nullptr;
    h->ggraph[i] = nullptr;
  }
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(h, hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(h, EG_ERR_HIP, "hipEventCreate");
  }
  eg_status st = EG_OK;
  for (int p = 0; p <= h->pmax && st == EG_OK; ++p) {
    const int N = nmodes_of(M.d, p);
    // free stream in phi coordinates as the timing state
    hipError_t e = eg::launch_freestream(M, N, h->tmp, h->st);
    if (e == hipSuccess) e = eg::launch_basis(M, N, h->tmp, h->tmp2, 0, h->st);
    for (int prec = 0; prec < 2 && e == hipSuccess; ++prec) {
      int best = 1;
      float tbest = 0.0f;
      for (int c = 0; c < 3 && e == hipSuccess; ++c) {
        M.res_tile_choice[p][prec] = c;
        e = eg::launch_residual(M, h->tabs[p], p, h->tmp2, nullptr, h->rt[p], prec, h->st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(a, h->st);
        for (int r = 0; r < reps && e == hipSuccess; ++r)
          e = eg::launch_residual(M, h->tabs[p], p, h->tmp2, nullptr, h->rt[p], prec, h->st);
        if (e == hipSuccess) e = hipEventRecord(b, h->st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && (c == 0 || ms < tbest)) {
          tbest = ms;
          best = c;
        }
      }
      M.res_tile_choice[p][prec] = best;
      if (tiles_host) tiles_host[2 * p + prec] = eg::residual_tile(M.d, p, prec, best);
    }
    if (e != hipSuccess) st = hipfail(h, e, "autotune");
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

eg_status eg_init_mesh(const eg_mesh* mesh, const eg_params* prm, void* hip_stream, eg_handle** out) {
  if (!out) return EG_ERR_ARG;
  *out = nullptr;
  if (!mesh || !prm || !mesh->xyz || !mesh->elem_vert || !mesh->bface_tag) return EG_ERR_ARG;
  if ((mesh->dim != 2 && mesh->dim != 3) || mesh->n_vert <= 0 || mesh->n_elem <= 0) return EG_ERR_ARG;
  eg_handle* h = new (std::nothrow) eg_handle;
  if (!h) return EG_ERR_ALLOC;
  *out = h;
  return init_common(h, mesh, prm, hip_stream, nullptr);
}

eg_status eg_init_batch(const eg_mesh* meshes, const eg_params* params, int n_solves, void* hip_stream,
                        eg_handle** out) {
  if (!out) return EG_ERR_ARG;
  *out = nullptr;
  if (!meshes || !params || n_solves < 1) return EG_ERR_ARG;
  const int d = meshes[0].dim;
  long long nv = 0, ne = 0;
  for (int i = 0; i < n_solves; ++i) {
    const eg_mesh& m = meshes[i];
    const eg_params& q = params[i];
    if (!m.xyz || !m.elem_vert || !m.bface_tag || m.dim != d || m.n_vert <= 0 || m.n_elem <= 0) return EG_ERR_ARG;
    if (q.p_max != params[0].p_max || q.rk_stages != params[0].rk_stages || q.krylov_m != params[0].krylov_m ||
        q.cfl_max != params[0].cfl_max || q.relative_ramp != params[0].relative_ramp ||
        q.gamma != params[0].gamma || q.precision != params[0].precision || q.flux != params[0].flux ||
        !(q.mach >= 0.0))
      return EG_ERR_ARG;
    nv += m.n_vert;
    ne += m.n_elem;
  }
  if (ne > (1LL << 28) || nv > (1LL << 30)) return EG_ERR_ARG;
  eg_handle* h = new (std::nothrow) eg_handle;
  if (!h) return EG_ERR_ALLOC;
  *out = h;
  // union mesh: vertices and elements of the solves one after another (no
  // shared vertices, so no face is matched across solves)
  const int nc = 1 << d, nf = 2 * d;
  std::vector<double> xyz((size_t)nv * d);
  std::vector<int32_t> ev((size_t)ne * nc);
  std::vector<int8_t> tag((size_t)ne * nf);
  bool curved = false;
  for (int i = 0; i < n_solves; ++i) curved = curved || meshes[i].elem_geo;
  const int gn = d == 2 ? 18 : 81;  // node coordinates per curved element
  std::vector<double> geo(curved ? (size_t)ne * gn : 0);
  BatchDef bd;
  bd.n = n_solves;
  bd.e0.push_back(0);
  long long ov = 0, oe = 0;
  for (int i = 0; i < n_solves; ++i) {
    const eg_mesh& m = meshes[i];
    std::memcpy(&xyz[(size_t)ov * d], m.xyz, sizeof(double) * (size_t)m.n_vert * d);
    for (long long k = 0; k < (long long)m.n_elem * nc; ++k) {
      if (m.elem_vert[k] < 0 || m.elem_vert[k] >= m.n_vert) {
        h->err = "element vertex index out of range";
        return EG_ERR_MESH;
      }
      ev[(size_t)oe * nc + k] = (int32_t)(m.elem_vert[k] + ov);
    }
    std::memcpy(&tag[(size_t)oe * nf], m.bface_tag, (size_t)m.n_elem * nf);
    if (curved && m.elem_geo) {
      std::memcpy(&geo[(size_t)oe * gn], m.elem_geo, sizeof(double) * gn * (size_t)m.n_elem);
    } else if (curved) {  // a straight mesh among curved ones: its multilinear nodes
      for (int e = 0; e < m.n_elem; ++e) {
        double Xc[8][3];
        for (int k = 0; k < nc; ++k)
          for (int a = 0; a < d; ++a) Xc[k][a] = m.xyz[(size_t)m.elem_vert[(size_t)e * nc + k] * d + a];
        if (d == 2) straight_nodes9(Xc, &geo[((size_t)oe + e) * gn]);
        else straight_nodes27(Xc, &geo[((size_t)oe + e) * gn]);
      }
    }
    ov += m.n_vert;
    oe += m.n_elem;
    bd.e0.push_back((int)oe);
    std::array<double, 5> U{};
    freestream_of(&params[i], d, U.data());
    bd.uinf.push_back(U);
  }
  eg_mesh um{d, (int)nv, xyz.data(), (int)ne, ev.data(), tag.data(), curved ? geo.data() : nullptr};
  return init_common(h, &um, &params[0], hip_stream, &bd);
}

eg_status eg_layout(const eg_handle* h, int solve, int p, int64_t* offset, int* n_modes, int* n_elem) {
  if (!h || p < 0 || p > h->pmax) return EG_ERR_ARG;
  const int nseg = h->M.nseg;
  if (solve < 0 || solve >= nseg) return EG_ERR_ARG;
  const int e0 = h->batch ? h->seg_e0[solve] : 0, e1 = h->batch ? h->seg_e0[solve + 1] : h->M.ne;
  const int N = nmodes_of(h->M.d, p);
  if (offset) *offset = (int64_t)e0 * h->M.V * N;
  if (n_modes) *n_modes = N;
  if (n_elem) *n_elem = e1 - e0;
  return EG_OK;
}



void eg_free(eg_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->st);
  for (void* p : h->allocs) (void)hipFree(p);
  for (hipEvent_t e : h->evpool) (void)hipEventDestroy(e);
  if (h->hpin) (void)hipHostFree(h->hpin);
  if (h->hcfl) (void)hipHostFree(h->hcfl);
  if (h->hcfl1) (void)hipHostFree(h->hcfl1);
  for (int i = 0; i < 2; ++i) {
    if (h->gexec[i]) (void)hipGraphExecDestroy(h->gexec[i]);
    if (h->ggraph[i]) (void)hipGraphDestroy(h->ggraph[i]);
  }
  if (h->gev) (void)hipEventDestroy(h->gev);
  if (h->gst) (void)hipStreamDestroy(h->gst);
  if (h->hnorm) (void)hipHostFree(h->hnorm);
  delete h;
}

const char* eg_last_error(const eg_handle* h) { return h ? h->err.c_str() : "null handle"; }

eg_status eg_sizes(const eg_handle* h, int p, int* n_elem, int* n_modes, int* n_vars) {
  if (!h || p < 0 || p > h->pmax) return EG_ERR_ARG;
  if (n_elem) *n_elem = h->M.ne;
  if (n_modes) *n_modes = nmodes_of(h->M.d, p);
  if (n_vars) *n_vars = h->M.V;
  return EG_OK;
}

eg_status eg_set_freestream(eg_handle* h, int p, double* u_dev) {
  if (!h || !u_dev) return EG_ERR_ARG;
  if (p < 0 || p > h->pmax) return fail(h, EG_ERR_ARG, "order out of range");
  HIPCHK(h, eg::launch_freestream(h->M, nmodes_of(h->M.d, p), u_dev, h->st));
  return EG_OK;
}

eg_status eg_residual(eg_handle* h, int p, const double* u_dev, double* r_dev) {
  if (!h || !u_dev || !r_dev) return EG_ERR_ARG;
  if (p < 0 || p > h->pmax) return fail(h, EG_ERR_ARG, "order out of range");
  const int N = nmodes_of(h->M.d, p);
  HIPCHK(h, eg::launch_basis(h->M, N, u_dev, h->tmp, 0, h->st));
  PCALL(h, EG_K_RESIDUAL, p, eg::launch_residual(h->M, h->tabs[p], p, h->tmp, nullptr, h->tmp2, blk_prec(h, p), h->st));
  HIPCHK(h, eg::launch_basis(h->M, N, h->tmp2, r_dev, 2, h->st));
  return EG_OK;
}

eg_status eg_timestep(eg_handle* h, int p, int p_level, double cfl, const double* u_dev, double* dtau_dev) {
  if (!h || !u_dev || !dtau_dev) return EG_ERR_ARG;
  if (p < 0 || p_level < 0 || p_level > h->pmax) return fail(h, EG_ERR_ARG, "order out of range");
  const int N = nmodes_of(h->M.d, p_level);
  HIPCHK(h, eg::launch_basis(h->M, N, u_dev, h->tmp, 0, h->st));
  HIPCHK(h, eg::launch_timestep(h->M, p, N, cfl, 1.0, h->tmp, dtau_dev, h->st));
  return EG_OK;
}

eg_status eg_element_jacobian(eg_handle* h, int p, const double* u_dev, double* D_dev) {
  if (!h || !u_dev || !D_dev) return EG_ERR_ARG;
  if (p < 1 || p > h->pmax) return fail(h, EG_ERR_ARG, "order out of range (p >= 1)");
  if (!eg::jacobian_supported(h->M.d, p)) return fail(h, EG_ERR_UNSUPPORTED, "element block too large");
  const int N = nmodes_of(h->M.d, p);
  HIPCHK(h, eg::launch_basis(h->M, N, u_dev, h->tmp, 0, h->st));
  HIPCHK(h, eg::launch_jacobian(h->M, h->tabs[p], p, h->tmp, h->dtau, D_dev, nullptr, h->dfail, false,
                                eg::PREC_FP64, h->st));
  HIPCHK(h, eg::launch_jac_to_psi(h->M, N, D_dev, h->st));
  return EG_OK;
}

eg_status eg_prk_step(eg_handle* h, int p, double cfl, double* u_dev, const double* f_dev) {
  if (!h || !u_dev) return EG_ERR_ARG;
  if (p < 1 || p > h->pmax) return fail(h, EG_ERR_ARG, "order out of range (p >= 1)");
  if (!eg::jacobian_supported(h->M.d, p)) return fail(h, EG_ERR_UNSUPPORTED, "element block too large");
  const int N = nmodes_of(h->M.d, p);
  HIPCHK(h, eg::launch_basis(h->M, N, u_dev, h->ut[p], 0, h->st));
  const double* ft = nullptr;
  if (f_dev) {
    HIPCHK(h, eg::launch_basis(h->M, N, f_dev, h->tmp, 3, h->st));
    ft = h->tmp;
  }
  h->phase_b = 0;  // one PRK step in the handle's smoother arithmetic (phase A in mixed mode)
  HIPCHK(h, eg::launch_residual(h->M, h->tabs[p], p, h->ut[p], ft, h->rt[p], res_prec(h, p), h->st));
  ECHK(run_prk(h, p, cfl, ft));
  HIPCHK(h, eg::launch_basis(h->M, N, h->ut[p], u_dev, 1, h->st));
  return EG_OK;
}

eg_status eg_jacobian_p0(eg_handle* h, const double* u0_dev, double* diag_dev, double* off_dev, int32_t* nbr_dev) {
  if (!h || !u0_dev || !diag_dev || !off_dev) return EG_ERR_ARG;
  HIPCHK(h, eg::launch_basis(h->M, 1, u0_dev, h->tmp, 0, h->st));
  HIPCHK(h, eg::launch_p0_setup(h->M, h->tmp, nullptr, h->pmax, 1.0, 0, h->u0, h->b0, diag_dev, off_dev, h->dt0,
                                h->st));
  if (nbr_dev) HIPCHK(h, eg::launch_nbr_export(h->M, nbr_dev, h->st));
  return EG_OK;
}

eg_status eg_exp1_step(eg_handle* h, double cfl, double* u0_dev, const double* f0_dev, int* m_used_host) {
  if (!h || !u0_dev) return EG_ERR_ARG;
  HIPCHK(h, eg::launch_basis(h->M, 1, u0_dev, h->ut[0], 0, h->st));
  const double* ft = nullptr;
  if (f0_dev) {
    HIPCHK(h, eg::launch_basis(h->M, 1, f0_dev, h->tmp, 3, h->st));
    ft = h->tmp;
  }
  ECHK(run_exp1(h, cfl, h->ut[0], ft));
  HIPCHK(h, eg::launch_basis(h->M, 1, h->ut[0], u0_dev, 1, h->st));
  if (m_used_host) {
    HIPCHK(h, hipMemcpyAsync(h->hpin, h->info, sizeof(double), hipMemcpyDeviceToHost, h->st));
    ECHK(sync_status(h));
    *m_used_host = (int)h->hpin[0];
  }
  return EG_OK;
}

eg_status eg_rnorm(eg_handle* h, const double* r_dev, double* rn_host) {
  if (!h || !r_dev || !rn_host) return EG_ERR_ARG;
  if (h->batch) return fail(h, EG_ERR_ARG, "batch handle: per-solve norms need eg_solve_batch");
  const int N = nmodes_of(h->M.d, h->pmax);
  HIPCHK(h, eg::launch_basis(h->M, N, r_dev, h->tmp, 3, h->st));
  HIPCHK(h, eg::launch_norm(h->M, N, h->tmp, h->npart, h->nout, h->st));
  HIPCHK(h, hipMemcpyAsync(h->hpin, h->nout, sizeof(double), hipMemcpyDeviceToHost, h->st));
  ECHK(sync_status(h));
  *rn_host = h->hpin[0];
  return EG_OK;
}

eg_status eg_rnorm_noalloc(eg_handle* h, const double* r_dev, double* rn_dev) {
  if (!h || !r_dev || !rn_dev) return EG_ERR_ARG;
  if (h->batch) return fail(h, EG_ERR_ARG, "batch handle: per-solve norms need eg_solve_batch");
  if (h->M.ne > eg::noalloc_max_elems())
    return fail(h, EG_ERR_ARG, "eg_rnorm_noalloc: " + std::to_string(h->M.ne) + " elements exceed the static workspace (" +
                                   std::to_string(eg::noalloc_max_elems()) + " elements)");
  HIPCHK(h, eg::launch_dnorm_noalloc(h->dev, h->M.ne, h->M.V, nmodes_of(h->M.d, h->pmax), h->M.omega, r_dev, rn_dev,
                                     h->st));
  return EG_OK;
}

eg_status eg_measure_peak(int kind, void* hip_stream, double* value_host) {
  if (kind < 0 || kind > 2 || !value_host) return EG_ERR_ARG;
  return eg::measure_peak(kind, static_cast<hipStream_t>(hip_stream), value_host) == hipSuccess ? EG_OK
                                                                                                 : EG_ERR_HIP;
}

eg_status eg_profile(eg_handle* h, int enable) {
  if (!h) return EG_ERR_ARG;
  HIPCHK(h, hipStreamSynchronize(h->st));
  h->recs.clear();
  h->evused = 0;
  h->prof = enable != 0;
  return EG_OK;
}

eg_status eg_profile_read(eg_handle* h, int kernel_class, int p, double* total_ms, int* launches) {
  if (!h || !total_ms || !launches || kernel_class < 0 || kernel_class >= EG_K_COUNT) return EG_ERR_ARG;
  HIPCHK(h, hipStreamSynchronize(h->st));
  double tot = 0.0;
  int cnt = 0;
  for (const auto& r : h->recs) {
    if (r.cls != kernel_class || (p >= 0 && r.p != p)) continue;
    float ms = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&ms, r.a, r.b));
    tot += ms;
    cnt++;
  }
  *total_ms = tot;
  *launches = cnt;
  return EG_OK;
}

eg_status eg_vcycle(eg_handle* h, double* u_dev, int n, double rref, double* rn_host, double* cfl_host) {
  if (!h || !u_dev || !rn_host || n < 1) return EG_ERR_ARG;
  if (h->batch) return fail(h, EG_ERR_ARG, "batch handle: per-solve norms need eg_solve_batch");
  if (!eg::jacobian_supported(h->M.d, h->pmax) && h->pmax > 0)
    return fail(h, EG_ERR_UNSUPPORTED, "element block too large");
  const int N = nmodes_of(h->M.d, h->pmax);
  HIPCHK(h, eg::launch_basis(h->M, N, u_dev, h->ut[h->pmax], 0, h->st));
  double rn = 0.0;
  ECHK(entry_norm(h, &rn));
  *rn_host = rn;
  if (!std::isfinite(rn)) return fail(h, EG_ERR_DIVERGED, "non-finite residual norm");
  const double cfl = cfl_ramp(h->cfl_max, rn, rref > 0.0 ? rref : rn, n, h->pmax);
  if (cfl_host) *cfl_host = cfl;
  h->phase_b = h->mixed && rn <= EG_PHASE_B_DROP * (rref > 0.0 ? rref : rn);
  ECHK(vc_rec(h, h->pmax, cfl));
  HIPCHK(h, eg::launch_basis(h->M, N, h->ut[h->pmax], u_dev, 1, h->st));
  ECHK(sync_status(h));
  return EG_OK;
}

namespace {
// Cycles n = n0, n0 + 1, ...: entry norm, stop test, V-cycle.  r1 < 0 means
// "take r_1 from this call's first norm".
eg_status solve_loop_body(eg_handle* h, double* u_dev, int n0, double r1, double drop_tol, int max_cycles,
                          double* hist_host, int* n_cycles_host);

eg_status solve_loop(eg_handle* h, double* u_dev, int n0, double r1, double drop_tol, int max_cycles,
                     double* hist_host, int* n_cycles_host) {
  StreamSwap sw{h, h->st};
  ECHK(sw.begin());
  eg_status st = solve_loop_body(h, u_dev, n0, r1, drop_tol, max_cycles, hist_host, n_cycles_host);
  sw.end();
  return st;
}

eg_status solve_loop_body(eg_handle* h, double* u_dev, int n0, double r1, double drop_tol, int max_cycles,
                          double* hist_host, int* n_cycles_host) {
  const int N = nmodes_of(h->M.d, h->pmax);
  HIPCHK(h, eg::launch_basis(h->M, N, u_dev, h->ut[h->pmax], 0, h->st));
  eg_status st = EG_OK;
  for (int n = n0;; ++n) {
    double rn = 0.0;
    st = entry_norm(h, &rn);
    if (st != EG_OK) break;
    hist_host[n - n0] = rn;
    *n_cycles_host = n - n0;
    if (r1 < 0.0) r1 = rn;
    h->sv_next = n;
    h->sv_r1 = r1;
    if (!std::isfinite(rn)) { st = fail(h, EG_ERR_DIVERGED, "non-finite residual norm"); break; }
    if (rn <= drop_tol * r1) break;
    if (n - n0 == max_cycles) { st = fail(h, EG_ERR_NOT_CONVERGED, "max_cycles reached"); break; }
    const double cfl = cfl_ramp(h->cfl_max, rn, h->relr ? r1 : 1.0, n, h->pmax);
    if (h->mixed && !h->sv_phase_b) {
      if (!(rn >= h->sv_rmin)) { h->sv_rmin = rn; h->sv_nmin = n; }
      if (phase_a_over(rn, r1, n, h->sv_nmin, h->sv_ring)) h->sv_phase_b = 1;
    }
    h->sv_ring[n % 64] = rn;
    h->phase_b = h->sv_phase_b;
    st = vcycle_run(h, cfl);
    if (st != EG_OK) break;
  }
  hipError_t e = eg::launch_basis(h->M, N, h->ut[h->pmax], u_dev, 1, h->st);
  if (e != hipSuccess && st == EG_OK) st = hipfail(h, e, "basis");
  hipError_t e2 = hipStreamSynchronize(h->st);
  if (e2 != hipSuccess && st == EG_OK) st = hipfail(h, e2, "sync");
  return st;
}
}  // namespace

eg_status eg_solve_steady(eg_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                          int* n_cycles_host) {
  if (!h || !u_dev || !hist_host || !n_cycles_host || max_cycles < 0) return EG_ERR_ARG;
  if (h->batch) return fail(h, EG_ERR_ARG, "batch handle: per-solve norms need eg_solve_batch");
  if (!eg::jacobian_supported(h->M.d, h->pmax) && h->pmax > 0)
    return fail(h, EG_ERR_UNSUPPORTED, "element block too large");
  h->sv_phase_b = 0;
  h->sv_nmin = 1;
  h->sv_rmin = HUGE_VAL;
  return solve_loop(h, u_dev, 1, -1.0, drop_tol, max_cycles, hist_host, n_cycles_host);
}

eg_status eg_drag(eg_handle* h, const double* u_dev, const double* dir_host, double sref, double* cd_host,
                  double* grad_dev) {
  if (!h || !u_dev || !dir_host || !cd_host || !(sref > 0.0)) return EG_ERR_ARG;
  if (h->batch) return fail(h, EG_ERR_ARG, "batch handle: per-solve norms need eg_solve_batch");
  if (!(h->mach > 0.0)) return fail(h, EG_ERR_ARG, "drag needs a free stream with mach > 0");
  const DevMesh& M = h->M;
  const int p = h->pmax, N = nmodes_of(M.d, p);
  double dir[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < M.d; ++a) dir[a] = dir_host[a];
  const double scale = -1.0 / (0.5 * h->mach * h->mach * sref);
  HIPCHK(h, eg::launch_basis(M, N, u_dev, h->tmp, 0, h->st));
  HIPCHK(h, eg::launch_drag(M, h->tabs[p], p, h->tmp, dir, scale, h->dpart, h->tmp2, h->st));
  HIPCHK(h, eg::launch_sum(h->dpart, nullptr, (size_t)M.ne, h->spart, 0, h->sout, h->st));
  if (grad_dev) HIPCHK(h, eg::launch_basis(M, N, h->tmp2, grad_dev, 2, h->st));
  HIPCHK(h, hipMemcpyAsync(h->hpin, h->sout, sizeof(double), hipMemcpyDeviceToHost, h->st));
  ECHK(sync_status(h));
  *cd_host = h->hpin[0];
  return EG_OK;
}

eg_status eg_jacobian_apply(eg_handle* h, int p, const double* u_dev, const double* v_dev, double* out_dev) {
  if (!h || !u_dev || !v_dev || !out_dev) return EG_ERR_ARG;
  if (p < 0 || p > h->pmax) return fail(h, EG_ERR_ARG, "order out of range");
  const DevMesh& M = h->M;
  const int N = nmodes_of(M.d, p);
  HIPCHK(h, eg::launch_basis(M, N, u_dev, h->tmp, 0, h->st));
  HIPCHK(h, eg::launch_basis(M, N, v_dev, h->tmp2, 0, h->st));
  HIPCHK(h, eg::launch_tangent(M, h->tabs[p], p, h->tmp, h->tmp2, h->rt[p], h->st));
  HIPCHK(h, eg::launch_basis(M, N, h->rt[p], out_dev, 2, h->st));
  return EG_OK;
}

eg_status eg_adjoint_apply(eg_handle* h, int p, const double* u_dev, const double* w_dev, double* out_dev) {
  if (!h || !u_dev || !w_dev || !out_dev) return EG_ERR_ARG;
  if (p < 1 || p > h->pmax) return fail(h, EG_ERR_ARG, "order out of range (p >= 1)");
  ECHK(adj_alloc(h));
  const DevMesh& M = h->M;
  const int N = nmodes_of(M.d, p);
  HIPCHK(h, eg::launch_basis(M, N, u_dev, h->tmp, 0, h->st));
  HIPCHK(h, eg::launch_basis(M, N, w_dev, h->tmp2, 0, h->st));
  HIPCHK(h, eg::launch_jac_points(M, h->tabs[p], p, h->tmp, h->adj_bc[p], h->st));
  HIPCHK(h, eg::launch_adj_residual(M, h->tabs[p], p, h->tmp2, nullptr, h->adj_bc[p], h->rho[p], h->st));
  HIPCHK(h, eg::launch_basis(M, N, h->rho[p], out_dev, 2, h->st));
  return EG_OK;
}

eg_status eg_param_sensitivity(eg_handle* hp, eg_handle* hm, double step, const double* u_dev, const double* lam_dev,
                               const double* dir_host, double sref, double* dj_host) {
  if (!hp || !hm || hp == hm || !u_dev || !lam_dev || !dir_host || !dj_host || !(step > 0.0) || !(sref > 0.0))
    return EG_ERR_ARG;
  if (hp->batch || hm->batch) return fail(hp, EG_ERR_ARG, "batch handle: per-solve sensitivities are not supported");
  if (hp->M.d != hm->M.d || hp->M.ne != hm->M.ne || hp->pmax != hm->pmax || hp->dev != hm->dev)
    return fail(hp, EG_ERR_ARG, "the two handles must have the same dimension, elements, order and device");
  const int p = hp->pmax, N = nmodes_of(hp->M.d, p);
  const size_t K = (size_t)hp->M.ne * hp->M.V * N;
  // R_p(u) on both handles (psi coordinates), each on its own stream
  eg_handle* hh[2] = {hp, hm};
  for (eg_handle* x : hh) {
    HIPCHK(hp, eg::launch_basis(x->M, N, u_dev, x->tmp, 0, x->st));
    HIPCHK(hp, eg::launch_residual(x->M, x->tabs[p], p, x->tmp, nullptr, x->tmp2, eg::PREC_FP64, x->st));
    HIPCHK(hp, eg::launch_basis(x->M, N, x->tmp2, x->un[p], 2, x->st));
  }
  HIPCHK(hp, hipStreamSynchronize(hm->st));
  // lambda . (R(theta + h) - R(theta - h)) on hp's stream, deterministic sums
  HIPCHK(hp, eg::launch_sub(hp->un[p], hm->un[p], hp->tmp2, K, hp->st));
  HIPCHK(hp, eg::launch_sum(hp->tmp2, lam_dev, K, hp->spart, 0, hp->sout, hp->st));
  HIPCHK(hp, hipMemcpyAsync(hp->hpin + 2, hp->sout, sizeof(double), hipMemcpyDeviceToHost, hp->st));
  ECHK(sync_status(hp));
  const double dr = hp->hpin[2];
  double cdp = 0.0, cdm = 0.0;
  eg_status st = eg_drag(hp, u_dev, dir_host, sref, &cdp, nullptr);
  if (st != EG_OK) return st;
  st = eg_drag(hm, u_dev, dir_host, sref, &cdm, nullptr);
  if (st != EG_OK) return fail(hp, st, std::string("drag on the theta - h handle: ") + hm->err);
  *dj_host = (cdp - cdm) / (2.0 * step) + dr / (2.0 * step);
  return EG_OK;
}

eg_status eg_adjoint_solve(eg_handle* h, const double* u_dev, const double* g_dev, double* lam_dev, double drop_tol,
                           int max_cycles, double* hist_host, int* n_cycles_host) {
  if (!h || !u_dev || !g_dev || !lam_dev || !hist_host || !n_cycles_host || max_cycles < 0) return EG_ERR_ARG;
  if (h->batch) return fail(h, EG_ERR_ARG, "batch handle: per-solve norms need eg_solve_batch");
  if (h->pmax < 1) return fail(h, EG_ERR_UNSUPPORTED, "adjoint needs p_max >= 1");
  ECHK(adj_supported(h));
  ECHK(adj_alloc(h));
  const DevMesh& M = h->M;
  const int pm = h->pmax, N = nmodes_of(M.d, pm);
  ECHK(adj_setup(h, u_dev));
  HIPCHK(h, eg::launch_basis(M, N, g_dev, h->gq[pm], 3, h->st));
  HIPCHK(h, eg::launch_basis(M, N, lam_dev, h->lam[pm], 0, h->st));
  eg_status st = EG_OK;
  double r1 = 0.0;
  for (int n = 0;; ++n) {
    double rn = 0.0;
    st = adj_norm(h, &rn);
    if (st != EG_OK) break;
    hist_host[n] = rn;
    *n_cycles_host = n;
    if (n == 0) r1 = rn;
    if (!std::isfinite(rn)) { st = fail(h, EG_ERR_DIVERGED, "non-finite adjoint residual"); break; }
    if (rn <= drop_tol * r1) break;
    if (n == max_cycles) { st = fail(h, EG_ERR_NOT_CONVERGED, "max_cycles reached"); break; }
    st = adj_vc(h, pm);
    if (st != EG_OK) break;
  }
  hipError_t e = eg::launch_basis(M, N, h->lam[pm], lam_dev, 1, h->st);
  if (e != hipSuccess && st == EG_OK) st = hipfail(h, e, "basis");
  hipError_t e2 = hipStreamSynchronize(h->st);
  if (e2 != hipSuccess && st == EG_OK) st = hipfail(h, e2, "sync");
  return st;
}

eg_status eg_solve_batch(eg_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                         int* n_cycles_host) {
  if (!h || !u_dev || !hist_host || !n_cycles_host || max_cycles < 0) return EG_ERR_ARG;
  if (!h->batch) return fail(h, EG_ERR_ARG, "not a batch handle (eg_init_batch)");
  if (!eg::jacobian_supported(h->M.d, h->pmax) && h->pmax > 0)
    return fail(h, EG_ERR_UNSUPPORTED, "element block too large");
  StreamSwap sw{h, h->st};
  ECHK(sw.begin());
  CflBind cb(h);  // per-solve CFL for the duration of the batch solve
  BatchRun br;
  br.h = h;
  br.u_dev = u_dev;
  br.drop_tol = drop_tol;
  br.max_cycles = max_cycles;
  br.hist = hist_host;
  br.ncyc = n_cycles_host;
  ECHK(br.begin());
  eg_status st = EG_OK;
  for (int n = 1;; ++n) {
    if ((st = br.launch_entry()) != EG_OK) break;
    if ((st = sync_status(h)) != EG_OK) break;
    if ((st = br.update(n)) != EG_OK) break;
    if (br.over) {
      st = br.result;
      break;
    }
    if ((st = br.launch_cfl()) != EG_OK) break;
    if ((st = vcycle_run(h, h->cfl_max)) != EG_OK) break;
  }
  const eg_status sf = br.finish();
  if (st == EG_OK) st = sf;
  hipError_t e2 = hipStreamSynchronize(h->st);
  if (e2 != hipSuccess && st == EG_OK) st = hipfail(h, e2, "sync");
  return st;
}

eg_status eg_solve_multi(eg_handle* const* hs, int nh, double* const* u_devs, double drop_tol, int max_cycles,
                         double* const* hist_hosts, int* const* n_cycles_hosts, int* status_host) {
  if (!hs || nh < 1 || !u_devs || !hist_hosts || !n_cycles_hosts || !status_host || max_cycles < 0)
    return EG_ERR_ARG;
  for (int k = 0; k < nh; ++k) {
    if (!hs[k] || !u_devs[k] || !hist_hosts[k] || !n_cycles_hosts[k]) return EG_ERR_ARG;
    if (!hs[k]->batch) return fail(hs[k], EG_ERR_ARG, "not a batch handle (eg_init_batch)");
    if (hs[k]->dev != hs[0]->dev) return fail(hs[0], EG_ERR_ARG, "handles on different devices");
    if (!eg::jacobian_supported(hs[k]->M.d, hs[k]->pmax) && hs[k]->pmax > 0)
      return fail(hs[k], EG_ERR_UNSUPPORTED, "element block too large");
    for (int j = 0; j < k; ++j)
      if (hs[j] == hs[k]) return fail(hs[0], EG_ERR_ARG, "a handle appears twice");
  }
  eg_handle* h0 = hs[0];
  bool graphs = true;
  for (int k = 0; k < nh; ++k) graphs = graphs && hs[k]->graphs && !hs[k]->prof;
  // every handle's work on one stream: h0's (its internal stream in graph
  // mode); the others' callers' work is complete on entry, and the call
  // synchronises before it returns
  StreamSwap sw{h0, h0->st};
  ECHK(sw.begin());
  std::vector<hipStream_t> caller(nh);
  for (int k = 1; k < nh; ++k) {
    caller[k] = hs[k]->st;
    HIPCHK(hs[k], hipStreamSynchronize(caller[k]));
  }
  for (int k = 1; k < nh; ++k) hs[k]->st = h0->st;
  std::vector<BatchRun> br(nh);
  std::vector<hipGraph_t> parents;
  std::vector<hipGraphExec_t> pexec;
  std::vector<unsigned> pkey;
  eg_status st = EG_OK;
  for (int k = 0; k < nh; ++k) {
    hs[k]->M.cfl_e = hs[k]->cfl_e_buf;  // per-solve CFL for the duration of the solve
    br[k].h = hs[k];
    br[k].u_dev = u_devs[k];
    br[k].drop_tol = drop_tol;
    br[k].max_cycles = max_cycles;
    br[k].hist = hist_hosts[k];
    br[k].ncyc = n_cycles_hosts[k];
    if (st == EG_OK) st = br[k].begin();
  }
  for (int n = 1; st == EG_OK; ++n) {
    for (int k = 0; k < nh && st == EG_OK; ++k)
      if (!br[k].over) st = br[k].launch_entry();
    if (st != EG_OK) break;
    if ((st = sync_status(h0)) != EG_OK) break;
    bool any = false;
    for (int k = 0; k < nh && st == EG_OK; ++k) {
      if (br[k].over) continue;
      st = br[k].update(n);
      any = any || !br[k].over;
    }
    if (st != EG_OK || !any) break;
    for (int k = 0; k < nh && st == EG_OK; ++k)
      if (!br[k].over) st = br[k].launch_cfl();
    if (st != EG_OK) break;
    if (!graphs) {
      for (int k = 0; k < nh && st == EG_OK; ++k)
        if (!br[k].over) st = vc_rec(hs[k], hs[k]->pmax, hs[k]->cfl_max);
      continue;
    }
    // one graph launch for the cycle: the running handles' captured
    // V-cycles as independent child graphs of one parent graph (one parent
    // per set of running handles and arithmetic phases)
    unsigned key = 0;
    for (int k = 0; k < nh; ++k)
      if (!br[k].over) key |= (1u << (2 * k)) | ((hs[k]->mixed && hs[k]->phase_b ? 1u : 0u) << (2 * k + 1));
    int slot = -1;
    for (size_t i = 0; i < pkey.size(); ++i)
      if (pkey[i] == key) slot = (int)i;
    if (slot < 0) {
      hipGraph_t parent = nullptr;
      const hipError_t ec = hipGraphCreate(&parent, 0);
      if (ec != hipSuccess) {
        st = hipfail(h0, ec, "hipGraphCreate");
        break;
      }
      parents.push_back(parent);
      for (int k = 0; k < nh && st == EG_OK; ++k) {
        if (br[k].over) continue;
        st = ensure_graph(hs[k], hs[k]->cfl_max);
        if (st != EG_OK) break;
        hipGraphNode_t node = nullptr;
        const hipError_t e =
            hipGraphAddChildGraphNode(&node, parent, nullptr, 0, hs[k]->ggraph[hs[k]->mixed && hs[k]->phase_b ? 1 : 0]);
        if (e != hipSuccess) st = hipfail(h0, e, "hipGraphAddChildGraphNode");
      }
      if (st != EG_OK) break;
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, parent, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        st = hipfail(h0, e, "hipGraphInstantiate");
        break;
      }
      pexec.push_back(ex);
      pkey.push_back(key);
      slot = (int)pkey.size() - 1;
    }
    const hipError_t e = hipGraphLaunch(pexec[slot], h0->st);
    if (e != hipSuccess) st = hipfail(h0, e, "hipGraphLaunch");
  }
  for (int k = 0; k < nh; ++k) {
    const eg_status sf = br[k].finish();
    if (st == EG_OK) st = sf;
  }
  hipError_t e2 = hipStreamSynchronize(h0->st);
  if (e2 != hipSuccess && st == EG_OK) st = hipfail(h0, e2, "sync");
  for (auto ex : pexec) (void)hipGraphExecDestroy(ex);
  for (auto g : parents) (void)hipGraphDestroy(g);
  eg_status worst = EG_OK;
  for (int k = 0; k < nh; ++k) {
    hs[k]->M.cfl_e = nullptr;
    if (k > 0) hs[k]->st = caller[k];
    status_host[k] = (int)(st != EG_OK ? st : br[k].result);
    if (worst == EG_OK || (worst == EG_ERR_NOT_CONVERGED && br[k].result == EG_ERR_DIVERGED))
      worst = br[k].result;
  }
  return st != EG_OK ? st : worst;
}

eg_status eg_solve_resume(eg_handle* h, double* u_dev, double drop_tol, int max_cycles, double* hist_host,
                          int* n_cycles_host) {
  if (!h || !u_dev || !hist_host || !n_cycles_host || max_cycles < 0) return EG_ERR_ARG;
  if (h->sv_next < 1) return fail(h, EG_ERR_ARG, "no steady solve to resume");
  return solve_loop(h, u_dev, h->sv_next, h->sv_r1, drop_tol, max_cycles, hist_host, n_cycles_host);
}

}  // extern "C"
