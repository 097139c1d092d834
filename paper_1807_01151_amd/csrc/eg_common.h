// Shared compile-time configuration and reference tables of the HIP path.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eg {

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// Geometry nodes per element: quads carry the nine nodes of a biquadratic
// map (quadratic curved elements, Section 5.1; straight ones have their edge
// and centre nodes at the bilinear positions), hexes their eight vertices.
constexpr int geo_nodes(int D) { return D == 2 ? 9 : 8; }

// Sizes of order P in dimension D: V variables, Q Gauss points per axis,
// N = (P+1)^D modes, QV volume points, QF points per face, NF faces, NC
// geometry nodes.
template <int D, int P>
struct Cfg {
  static constexpr int V = D + 2;
  static constexpr int Q = P + 2;
  static constexpr int N = ipow(P + 1, D);
  static constexpr int QV = ipow(Q, D);
  static constexpr int QF = ipow(Q, D - 1);
  static constexpr int NF = 2 * D;
  static constexpr int NC = geo_nodes(D);
  static constexpr int NB = V * N;  // block size of the element operator
};

// One-dimensional tables of order P, copied to LDS by every kernel:
// Gauss points / weights of the (P+2)-point rule, orthonormal Legendre
// values and derivatives at those points and at the interval ends, and the
// multi-index of every mode in hierarchical order.  R is the arithmetic type
// of the kernel that reads them (double, or float for the FP32 smoother).
template <int D, int P, class R = double>
struct Tab {
  R x[P + 2];
  R w[P + 2];
  R L[P + 1][P + 2];
  R dL[P + 1][P + 2];
  R Lb[P + 1][2];
  int8_t m[Cfg<D, P>::N][3];
};

// Numerical flux of the face integrals (Section 3.1 after eq. (euler3)).
constexpr int FLUX_RUSANOV = 0;
constexpr int FLUX_ROE = 1;

// Free stream, gas constant and numerical flux passed to kernels by value.
template <class R = double>
struct GasT {
  R g;
  R Uinf[5];
  int flux;  // FLUX_RUSANOV or FLUX_ROE
};
using Gas = GasT<double>;

// Boundary codes stored in the neighbour array for faces without neighbour.
constexpr int NB_WALL = -1;
constexpr int NB_FAR = -2;
// Neighbour code of a slip face that is a symmetry plane rather than the
// body: same ghost state, left out of the drag integral.
constexpr uint8_t NCODE_SYMMETRY = 1;

}  // namespace eg
