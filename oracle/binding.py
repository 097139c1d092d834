"""ctypes binding of the C++ oracle (test infrastructure only)."""

from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eg_oracle.cpp")
_LIB = os.path.join(_HERE, "libeg_oracle.so")
_lib = None

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with plain FP64 semantics (no contraction, no fast math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-shared", "-fPIC", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = C.CDLL(_LIB)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, _d, C.c_int, _i32, C.POINTER(C.c_int8), _d, C.c_int,
                                 C.c_double, C.c_double, C.c_double, C.c_double, C.c_char_p, C.c_int]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_nmodes.restype = C.c_int
        L.orc_nmodes.argtypes = [C.c_int, C.c_int]
        L.orc_nfaces.restype = C.c_int
        L.orc_nfaces.argtypes = [C.c_void_p]
        L.orc_gauss.argtypes = [C.c_int, _d, _d]
        L.orc_modes.argtypes = [C.c_int, C.c_int, _i32]
        L.orc_geometry.argtypes = [C.c_void_p, _d, _d, _d, _d]
        L.orc_basis_T.argtypes = [C.c_void_p, _d]
        L.orc_neighbours.argtypes = [C.c_void_p, _i32]
        L.orc_eval_point.argtypes = [C.c_void_p, C.c_int, C.c_int, _d, _d, _d, _d]
        L.orc_freestream_state.argtypes = [C.c_void_p, _d]
        L.orc_freestream.argtypes = [C.c_void_p, C.c_int, _d]
        L.orc_residual.argtypes = [C.c_void_p, C.c_int, _d, _d]
        L.orc_residual_complex.argtypes = [C.c_void_p, C.c_int, _d, _d, _d, _d]
        L.orc_jacobian_blocks.argtypes = [C.c_void_p, C.c_int, _d, _d, _d]
        L.orc_flux_jac.argtypes = [C.c_int, C.c_double, _d, _d, _d]
        L.orc_rusanov.argtypes = [C.c_int, C.c_double, _d, _d, _d, _d]
        L.orc_ghost.argtypes = [C.c_void_p, C.c_int, _d, _d, _d, _d]
        L.orc_rusanov_jac.argtypes = [C.c_int, C.c_double, _d, _d, _d, _d, _d]
        L.orc_roe_jac.argtypes = [C.c_int, C.c_double, _d, _d, _d, _d, _d]
        L.orc_roe.argtypes = [C.c_int, C.c_double, _d, _d, _d, _d]
        L.orc_set_flux.argtypes = [C.c_void_p, C.c_int]
        L.orc_timestep.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _d, _d]
        L.orc_rnorm.restype = C.c_double
        L.orc_rnorm.argtypes = [C.c_void_p, C.c_int, _d]
        L.orc_cfl_ramp.restype = C.c_double
        L.orc_cfl_ramp.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
        L.orc_drag.argtypes = [C.c_void_p, C.c_int, _d, _d, C.c_double, _d]
        L.orc_drag.restype = C.c_double
        L.orc_prk.restype = C.c_int
        L.orc_prk.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _d, _d]
        L.orc_exp1.restype = C.c_int
        L.orc_exp1.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _d, _d, C.POINTER(C.c_int), _d]
        L.orc_expm.restype = C.c_int
        L.orc_expm.argtypes = [C.c_int, _d, _d]
        L.orc_phi1_e1.restype = C.c_int
        L.orc_phi1_e1.argtypes = [C.c_int, _d, _d]
        L.orc_arnoldi_dense.restype = C.c_int
        L.orc_arnoldi_dense.argtypes = [C.c_int, C.c_int, _d, _d, _d, _d, _d]
        L.orc_vcycle.restype = C.c_int
        L.orc_vcycle.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _d, _d, _d, _d]
        L.orc_solve.restype = C.c_int
        L.orc_solve.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_int,
                                _d, _d, _d, C.POINTER(C.c_int)]
        L.orc_mms_project.argtypes = [C.c_void_p, C.c_int, _d]
        L.orc_mms_forcing.argtypes = [C.c_void_p, C.c_int, _d]
        L.orc_mms_error.restype = C.c_double
        L.orc_mms_error.argtypes = [C.c_void_p, C.c_int, _d]
        L.porc_create.restype = C.c_void_p
        L.porc_create.argtypes = [C.c_int, _d, C.c_int, C.POINTER(C.c_int8), _i32, C.POINTER(C.c_int8), C.c_int,
                                  C.c_double, C.c_double, C.c_double, C.c_double, C.c_char_p, C.c_int]
        L.porc_free.argtypes = [C.c_void_p]
        L.porc_set_flux.argtypes = [C.c_void_p, C.c_int]
        L.porc_nmodes.restype = C.c_int
        L.porc_nmodes.argtypes = [C.c_int]
        L.porc_nfaces.restype = C.c_int
        L.porc_nfaces.argtypes = [C.c_void_p]
        L.porc_monomials.argtypes = [C.c_int, _i32]
        L.porc_geometry.argtypes = [C.c_void_p, _d, _d, _d]
        L.porc_basis_S.argtypes = [C.c_void_p, _d]
        L.porc_vol_rule.argtypes = [C.c_void_p, C.c_int, C.c_int, _d, _d]
        L.porc_faces.argtypes = [C.c_void_p, _i32, _i32, _d]
        L.porc_face_rule.argtypes = [C.c_void_p, C.c_int, C.c_int, _d, _d, _d]
        L.porc_psi.argtypes = [C.c_void_p, C.c_int, C.c_int, _d, _d, _d]
        L.porc_freestream.argtypes = [C.c_void_p, C.c_int, _d]
        L.porc_residual.argtypes = [C.c_void_p, C.c_int, _d, _d]
        L.porc_residual_complex.argtypes = [C.c_void_p, C.c_int, _d, _d, _d, _d]
        L.porc_mms_project.argtypes = [C.c_void_p, C.c_int, _d]
        L.porc_mms_forcing.argtypes = [C.c_void_p, C.c_int, _d]
        L.porc_timestep.argtypes = [C.c_void_p, C.c_int, C.c_double, _d, _d]
        L.porc_element_blocks.argtypes = [C.c_void_p, C.c_int, _d, _d]
        L.porc_exp1.restype = C.c_int
        L.porc_exp1.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _d, _d]
        L.porc_vcycle.restype = C.c_int
        L.porc_vcycle.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _d, _d, _d]
        L.porc_solve.restype = C.c_int
        L.porc_solve.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _d, _d,
                                 C.POINTER(C.c_int)]
        L.porc_prk.restype = C.c_int
        L.porc_prk.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, _d, _d]
        L.porc_rnorm.restype = C.c_double
        L.porc_rnorm.argtypes = [C.c_void_p, C.c_int, _d]
        L.porc_surface.argtypes = [C.c_void_p, _d, _d]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    if a.dtype == np.float64:
        return a.ctypes.data_as(_d)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_i32)
    if a.dtype == np.int8:
        return a.ctypes.data_as(C.POINTER(C.c_int8))
    raise TypeError(a.dtype)


def gauss(Q: int):
    x = np.zeros(Q)
    w = np.zeros(Q)
    lib().orc_gauss(Q, _p(x), _p(w))
    return x, w


def modes(dim: int, p: int) -> np.ndarray:
    n = (p + 1) ** dim
    a = np.zeros((n, 3), dtype=np.int32)
    lib().orc_modes(dim, p, _p(a))
    return a


def expm(A: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    E = np.zeros_like(A)
    if lib().orc_expm(A.shape[0], _p(A), _p(E)) != 0:
        raise RuntimeError("expm failed")
    return E


def phi1_e1(H: np.ndarray) -> np.ndarray:
    H = np.ascontiguousarray(H, dtype=np.float64)
    y = np.zeros(H.shape[0])
    if lib().orc_phi1_e1(H.shape[0], _p(H), _p(y)) != 0:
        raise RuntimeError("phi1 failed")
    return y


def arnoldi_dense(A: np.ndarray, b: np.ndarray, m: int):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    K = A.shape[0]
    Vb = np.zeros((m + 1, K))
    H = np.zeros((m + 1, m))
    beta = C.c_double(0.0)
    mu = lib().orc_arnoldi_dense(K, m, _p(A), _p(b), _p(Vb), _p(H), C.byref(beta))
    return mu, Vb, H, beta.value


def rusanov(dim, gamma, UL, UR, nh):
    UL, UR, nh = (np.ascontiguousarray(a, dtype=np.float64) for a in (UL, UR, nh))
    F = np.zeros(dim + 2)
    lib().orc_rusanov(dim, gamma, _p(UL), _p(UR), _p(nh), _p(F))
    return F


def rusanov_jac(dim, gamma, UL, UR, nh):
    """(dF/dUL, dF/dUR) of the Rusanov flux by complex step."""
    UL, UR, nh = (np.ascontiguousarray(a, dtype=np.float64) for a in (UL, UR, nh))
    JL = np.zeros((dim + 2, dim + 2))
    JR = np.zeros((dim + 2, dim + 2))
    lib().orc_rusanov_jac(dim, gamma, _p(UL), _p(UR), _p(nh), _p(JL), _p(JR))
    return JL, JR


def roe(dim, gamma, UL, UR, nh):
    UL, UR, nh = (np.ascontiguousarray(a, dtype=np.float64) for a in (UL, UR, nh))
    F = np.zeros(dim + 2)
    lib().orc_roe(dim, gamma, _p(UL), _p(UR), _p(nh), _p(F))
    return F


def roe_jac(dim, gamma, UL, UR, nh):
    """(dF/dUL, dF/dUR) of the Roe flux by complex step."""
    UL, UR, nh = (np.ascontiguousarray(a, dtype=np.float64) for a in (UL, UR, nh))
    JL = np.zeros((dim + 2, dim + 2))
    JR = np.zeros((dim + 2, dim + 2))
    lib().orc_roe_jac(dim, gamma, _p(UL), _p(UR), _p(nh), _p(JL), _p(JR))
    return JL, JR


def flux_jac(dim, gamma, U, g):
    U, g = (np.ascontiguousarray(a, dtype=np.float64) for a in (U, g))
    K = np.zeros((dim + 2, dim + 2))
    lib().orc_flux_jac(dim, gamma, _p(U), _p(g), _p(K))
    return K


class Oracle:
    """One mesh + free stream + p_max.  Level-p vectors are float64[E, V, N_p]."""

    def __init__(self, mesh, pmax: int, gamma: float = 1.4, mach: float = 0.3,
                 alpha_deg: float = 0.0, beta_deg: float = 0.0, flux: str = "rusanov"):
        m = mesh.contiguous()
        self.mesh = m
        self.dim = m.dim
        self.V = m.dim + 2
        self.ne = m.n_elem
        self.pmax = pmax
        self.gamma = gamma
        self.mach = mach
        self.alpha_deg, self.beta_deg = alpha_deg, beta_deg
        err = C.create_string_buffer(256)
        h = lib().orc_create(m.dim, m.n_vert, _p(m.xyz), m.n_elem, _p(m.elem_vert), _p(m.bface_tag),
                             _p(getattr(m, "elem_geo", None)), pmax, gamma, mach, alpha_deg, beta_deg, err, 256)
        if not h:
            raise ValueError("oracle mesh set-up failed: " + err.value.decode())
        self._h = C.c_void_p(h)
        if flux not in ("rusanov", "roe"):
            raise ValueError("flux must be 'rusanov' or 'roe'")
        self.flux = flux
        lib().orc_set_flux(self._h, 1 if flux == "roe" else 0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def N(self, p: int) -> int:
        return (p + 1) ** self.dim

    def zeros(self, p: int) -> np.ndarray:
        return np.zeros((self.ne, self.V, self.N(p)))

    def geometry(self):
        vol, surf, h = (np.zeros(self.ne) for _ in range(3))
        om = C.c_double(0.0)
        lib().orc_geometry(self._h, _p(vol), _p(surf), _p(h), C.byref(om))
        return vol, surf, h, om.value

    def basis_T(self) -> np.ndarray:
        n = self.N(self.pmax)
        T = np.zeros((self.ne, n, n))
        lib().orc_basis_T(self._h, _p(T))
        return T

    def neighbours(self) -> np.ndarray:
        nb = np.zeros((self.ne, 2 * self.dim), dtype=np.int32)
        lib().orc_neighbours(self._h, _p(nb))
        return nb

    def eval_point(self, p, e, u, xi):
        U = np.zeros(self.V)
        x = np.zeros(self.dim)
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        lib().orc_eval_point(self._h, p, e, _p(np.ascontiguousarray(u)), _p(xi), _p(U), _p(x))
        return U, x

    def freestream_state(self) -> np.ndarray:
        U = np.zeros(self.V)
        lib().orc_freestream_state(self._h, _p(U))
        return U

    def freestream(self, p: int) -> np.ndarray:
        u = self.zeros(p)
        lib().orc_freestream(self._h, p, _p(u))
        return u

    def residual(self, p: int, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == (self.ne, self.V, self.N(p))
        r = np.zeros_like(u)
        lib().orc_residual(self._h, p, _p(u), _p(r))
        return r

    def residual_complex(self, p: int, u: np.ndarray) -> np.ndarray:
        ure = np.ascontiguousarray(u.real, dtype=np.float64)
        uim = np.ascontiguousarray(u.imag, dtype=np.float64)
        rre, rim = np.zeros_like(ure), np.zeros_like(ure)
        lib().orc_residual_complex(self._h, p, _p(ure), _p(uim), _p(rre), _p(rim))
        return rre + 1j * rim

    def jacobian_blocks(self, p: int, u: np.ndarray, offdiag: bool = False):
        u = np.ascontiguousarray(u, dtype=np.float64)
        n = self.V * self.N(p)
        D = np.zeros((self.ne, n, n))
        Off = np.zeros((self.ne, 2 * self.dim, n, n)) if offdiag else None
        lib().orc_jacobian_blocks(self._h, p, _p(u), _p(D), _p(Off))
        return (D, Off) if offdiag else D

    def ghost(self, tag, U, nh, x):
        Ug = np.zeros(self.V)
        lib().orc_ghost(self._h, tag, _p(np.ascontiguousarray(U, dtype=np.float64)),
                        _p(np.ascontiguousarray(nh, dtype=np.float64)),
                        _p(np.ascontiguousarray(x, dtype=np.float64)), _p(Ug))
        return Ug

    def timestep(self, p: int, cfl: float, u: np.ndarray) -> np.ndarray:
        dt = np.zeros(self.ne)
        u = np.ascontiguousarray(u, dtype=np.float64)
        lib().orc_timestep(self._h, p, u.shape[2], cfl, _p(u), _p(dt))
        return dt

    def drag(self, p: int, u: np.ndarray, direction=None, sref: float = 1.0, grad: bool = False):
        """Pressure drag coefficient C_D of the level-p state u on the slip
        walls along ``direction`` (default: the free-stream direction), and
        optionally dC_D/du."""
        if direction is None:
            direction = self.freestream_direction()
        dv = np.zeros(3)
        dv[: self.dim] = np.asarray(direction, dtype=np.float64)[: self.dim]
        u = np.ascontiguousarray(u, dtype=np.float64)
        g = np.zeros_like(u) if grad else None
        c = lib().orc_drag(self._h, p, _p(u), _p(dv), float(sref), _p(g) if grad else None)
        return (c, g) if grad else c

    def jacobian_sparse(self, p: int, u: np.ndarray):
        """dR_p/du as a scipy CSR matrix assembled from the exact element
        blocks (Section 3.3, eqs. (jac1), (jac2)); unknowns ordered as the
        flattened [E][V][N_p] vector."""
        import scipy.sparse as sp
        D, Off = self.jacobian_blocks(p, u, offdiag=True)
        n = self.V * self.N(p)
        nb = self.neighbours()
        I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        rows, cols, vals = [], [], []
        for e in range(self.ne):
            rows.append(e * n + I.ravel()); cols.append(e * n + J.ravel()); vals.append(D[e].ravel())
            for lf in range(2 * self.dim):
                if nb[e, lf] >= 0:
                    rows.append(e * n + I.ravel()); cols.append(nb[e, lf] * n + J.ravel())
                    vals.append(Off[e, lf].ravel())
        K = self.ne * n
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(K, K))

    def adjoint(self, p: int, u: np.ndarray, g: np.ndarray) -> np.ndarray:
        """The discrete adjoint: lambda with (dR_p/du)^T lambda + g = 0, by a
        sparse direct solve (for g = dJ/du, dJ/dtheta = dJ/dtheta|_u +
        lambda . dR/dtheta|_u)."""
        import scipy.sparse.linalg as spla
        Jm = self.jacobian_sparse(p, u)
        lam = spla.spsolve(Jm.T.tocsc(), -np.ascontiguousarray(g).ravel())
        return lam.reshape(u.shape)

    def freestream_direction(self) -> np.ndarray:
        a, b = math.radians(self.alpha_deg), math.radians(self.beta_deg)
        v = np.array([math.cos(a) * math.cos(b), math.sin(a) * math.cos(b), math.sin(b)])
        return v[: self.dim]

    def rnorm(self, p: int, r: np.ndarray) -> float:
        return lib().orc_rnorm(self._h, p, _p(np.ascontiguousarray(r)))

    def prk(self, p, s, cfl, u, f=None):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        if lib().orc_prk(self._h, p, s, cfl, _p(u), _p(f)) != 0:
            raise RuntimeError("PRK failed (singular block)")
        return u

    def exp1(self, m, cfl, u0, f0=None):
        u0 = np.array(u0, dtype=np.float64, copy=True, order="C")
        mu = C.c_int(0)
        beta = C.c_double(0.0)
        if lib().orc_exp1(self._h, self.pmax, m, cfl, _p(u0), _p(f0), C.byref(mu), C.byref(beta)) != 0:
            raise RuntimeError("EXP1 failed")
        return u0, mu.value, beta.value

    def vcycle(self, u, n, s=4, m=30, cfl_max=100.0, rref=1.0, f=None):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        rn = C.c_double(0.0)
        cfl = C.c_double(0.0)
        st = lib().orc_vcycle(self._h, self.pmax, s, m, cfl_max, rref, n, _p(u), _p(f), C.byref(rn), C.byref(cfl))
        if st != 0:
            raise RuntimeError(f"V-cycle failed ({st})")
        return u, rn.value, cfl.value

    def solve(self, u, s=4, m=30, cfl_max=100.0, drop=1e-10, max_cycles=200, f=None, relative_ramp=True):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        hist = np.zeros(max_cycles + 1)
        nc = C.c_int(0)
        st = lib().orc_solve(self._h, self.pmax, s, m, cfl_max, int(relative_ramp), drop, max_cycles, _p(u), _p(f),
                             _p(hist), C.byref(nc))
        return u, hist[: nc.value + 1], st

    def mms_project(self, p):
        u = self.zeros(p)
        lib().orc_mms_project(self._h, p, _p(u))
        return u

    def mms_forcing(self, p):
        f = self.zeros(p)
        lib().orc_mms_forcing(self._h, p, _p(f))
        return f

    def mms_error(self, p, u):
        return lib().orc_mms_error(self._h, p, _p(np.ascontiguousarray(u)))


def poly_nmodes(p: int) -> int:
    """N = (p+1)(p+2)(p+3)/6 Cartesian monomials of total degree <= p."""
    return (p + 1) * (p + 2) * (p + 3) // 6


def poly_monomials(p: int) -> np.ndarray:
    """int32[N, 3]: exponents (a_x, a_y, a_z) of chi_j in the oracle's order."""
    a = np.zeros((poly_nmodes(p), 3), dtype=np.int32)
    lib().porc_monomials(p, _p(a))
    return a


class PolyOracle:
    """Tetrahedra and prisms with the Cartesian P_p basis orthonormalised by
    MGS (Section 3.2).  Level-p vectors are float64[E, 5, N_p]."""

    def __init__(self, mesh, pmax: int, gamma: float = 1.4, mach: float = 0.3,
                 alpha_deg: float = 0.0, beta_deg: float = 0.0, flux: str = "rusanov"):
        m = mesh.contiguous()
        self.mesh = m
        self.V = 5
        self.ne = m.n_elem
        self.pmax = pmax
        self.gamma = gamma
        err = C.create_string_buffer(256)
        h = lib().porc_create(m.n_vert, _p(m.xyz), m.n_elem, _p(m.elem_type), _p(m.elem_vert), _p(m.bface_tag),
                              pmax, gamma, mach, alpha_deg, beta_deg, err, 256)
        if not h:
            raise ValueError("oracle mesh set-up failed: " + err.value.decode())
        self._h = C.c_void_p(h)
        if flux not in ("rusanov", "roe"):
            raise ValueError("flux must be 'rusanov' or 'roe'")
        self.flux = flux
        lib().porc_set_flux(self._h, 1 if flux == "roe" else 0)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.porc_free(h)
            self._h = None

    def N(self, p: int) -> int:
        return poly_nmodes(p)

    def zeros(self, p: int) -> np.ndarray:
        return np.zeros((self.ne, 5, self.N(p)))

    def geometry(self):
        """(volume [E], centroid xc [E, 3], half extents L [E, 3])."""
        vol = np.zeros(self.ne)
        xc, L = np.zeros((self.ne, 3)), np.zeros((self.ne, 3))
        lib().porc_geometry(self._h, _p(vol), _p(xc), _p(L))
        return vol, xc, L

    def basis_S(self) -> np.ndarray:
        n = self.N(self.pmax)
        S = np.zeros((self.ne, n, n))
        lib().porc_basis_S(self._h, _p(S))
        return S

    def vol_rule(self, e: int, Q: int):
        X, W = np.zeros((Q ** 3, 3)), np.zeros(Q ** 3)
        lib().porc_vol_rule(self._h, e, Q, _p(X), _p(W))
        return X, W

    def faces(self):
        nf = lib().porc_nfaces(self._h)
        info = np.zeros((nf, 6), dtype=np.int32)
        cv = np.zeros((nf, 4), dtype=np.int32)
        sgn = np.zeros(nf)
        lib().porc_faces(self._h, _p(info), _p(cv), _p(sgn))
        return info, cv, sgn

    def face_rule(self, f: int, Q: int):
        X, W, Nh = np.zeros((Q * Q, 3)), np.zeros(Q * Q), np.zeros((Q * Q, 3))
        lib().porc_face_rule(self._h, f, Q, _p(X), _p(W), _p(Nh))
        return X, W, Nh

    def psi(self, e: int, p: int, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = self.N(p)
        psi, g = np.zeros(n), np.zeros((n, 3))
        lib().porc_psi(self._h, e, n, _p(x), _p(psi), _p(g))
        return psi, g

    def freestream(self, p: int) -> np.ndarray:
        u = self.zeros(p)
        lib().porc_freestream(self._h, p, _p(u))
        return u

    def residual(self, p: int, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == (self.ne, 5, self.N(p))
        r = np.zeros_like(u)
        lib().porc_residual(self._h, p, _p(u), _p(r))
        return r

    def residual_complex(self, p: int, u: np.ndarray) -> np.ndarray:
        ure = np.ascontiguousarray(u.real, dtype=np.float64)
        uim = np.ascontiguousarray(u.imag, dtype=np.float64)
        rre, rim = np.zeros_like(ure), np.zeros_like(ure)
        lib().porc_residual_complex(self._h, p, _p(ure), _p(uim), _p(rre), _p(rim))
        return rre + 1j * rim

    def surface(self):
        """(|dE| [E], h_E = 6 |E| / |dE| [E])."""
        surf, hE = np.zeros(self.ne), np.zeros(self.ne)
        lib().porc_surface(self._h, _p(surf), _p(hE))
        return surf, hE

    def timestep(self, p: int, cfl: float, u: np.ndarray) -> np.ndarray:
        u = np.ascontiguousarray(u, dtype=np.float64)
        assert u.shape == (self.ne, 5, self.N(p))
        dt = np.zeros(self.ne)
        lib().porc_timestep(self._h, p, cfl, _p(u), _p(dt))
        return dt

    def rnorm(self, p: int, r: np.ndarray) -> float:
        r = np.ascontiguousarray(r, dtype=np.float64)
        assert r.shape == (self.ne, 5, self.N(p))
        return lib().porc_rnorm(self._h, p, _p(r))

    def element_blocks(self, p: int, u: np.ndarray) -> np.ndarray:
        """D_E = dR_E/du_E by complex step: [E, 5 N, 5 N], rows / columns (v, i)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        n = 5 * self.N(p)
        D = np.zeros((self.ne, n, n))
        lib().porc_element_blocks(self._h, p, _p(u), _p(D))
        return D

    def exp1(self, m: int, cfl: float, u0: np.ndarray, f0=None):
        """EXP1 on the level-0 state u0 (time steps at p_max), returns (u0 new, status)."""
        u = np.array(u0, dtype=np.float64, copy=True, order="C")
        f = None if f0 is None else np.ascontiguousarray(f0, dtype=np.float64)
        st = lib().porc_exp1(self._h, self.pmax, m, cfl, _p(u), _p(f))
        return u, st

    def vcycle(self, u, n, s=4, m=30, cfl_max=100.0, rref=0.0):
        """One V-cycle from the level-p_max state u: (u new, r_n, cfl, status)."""
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        rn, cfl = C.c_double(0.0), C.c_double(0.0)
        st = lib().porc_vcycle(self._h, self.pmax, s, m, cfl_max, rref, n, _p(u), C.byref(rn), C.byref(cfl))
        return u, rn.value, cfl.value, st

    def solve(self, u, s=4, m=30, cfl_max=100.0, drop=1e-10, max_cycles=200):
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        hist = np.zeros(max_cycles + 1)
        nc = C.c_int(0)
        st = lib().porc_solve(self._h, self.pmax, s, m, cfl_max, drop, max_cycles, _p(u), _p(hist), C.byref(nc))
        return u, hist[: nc.value + 1], st

    def prk(self, p: int, s: int, cfl: float, u: np.ndarray, f=None):
        """One s-stage PRK step from u (returns the new state and the status)."""
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        st = lib().porc_prk(self._h, p, s, cfl, _p(u), _p(f))
        return u, st

    def mms_project(self, p):
        u = self.zeros(p)
        lib().porc_mms_project(self._h, p, _p(u))
        return u

    def mms_forcing(self, p):
        f = self.zeros(p)
        lib().porc_mms_forcing(self._h, p, _p(f))
        return f
