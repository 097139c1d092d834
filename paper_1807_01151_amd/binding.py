"""ctypes binding of libeg.so: argument marshalling only."""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libeg.so")
_lib = None

# every symbol include/eg.h declares
EXPORTED_SYMBOLS = (
    "eg_init_mesh", "eg_free", "eg_last_error", "eg_sizes", "eg_set_freestream", "eg_residual",
    "eg_timestep", "eg_element_jacobian", "eg_prk_step", "eg_jacobian_p0", "eg_exp1_step", "eg_rnorm",
    "eg_vcycle", "eg_solve_steady", "eg_solve_resume", "eg_profile", "eg_profile_read",
    "eg_drag", "eg_adjoint_apply", "eg_adjoint_solve", "eg_init_batch", "eg_layout", "eg_solve_batch", "eg_autotune",
    "eg_set_graphs", "eg_measure_peak", "eg_rnorm_noalloc",
    "eg_param_sensitivity", "eg_jacobian_apply", "eg_solve_multi",
    "eg_poly_init", "eg_poly_free", "eg_poly_last_error", "eg_poly_freestream", "eg_poly_residual",
    "eg_poly_basis", "eg_poly_timestep", "eg_poly_rnorm", "eg_poly_restrict", "eg_poly_prolong_add",
    "eg_poly_element_block", "eg_poly_prk_step", "eg_poly_exp1_step", "eg_poly_vcycle", "eg_poly_solve_steady",
)

KERNEL_CLASSES = ("residual", "jacobian_lu", "prk_stage", "transfer", "timestep", "p0_setup", "arnoldi",
                  "phi1", "exp1_update", "norm")

STATUS = {0: "EG_OK", 1: "EG_ERR_ARG", 2: "EG_ERR_MESH", 3: "EG_ERR_ALLOC", 4: "EG_ERR_HIP",
          5: "EG_ERR_NOT_CONVERGED", 6: "EG_ERR_DIVERGED", 7: "EG_ERR_UNSUPPORTED"}


class EgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_vert", C.c_int), ("xyz", C.POINTER(C.c_double)), ("n_elem", C.c_int),
                ("elem_vert", C.POINTER(C.c_int32)), ("bface_tag", C.POINTER(C.c_int8)),
                ("elem_geo", C.POINTER(C.c_double))]


def _c_mesh(m) -> _Mesh:
    """eg_mesh view of a contiguous mesh (the arrays must outlive the call)."""
    geo = getattr(m, "elem_geo", None)
    if geo is not None and geo.shape != (m.n_elem, 3 ** m.dim, m.dim):
        raise ValueError(f"elem_geo must have shape {(m.n_elem, 3 ** m.dim, m.dim)}, got {geo.shape}")
    return _Mesh(m.dim, m.n_vert, m.xyz.ctypes.data_as(C.POINTER(C.c_double)), m.n_elem,
                 m.elem_vert.ctypes.data_as(C.POINTER(C.c_int32)),
                 m.bface_tag.ctypes.data_as(C.POINTER(C.c_int8)),
                 None if geo is None else geo.ctypes.data_as(C.POINTER(C.c_double)))


class _PolyMesh(C.Structure):
    _fields_ = [("n_vert", C.c_int), ("xyz", C.POINTER(C.c_double)), ("n_elem", C.c_int),
                ("elem_type", C.POINTER(C.c_int8)), ("elem_vert", C.POINTER(C.c_int32)),
                ("bface_tag", C.POINTER(C.c_int8))]


class _Params(C.Structure):
    _fields_ = [("p_max", C.c_int), ("rk_stages", C.c_int), ("cfl_max", C.c_double), ("krylov_m", C.c_int),
                ("relative_ramp", C.c_int), ("gamma", C.c_double), ("mach", C.c_double),
                ("alpha_deg", C.c_double), ("beta_deg", C.c_double), ("precision", C.c_int),
                ("flux", C.c_int)]

PRECISIONS = {"fp64": 0, "mixed": 1}
FLUXES = {"rusanov": 0, "roe": 1}


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libeg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with paper_1807_01151_amd/build.py")
        L = C.CDLL(_LIB_PATH)
        vp, d, i = C.c_void_p, C.c_double, C.c_int
        pd = C.POINTER(C.c_double)
        L.eg_init_mesh.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), vp, C.POINTER(vp)]
        L.eg_init_mesh.restype = i
        L.eg_free.argtypes = [vp]
        L.eg_free.restype = None
        L.eg_last_error.argtypes = [vp]
        L.eg_last_error.restype = C.c_char_p
        L.eg_sizes.argtypes = [vp, i, C.POINTER(i), C.POINTER(i), C.POINTER(i)]
        L.eg_set_freestream.argtypes = [vp, i, vp]
        L.eg_residual.argtypes = [vp, i, vp, vp]
        L.eg_timestep.argtypes = [vp, i, i, d, vp, vp]
        L.eg_element_jacobian.argtypes = [vp, i, vp, vp]
        L.eg_prk_step.argtypes = [vp, i, d, vp, vp]
        L.eg_jacobian_p0.argtypes = [vp, vp, vp, vp, vp]
        L.eg_exp1_step.argtypes = [vp, d, vp, vp, C.POINTER(i)]
        L.eg_rnorm.argtypes = [vp, vp, pd]
        L.eg_rnorm_noalloc.argtypes = [vp, vp, vp]
        L.eg_rnorm_noalloc.restype = i
        L.eg_measure_peak.argtypes = [i, vp, pd]
        L.eg_measure_peak.restype = i
        L.eg_vcycle.argtypes = [vp, vp, i, d, pd, pd]
        L.eg_solve_steady.argtypes = [vp, vp, d, i, pd, C.POINTER(i)]
        L.eg_solve_resume.argtypes = [vp, vp, d, i, pd, C.POINTER(i)]
        L.eg_profile.argtypes = [vp, i]
        L.eg_profile_read.argtypes = [vp, i, i, pd, C.POINTER(i)]
        L.eg_drag.argtypes = [vp, vp, pd, d, pd, vp]
        L.eg_set_graphs.argtypes = [vp, i]
        L.eg_autotune.argtypes = [vp, i, C.POINTER(i)]
        L.eg_init_batch.argtypes = [C.POINTER(_Mesh), C.POINTER(_Params), i, vp, C.POINTER(vp)]
        L.eg_layout.argtypes = [vp, i, i, C.POINTER(C.c_int64), C.POINTER(i), C.POINTER(i)]
        L.eg_solve_batch.argtypes = [vp, vp, d, i, pd, C.POINTER(i)]
        L.eg_adjoint_apply.argtypes = [vp, i, vp, vp, vp]
        L.eg_jacobian_apply.argtypes = [vp, i, vp, vp, vp]
        L.eg_param_sensitivity.argtypes = [vp, vp, d, vp, vp, pd, d, pd]
        L.eg_param_sensitivity.restype = i
        L.eg_adjoint_solve.argtypes = [vp, vp, vp, vp, d, i, pd, C.POINTER(i)]
        L.eg_solve_multi.argtypes = [C.POINTER(vp), i, C.POINTER(vp), d, i, C.POINTER(vp), C.POINTER(vp),
                                     C.POINTER(i)]
        L.eg_solve_multi.restype = i
        L.eg_poly_init.argtypes = [C.POINTER(_PolyMesh), C.POINTER(_Params), vp, C.POINTER(vp)]
        L.eg_poly_init.restype = i
        L.eg_poly_free.argtypes = [vp]
        L.eg_poly_free.restype = None
        L.eg_poly_last_error.argtypes = [vp]
        L.eg_poly_last_error.restype = C.c_char_p
        L.eg_poly_freestream.argtypes = [vp, i, vp]
        L.eg_poly_freestream.restype = i
        L.eg_poly_residual.argtypes = [vp, i, vp, vp]
        L.eg_poly_residual.restype = i
        L.eg_poly_basis.argtypes = [vp, pd, pd, pd, pd]
        L.eg_poly_basis.restype = i
        L.eg_poly_element_block.argtypes = [vp, i, vp, vp]
        L.eg_poly_prk_step.argtypes = [vp, i, i, d, vp, vp]
        L.eg_poly_exp1_step.argtypes = [vp, d, vp, vp]
        L.eg_poly_exp1_step.restype = i
        L.eg_poly_vcycle.argtypes = [vp, vp, i, d, pd, pd]
        L.eg_poly_vcycle.restype = i
        L.eg_poly_solve_steady.argtypes = [vp, vp, d, i, pd, C.POINTER(i)]
        L.eg_poly_solve_steady.restype = i
        L.eg_poly_prk_step.restype = i
        L.eg_poly_element_block.restype = i
        L.eg_poly_timestep.argtypes = [vp, i, d, vp, vp]
        L.eg_poly_timestep.restype = i
        L.eg_poly_rnorm.argtypes = [vp, i, vp, pd]
        L.eg_poly_rnorm.restype = i
        L.eg_poly_restrict.argtypes = [vp, i, i, vp, vp]
        L.eg_poly_restrict.restype = i
        L.eg_poly_prolong_add.argtypes = [vp, i, i, vp, vp]
        L.eg_poly_prolong_add.restype = i
        for name in ("eg_sizes", "eg_set_freestream", "eg_residual", "eg_timestep", "eg_element_jacobian",
                     "eg_prk_step", "eg_jacobian_p0", "eg_exp1_step", "eg_rnorm", "eg_vcycle",
                     "eg_solve_steady", "eg_solve_resume", "eg_profile", "eg_profile_read"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def check_tensor(t, numel=None, dtype="float64", device=None, name="tensor"):
    """Checks a caller tensor before its pointer crosses the C ABI: a torch
    tensor of the given dtype and element count, contiguous, on the handle's
    device.  The kernels read and write exactly numel values, so a mismatch
    is refused here rather than left to the device.  Raises TypeError
    (type, dtype, device) or ValueError (size)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    want = getattr(torch, dtype)
    if t.dtype != want:
        raise TypeError(f"{name}: expected dtype {want}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()} (shape {tuple(t.shape)})")
    if not t.is_contiguous():
        raise TypeError(f"{name}: expected a contiguous tensor")
    if t.device.type != "cuda":
        raise TypeError(f"{name}: expected a device tensor, got one on {t.device}")
    if device is not None and t.device.index != device:
        raise TypeError(f"{name}: tensor on cuda:{t.device.index}, handle on cuda:{device}")
    return C.c_void_p(t.data_ptr())


class Solver:
    """One mesh on one device stream.  Level-p state tensors are float64
    [n_elem, V, N_p] on the device (C ABI layout [elem][var][mode])."""

    def __init__(self, mesh, p_max: int, rk_stages: int = 4, cfl_max: float = 100.0, krylov_m: int = 30,
                 relative_ramp: bool = True, gamma: float = 1.4, mach: float = 0.3, alpha_deg: float = 0.0,
                 beta_deg: float = 0.0, precision: str = "fp64", flux: str = "rusanov", stream=None):
        import numpy as np
        import torch
        L = lib()
        m = mesh.contiguous()
        self._keep = (m.xyz, m.elem_vert, m.bface_tag, m.elem_geo)
        cm = _c_mesh(m)
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        if flux not in FLUXES:
            raise ValueError(f"flux must be one of {sorted(FLUXES)}")
        self.precision, self.flux = precision, flux
        cp = _Params(p_max, rk_stages, cfl_max, krylov_m, int(relative_ramp), gamma, mach, alpha_deg, beta_deg,
                     PRECISIONS[precision], FLUXES[flux])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = L.eg_init_mesh(C.byref(cm), C.byref(cp), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if st != 0:
            msg = L.eg_last_error(h).decode() if h.value else ""
            if h.value:
                L.eg_free(h)
            self._h = None
            raise EgError(st, msg)
        self.dim, self.p_max, self.n_elem, self.V = m.dim, p_max, m.n_elem, m.dim + 2
        self.mach, self.alpha_deg, self.beta_deg = mach, alpha_deg, beta_deg
        self.krylov_m = krylov_m
        self.device = torch.cuda.current_device()
        self._np = np

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().eg_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != 0:
            raise EgError(st, lib().eg_last_error(self._h).decode())

    def N(self, p: int) -> int:
        return (p + 1) ** self.dim

    def _vec(self, t, p: int, name: str = "u"):
        """Pointer of a level-p coefficient vector (n_elem * V * N_p FP64
        values on the handle's device); None passes through."""
        if t is None:
            return None
        if not 0 <= p <= self.p_max:
            raise ValueError(f"order p = {p} outside 0..{self.p_max}")
        return check_tensor(t, self.n_elem * self.V * self.N(p), "float64", self.device, name)

    def _arr(self, t, numel: int, name: str, dtype: str = "float64"):
        return check_tensor(t, numel, dtype, self.device, name)

    def empty(self, p: int):
        import torch
        return torch.empty((self.n_elem, self.V, self.N(p)), dtype=torch.float64, device="cuda")

    def freestream(self, p: int):
        u = self.empty(p)
        pu = self._vec(u, p)
        self._chk(lib().eg_set_freestream(self._h, p, pu))
        return u

    def residual(self, p: int, u, out=None):
        pu = self._vec(u, p, "u")
        r = self.empty(p) if out is None else out
        pr = self._vec(r, p, "out")
        self._chk(lib().eg_residual(self._h, p, pu, pr))
        return r

    def timestep(self, p: int, cfl: float, u):
        import torch
        if u.dim() != 3:
            raise ValueError("u: expected a [n_elem, V, N_p] tensor")
        p_level = round(u.shape[2] ** (1.0 / self.dim)) - 1
        pu = self._vec(u, p_level, "u")
        dt = torch.empty(self.n_elem, dtype=torch.float64, device="cuda")
        self._chk(lib().eg_timestep(self._h, p, p_level, cfl, pu, self._arr(dt, self.n_elem, "dtau")))
        return dt

    def element_jacobian(self, p: int, u):
        import torch
        pu = self._vec(u, p, "u")
        n = self.V * self.N(p)
        D = torch.empty((self.n_elem, n, n), dtype=torch.float64, device="cuda")
        self._chk(lib().eg_element_jacobian(self._h, p, pu, self._arr(D, self.n_elem * n * n, "D")))
        return D

    def prk_step(self, p: int, cfl: float, u, f=None):
        pu, pf = self._vec(u, p, "u"), self._vec(f, p, "f")
        self._chk(lib().eg_prk_step(self._h, p, cfl, pu, pf))
        return u

    def jacobian_p0(self, u0):
        import torch
        pu = self._vec(u0, 0, "u0")
        V, nf = self.V, 2 * self.dim
        Dg = torch.empty((self.n_elem, V, V), dtype=torch.float64, device="cuda")
        Off = torch.empty((self.n_elem, nf, V, V), dtype=torch.float64, device="cuda")
        nb = torch.empty((self.n_elem, nf), dtype=torch.int32, device="cuda")
        self._chk(lib().eg_jacobian_p0(self._h, pu, self._arr(Dg, Dg.numel(), "diag"),
                                       self._arr(Off, Off.numel(), "off"),
                                       self._arr(nb, nb.numel(), "nbr", "int32")))
        return Dg, Off, nb

    def exp1_step(self, cfl: float, u0, f0=None):
        pu, pf = self._vec(u0, 0, "u0"), self._vec(f0, 0, "f0")
        mu = C.c_int(0)
        self._chk(lib().eg_exp1_step(self._h, cfl, pu, pf, C.byref(mu)))
        return u0, mu.value

    def rnorm(self, r) -> float:
        pr = self._vec(r, self.p_max, "r")
        v = C.c_double(0.0)
        self._chk(lib().eg_rnorm(self._h, pr, C.byref(v)))
        return v.value

    def rnorm_noalloc(self, r, out=None):
        """eg_rnorm's norm written into a one-element device tensor, with no
        allocation inside the library and no synchronisation."""
        import torch
        pr = self._vec(r, self.p_max, "r")
        o = torch.empty(1, dtype=torch.float64, device="cuda") if out is None else out
        self._chk(lib().eg_rnorm_noalloc(self._h, pr, self._arr(o, 1, "out")))
        return o

    def vcycle(self, u, n: int, rref: float = 0.0):
        pu = self._vec(u, self.p_max, "u")
        rn = C.c_double(0.0)
        cfl = C.c_double(0.0)
        self._chk(lib().eg_vcycle(self._h, pu, n, rref, C.byref(rn), C.byref(cfl)))
        return rn.value, cfl.value

    def profile(self, enable: bool):
        self._chk(lib().eg_profile(self._h, int(enable)))

    def set_graphs(self, enable: bool):
        """Replay the V-cycle as a captured HIP graph in the steady solves."""
        self._chk(lib().eg_set_graphs(self._h, int(enable)))

    def autotune(self, reps: int = 5):
        """Time the residual's element tiles per order and precision and keep
        the fastest (eg_autotune); returns {(p, "fp64" | "fp32"): elements
        per workgroup}."""
        return _autotune(self, reps)

    def profile_read(self, kernel_class: str, p: int = -1):
        """(total milliseconds, launches) of one kernel class at level p (-1: all)."""
        ms = C.c_double(0.0)
        n = C.c_int(0)
        self._chk(lib().eg_profile_read(self._h, KERNEL_CLASSES.index(kernel_class), p, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def solve_steady(self, u, drop_tol: float = 1e-10, max_cycles: int = 1000, raise_on_fail: bool = False,
                     resume: bool = False):
        np = self._np
        pu = self._vec(u, self.p_max, "u")
        hist = np.zeros(max_cycles + 1)
        nc = C.c_int(0)
        fn = lib().eg_solve_resume if resume else lib().eg_solve_steady
        st = fn(self._h, pu, drop_tol, max_cycles, hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nc))
        if st not in (0, 5, 6) or (raise_on_fail and st != 0):
            self._chk(st)
        return hist[: nc.value + 1], st


def measure_peak(kind: str, stream=None) -> float:
    """Achievable peak of the current device: "hbm" (GB/s, streaming copy),
    "fp64_mfma" or "fp64_fma" (TFLOP/s)."""
    import torch
    kinds = {"hbm": 0, "fp64_mfma": 1, "fp64_fma": 2}
    st = stream if stream is not None else torch.cuda.current_stream()
    v = C.c_double(0.0)
    s = lib().eg_measure_peak(kinds[kind], C.c_void_p(st.cuda_stream), C.byref(v))
    if s != 0:
        raise EgError(s, "eg_measure_peak failed")
    return v.value


def _autotune(obj, reps):
    pmax = obj.p_max
    tiles = (C.c_int * (2 * (pmax + 1)))()
    obj._chk(lib().eg_autotune(obj._h, int(reps), tiles))
    return {(p, prec): tiles[2 * p + k] for p in range(pmax + 1) for k, prec in enumerate(("fp64", "fp32"))}


def _freestream_direction(dim, alpha_deg, beta_deg):
    import math
    a, b = math.radians(alpha_deg), math.radians(beta_deg)
    v = (math.cos(a) * math.cos(b), math.sin(a) * math.cos(b), math.sin(b))
    return v[:dim]


def _solver_drag(self, u, direction=None, sref: float = 1.0, grad: bool = False):
    """Pressure drag coefficient C_D of the level-p_max state u (and
    optionally dC_D/du on the device)."""
    if direction is None:
        direction = _freestream_direction(self.dim, self.alpha_deg, self.beta_deg)
    dv = (C.c_double * 3)(*([float(x) for x in direction] + [0.0] * (3 - len(direction))))
    cd = C.c_double(0.0)
    pu = self._vec(u, self.p_max, "u")
    g = self.empty(self.p_max) if grad else None
    self._chk(lib().eg_drag(self._h, pu, dv, float(sref), C.byref(cd), self._vec(g, self.p_max, "grad")))
    return (cd.value, g) if grad else cd.value


def _solver_jacobian_apply(self, p: int, u, v, out=None):
    """(dR_p/du)(u) v (matrix free, forward-mode dual numbers)."""
    pu, pv = self._vec(u, p, "u"), self._vec(v, p, "v")
    o = self.empty(p) if out is None else out
    self._chk(lib().eg_jacobian_apply(self._h, p, pu, pv, self._vec(o, p, "out")))
    return o


def _solver_adjoint_apply(self, p: int, u, w, out=None):
    """(dR_p/du)(u)^T w."""
    pu, pw = self._vec(u, p, "u"), self._vec(w, p, "w")
    o = self.empty(p) if out is None else out
    self._chk(lib().eg_adjoint_apply(self._h, p, pu, pw, self._vec(o, p, "out")))
    return o


def _solver_adjoint_solve(self, u, g, lam=None, drop_tol: float = 1e-10, max_cycles: int = 500,
                          raise_on_fail: bool = True):
    """lambda with (dR/du)(u)^T lambda + g = 0 (adjoint V-cycles); returns
    (lambda, history of the adjoint residual 2-norm, status)."""
    import torch
    np = self._np
    pu, pg = self._vec(u, self.p_max, "u"), self._vec(g, self.p_max, "g")
    lam = torch.zeros_like(g) if lam is None else lam
    pl = self._vec(lam, self.p_max, "lam")
    hist = np.zeros(max_cycles + 1)
    nc = C.c_int(0)
    st = lib().eg_adjoint_solve(self._h, pu, pg, pl, drop_tol, max_cycles,
                                hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nc))
    if st not in (0, 5) or (raise_on_fail and st != 0):
        self._chk(st)
    return lam, hist[: nc.value + 1], st


def _solver_param_sensitivity(self, minus, step: float, u, lam, direction=None, sref: float = 1.0):
    """dC_D/dtheta = dC_D/dtheta|_u + lambda . dR/dtheta|_u by central
    differences over this handle (built at theta + step) and ``minus``
    (theta - step), evaluated inside the library (eg_param_sensitivity)."""
    if direction is None:
        direction = _freestream_direction(self.dim, self.alpha_deg, self.beta_deg)
    dv = (C.c_double * 3)(*([float(x) for x in direction] + [0.0] * (3 - len(direction))))
    pu, pl = self._vec(u, self.p_max, "u"), self._vec(lam, self.p_max, "lam")
    out = C.c_double(0.0)
    self._chk(lib().eg_param_sensitivity(self._h, minus._h, float(step), pu, pl, dv, float(sref), C.byref(out)))
    return out.value


Solver.drag = _solver_drag
Solver.adjoint_apply = _solver_adjoint_apply
Solver.jacobian_apply = _solver_jacobian_apply
Solver.param_sensitivity = _solver_param_sensitivity
Solver.adjoint_solve = _solver_adjoint_solve


class BatchSolver:
    """n independent steady solves (same dim, p_max and solver settings; own
    mesh, Mach number and angles) in one handle of the library: every kernel
    launch covers all solves, norms, CFL ramps and the EXP1 Krylov process
    are per solve.  The state is one device tensor of the solves' level-p_max
    vectors one after another (``views`` splits it)."""

    def __init__(self, meshes, p_max: int, machs, alphas=None, betas=None, rk_stages: int = 4,
                 cfl_max: float = 100.0, krylov_m: int = 30, relative_ramp: bool = True, gamma: float = 1.4,
                 precision: str = "fp64", flux: str = "rusanov", stream=None):
        import numpy as np
        import torch
        L = lib()
        n = len(meshes)
        alphas = [0.0] * n if alphas is None else list(alphas)
        betas = [0.0] * n if betas is None else list(betas)
        ms = [m.contiguous() for m in meshes]
        self._keep = [(m.xyz, m.elem_vert, m.bface_tag, m.elem_geo) for m in ms]
        cms = (_Mesh * n)(*[_c_mesh(m) for m in ms])
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        if flux not in FLUXES:
            raise ValueError(f"flux must be one of {sorted(FLUXES)}")
        cps = (_Params * n)(*[_Params(p_max, rk_stages, cfl_max, krylov_m, int(relative_ramp), gamma, float(machs[i]),
                                      float(alphas[i]), float(betas[i]), PRECISIONS[precision], FLUXES[flux])
                              for i in range(n)])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = L.eg_init_batch(cms, cps, n, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if st != 0:
            msg = L.eg_last_error(h).decode() if h.value else ""
            if h.value:
                L.eg_free(h)
            self._h = None
            raise EgError(st, msg)
        self.n, self.dim, self.p_max, self.V = n, ms[0].dim, p_max, ms[0].dim + 2
        self.n_elem = sum(m.n_elem for m in ms)
        self.elems = [m.n_elem for m in ms]
        self.device = torch.cuda.current_device()
        self._np = np

    close = Solver.close
    __del__ = Solver.__del__
    set_graphs = Solver.set_graphs
    _chk = Solver._chk
    N = Solver.N
    _vec = Solver._vec
    _arr = Solver._arr
    empty = Solver.empty
    freestream = Solver.freestream
    residual = Solver.residual

    def autotune(self, reps: int = 5):
        """Residual tiles per order and precision of the batch (see Solver.autotune)."""
        return _autotune(self, reps)

    def profile(self, enable: bool):
        """Event timing of every kernel class (see Solver.profile)."""
        self._chk(lib().eg_profile(self._h, int(enable)))

    def profile_read(self, kernel_class: str, p: int = -1):
        """(total milliseconds, launches) of one kernel class at level p (-1: all)."""
        ms = C.c_double(0.0)
        n = C.c_int(0)
        self._chk(lib().eg_profile_read(self._h, KERNEL_CLASSES.index(kernel_class), p, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def layout(self, solve: int, p: int):
        off = C.c_int64(0)
        nm, ne = C.c_int(0), C.c_int(0)
        self._chk(lib().eg_layout(self._h, solve, p, C.byref(off), C.byref(nm), C.byref(ne)))
        return off.value, nm.value, ne.value

    def views(self, u):
        """Per-solve [n_elem_s, V, N] views of a batch vector."""
        out, e0 = [], 0
        for ne in self.elems:
            out.append(u[e0:e0 + ne])
            e0 += ne
        return out

    def solve(self, u, drop_tol: float = 1e-10, max_cycles: int = 1000):
        """Returns (list of per-solve residual histories, cycles per solve, status)."""
        np = self._np
        pu = self._vec(u, self.p_max, "u")
        hist = np.zeros((self.n, max_cycles + 1))
        nc = (C.c_int * self.n)()
        st = lib().eg_solve_batch(self._h, pu, drop_tol, max_cycles,
                                  hist.ctypes.data_as(C.POINTER(C.c_double)), nc)
        if st not in (0, 5, 6):
            self._chk(st)
        cyc = [int(nc[i]) for i in range(self.n)]
        return [hist[i, : cyc[i] + 1] for i in range(self.n)], cyc, st


def solve_multi(batches, us, drop_tol: float = 1e-10, max_cycles: int = 1000):
    """Several BatchSolvers (e.g. one per polynomial order) advanced together
    by eg_solve_multi: per V-cycle one synchronisation and one launch (a
    single graph of every handle's V-cycle when all have graph replay
    enabled).  Returns, per handle, (per-solve histories, cycles per solve,
    status) as BatchSolver.solve."""
    import numpy as np
    batches, us = list(batches), list(us)
    if not batches or len(batches) != len(us):
        raise ValueError("solve_multi: one state per batch handle")
    if len({id(b) for b in batches}) != len(batches):
        raise ValueError("solve_multi: a handle appears twice")
    nh = len(batches)
    hs = (C.c_void_p * nh)(*[b._h for b in batches])
    pu = (C.c_void_p * nh)(*[b._vec(u, b.p_max, "u") for b, u in zip(batches, us)])
    hists = [np.zeros((b.n, max_cycles + 1)) for b in batches]
    ncs = [(C.c_int * b.n)() for b in batches]
    ph = (C.c_void_p * nh)(*[h.ctypes.data for h in hists])
    pn = (C.c_void_p * nh)(*[C.cast(nc, C.c_void_p).value for nc in ncs])
    status = (C.c_int * nh)()
    st = lib().eg_solve_multi(hs, nh, pu, drop_tol, max_cycles, ph, pn, status)
    if st not in (0, 5, 6):
        batches[0]._chk(st)
    out = []
    for k, b in enumerate(batches):
        cyc = [int(ncs[k][i]) for i in range(b.n)]
        out.append(([hists[k][i, : cyc[i] + 1] for i in range(b.n)], cyc, int(status[k])))
    return out


class PolySolver:
    """Tetrahedra and prisms with the Cartesian basis (eg_poly_* entry
    points).  Level-p tensors are float64 [n_elem, 5, N_p] on the device,
    N_p = (p+1)(p+2)(p+3)/6."""

    def __init__(self, mesh, p_max: int, rk_stages: int = 4, cfl_max: float = 100.0, krylov_m: int = 30,
                 gamma: float = 1.4, mach: float = 0.3, alpha_deg: float = 0.0, beta_deg: float = 0.0,
                 flux: str = "rusanov", stream=None):
        import torch
        L = lib()
        m = mesh.contiguous()
        self._keep = (m.xyz, m.elem_type, m.elem_vert, m.bface_tag)
        if m.elem_vert.shape != (m.n_elem, 6) or m.bface_tag.shape != (m.n_elem, 5) or m.xyz.shape[1:] != (3,):
            raise ValueError("poly mesh arrays must be xyz [n_vert, 3], elem_vert [n_elem, 6], bface_tag [n_elem, 5]")
        if flux not in FLUXES:
            raise ValueError(f"flux must be one of {sorted(FLUXES)}")
        cm = _PolyMesh(m.n_vert, m.xyz.ctypes.data_as(C.POINTER(C.c_double)), m.n_elem,
                       m.elem_type.ctypes.data_as(C.POINTER(C.c_int8)),
                       m.elem_vert.ctypes.data_as(C.POINTER(C.c_int32)),
                       m.bface_tag.ctypes.data_as(C.POINTER(C.c_int8)))
        cp = _Params(p_max, rk_stages, cfl_max, krylov_m, 1, gamma, mach, alpha_deg, beta_deg, 0, FLUXES[flux])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        st = L.eg_poly_init(C.byref(cm), C.byref(cp), C.c_void_p(self.stream.cuda_stream), C.byref(h))
        self._h = h
        if st != 0:
            msg = L.eg_poly_last_error(h).decode() if h.value else ""
            if h.value:
                L.eg_poly_free(h)
            self._h = None
            raise EgError(st, msg)
        self.p_max, self.n_elem, self.V = p_max, m.n_elem, 5
        self.device = torch.cuda.current_device()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().eg_poly_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != 0:
            raise EgError(st, lib().eg_poly_last_error(self._h).decode())

    @staticmethod
    def N(p: int) -> int:
        return (p + 1) * (p + 2) * (p + 3) // 6

    def _vec(self, t, p: int, name: str):
        if not 0 <= p <= self.p_max:
            raise ValueError(f"order p = {p} outside 0..{self.p_max}")
        return check_tensor(t, self.n_elem * 5 * self.N(p), "float64", self.device, name)

    def empty(self, p: int):
        import torch
        return torch.empty((self.n_elem, 5, self.N(p)), dtype=torch.float64, device="cuda")

    def freestream(self, p: int):
        u = self.empty(p)
        self._chk(lib().eg_poly_freestream(self._h, p, self._vec(u, p, "u")))
        return u

    def residual(self, p: int, u, out=None):
        pu = self._vec(u, p, "u")
        r = self.empty(p) if out is None else out
        pr = self._vec(r, p, "out")
        if pr.value == pu.value:
            raise ValueError("out must not alias u")
        self._chk(lib().eg_poly_residual(self._h, p, pu, pr))
        return r

    def element_block(self, p: int, u, out=None):
        """D_E = dR_E/du_E for every element: float64 [n_elem, 5 N_p, 5 N_p]."""
        import torch
        n = 5 * self.N(p)
        pu = self._vec(u, p, "u")
        D = torch.empty((self.n_elem, n, n), dtype=torch.float64, device="cuda") if out is None else out
        self._chk(lib().eg_poly_element_block(self._h, p, pu,
                                              check_tensor(D, self.n_elem * n * n, "float64", self.device, "out")))
        return D

    def prk_step(self, p: int, s: int, cfl: float, u, f=None):
        """One s-stage PRK step on u (level p >= 1), in place."""
        pu = self._vec(u, p, "u")
        pf = None if f is None else self._vec(f, p, "f")
        if pf is not None and pf.value == pu.value:
            raise ValueError("f must not alias u")
        self._chk(lib().eg_poly_prk_step(self._h, p, int(s), float(cfl), pu, pf))
        return u

    def exp1_step(self, cfl: float, u0, f0=None):
        """EXP1 on the level-0 state u0, in place."""
        pu = self._vec(u0, 0, "u0")
        pf = None if f0 is None else self._vec(f0, 0, "f0")
        if pf is not None and pf.value == pu.value:
            raise ValueError("f0 must not alias u0")
        self._chk(lib().eg_poly_exp1_step(self._h, float(cfl), pu, pf))
        return u0

    def vcycle(self, u, n: int, rref: float = 0.0):
        """One V-cycle on the level-p_max state u, in place: (r_n, cfl)."""
        rn, cfl = C.c_double(0.0), C.c_double(0.0)
        self._chk(lib().eg_poly_vcycle(self._h, self._vec(u, self.p_max, "u"), int(n), float(rref),
                                       C.byref(rn), C.byref(cfl)))
        return rn.value, cfl.value

    def solve_steady(self, u, drop_tol: float = 1e-10, max_cycles: int = 1000):
        """V-cycles in place until the drop or max_cycles: (history, status)."""
        import numpy as np
        hist = np.zeros(max_cycles + 1)
        nc = C.c_int(0)
        st = lib().eg_poly_solve_steady(self._h, self._vec(u, self.p_max, "u"), float(drop_tol), int(max_cycles),
                                        hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(nc))
        if st not in (0, 5, 6):
            self._chk(st)
        return hist[: nc.value + 1], st

    def timestep(self, p: int, cfl: float, u):
        import torch
        pu = self._vec(u, p, "u")
        dt = torch.empty(self.n_elem, dtype=torch.float64, device="cuda")
        self._chk(lib().eg_poly_timestep(self._h, p, float(cfl), pu,
                                         check_tensor(dt, self.n_elem, "float64", self.device, "dtau")))
        return dt

    def rnorm(self, p: int, r) -> float:
        out = C.c_double(0.0)
        self._chk(lib().eg_poly_rnorm(self._h, p, self._vec(r, p, "r"), C.byref(out)))
        return out.value

    def restrict(self, pf: int, pc: int, x, out=None):
        if not 0 <= pc <= pf:
            raise ValueError("restrict needs 0 <= pc <= pf")
        px = self._vec(x, pf, "x")
        y = self.empty(pc) if out is None else out
        self._chk(lib().eg_poly_restrict(self._h, pf, pc, px, self._vec(y, pc, "out")))
        return y

    def prolong_add(self, pc: int, pf: int, y, x):
        """x (level pf) += zero-padded y (level pc), in place."""
        if not 0 <= pc <= pf:
            raise ValueError("prolong_add needs 0 <= pc <= pf")
        py, px = self._vec(y, pc, "y"), self._vec(x, pf, "x")
        if px.value == py.value:
            raise ValueError("x must not alias y")
        self._chk(lib().eg_poly_prolong_add(self._h, pc, pf, py, px))
        return x

    def basis(self):
        """(S [n_elem, N_pmax, N_pmax], xc [n_elem, 3], L [n_elem, 3], vol [n_elem]) of the set-up."""
        import numpy as np
        n = self.N(self.p_max)
        S = np.zeros((self.n_elem, n, n))
        xc, Lh, vol = np.zeros((self.n_elem, 3)), np.zeros((self.n_elem, 3)), np.zeros(self.n_elem)
        pd = C.POINTER(C.c_double)
        self._chk(lib().eg_poly_basis(self._h, S.ctypes.data_as(pd), xc.ctypes.data_as(pd), Lh.ctypes.data_as(pd),
                                      vol.ctypes.data_as(pd)))
        return S, xc, Lh, vol
