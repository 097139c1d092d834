"""Mixed precision (FP32 smoother on p >= 1, FP64 state, norms, EXP1 and
defect correction) against the FP64 oracle, through the C ABI.

Errors stated per result.  A single FP32 residual evaluation sums O(50)
terms of size O(|F|) per coefficient in single precision (unit roundoff
6e-8), so against the FP64 residual of a state perturbed by 2 % its error is
a few 1e-6 of the residual's largest entry; one PRK step adds the FP32 LU
solve of blocks with condition numbers up to ~1e3.  The defect-corrected
V-cycle has the FP64 steady state as its fixed point, so converged solves
are compared at FP64 accuracy."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell
from tests.gpu_util import perturbed, to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu

CASES = [
    ("ogrid16x6-p3", ogrid(16, 6), 3, 3.0),
    ("ogrid10x3-p4", ogrid(10, 3), 4, -2.0),
    ("sphere6x2x2x2-p2", cubed_sphere_shell(2, 2), 2, 2.0),
    ("sphere6x2x2x2-p3", cubed_sphere_shell(2, 2), 3, 2.0),
    ("ogrid10x3c-p4-curved", ogrid(10, 3, curved=True), 4, -2.0),
    ("sphere6x2x2x2c-p2-curved", cubed_sphere_shell(2, 2, curved=True), 2, 2.0),
    ("sphere6x2x2x2c-p3-curved", cubed_sphere_shell(2, 2, curved=True), 3, 2.0),
]


def _solver(mesh, p, alpha, **kw):
    import paper_1807_01151_amd as P
    return P.Solver(mesh, p, alpha_deg=alpha, precision="mixed", **kw)


@pytest.mark.parametrize("name,mesh,p,alpha", CASES, ids=[c[0] for c in CASES])
def test_mixed_residual_error(name, mesh, p, alpha):
    """FP32 residual kernel vs the FP64 oracle residual: error <= 2e-5 of the
    largest entry at every level p >= 1 (FP64 at p = 0)."""
    print("case", name, flush=True)
    O = oracle.Oracle(mesh, p, alpha_deg=alpha)
    S = _solver(mesh, p, alpha)
    for lev in range(p + 1):
        u = perturbed(O, lev, 100 + lev)
        r_o = O.residual(lev, u)
        r_g = to_host(S.residual(lev, to_dev(u)))
        e = rel_err(r_g, r_o)
        print(f"  p={lev} residual error {e:.3e}", flush=True)
        assert e < (1e-12 if lev == 0 else 2e-5), (lev, e)


@pytest.mark.parametrize("name,mesh,p,alpha", CASES, ids=[c[0] for c in CASES])
def test_mixed_prk_step_error(name, mesh, p, alpha):
    """One FP32 PRK step (FP32 blocks, LU and stage solves) vs the FP64
    oracle step: the update agrees to 2e-4 of its largest entry."""
    print("case", name, flush=True)
    O = oracle.Oracle(mesh, p, alpha_deg=alpha)
    S = _solver(mesh, p, alpha, rk_stages=3)
    for lev in range(1, p + 1):
        u = perturbed(O, lev, 200 + lev)
        out_o = O.prk(lev, 3, 5.0, u)
        ud = to_dev(u)
        S.prk_step(lev, 5.0, ud)
        e = rel_err(to_host(ud) - u, out_o - u)
        print(f"  p={lev} PRK update error {e:.3e}", flush=True)
        assert e < 2e-4, (lev, e)


@pytest.fixture(scope="module")
def c1_steady():
    """The oracle's FP64 steady state of the c1 workload (O-grid 24 x 12,
    p = 1, s = 4, CFL_max = 100, m = 30), solved to a 1e-10 drop."""
    mesh = ogrid(24, 12)
    O = oracle.Oracle(mesh, 1)
    u, h, st = O.solve(O.freestream(1), s=4, m=30, cfl_max=100.0, drop=1e-10, max_cycles=4000)
    assert st == 0
    return mesh, O, u, h


def test_mixed_vcycle_keeps_fp64_fixed_point(c1_steady):
    """A mixed V-cycle started at the FP64 steady state moves it by no more
    than an FP64 V-cycle does (the defect correction makes R64 = 0 its fixed
    point; without it the FP32 residual's 1e-7 error would move it)."""
    mesh, O, u, h = c1_steady
    S = _solver(mesh, 1, 0.0, rk_stages=4, cfl_max=100.0, krylov_m=30)
    ud = to_dev(u)
    rn, cfl = S.vcycle(ud, 200, rref=h[0])
    du = np.max(np.abs(to_host(ud) - u)) / np.max(np.abs(u))
    un, rn_o, _ = O.vcycle(u, 200, s=4, m=30, cfl_max=100.0, rref=h[0])
    du_o = np.max(np.abs(un - u)) / np.max(np.abs(u))
    print("mixed move", du, "FP64 move", du_o, flush=True)
    assert abs(rn - rn_o) <= 1e-12 * h[0]
    assert du <= max(10 * du_o, 1e-12)


def test_mixed_solve_reaches_fp64_steady_state(c1_steady):
    """From the free stream the mixed solve reaches the 1e-10 FP64 residual
    drop; continued to a 1e-12 drop, its state equals the FP64 oracle's state
    continued to the same drop to 1e-9 (relative, max norm)."""
    mesh, O, u_o, h_o = c1_steady
    S = _solver(mesh, 1, 0.0, rk_stages=4, cfl_max=100.0, krylov_m=30)
    ud = S.freestream(1)
    h_m, st = S.solve_steady(ud, drop_tol=1e-10, max_cycles=6000)
    print("mixed cycles to 1e-10:", len(h_m) - 1, "FP64 oracle:", len(h_o) - 1, flush=True)
    assert st == 0
    assert h_m[-1] <= 1e-10 * h_m[0]
    # both continued to a 1e-12 drop: the states agree to 1e-9
    h_m2, st2 = S.solve_steady(ud, drop_tol=1e-12, max_cycles=3000, resume=True)
    u_m = to_host(ud)
    u_o2, h_o2, st_o2 = O.solve(u_o, s=4, m=30, cfl_max=100.0, drop=1e-12 * h_o[0] / O.rnorm(1, O.residual(1, u_o)),
                                max_cycles=3000)
    e = rel_err(u_m, u_o2)
    print("mixed vs FP64 steady state", e, "final drops", h_m2[-1] / h_m[0], flush=True)
    assert st2 == 0
    assert e <= 1e-9
    assert O.rnorm(1, O.residual(1, u_m)) <= 2e-12 * h_m[0]
