"""Adjoint drag sensitivity on the GPU against the FP64 oracle: the drag
functional and its gradient, the transposed-Jacobian kernel against the
oracle's assembled Jacobian, the adjoint V-cycle against the oracle's sparse
direct adjoint, and the torch.autograd gradient dC_D/dtheta (Mach number and
wall-bump amplitudes) against central finite differences of converged GPU
solves (step 1e-6, FP64).

Tolerances: the functional and the matrix-free products are single FP64
evaluations (1e-12 of the largest entry, as for the residual); the adjoint
solution is iterated to a 1e-12 drop of its residual, so it matches the
direct solve to ~1e-12 times the conditioning (1e-8 bound); the FD check is
limited by the steady solves' 1e-12 drop over a step of 1e-6 (1e-5 bound)."""

import numpy as np
import pytest
import torch

import oracle
from eg_inputs import ogrid, cubed_sphere_shell, wall_bumps, bump_centers, clip
from tests.gpu_util import perturbed, to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu


def _quarter(mesh):
    """y > 0, z > 0 part of the shell; the cut faces are symmetry planes."""
    return clip(mesh, np.all(mesh.xyz[mesh.elem_vert].mean(axis=1)[:, 1:] > 0.0, axis=1))


CASES = [
    ("ogrid16x6-p3", ogrid(16, 6), 3, 3.0),
    ("ogrid12x4-p2", ogrid(12, 4), 2, -2.0),
    ("sphere6x2x2x2-p1", cubed_sphere_shell(2, 2), 1, 2.0),
    ("ogrid10x3-p4", ogrid(10, 3), 4, 1.0),
    ("sphere6x2x2x2-p2", cubed_sphere_shell(2, 2), 2, -1.0),
    ("sphere6x2x2x2-p3", cubed_sphere_shell(2, 2), 3, 1.0),
    ("ogrid12x4c-p3-curved", ogrid(12, 4, curved=True), 3, 2.0),
    ("sphere6x4x4x2-quarter-p2-symmetry", _quarter(cubed_sphere_shell(4, 2)), 2, 0.0),
    ("sphere6x2x2x2c-p3-curved", cubed_sphere_shell(2, 2, curved=True), 3, 1.0),
]


def _solver(mesh, p, alpha, **kw):
    import paper_1807_01151_amd as P
    return P.Solver(mesh, p, alpha_deg=alpha, **kw)


@pytest.mark.parametrize("name,mesh,p,alpha", CASES, ids=[c[0] for c in CASES])
def test_drag_parity(name, mesh, p, alpha):
    O = oracle.Oracle(mesh, p, alpha_deg=alpha)
    S = _solver(mesh, p, alpha)
    u = perturbed(O, p, 300)
    c_o, g_o = O.drag(p, u, sref=0.7, grad=True)
    c_g, g_g = S.drag(to_dev(u), sref=0.7, grad=True)
    print(name, "C_D", c_o, c_g, flush=True)
    # C_D is a sum of O(1) wall-pressure terms whose free-stream part cancels
    # over the closed wall, so its round-off is relative to O(1), not to C_D
    assert abs(c_g - c_o) <= 1e-12 * max(abs(c_o), 1.0)
    assert rel_err(to_host(g_g), g_o) < 1e-12


@pytest.mark.parametrize("name,mesh,p,alpha", CASES, ids=[c[0] for c in CASES])
def test_adjoint_apply_parity(name, mesh, p, alpha):
    """(dR_p/du)^T w against the oracle's assembled Jacobian (exact blocks,
    pinned to complex step) at every level p >= 1."""
    O = oracle.Oracle(mesh, p, alpha_deg=alpha)
    S = _solver(mesh, p, alpha)
    rng = np.random.default_rng(301)
    for lev in range(1, p + 1):
        u = perturbed(O, lev, 310 + lev)
        w = rng.standard_normal(u.shape)
        ref = (O.jacobian_sparse(lev, u).T @ w.ravel()).reshape(u.shape)
        got = to_host(S.adjoint_apply(lev, to_dev(u), to_dev(w)))
        e = rel_err(got, ref)
        print(f"  {name} p={lev} J^T w error {e:.3e}", flush=True)
        assert e < 1e-12


@pytest.fixture(scope="module")
def c1_steady():
    mesh = ogrid(24, 12)
    O = oracle.Oracle(mesh, 1)
    u, h, st = O.solve(O.freestream(1), s=4, m=30, cfl_max=100.0, drop=1e-12, max_cycles=6000)
    assert st == 0
    return mesh, O, u


def test_adjoint_solve_parity(c1_steady):
    """The adjoint V-cycle at the converged c1 state (O-grid 24 x 12, p = 1)
    against the oracle's sparse direct solve of (dR/du)^T lambda + dC_D/du = 0."""
    mesh, O, u = c1_steady
    S = _solver(mesh, 1, 0.0, rk_stages=4, cfl_max=100.0, krylov_m=30)
    _, g = O.drag(1, u, grad=True)
    lam_o = O.adjoint(1, u, g)
    lam_g, hist, st = S.adjoint_solve(to_dev(u), to_dev(g), drop_tol=1e-12, max_cycles=10000)
    e = rel_err(to_host(lam_g), lam_o)
    print("adjoint cycles", len(hist) - 1, "drop", hist[-1] / hist[0], "lambda error", e, flush=True)
    assert st == 0
    assert e < 1e-8


@pytest.mark.parametrize("name,mesh,p,alpha", CASES[4:6], ids=[c[0] for c in CASES[4:6]])
def test_adjoint_solve_large_blocks(name, mesh, p, alpha):
    """Adjoint V-cycles with the 135 x 135 and 320 x 320 blocks of 3D p = 2
    and 3 at a perturbed state: the adjoint problem is linear in lambda, so its residual
    (dR/du)^T lambda + dC_D/du, with the oracle's assembled Jacobian, is
    checked directly (10^-8 of |g| after a 10^-11 drop of the V-cycle's own
    residual)."""
    O = oracle.Oracle(mesh, p, alpha_deg=alpha)
    S = _solver(mesh, p, alpha, rk_stages=4, cfl_max=20.0, krylov_m=30)
    u = perturbed(O, p, 320, amp=0.005)
    _, g = O.drag(p, u, grad=True)
    lam, hist, st = S.adjoint_solve(to_dev(u), to_dev(g), drop_tol=1e-11, max_cycles=4000)
    lam = to_host(lam)
    r = (O.jacobian_sparse(p, u).T @ lam.ravel()).reshape(g.shape) + g
    e = np.linalg.norm(r) / np.linalg.norm(g)
    print(f"{name}: adjoint cycles {len(hist) - 1}, drop {hist[-1] / hist[0]:.2e}, equation residual {e:.2e}",
          flush=True)
    assert st == 0
    assert e < 1e-8


def test_adjoint_solve_2d_p4_curved():
    """2D p = 4 (100 x 100 blocks, transposed stage k_prk_stage_trc<100>) at
    the converged state of the curved O-grid 16 x 8: the adjoint V-cycle
    reaches a 1e-11 drop and lambda equals the oracle's sparse direct solve
    of (dR/du)^T lambda + dC_D/du = 0 at the same state.  (On straight-sided
    O-grids the forward cycle map is unstable at the steady state and the
    transposed one diverged likewise.)"""
    mesh = ogrid(16, 8, curved=True)
    O = oracle.Oracle(mesh, 4)
    S = _solver(mesh, 4, 0.0, rk_stages=4, cfl_max=100.0, krylov_m=30)
    ud = S.freestream(4)
    h, st = S.solve_steady(ud, drop_tol=1e-12, max_cycles=4000)
    assert st == 0, (len(h), h[-1] / h[0])
    u = to_host(ud)
    _, g = O.drag(4, u, grad=True)
    lam_o = O.adjoint(4, u, g)
    lam_g, hist, st = S.adjoint_solve(ud, to_dev(g), drop_tol=1e-11, max_cycles=8000)
    e = rel_err(to_host(lam_g), lam_o)
    print("2D p4 adjoint cycles", len(hist) - 1, "drop", hist[-1] / hist[0], "lambda error", e, flush=True)
    assert st == 0
    assert e < 1e-8


def test_steady_drag_gradient_matches_finite_differences():
    """dC_D/dtheta by torch.autograd through the adjoint, theta = (Mach, two
    wall-bump amplitudes), against central differences of converged GPU
    solves at theta +- 1e-6."""
    import paper_1807_01151_amd as P
    base = ogrid(12, 4)
    prob = P.autograd.SteadyDragProblem(base=base, centers=bump_centers(2, 2, seed=5), sigma=0.4, p_max=1,
                                        solver_kw=dict(rk_stages=4, cfl_max=100.0, krylov_m=30),
                                        drop=1e-13, adjoint_drop=1e-12)
    theta = torch.tensor([0.3, 0.0, 0.0], dtype=torch.float64, requires_grad=True)
    cd = P.autograd.SteadyDrag.apply(theta, prob)
    cd.backward()
    grad = theta.grad.numpy()
    h = 1e-6
    fd = np.zeros(3)
    for i in range(3):
        tp, tm = theta.detach().clone(), theta.detach().clone()
        tp[i] += h
        tm[i] -= h
        Sp, Sm = prob.solver(tp.tolist()), prob.solver(tm.tolist())
        cp = Sp.drag(prob.steady(Sp), sref=prob.sref)
        cm = Sm.drag(prob.steady(Sm), sref=prob.sref)
        fd[i] = (cp - cm) / (2 * h)
    print("C_D", cd.item(), "adjoint gradient", grad, "FD", fd, flush=True)
    assert np.all(np.abs(grad - fd) <= 1e-5 * np.abs(fd) + 1e-9)


@pytest.mark.timeout(900)
def test_steady_drag_gradient_3d_p3_matches_finite_differences():
    """The adjoint workload's check at 3D p = 3 (320 x 320 blocks): dC_D/dtheta
    by torch.autograd through the adjoint, theta = (Mach, one seeded
    Gaussian wall-bump amplitude), on the shell 6 x 3 x 3 x 4, against
    central differences (h = 1e-6) of converged FP64 GPU solves."""
    import paper_1807_01151_amd as P
    base = cubed_sphere_shell(3, 4)
    prob = P.autograd.SteadyDragProblem(base=base, centers=bump_centers(3, 1, seed=5), sigma=0.4, p_max=3,
                                        solver_kw=dict(rk_stages=4, cfl_max=100.0, krylov_m=30),
                                        drop=1e-12, max_cycles=10000, adjoint_drop=1e-11,
                                        adjoint_max_cycles=10000)
    theta = torch.tensor([0.3, 0.0], dtype=torch.float64, requires_grad=True)
    cd = P.autograd.SteadyDrag.apply(theta, prob)
    cd.backward()
    grad = theta.grad.numpy()
    h = 1e-6
    fd = np.zeros(2)
    for i in range(2):
        tp, tm = theta.detach().clone(), theta.detach().clone()
        tp[i] += h
        tm[i] -= h
        Sp, Sm = prob.solver(tp.tolist()), prob.solver(tm.tolist())
        cp = Sp.drag(prob.steady(Sp), sref=prob.sref)
        cm = Sm.drag(prob.steady(Sm), sref=prob.sref)
        fd[i] = (cp - cm) / (2 * h)
    print("3D p=3 C_D", cd.item(), "adjoint gradient", grad, "FD", fd, flush=True)
    assert np.all(np.abs(grad - fd) <= 1e-4 * np.abs(fd) + 1e-9)


def test_param_sensitivity_matches_separate_evaluations():
    """eg_param_sensitivity (central differences over the theta +- h handles,
    formed in the library) against the same formula assembled from the
    library's residual and drag calls, and from the oracle's: the theta
    derivative at a fixed state of C_D plus lambda . R, theta = Mach."""
    import paper_1807_01151_amd as P
    import torch
    mesh, p, mach, h = ogrid(12, 4), 2, 0.3, 1e-6
    O = oracle.Oracle(mesh, p, mach=mach)
    u = perturbed(O, p, 930)
    lam = np.random.default_rng(931).standard_normal(u.shape)
    Sp = P.Solver(mesh, p, mach=mach + h)
    Sm = P.Solver(mesh, p, mach=mach - h)
    ud, ld = to_dev(u), to_dev(lam)
    got = Sp.param_sensitivity(Sm, h, ud, ld, direction=(1.0, 0.0))
    dR = (Sp.residual(p, ud) - Sm.residual(p, ud)) / (2 * h)
    ref = (Sp.drag(ud, direction=(1.0, 0.0)) - Sm.drag(ud, direction=(1.0, 0.0))) / (2 * h) + float(torch.sum(ld * dR))
    Op, Om = oracle.Oracle(mesh, p, mach=mach + h), oracle.Oracle(mesh, p, mach=mach - h)
    orc = ((Op.drag(p, u, (1.0, 0.0)) - Om.drag(p, u, (1.0, 0.0))) / (2 * h)
           + float(np.sum(lam * (Op.residual(p, u) - Om.residual(p, u)))) / (2 * h))
    print(f"param sensitivity: library {got:.12e}, separate calls {ref:.12e}, oracle {orc:.12e}", flush=True)
    assert abs(got - ref) <= 1e-12 * max(abs(ref), 1.0)
    # central differences of O(1) sums over 2h = 2e-6: rounding of 1e-16 becomes ~1e-10
    assert abs(got - orc) <= 1e-8 * max(abs(orc), 1.0)
