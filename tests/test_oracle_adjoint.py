"""Pin of the oracle adjoint (sparse direct solve of (dR/du)^T lambda + g = 0)
end to end: the adjoint drag sensitivity to the Mach number and to a wall
bump amplitude equals central differences of converged steady solves."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, wall_bumps, bump_centers

P = 1
SOLVE = dict(s=4, m=30, cfl_max=100.0, max_cycles=6000)


def _steady(O, u0, drop):
    r0 = O.rnorm(P, O.residual(P, u0))
    u, h, st = O.solve(u0, drop=drop, **SOLVE)
    assert st == 0
    return u


def _converge(O, u0, abs_tol):
    """Steady state with ||R|| <= abs_tol (the solve's drop is relative to its
    own first norm)."""
    r0 = O.rnorm(P, O.residual(P, u0))
    return _steady(O, u0, abs_tol / r0) if r0 > abs_tol else u0


@pytest.mark.slow
def test_adjoint_gradient_matches_finite_differences():
    base = ogrid(12, 4)
    cen = bump_centers(2, 1, seed=3)
    ma, h = 0.3, 1e-5

    def mesh_of(a):
        return wall_bumps(base, [a], cen, 0.4)

    O = oracle.Oracle(mesh_of(0.0), P, mach=ma)
    u = _converge(O, O.freestream(P), 1e-16)
    c, g = O.drag(P, u, grad=True)
    lam = O.adjoint(P, u, g)
    # Mach: dR/dMa and dC/dMa at fixed u by central differences of the
    # residual and the functional
    Op, Om = oracle.Oracle(mesh_of(0.0), P, mach=ma + h), oracle.Oracle(mesh_of(0.0), P, mach=ma - h)
    dR = (Op.residual(P, u) - Om.residual(P, u)) / (2 * h)
    dC = (Op.drag(P, u) - Om.drag(P, u)) / (2 * h)
    adj_ma = dC + float(np.sum(lam * dR))
    fd_ma = (Op.drag(P, _converge(Op, u, 1e-16)) - Om.drag(P, _converge(Om, u, 1e-16))) / (2 * h)
    print("dC/dMa adjoint", adj_ma, "FD", fd_ma)
    assert abs(adj_ma - fd_ma) < 1e-5 * abs(fd_ma)
    # wall bump amplitude
    Bp, Bm = oracle.Oracle(mesh_of(h), P, mach=ma), oracle.Oracle(mesh_of(-h), P, mach=ma)
    dR = (Bp.residual(P, u) - Bm.residual(P, u)) / (2 * h)
    dC = (Bp.drag(P, u) - Bm.drag(P, u)) / (2 * h)
    adj_a = dC + float(np.sum(lam * dR))
    fd_a = (Bp.drag(P, _converge(Bp, u, 1e-16)) - Bm.drag(P, _converge(Bm, u, 1e-16))) / (2 * h)
    print("dC/da adjoint", adj_a, "FD", fd_a)
    assert abs(adj_a - fd_a) < 1e-5 * abs(fd_a)
