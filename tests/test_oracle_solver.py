"""Pins of the oracle's Jacobian blocks (Section 3.3), time step (Section 4),
PRK smoother (Section 2.3), EXP1 step (Sections 2.1-2.2) and V-cycle
(Section 2.4) against brute force: complex-step Jacobians of the whole
residual, dense matrix functions from scipy and an independent Newton solve."""

import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from eg_inputs import ogrid, cubed_sphere_shell


def perturbed(O, p, seed, amp=0.02):
    rng = np.random.default_rng(seed)
    u = O.freestream(p)
    vol, *_ = O.geometry()
    deg = oracle.modes(O.dim, p)[:, : O.dim].max(axis=1)
    return u + amp * rng.uniform(-1, 1, u.shape) * np.sqrt(vol)[:, None, None] * (0.25 ** deg)[None, None, :]


def brute_jacobian(O, p, u):
    """Dense dR/du by complex step of the full residual, one column at a time."""
    K = u.size
    J = np.zeros((K, K))
    for c in range(K):
        du = np.zeros(K, dtype=complex)
        du[c] = 1e-30j
        J[:, c] = (O.residual_complex(p, u + du.reshape(u.shape)).imag / 1e-30).ravel()
    return J


@pytest.mark.parametrize("mesh,p", [(ogrid(6, 3), 0), (ogrid(6, 3), 2), (ogrid(4, 2), 4),
                                    (cubed_sphere_shell(1, 2), 1)])
def test_jacobian_blocks_match_full_complex_step(mesh, p):
    O = oracle.Oracle(mesh, p, alpha_deg=3.0)
    u = perturbed(O, p, 21)
    D, Off = O.jacobian_blocks(p, u, offdiag=True)
    J = brute_jacobian(O, p, u)
    n = O.V * O.N(p)
    nb = O.neighbours()
    scale = np.max(np.abs(J))
    Jb = np.zeros_like(J)
    for e in range(O.ne):
        Jb[e * n:(e + 1) * n, e * n:(e + 1) * n] += D[e]
        for lf in range(2 * O.dim):
            if nb[e, lf] >= 0:
                f = nb[e, lf]
                Jb[e * n:(e + 1) * n, f * n:(f + 1) * n] += Off[e, lf]
    assert np.max(np.abs(Jb - J)) < 1e-13 * scale


def test_timestep_closed_form():
    """dtau = CFL h / ((2p+1)(|v|+c)) with h = 2d|E|/|dE| at the free stream
    (c = 1, |v| = Ma); |E| and |dE| from the polygon."""
    m = ogrid(12, 3)
    p, cfl, ma = 2, 7.0, 0.3
    O = oracle.Oracle(m, p, mach=ma)
    dt = O.timestep(p, cfl, O.freestream(p))
    for e in range(m.n_elem):
        v = m.xyz[m.elem_vert[e]][[0, 1, 3, 2]]
        x, y = v[:, 0], v[:, 1]
        area = 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)
        perim = sum(np.linalg.norm(v[k] - v[(k + 1) % 4]) for k in range(4))
        ref = cfl * (4 * area / perim) / ((2 * p + 1) * (ma + 1.0))
        assert abs(dt[e] - ref) < 1e-13 * ref


def test_prk_step_matches_dense_statement():
    """One s-stage PRK step against a numpy statement of eq. (prk_scalar) that
    uses brute-force Jacobian blocks and numpy's dense solver."""
    p, s, cfl = 1, 3, 5.0
    O = oracle.Oracle(ogrid(6, 3), p, alpha_deg=2.0)
    u = perturbed(O, p, 31)
    f = 1e-3 * np.random.default_rng(32).standard_normal(u.shape)
    out = O.prk(p, s, cfl, u, f)
    n = O.V * O.N(p)
    J = brute_jacobian(O, p, u)
    dt = O.timestep(p, cfl, u)
    Pb = [np.eye(n) / dt[e] - J[e * n:(e + 1) * n, e * n:(e + 1) * n] for e in range(O.ne)]
    uk = u.copy()
    for k in range(1, s + 1):
        R = O.residual(p, uk) + f
        x = np.stack([np.linalg.solve(Pb[e], R[e].ravel()) for e in range(O.ne)]).reshape(u.shape)
        uk = u + x / (s - k + 1)
    assert np.max(np.abs(out - uk)) < 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("mesh", [ogrid(8, 4), cubed_sphere_shell(1, 2)])
def test_exp1_full_krylov_matches_dense_phi1(mesh):
    """With m >= K_0 the EXP1 step equals v0 + phi_1(T J) T (R_0 + f), T =
    diag(dt_E), evaluated densely (brute-force J, scipy expm)."""
    pmax, cfl = 2, 20.0
    O = oracle.Oracle(mesh, pmax, alpha_deg=1.0)
    u0 = perturbed(O, 0, 41)
    f0 = 1e-3 * np.random.default_rng(42).standard_normal(u0.shape)
    K = u0.size
    out, mu, beta = O.exp1(K, cfl, u0, f0)
    dt = (pmax + 1) * O.timestep(pmax, cfl, u0)
    T = np.repeat(dt, O.V)
    J = brute_jacobian(O, 0, u0)
    A = T[:, None] * J
    b = T * (O.residual(0, u0) + f0).ravel()
    ref = u0.ravel() + np.linalg.solve(A, (sla.expm(A) - np.eye(K)) @ b)
    assert np.max(np.abs(out.ravel() - ref)) < 1e-10 * np.max(np.abs(ref - u0.ravel()))
    # m = 30 is already close, and the error falls with m
    e10 = np.max(np.abs(O.exp1(10, cfl, u0, f0)[0].ravel() - ref))
    e30 = np.max(np.abs(O.exp1(30, cfl, u0, f0)[0].ravel() - ref))
    assert e30 < e10


def test_exp1_large_step_is_newton():
    """As dt grows the EXP1 step tends to the Newton step -J^{-1}(R + f)
    (the scheme 'behaves like a fully implicit method')."""
    pmax = 1
    O = oracle.Oracle(ogrid(8, 4), pmax)
    u0 = perturbed(O, 0, 51, amp=0.01)
    K = u0.size
    J = brute_jacobian(O, 0, u0)
    newton = u0.ravel() - np.linalg.solve(J, O.residual(0, u0).ravel())
    assert np.max(np.linalg.eigvals(J).real) < 0  # stable first-order Jacobian
    out, mu, beta = O.exp1(K, 1e9, u0)
    assert np.max(np.abs(out.ravel() - newton)) < 1e-6 * np.max(np.abs(newton - u0.ravel()))


def _newton(O, p, u, iters=8):
    n = O.V * O.N(p)
    nb = O.neighbours()
    for _ in range(iters):
        r = O.residual(p, u)
        if np.max(np.abs(r)) < 1e-14:
            break
        D, Off = O.jacobian_blocks(p, u, offdiag=True)
        rows, cols, vals = [], [], []
        I, Jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        for e in range(O.ne):
            rows.append(e * n + I.ravel()); cols.append(e * n + Jj.ravel()); vals.append(D[e].ravel())
            for lf in range(2 * O.dim):
                if nb[e, lf] >= 0:
                    rows.append(e * n + I.ravel()); cols.append(nb[e, lf] * n + Jj.ravel())
                    vals.append(Off[e, lf].ravel())
        Jm = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(u.size, u.size))
        u = u - spla.spsolve(Jm, r.ravel()).reshape(u.shape)
    return u


@pytest.mark.slow
def test_vcycle_converges_to_newton_steady_state_and_keeps_it():
    """The eMG fixed point is the DG steady state R(u) = 0: the V-cycle solve
    reaches the state an independent Newton solve finds, and a V-cycle started
    at that state leaves it in place."""
    p = 2
    O = oracle.Oracle(ogrid(12, 4), p, alpha_deg=2.0)
    u, hist, st = O.solve(O.freestream(p), s=4, m=30, cfl_max=100.0, drop=1e-9, max_cycles=3000)
    assert st == 0
    un = _newton(O, p, u.copy())
    assert np.max(np.abs(O.residual(p, un))) < 1e-13
    assert np.max(np.abs(u - un)) < 1e-6 * np.max(np.abs(un))
    u2, rn, cfl = O.vcycle(un, 50, s=4, m=30, cfl_max=100.0)
    assert np.max(np.abs(u2 - un)) < 1e-12 * np.max(np.abs(un))
    # the fixed point does not depend on the smoother's settings
    u3, h3, st3 = O.solve(O.freestream(p), s=3, m=20, cfl_max=10.0, drop=1e-9, max_cycles=4000)
    assert st3 == 0
    assert np.max(np.abs(u3 - un)) < 1e-6 * np.max(np.abs(un))


def test_cfl_ramp():
    L = oracle.lib()
    # literal: r_n^-1 dominates; relative: starts at 1 and grows as r falls
    assert L.orc_cfl_ramp(100.0, 1e-3, 1.0, 1, 3) == 100.0
    assert L.orc_cfl_ramp(100.0, 1e-3, 1e-3, 1, 3) == 1.0
    assert L.orc_cfl_ramp(100.0, 1e-3, 1e-3, 8, 3) == 2.0
    assert math.isclose(L.orc_cfl_ramp(100.0, 1e-5, 1e-3, 2, 3), 100.0)
    assert math.isclose(L.orc_cfl_ramp(1000.0, 1e-5, 1e-3, 2, 3), 100.0)
