"""Pins of the oracle's Roe flux (the paper's Riemann solver, Section 3.1
after eq. (euler3) and Section 3.3, from Roe's 1981 linearisation), with the
reading of the entropy fix (Harten's on the acoustic waves, delta = 0.1 c).

* Consistency: F~(U, U; n) = F(U) . n, the textbook Euler flux written here.
* Conservation form: F~(UL, UR; n) = -F~(UR, UL; -n).
* Roe's property A(UL, UR) (UR - UL) = F(UR) - F(UL): when every wave speed
  has one sign (supersonic normal flow, entropy fix inactive) the flux is
  exactly the upwind physical flux; any slip in the averages, strengths or
  eigenvectors breaks it.
* Exact resolution of a stationary contact (equal pressure, zero velocity,
  different densities): no mass flux.
* Continuity through the entropy-fix zone (no jump where |lambda| = delta).
* Complex-step Jacobians against central finite differences of the flux.
* Residual level with the Roe flux: free-stream preservation, conservation
  with closed slip walls, manufactured-solution order p + 1.
"""

import math

import numpy as np
import pytest

import oracle
from eg_inputs import box, cubed_sphere_shell, ogrid, TAG_EXACT, TAG_FARFIELD, TAG_WALL

G = 1.4


def cons(rho, v, p):
    v = np.asarray(v, dtype=np.float64)
    return np.concatenate([[rho], rho * v, [p / (G - 1.0) + 0.5 * rho * float(v @ v)]])


def euler_flux(U, n):
    """F(U) . n of the Euler equations from the definition (mass, momentum
    and energy flux through a surface of normal n)."""
    d = len(n)
    rho, m, E = U[0], U[1:1 + d], U[d + 1]
    v = m / rho
    p = (G - 1.0) * (E - 0.5 * rho * float(v @ v))
    vn = float(v @ n)
    return np.concatenate([[rho * vn], rho * v * vn + p * np.asarray(n), [(E + p) * vn]])


def unit(rng, d):
    n = rng.standard_normal(d)
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("d", [2, 3])
def test_consistency_and_conservation_form(d):
    rng = np.random.default_rng(40 + d)
    for _ in range(20):
        n = unit(rng, d)
        U = cons(rng.uniform(0.5, 2.0), rng.uniform(-0.8, 0.8, d), rng.uniform(0.3, 2.0))
        F = oracle.roe(d, G, U, U, n)
        assert np.max(np.abs(F - euler_flux(U, n))) <= 1e-14 * np.max(np.abs(F))
        UR = cons(rng.uniform(0.5, 2.0), rng.uniform(-0.8, 0.8, d), rng.uniform(0.3, 2.0))
        F1 = oracle.roe(d, G, U, UR, n)
        F2 = oracle.roe(d, G, UR, U, -n)
        assert np.max(np.abs(F1 + F2)) <= 1e-14 * np.max(np.abs(F1))


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("direction", [+1, -1])
def test_supersonic_states_are_upwinded_exactly(d, direction):
    """Normal Mach numbers 2..3 on both sides towards +n (or -n): every Roe
    wave speed has the same sign, so F~ = F(UL) . n (or F(UR) . n)."""
    rng = np.random.default_rng(50 + d + direction)
    for _ in range(20):
        n = unit(rng, d)
        states = []
        for _s in range(2):
            rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.3, 2.0)
            c = math.sqrt(G * p / rho)
            t = rng.standard_normal(d)
            t -= float(t @ n) * n
            v = direction * rng.uniform(2.0, 3.0) * c * n + 0.3 * c * t
            states.append(cons(rho, v, p))
        UL, UR = states
        F = oracle.roe(d, G, UL, UR, n)
        up = euler_flux(UL if direction > 0 else UR, n)
        assert np.max(np.abs(F - up)) <= 1e-13 * np.max(np.abs(up))


@pytest.mark.parametrize("d", [2, 3])
def test_stationary_contact_is_exact(d):
    rng = np.random.default_rng(60 + d)
    for _ in range(10):
        n = unit(rng, d)
        p = rng.uniform(0.3, 2.0)
        UL = cons(rng.uniform(0.5, 2.0), np.zeros(d), p)
        UR = cons(rng.uniform(0.5, 2.0), np.zeros(d), p)
        F = oracle.roe(d, G, UL, UR, n)
        want = np.concatenate([[0.0], p * n, [0.0]])
        assert np.max(np.abs(F - want)) <= 1e-14 * p


def test_continuous_through_the_entropy_fix():
    """A sweep of the normal velocity through the sonic point of the left
    acoustic wave: the flux changes by O(step) everywhere (Lipschitz), also
    where |v_n - c| crosses the fix width."""
    d, n = 2, np.array([1.0, 0.0])
    steps = np.linspace(0.85, 1.15, 3001)
    Fs = []
    for s in steps:
        UL = cons(1.0, [s, 0.1], 1.0 / G)        # c = 1 on the left
        UR = cons(0.9, [s * 1.05, 0.1], 0.95 / G)
        Fs.append(oracle.roe(d, G, UL, UR, n))
    Fs = np.array(Fs)
    h = steps[1] - steps[0]
    slopes = np.max(np.abs(np.diff(Fs, axis=0)), axis=1) / h
    assert np.max(slopes) <= 20.0 * np.median(slopes) + 10.0


@pytest.mark.parametrize("d", [2, 3])
def test_complex_step_jacobian_matches_finite_differences(d):
    rng = np.random.default_rng(70 + d)
    for _ in range(5):
        n = unit(rng, d)
        UL = cons(rng.uniform(0.7, 1.5), rng.uniform(-0.5, 0.5, d), rng.uniform(0.5, 1.5))
        UR = cons(rng.uniform(0.7, 1.5), rng.uniform(-0.5, 0.5, d), rng.uniform(0.5, 1.5))
        JL, JR = oracle.roe_jac(d, G, UL, UR, n)
        for J, side in ((JL, 0), (JR, 1)):
            Jfd = np.zeros_like(J)
            for w in range(d + 2):
                h = 1e-6 * max(1.0, abs((UL, UR)[side][w]))
                a, b = [UL.copy(), UR.copy()], [UL.copy(), UR.copy()]
                a[side][w] += h
                b[side][w] -= h
                Jfd[:, w] = (oracle.roe(d, G, a[0], a[1], n) - oracle.roe(d, G, b[0], b[1], n)) / (2 * h)
            assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J)), side


@pytest.mark.parametrize("mesh,p,alpha", [(ogrid(12, 5, inner=TAG_FARFIELD), 3, 4.0),
                                          (cubed_sphere_shell(2, 2, inner=TAG_FARFIELD), 2, 3.0)])
def test_roe_freestream_preservation(mesh, p, alpha):
    O = oracle.Oracle(mesh, p, alpha_deg=alpha, flux="roe")
    r = O.residual(p, O.freestream(p))
    vol, *_ = O.geometry()
    assert np.max(np.abs(r) / (2.0 * np.sqrt(vol)[:, None, None])) < 1e-13


def test_roe_conservation_closed_walls():
    mesh = ogrid(12, 4, inner=TAG_WALL, outer=TAG_WALL)
    p = 2
    O = oracle.Oracle(mesh, p, flux="roe")
    rng = np.random.default_rng(3)
    vol, *_ = O.geometry()
    u = O.freestream(p) + 0.02 * rng.uniform(-1, 1, (mesh.n_elem, 4, 9)) * np.sqrt(vol)[:, None, None]
    r = O.residual(p, u)
    for v in (0, 3):
        tot = np.sum(np.sqrt(vol) * r[:, v, 0])
        assert abs(tot) < 1e-13 * np.sum(np.abs(np.sqrt(vol) * r[:, v, 0]))


@pytest.mark.slow
def test_roe_mms_order():
    """Steady manufactured solution with the Roe flux on 2D boxes: the L2
    error of the converged p = 1 solution falls at rate >= 1.5."""
    p, errs = 1, []
    for n in (4, 8):
        O = oracle.Oracle(box(2, n, tag=TAG_EXACT), p, flux="roe")
        u, hist, st = O.solve(O.mms_project(p), s=4, m=30, cfl_max=100.0, drop=1e-8, max_cycles=3000,
                              f=O.mms_forcing(p))
        assert st == 0, (st, hist[-1] / hist[0])
        errs.append(O.mms_error(p, u))
    rate = math.log2(errs[0] / errs[1])
    assert rate >= p + 0.5, (errs, rate)
