"""Pins of the oracle's flux, ghost states and flux Jacobian (Section 3.3 and
Appendix A) against textbook Euler relations written out here."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid

G = 1.4


def euler_flux_n(U, n):
    """Textbook Euler flux F(U) . n (d = len(n))."""
    d = len(n)
    rho, m, E = U[0], U[1:1 + d], U[1 + d]
    v = m / rho
    p = (G - 1) * (E - 0.5 * rho * v @ v)
    vn = v @ n
    return np.concatenate([[rho * vn], m * vn + p * n, [(E + p) * vn]])


def random_state(rng, d):
    rho = rng.uniform(0.5, 2.0)
    v = rng.uniform(-0.6, 0.6, d)
    p = rng.uniform(0.3, 1.5)
    return np.concatenate([[rho], rho * v, [p / (G - 1) + 0.5 * rho * v @ v]])


@pytest.mark.parametrize("d", [2, 3])
def test_rusanov_consistency_and_antisymmetry(d):
    rng = np.random.default_rng(11)
    for _ in range(50):
        UL, UR = random_state(rng, d), random_state(rng, d)
        n = rng.standard_normal(d)
        n /= np.linalg.norm(n)
        F = oracle.rusanov(d, G, UL, UL, n)
        assert np.allclose(F, euler_flux_n(UL, n), rtol=1e-14, atol=1e-14)
        F1 = oracle.rusanov(d, G, UL, UR, n)
        F2 = oracle.rusanov(d, G, UR, UL, -n)
        assert np.array_equal(F1, -F2)  # bitwise: built without contraction


@pytest.mark.parametrize("d", [2, 3])
def test_rusanov_upwind_limit(d):
    """With equal wave-speed bound lambda the flux is the central average minus
    lambda/2 times the jump; check against that value with lambda computed here."""
    rng = np.random.default_rng(12)
    for _ in range(20):
        UL, UR = random_state(rng, d), random_state(rng, d)
        n = rng.standard_normal(d)
        n /= np.linalg.norm(n)

        def lam(U):
            v = U[1:1 + d] / U[0]
            p = (G - 1) * (U[-1] - 0.5 * U[0] * v @ v)
            return abs(v @ n) + np.sqrt(G * p / U[0])

        ref = 0.5 * (euler_flux_n(UL, n) + euler_flux_n(UR, n)) - 0.5 * max(lam(UL), lam(UR)) * (UR - UL)
        assert np.allclose(oracle.rusanov(d, G, UL, UR, n), ref, rtol=1e-13, atol=1e-14)


def test_wall_ghost_zero_mass_energy_flux():
    O = oracle.Oracle(ogrid(8, 2), 1)
    rng = np.random.default_rng(3)
    for _ in range(20):
        U = random_state(rng, 2)
        n = rng.standard_normal(2)
        n /= np.linalg.norm(n)
        Ug = O.ghost(1, U, n, np.zeros(2))
        F = oracle.rusanov(2, G, U, Ug, n)
        assert abs(F[0]) < 1e-15 and abs(F[3]) < 1e-14
        p = (G - 1) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0])
        # momentum flux is normal; with the mirror ghost both sides share |v.n|
        # and c, so its size is p + (m.n)(v.n + |v.n| + c)
        assert abs(F[1] * n[1] - F[2] * n[0]) < 1e-13
        mn = U[1:3] @ n
        vn = mn / U[0]
        c = np.sqrt(G * p / U[0])
        assert abs(F[1:3] @ n - (p + mn * (vn + abs(vn) + c))) < 1e-13


def test_farfield_ghost_freestream_fixed_point():
    for alpha in (0.0, 3.0, -5.0):
        O = oracle.Oracle(ogrid(8, 2), 1, mach=0.3, alpha_deg=alpha)
        Uinf = O.freestream_state()
        for th in np.linspace(0, 2 * np.pi, 13):
            n = np.array([np.cos(th), np.sin(th)])
            Ug = O.ghost(2, Uinf, n, np.zeros(2))
            assert np.allclose(Ug, Uinf, rtol=1e-14, atol=1e-14)


def test_farfield_ghost_riemann_invariants():
    """The ghost state carries the outgoing invariant from inside and the
    incoming one from the free stream (textbook characteristic BC)."""
    O = oracle.Oracle(ogrid(8, 2), 1, mach=0.3, alpha_deg=2.0)
    Uinf = O.freestream_state()
    rng = np.random.default_rng(5)

    def prim(U):
        v = U[1:3] / U[0]
        p = (G - 1) * (U[3] - 0.5 * U[0] * v @ v)
        return U[0], v, p, np.sqrt(G * p / U[0])

    for _ in range(20):
        U = Uinf + 0.05 * rng.standard_normal(4) * np.array([1, 0.3, 0.3, 1])
        n = rng.standard_normal(2)
        n /= np.linalg.norm(n)
        Ug = O.ghost(2, U, n, np.zeros(2))
        r, v, p, c = prim(U)
        rb, vb, pb, cb = prim(Ug)
        ri, vi, pi, ci = prim(Uinf)
        assert abs((vb @ n + 2 * cb / (G - 1)) - (v @ n + 2 * c / (G - 1))) < 1e-13
        assert abs((vb @ n - 2 * cb / (G - 1)) - (vi @ n - 2 * ci / (G - 1))) < 1e-13
        src = (r, v, p) if vb @ n > 0 else (ri, vi, pi)
        t = np.array([-n[1], n[0]])
        assert abs(vb @ t - src[1] @ t) < 1e-13
        assert abs(pb / rb ** G - src[2] / src[0] ** G) < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_flux_jacobian_matches_finite_differences(d):
    """Appendix A matrix (with a_1 read as the total enthalpy) against central
    differences of the textbook flux."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        U = random_state(rng, d)
        g = rng.standard_normal(d)
        K = oracle.flux_jac(d, G, U, g)
        h = 1e-6
        Kfd = np.zeros_like(K)
        for w in range(d + 2):
            e = np.zeros(d + 2)
            e[w] = h
            Kfd[:, w] = (euler_flux_n(U + e, g) - euler_flux_n(U - e, g)) / (2 * h)
        assert np.max(np.abs(K - Kfd)) < 1e-8 * max(1.0, np.abs(K).max())
