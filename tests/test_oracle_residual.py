"""Pins of the oracle's DG residual (Section 3.1, eq. (euler3)): free-stream
preservation, conservation, mirror symmetry, rotation invariance and the
order of accuracy on a manufactured solution."""

import math

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell, box, Mesh, TAG_FARFIELD, TAG_WALL


def perturbed(O, p, seed, amp=0.02):
    """Free stream plus a seeded perturbation scaled with the element size."""
    rng = np.random.default_rng(seed)
    u = O.freestream(p)
    vol, *_ = O.geometry()
    return u + amp * rng.uniform(-1, 1, u.shape) * np.sqrt(vol)[:, None, None]


@pytest.mark.parametrize("mesh,p,alpha", [
    (ogrid(12, 5, inner=TAG_FARFIELD), 3, 4.0),
    (ogrid(16, 4, inner=TAG_FARFIELD), 1, -2.0),
    (ogrid(10, 3, inner=TAG_FARFIELD), 4, 1.0),
    (cubed_sphere_shell(2, 2, inner=TAG_FARFIELD), 2, 3.0),
    (box(2, 4, skew=0.2, seed=1, tag=TAG_FARFIELD), 2, 10.0),
])
def test_freestream_preservation(mesh, p, alpha):
    O = oracle.Oracle(mesh, p, mach=0.3, alpha_deg=alpha)
    u = O.freestream(p)
    r = O.residual(p, u)
    vol, *_ = O.geometry()
    # residual coefficients scale like sqrt(|E|) * flux / h; compare relative to that
    scale = np.sqrt(vol)[:, None, None] * 2.0
    assert np.max(np.abs(r) / scale) < 1e-13


@pytest.mark.parametrize("mesh,p", [(ogrid(12, 4, inner=TAG_WALL, outer=TAG_WALL), 2),
                                    (cubed_sphere_shell(2, 2, inner=TAG_WALL, outer=TAG_WALL), 1)])
def test_conservation_closed_walls(mesh, p):
    """With slip walls only, interior fluxes cancel and the wall mass and energy
    fluxes vanish, so sum_E int_E R_v = sum_E sqrt|E| R_{E,v,0} = 0 for v = mass,
    energy (the cell mean of R is R_0 psi_0 with psi_0 = 1/sqrt|E|)."""
    O = oracle.Oracle(mesh, p)
    u = perturbed(O, p, 1)
    r = O.residual(p, u)
    vol, *_ = O.geometry()
    for v in (0, O.V - 1):
        tot = np.sum(np.sqrt(vol) * r[:, v, 0])
        mag = np.sum(np.abs(np.sqrt(vol) * r[:, v, 0]))
        assert abs(tot) < 1e-13 * mag


def test_mirror_symmetry_alpha0():
    """At alpha = 0 on the O-grid (symmetric about y = 0), mirroring the state
    mirrors the residual."""
    nt, nr, p = 16, 4, 2
    m = ogrid(nt, nr)
    O = oracle.Oracle(m, p, alpha_deg=0.0)
    u = perturbed(O, p, 2)
    modes = oracle.modes(2, p)
    # mirror y -> -y maps element (i, j) to (nt-1-i, j) and flips eta: mode (a, b) gets (-1)^b,
    # the y-momentum changes sign
    perm = np.array([j * nt + (nt - 1 - i) for j in range(nr) for i in range(nt)])
    sgn_mode = (-1.0) ** modes[:, 1]
    sgn_var = np.array([1, 1, -1, 1.0])

    def mirror(x):
        return x[perm] * sgn_var[None, :, None] * sgn_mode[None, None, :]

    r1 = O.residual(p, mirror(u))
    r2 = mirror(O.residual(p, u))
    assert np.max(np.abs(r1 - r2)) < 1e-12 * np.max(np.abs(r2))


def test_rotation_invariance():
    """Rotating mesh, free stream and momentum together rotates the residual's
    momentum components and leaves the rest unchanged."""
    p = 2
    m = ogrid(12, 3)
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    m2 = Mesh(2, m.xyz @ Rm.T, m.elem_vert, m.bface_tag)
    O1 = oracle.Oracle(m, p, alpha_deg=5.0)
    O2 = oracle.Oracle(m2, p, alpha_deg=5.0 + math.degrees(th))
    u = perturbed(O1, p, 4)
    u2 = u.copy()
    u2[:, 1:3, :] = np.einsum("ab,ebi->eai", Rm, u[:, 1:3, :])
    r1 = O1.residual(p, u)
    r2 = O2.residual(p, u2)
    r1[:, 1:3, :] = np.einsum("ab,ebi->eai", Rm, r1[:, 1:3, :])
    assert np.max(np.abs(r1 - r2)) < 1e-11 * np.max(np.abs(r1))


@pytest.mark.slow
@pytest.mark.parametrize("p", [1, 3])
def test_mms_order_of_accuracy(p):
    """Steady manufactured solution (exact-state ghost on the box boundary):
    the L2 error of the converged DG solution falls at rate >= p + 0.5 (the
    expected rate is p + 1; p = 2 is still pre-asymptotic on boxes this small,
    2.2 / 2.5 / 2.7 from 2 to 16 cells per side)."""
    errs = []
    hs = []
    for n in (4, 8):
        m = box(2, n, skew=0.0, tag=3)
        O = oracle.Oracle(m, p)
        f = O.mms_forcing(p)
        u = O.mms_project(p)
        u, hist, st = O.solve(u, s=4, m=30, cfl_max=100.0, drop=1e-8, max_cycles=3000, f=f)
        assert st == 0, (st, hist[-1] / hist[0])
        errs.append(O.mms_error(p, u))
        hs.append(1.0 / n)
    rate = math.log(errs[0] / errs[1]) / math.log(hs[0] / hs[1])
    assert rate >= p + 0.5, (errs, rate)
