"""Pins of the oracle's quadratic curved elements (biquadratic nine-node quads
and triquadratic 27-node hexes; the cylinder grid of Section 5.1 and the
sphere grid of Section 5.2 are curved): the straight special case,
closed-form areas and volumes, the h^4 geometric error of curved circles
and spheres against h^2 of straight facets, free-stream preservation,
local-frame invariance, mirror symmetry and the consistency rate of the
residual on curved annuli and shells."""

import math

import numpy as np
import pytest

import oracle
from eg_inputs import (ogrid, box, cubed_sphere_shell, mapped, straight_nodes, reorient, wall_bumps, Mesh,
                       node_of_vertex, TAG_FARFIELD, TAG_EXACT)
from tests.test_oracle_norm_ties_orientation import truncation
from tests.test_oracle_residual import perturbed


def _as_nine_node(m):
    return Mesh(m.dim, m.xyz, m.elem_vert, m.bface_tag, m.name + "+9", straight_nodes(m))


@pytest.mark.parametrize("p", [1, 3])
def test_straight_nodes_reduce_to_bilinear(p):
    """Nine nodes at the bilinear positions describe the same element map, so
    geometry, residual and element blocks equal those of the multilinear
    vertex map (a separate code path of the oracle) to rounding."""
    m = reorient(wall_bumps(ogrid(12, 4), [0.05], [[1.0, 0.3]], 0.4), 5)
    O1, O2 = oracle.Oracle(m, p, alpha_deg=3.0), oracle.Oracle(_as_nine_node(m), p, alpha_deg=3.0)
    g1, g2 = O1.geometry(), O2.geometry()
    for a, b in zip(g1[:3], g2[:3]):
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))
    u = perturbed(O1, p, 3)
    r1, r2 = O1.residual(p, u), O2.residual(p, u)
    assert np.max(np.abs(r1 - r2)) <= 1e-13 * np.max(np.abs(r1))
    b1, b2 = O1.jacobian_blocks(p, u), O2.jacobian_blocks(p, u)
    assert np.max(np.abs(b1 - b2)) <= 1e-13 * np.max(np.abs(b1))


# x = s + a t^2 + c s t^2, y = t + b s^2 + e s^2 t: biquadratic in (s, t), so
# the nine-node interpolant of every element of a uniform box reproduces it
_A, _B, _C, _E = 0.1, 0.15, 0.2, 0.1


def _biquad(x):
    s, t = x[:, 0], x[:, 1]
    return np.stack([s + _A * t * t + _C * s * t * t, t + _B * s * s + _E * s * s * t], axis=1)


def _biquad_area(s0, s1, t0, t1):
    """Integral of det = 1 + e s^2 + c t^2 - 3 c e s^2 t^2 - 4 a b s t
    - 4 a e s t^2 - 4 b c s^2 t over [s0, s1] x [t0, t1]."""
    S = [(s1 ** (k + 1) - s0 ** (k + 1)) / (k + 1) for k in range(3)]
    T = [(t1 ** (k + 1) - t0 ** (k + 1)) / (k + 1) for k in range(3)]
    return (S[0] * T[0] + _E * S[2] * T[0] + _C * S[0] * T[2] - 3 * _C * _E * S[2] * T[2]
            - 4 * _A * _B * S[1] * T[1] - 4 * _A * _E * S[1] * T[2] - 4 * _B * _C * S[2] * T[1])


@pytest.mark.parametrize("p", [0, 2])
def test_exact_area_of_biquadratic_map(p):
    """Element areas of a box under a global biquadratic map equal the closed
    form (det is a polynomial the (p+2)-point rule integrates exactly);
    the straight-sided version of the same mesh misses them at O(h^2)."""
    n = 5
    base = box(2, n, tag=TAG_FARFIELD)
    m = mapped(base, _biquad)
    vol, *_ = oracle.Oracle(m, p).geometry()
    want = np.empty(m.n_elem)
    for e in range(m.n_elem):
        lo = base.xyz[base.elem_vert[e, 0]]
        hi = base.xyz[base.elem_vert[e, 3]]
        want[e] = _biquad_area(lo[0], hi[0], lo[1], hi[1])
    assert np.max(np.abs(vol - want)) <= 1e-14
    straight = Mesh(2, m.xyz, m.elem_vert, m.bface_tag)
    vol_s, *_ = oracle.Oracle(straight, p).geometry()
    assert np.max(np.abs(vol_s - want)) > 1e-5


def test_annulus_area_rate():
    """Total area of an O-grid annulus against pi (r_out^2 - r_in^2): the
    curved mesh (mid-arc nodes on the circles) converges at rate 4 in the
    number of cells per circle, the straight one at rate 2 (chords)."""
    exact = math.pi * (2.0 ** 2 - 0.5 ** 2)
    for curved, lo, hi in ((True, 3.9, 4.1), (False, 1.9, 2.1)):
        err = []
        for nt in (16, 32):
            m = ogrid(nt, 3, r_in=0.5, r_out=2.0, stretch=1.01, curved=curved)
            vol, *_ = oracle.Oracle(m, 1).geometry()
            err.append(abs(vol.sum() - exact))
        rate = math.log2(err[0] / err[1])
        assert lo <= rate <= hi, (curved, err, rate)


@pytest.mark.parametrize("mesh,p,alpha", [
    (ogrid(12, 5, inner=TAG_FARFIELD, curved=True), 3, 4.0),
    (reorient(ogrid(10, 3, inner=TAG_FARFIELD, curved=True), 2), 4, 1.0),
    (mapped(box(2, 4, skew=0.2, seed=1, tag=TAG_FARFIELD), _biquad), 2, 10.0),
])
def test_freestream_preservation_curved(mesh, p, alpha):
    """A uniform state has zero residual on curved meshes too: the discrete
    metric terms of the biquadratic map satisfy the metric identities and
    the rule integrates them exactly."""
    O = oracle.Oracle(mesh, p, mach=0.3, alpha_deg=alpha)
    r = O.residual(p, O.freestream(p))
    vol, *_ = O.geometry()
    assert np.max(np.abs(r) / (2.0 * np.sqrt(vol)[:, None, None])) < 1e-13


@pytest.mark.parametrize("p", [1, 2])
def test_residual_invariant_under_local_frames_curved(p):
    """Random rotations of each curved element's reference frame (the nine
    nodes relabelled with the vertices) leave the per-element residual norm of
    the same function unchanged."""
    mesh = ogrid(12, 4, r_in=0.5, r_out=1.5, stretch=1.05, inner=TAG_EXACT, outer=TAG_EXACT, curved=True)
    t1, s1 = truncation(oracle.Oracle(mesh, p), p)
    t2, s2 = truncation(oracle.Oracle(reorient(mesh, 7), p), p)
    assert np.max(np.abs(t1 - t2)) <= 1e-12 * np.max(s1)
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * np.max(s1)


def test_mirror_symmetry_curved_alpha0():
    """At alpha = 0 the curved O-grid is symmetric about y = 0, so mirroring
    the state mirrors the residual (element (i, j) <-> (nt-1-i, j), eta
    flipped: mode (a, b) takes (-1)^b, y-momentum changes sign)."""
    nt, nr, p = 16, 4, 2
    O = oracle.Oracle(ogrid(nt, nr, curved=True), p, alpha_deg=0.0)
    u = perturbed(O, p, 2)
    modes = oracle.modes(2, p)
    perm = np.array([j * nt + (nt - 1 - i) for j in range(nr) for i in range(nt)])
    sgn = np.array([1, 1, -1, 1.0])[None, :, None] * ((-1.0) ** modes[:, 1])[None, None, :]
    r1 = O.residual(p, u[perm] * sgn)
    r2 = O.residual(p, u)[perm] * sgn
    assert np.max(np.abs(r1 - r2)) < 1e-12 * np.max(np.abs(r2))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_truncation_rate_curved_annulus(p):
    """Consistency of the residual on curved elements: with exact-state
    ghosts on both circles, ||R(Pi u) + f||_E / sqrt|E| of the projected
    manufactured state falls like h^p (rms rate >= p - 0.3 from 16 to 32
    cells per circle, radial cells doubled too; 0.85, 1.86, 2.85 measured,
    from 8 cells the rates are still pre-asymptotic, as for straight
    elements)."""
    rms = []
    for nt, nr in ((16, 6), (32, 12)):
        m = ogrid(nt, nr, r_in=0.5, r_out=1.5, stretch=1.0001, inner=TAG_EXACT, outer=TAG_EXACT, curved=True)
        t, _ = truncation(oracle.Oracle(m, p), p)
        rms.append(math.sqrt(float(np.mean(t ** 2))))
    rate = math.log2(rms[0] / rms[1])
    assert rate >= p - 0.3, (rms, rate)


def test_curved_mesh_checks():
    """Corner nodes off their vertices and edges whose two sides disagree on
    the middle node are rejected."""
    m = ogrid(8, 2, curved=True)
    bad = m.elem_geo.copy()
    bad[3, 0, 0] += 1e-6
    with pytest.raises(ValueError, match="corner"):
        oracle.Oracle(Mesh(2, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)
    bad = m.elem_geo.copy()
    bad[3, 7, 1] += 1e-6  # middle node of face 3 (eta = +1), shared with element 4
    with pytest.raises(ValueError, match="non-conforming curved"):
        oracle.Oracle(Mesh(2, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)


# ------------------------------------------------------------------ 3D hexes
@pytest.mark.parametrize("p", [1, 2])
def test_straight_nodes_reduce_to_trilinear(p):
    """27 nodes at the trilinear positions describe the same hex map."""
    m = reorient(wall_bumps(cubed_sphere_shell(2, 2, r_in=0.5, r_out=1.5), [0.05], [[0.3, 0.5, 0.8]], 0.5,
                            r_out=1.5), 3)
    O1 = oracle.Oracle(m, p, alpha_deg=2.0)
    O2 = oracle.Oracle(Mesh(3, m.xyz, m.elem_vert, m.bface_tag, "", straight_nodes(m)), p, alpha_deg=2.0)
    for a, b in zip(O1.geometry()[:3], O2.geometry()[:3]):
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))
    u = perturbed(O1, p, 5)
    r1, r2 = O1.residual(p, u), O2.residual(p, u)
    assert np.max(np.abs(r1 - r2)) <= 1e-13 * np.max(np.abs(r1))
    b1, b2 = O1.jacobian_blocks(p, u), O2.jacobian_blocks(p, u)
    assert np.max(np.abs(b1 - b2)) <= 1e-13 * np.max(np.abs(b1))


# a triquadratic map of the unit cube (each component of degree <= 2 in every
# variable) and its Jacobian matrix
_TQ = (0.2, 0.15, 0.25, 0.1, -0.12, 0.08)


def _triquad(x):
    s, t, u = x[:, 0], x[:, 1], x[:, 2]
    a, b, c, d, e, f = _TQ
    return np.stack([s + a * t * t + d * t * u, t + b * u * u + e * s * u, u + c * s * s + f * s * t], axis=1)


def _triquad_det(s, t, u):
    a, b, c, d, e, f = _TQ
    J = np.array([[1.0, 2 * a * t + d * u, d * t],
                  [e * u, 1.0, 2 * b * u + e * s],
                  [2 * c * s + f * t, f * s, 1.0]])
    return np.linalg.det(J)


def test_exact_volume_of_triquadratic_map():
    """Element volumes of a box under a global triquadratic map equal the
    integral of its Jacobian determinant (a polynomial of degree <= 6 per
    variable, integrated here with numpy's 8-point Gauss-Legendre rule per
    axis); the straight-sided version of the same mesh misses them."""
    base = box(3, 3, tag=TAG_FARFIELD)
    m = mapped(base, _triquad)
    vol, *_ = oracle.Oracle(m, 1).geometry()
    gx, gw = np.polynomial.legendre.leggauss(8)
    want = np.zeros(m.n_elem)
    for e in range(m.n_elem):
        lo, hi = base.xyz[base.elem_vert[e, 0]], base.xyz[base.elem_vert[e, 7]]
        h = 0.5 * (hi - lo)
        for i, wi in zip(gx, gw):
            for j, wj in zip(gx, gw):
                for k, wk in zip(gx, gw):
                    pt = lo + h * (1.0 + np.array([i, j, k]))
                    want[e] += wi * wj * wk * _triquad_det(*pt) * h.prod()
    assert np.max(np.abs(vol - want)) <= 1e-14
    vol_s, *_ = oracle.Oracle(Mesh(3, m.xyz, m.elem_vert, m.bface_tag), 1).geometry()
    assert np.max(np.abs(vol_s - want)) > 1e-6


def test_shell_volume_rate():
    """Volume of a cubed-sphere shell against 4/3 pi (r_out^3 - r_in^3): rate
    4 with curved hexes, 2 with straight ones (3.99 / 4.00 and 1.84 / 1.96
    measured from 2 to 4 to 8 cells per panel side)."""
    exact = 4.0 / 3.0 * math.pi * (1.0 - 0.5 ** 3)
    for curved, lo, hi in ((True, 3.9, 4.1), (False, 1.8, 2.1)):
        err = []
        for n in (4, 8):
            m = cubed_sphere_shell(n, 2, r_in=0.5, r_out=1.0, stretch=1.0001, curved=curved)
            vol, *_ = oracle.Oracle(m, 1).geometry()
            err.append(abs(vol.sum() - exact))
        rate = math.log2(err[0] / err[1])
        assert lo <= rate <= hi, (curved, err, rate)


@pytest.mark.parametrize("p", [1, 3])
def test_freestream_preservation_curved_shell(p):
    """The triquadratic map's cofactor metric terms satisfy the metric
    identities exactly and the rule integrates them exactly: zero residual
    of a uniform state."""
    m = reorient(cubed_sphere_shell(2, 2, inner=TAG_FARFIELD, curved=True), 4)
    O = oracle.Oracle(m, p, alpha_deg=3.0, beta_deg=-2.0)
    r = O.residual(p, O.freestream(p))
    vol, *_ = O.geometry()
    assert np.max(np.abs(r) / (2.0 * np.sqrt(vol)[:, None, None])) < 1e-13


@pytest.mark.parametrize("p", [1, 2])
def test_curved_shell_local_frames_and_truncation_rate(p):
    """Random local frames leave the per-element residual norms unchanged,
    and the truncation error of the projected manufactured state falls like
    h^p on curved shells (1.08 and 1.97 measured from 4 to 8 cells)."""
    m4 = cubed_sphere_shell(4, 4, r_in=0.5, r_out=1.0, inner=TAG_EXACT, outer=TAG_EXACT, curved=True)
    t1, s1 = truncation(oracle.Oracle(m4, p), p)
    t2, s2 = truncation(oracle.Oracle(reorient(m4, 8), p), p)
    assert np.max(np.abs(t1 - t2)) <= 1e-12 * np.max(s1)
    assert np.max(np.abs(s1 - s2)) <= 1e-12 * np.max(s1)
    m8 = cubed_sphere_shell(8, 8, r_in=0.5, r_out=1.0, inner=TAG_EXACT, outer=TAG_EXACT, curved=True)
    t8, _ = truncation(oracle.Oracle(m8, p), p)
    rate = math.log2(math.sqrt(float(np.mean(t1 ** 2))) / math.sqrt(float(np.mean(t8 ** 2))))
    assert rate >= p - 0.3, rate


def test_curved_hex_checks():
    m = cubed_sphere_shell(2, 1, curved=True)
    bad = m.elem_geo.copy()
    bad[5, node_of_vertex(3)[6], 2] += 1e-6
    with pytest.raises(ValueError, match="corner"):
        oracle.Oracle(Mesh(3, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)
    bad = m.elem_geo.copy()
    bad[5, 4 + 9 * 2, 1] += 1e-6  # centre node of face 5 (zeta = +1), an interior face
    with pytest.raises(ValueError, match="non-conforming curved"):
        oracle.Oracle(Mesh(3, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)
    bad = m.elem_geo.copy()
    bad[5, 13, 0] += 1e-6  # the centre node belongs to no face
    oracle.Oracle(Mesh(3, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)
