"""Pins of the oracle's symmetry-plane boundary (Section 5.2: the sphere mesh
is cut along the flow's planes of symmetry, which carry a symmetry
condition).  On a mirror-symmetric state the neighbour across the plane holds
the mirror image of the inside state, which is the slip ghost; so the half
(quarter) domain's residual and its Jacobian on mirror-symmetric
perturbations equal the full domain's on the kept elements, and its drag is
a half (quarter) of the full drag."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell, clip, TAG_WALL, TAG_SYMMETRY
from tests.test_oracle_residual import perturbed


def mirror_partners(mesh, axis):
    """For every element, the element whose vertices are its mirror images
    across the plane x_axis = 0, and the signed permutation S between their
    reference frames (the partner's corner xi sits at the mirror of this
    element's corner S xi)."""
    X = mesh.xyz[mesh.elem_vert]
    dim, nc = mesh.dim, 2 ** mesh.dim

    def key(pts):
        return frozenset(tuple(np.round(p, 9) + 0.0) for p in pts)

    index = {key(X[e]): e for e in range(mesh.n_elem)}
    corners = np.array([[2 * ((k >> r) & 1) - 1 for r in range(dim)] for k in range(nc)])
    out = []
    for e in range(mesh.n_elem):
        Y = X[e].copy()
        Y[:, axis] *= -1.0
        e2 = index[key(Y)]
        img = np.array([corners[int(np.argmin(np.sum((Y - X[e2][k]) ** 2, axis=1)))] for k in range(nc)])
        S = np.rint(np.linalg.lstsq(corners.astype(float), img.astype(float), rcond=None)[0].T).astype(int)
        assert np.array_equal(corners @ S.T, img)
        out.append((e2, S))
    return out


def symmetric_full_state(mesh, O, p, keep, u_keep, axes, everywhere=False):
    """Full-domain state: u_keep on the kept elements, the mirror image of a
    kept element's state on its face neighbour across each plane (a diagonal S
    flips the modes of odd degree along the flipped axes, the momentum normal
    to the plane changes sign), free stream elsewhere; ``everywhere`` mirrors
    every kept element onto its partner (a fully symmetric state)."""
    u = O.freestream(p)
    kept = np.nonzero(keep)[0]
    u[kept] = u_keep
    modes = oracle.modes(mesh.dim, p)[:, : mesh.dim]
    done = np.zeros(mesh.n_elem, dtype=bool)
    for axis in axes:
        for e, (e2, S) in enumerate(mirror_partners(mesh, axis)):
            shared = len(set(mesh.elem_vert[e].tolist()) & set(mesh.elem_vert[e2].tolist()))
            if not keep[e] or keep[e2] or (shared != 2 ** (mesh.dim - 1) and not everywhere):
                continue  # only the kept elements' neighbours across the plane matter
            assert np.count_nonzero(S - np.diag(np.diag(S))) == 0, "partner frames differ by an axis swap"
            sgn_mode = np.prod(np.diag(S)[None, :] ** modes, axis=1)
            sgn_var = np.ones(mesh.dim + 2)
            sgn_var[1 + axis] = -1.0
            u[e2] = u[e] * sgn_var[:, None] * sgn_mode[None, :]
            done[e2] = True
    return u, done


def _cut(mesh, axes, tag=TAG_SYMMETRY):
    c = mesh.xyz[mesh.elem_vert].mean(axis=1)
    keep = np.all(c[:, list(axes)] > 0.0, axis=1)
    return keep, clip(mesh, keep, tag)


CASES = [
    ("ogrid-half", ogrid(16, 4), (1,), 2, "rusanov"),
    ("ogrid-curved-half-roe", ogrid(16, 4, curved=True), (1,), 3, "roe"),
    ("sphere-quarter", cubed_sphere_shell(4, 2), (1, 2), 2, "rusanov"),
    ("sphere-half-roe", cubed_sphere_shell(2, 2), (2,), 1, "roe"),
]


@pytest.mark.parametrize("name,mesh,axes,p,flux", CASES, ids=[c[0] for c in CASES])
def test_cut_domain_equals_full_domain(name, mesh, axes, p, flux):
    keep, part = _cut(mesh, axes)
    assert np.count_nonzero(part.bface_tag == TAG_SYMMETRY) > 0
    # every cut face lies on a plane of symmetry
    for e, lf in zip(*np.nonzero(part.bface_tag == TAG_SYMMETRY)):
        r, s = divmod(int(lf), 2)
        pts = part.xyz[[part.elem_vert[e, k] for k in range(2 ** part.dim) if (k >> r) & 1 == s]]
        assert any(np.max(np.abs(pts[:, a])) < 1e-12 for a in axes)
    Op = oracle.Oracle(part, p, flux=flux)
    Of = oracle.Oracle(mesh, p, flux=flux)
    u_part = perturbed(Op, p, 31)
    u_full, _ = symmetric_full_state(mesh, Of, p, keep, u_part, axes)
    r_part = Op.residual(p, u_part)
    r_full = Of.residual(p, u_full)[keep]
    assert np.max(np.abs(r_part - r_full)) <= 1e-12 * np.max(np.abs(r_full))
    # the linearisation too, on a mirror-symmetric perturbation (the element
    # blocks alone differ: at a symmetry face the ghost's derivative folds
    # into the diagonal block, across an interior face it is off-diagonal)
    dv = np.random.default_rng(34).uniform(-1, 1, u_part.shape)
    d_full = (symmetric_full_state(mesh, Of, p, keep, dv, axes)[0]
              - symmetric_full_state(mesh, Of, p, keep, 0.0 * dv, axes)[0])
    jv_part = (Op.jacobian_sparse(p, u_part) @ dv.ravel()).reshape(dv.shape)
    jv_full = (Of.jacobian_sparse(p, u_full) @ d_full.ravel()).reshape(d_full.shape)[keep]
    assert np.max(np.abs(jv_part - jv_full)) <= 1e-12 * np.max(np.abs(jv_full))


@pytest.mark.parametrize("name,mesh,axes,p,flux", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_drag_leaves_out_symmetry_planes(name, mesh, axes, p, flux):
    """On a symmetric state the half O-grid's drag (and its gradient on the
    kept elements) is half the full drag; the force normal to the plane is
    the upper half-body's alone, and tagging the cut faces as walls instead
    adds their pressure force.  (On the cubed sphere
    some mirror partners' frames differ by an axis swap, so a fully symmetric
    state is not written here; the GPU tests compare quarter and full sphere
    drags at their steady states.)"""
    keep, part = _cut(mesh, axes)
    Op, Of = oracle.Oracle(part, p, flux=flux), oracle.Oracle(mesh, p, flux=flux)
    u_part = perturbed(Op, p, 32)
    u_full, done = symmetric_full_state(mesh, Of, p, keep, u_part, axes, everywhere=True)
    assert np.all(done | keep)
    f = 2 ** len(axes)
    cd_p, g_p = Op.drag(p, u_part, grad=True)
    cd_f, g_f = Of.drag(p, u_full, grad=True)
    assert abs(f * cd_p - cd_f) <= 1e-12 * abs(cd_f)
    assert np.max(np.abs(g_p - g_f[keep])) <= 1e-12 * np.max(np.abs(g_f))
    # The force normal to the plane tells a symmetry face from a wall.  On the
    # full grid with the free stream below y = 0, the lower half-body feels
    # the constant pressure p_inf, whose force along +y is p_inf times the
    # chord 2 r_in (the integral of the scaled normal along an open curve is
    # its rotated chord, exact for straight and quadratic edges); the rest is
    # the upper half-body, i.e. what the half grid integrates.
    up = np.array([0.0, 1.0])
    u_upper, _ = symmetric_full_state(mesh, Of, p, keep, u_part, axes)
    Uf = Of.freestream_state()
    p_inf = 0.4 * (Uf[3] - 0.5 * (Uf[1] ** 2 + Uf[2] ** 2) / Uf[0])
    scale = -1.0 / (0.5 * 0.3 ** 2)
    lower = scale * p_inf * 2.0 * 0.5
    u_free_below = u_upper.copy()
    u_free_below[~keep] = Of.freestream(p)[~keep]
    cl_f = Of.drag(p, u_free_below, direction=up)
    cl_p = Op.drag(p, u_part, direction=up)
    assert abs(cl_p - (cl_f - lower)) <= 1e-12 * abs(lower)
    _, walls = _cut(mesh, axes, tag=TAG_WALL)
    cl_w = oracle.Oracle(walls, p, flux=flux).drag(p, u_part, direction=up)
    assert abs(cl_w - cl_p) > 1e-3 * abs(cl_p)


def test_symmetry_ghost_is_the_mirror_state():
    """The symmetry ghost equals the slip-wall ghost (mirror image of the
    inside state across the face)."""
    O = oracle.Oracle(ogrid(8, 2), 1)
    rng = np.random.default_rng(5)
    U = np.array([1.1, 0.2, -0.1, 2.6])
    for _ in range(5):
        n = rng.normal(size=2)
        n /= np.linalg.norm(n)
        g4 = O.ghost(TAG_SYMMETRY, U, n, np.zeros(2))
        g1 = O.ghost(TAG_WALL, U, n, np.zeros(2))
        assert np.array_equal(g4, g1)
        vn = U[1:3] @ n
        assert np.allclose(g4[1:3], U[1:3] - 2.0 * vn * n, rtol=0, atol=1e-15)

