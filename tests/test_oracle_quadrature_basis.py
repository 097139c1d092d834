"""Pins of the oracle's quadrature and basis (Section 3.2) against numpy's
Gauss-Legendre routine, exact areas and an independent numpy integration."""

import math

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell, box


@pytest.mark.parametrize("Q", list(range(1, 11)))
def test_gauss_matches_numpy(Q):
    x, w = oracle.gauss(Q)
    xr, wr = np.polynomial.legendre.leggauss(Q)
    assert np.max(np.abs(x - xr)) < 2e-15
    assert np.max(np.abs(w - wr)) < 2e-15
    # exact for monomials up to degree 2Q-1
    for k in range(2 * Q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


def test_modes_hierarchical():
    for d in (2, 3):
        full = oracle.modes(d, 4)
        for p in range(4):
            lvl = oracle.modes(d, p)
            assert np.array_equal(full[: len(lvl)], lvl)
            assert len(lvl) == (p + 1) ** d
            assert lvl[:, :d].max() == p


def _shoelace(P):
    x, y = P[:, 0], P[:, 1]
    return 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)


def test_volumes_are_exact_polygon_areas():
    m = ogrid(24, 12)
    O = oracle.Oracle(m, 2)
    vol, surf, h, om = O.geometry()
    for e in range(m.n_elem):
        v = m.xyz[m.elem_vert[e]]
        poly = v[[0, 1, 3, 2]]  # corners (xi, eta) = (-,-), (+,-), (+,+), (-,+)
        assert abs(vol[e] - _shoelace(poly)) < 1e-13 * max(1.0, vol[e])
        edges = sum(np.linalg.norm(poly[k] - poly[(k + 1) % 4]) for k in range(4))
        assert abs(surf[e] - edges) < 1e-13 * edges
    # whole annulus between two regular 24-gons
    r_in, r_out = 0.5, 20.0
    area = 0.5 * 24 * math.sin(2 * math.pi / 24) * (r_out ** 2 - r_in ** 2)
    assert abs(om - area) < 1e-11 * area
    assert np.allclose(h, 4 * vol / surf, rtol=1e-15)


def test_hex_volumes_sum_to_box():
    m = box(3, 3, skew=0.15, seed=3, tag=2)
    O = oracle.Oracle(m, 1)
    vol, surf, h, om = O.geometry()
    assert abs(om - 1.0) < 1e-14
    assert np.all(vol > 0)


def _ref_points(Q, d):
    x, w = np.polynomial.legendre.leggauss(Q)
    pts = np.stack(np.meshgrid(*([x] * d), indexing="ij"), -1).reshape(-1, d)
    wts = np.prod(np.stack(np.meshgrid(*([w] * d), indexing="ij"), -1).reshape(-1, d), axis=1)
    return pts, wts


def _det_multilinear(X, xi):
    d = X.shape[1]
    J = np.zeros((d, d))
    for c in range(2 ** d):
        bits = [(c >> r) & 1 for r in range(d)]
        for r in range(d):
            g = 1.0
            for q in range(d):
                s = 1.0 if bits[q] else -1.0
                g *= 0.5 * s if q == r else 0.5 * (1 + s * xi[q])
            J[:, r] += g * X[c]
    return np.linalg.det(J)


@pytest.mark.parametrize("mesh,p", [(ogrid(8, 4), 3), (cubed_sphere_shell(1, 2), 2)])
def test_basis_orthonormal_by_independent_integration(mesh, p):
    """Evaluate psi_i through the oracle at numpy's Gauss points of a finer
    rule and integrate psi_i psi_j |det| with a test-side multilinear map."""
    O = oracle.Oracle(mesh, p)
    N, V, d = O.N(p), O.V, mesh.dim
    pts, wts = _ref_points(p + 3, d)
    vol, *_ = O.geometry()
    for e in (0, mesh.n_elem // 2, mesh.n_elem - 1):
        X = mesh.xyz[mesh.elem_vert[e]]
        Psi = np.zeros((len(pts), N))
        dets = np.array([_det_multilinear(X, xi) for xi in pts])
        for i in range(N):
            u = O.zeros(p)
            u[e, 0, i] = 1.0
            for q, xi in enumerate(pts):
                Psi[q, i] = O.eval_point(p, e, u, xi)[0][0]
        G = Psi.T @ (Psi * (wts * dets)[:, None])
        assert np.max(np.abs(G - np.eye(N))) < 1e-12
        assert np.max(np.abs(Psi[:, 0] - 1.0 / math.sqrt(vol[e]))) < 1e-12 / math.sqrt(vol[e])
