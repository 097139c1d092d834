"""The seeded input generators for curved elements and cut grids: curved
nodes on the true circles and spheres, face nodes shared bit-identically by
neighbours (also across cubed-sphere panel seams and after reorientation),
and the topology of clip().  Inputs only: no method arithmetic here."""

import numpy as np
import pytest

from eg_inputs import (ogrid, cubed_sphere_shell, clip, reorient, wall_bumps, node_ref, node_of_vertex,
                       straight_nodes, TAG_INTERIOR, TAG_SYMMETRY, TAG_WALL)


def _face_nodes(mesh, e, lf):
    """Coordinates of the 3^(d-1) nodes of local face lf, as a set of tuples."""
    r, s = divmod(lf, 2)
    ref = node_ref(mesh.dim) + 1
    return {tuple(mesh.elem_geo[e, k]) for k in range(3 ** mesh.dim) if ref[k, r] == 2 * s}


def _interior_pairs(mesh):
    nc = 2 ** mesh.dim
    owners = {}
    for e in range(mesh.n_elem):
        for lf in range(2 * mesh.dim):
            if mesh.bface_tag[e, lf] != TAG_INTERIOR:
                continue
            r, s = divmod(lf, 2)
            key = frozenset(int(mesh.elem_vert[e, k]) for k in range(nc) if (k >> r) & 1 == s)
            owners.setdefault(key, []).append((e, lf))
    return list(owners.values())


@pytest.mark.parametrize("mesh", [ogrid(12, 4, curved=True), reorient(ogrid(10, 3, curved=True), 3),
                                  cubed_sphere_shell(3, 2, curved=True),
                                  reorient(cubed_sphere_shell(2, 2, curved=True), 5)],
                         ids=["ogrid", "ogrid-reoriented", "shell", "shell-reoriented"])
def test_shared_face_nodes_are_bit_identical(mesh):
    pairs = _interior_pairs(mesh)
    assert all(len(p) == 2 for p in pairs)
    for (e1, l1), (e2, l2) in pairs:
        assert _face_nodes(mesh, e1, l1) == _face_nodes(mesh, e2, l2)
    # corner nodes are the vertices
    for i, k in enumerate(node_of_vertex(mesh.dim)):
        assert np.array_equal(mesh.elem_geo[:, k], mesh.xyz[mesh.elem_vert[:, i]])


def test_curved_nodes_on_the_true_circles_and_spheres():
    m = ogrid(16, 4, r_in=0.5, r_out=20.0, curved=True)
    r = np.linalg.norm(m.elem_geo, axis=2)
    inner = [k for k in range(9) if node_ref(2)[k, 0] == -1]  # xi = -1: the body
    assert np.max(np.abs(r[:16][:, inner] - 0.5)) < 1e-15  # the first ring (j = 0) touches the body
    s = cubed_sphere_shell(4, 3, r_in=0.5, r_out=20.0, curved=True)
    rs = np.linalg.norm(s.elem_geo, axis=2)
    inner3 = [k for k in range(27) if node_ref(3)[k, 0] == -1]
    ring0 = np.arange(6 * 16)  # layer j = 0
    assert np.max(np.abs(rs[ring0][:, inner3] - 0.5)) < 1e-15
    outer3 = [k for k in range(27) if node_ref(3)[k, 0] == 1]
    ring_last = np.arange(6 * 16 * 2, 6 * 16 * 3)
    assert np.max(np.abs(rs[ring_last][:, outer3] - 20.0)) < 1e-13


def test_straight_nodes_reproduce_the_vertices():
    for m in (ogrid(8, 2), cubed_sphere_shell(2, 1)):
        g = straight_nodes(m)
        for i, k in enumerate(node_of_vertex(m.dim)):
            assert np.array_equal(g[:, k], m.xyz[m.elem_vert[:, i]])


def test_wall_bumps_move_curved_nodes_consistently():
    m = wall_bumps(cubed_sphere_shell(2, 2, curved=True), [0.05], [[0.0, 0.6, 0.8]], 0.4)
    for (e1, l1), (e2, l2) in _interior_pairs(m):
        assert _face_nodes(m, e1, l1) == _face_nodes(m, e2, l2)


@pytest.mark.parametrize("mesh,axes,n_keep", [(ogrid(16, 4), (1,), 32), (ogrid(16, 4, curved=True), (1,), 32),
                                               (cubed_sphere_shell(4, 2), (1, 2), 48)])
def test_clip_topology(mesh, axes, n_keep):
    c = mesh.xyz[mesh.elem_vert].mean(axis=1)
    keep = np.all(c[:, list(axes)] > 0.0, axis=1)
    part = clip(mesh, keep)
    assert part.n_elem == n_keep
    # vertices compacted, all used
    assert np.array_equal(np.unique(part.elem_vert), np.arange(part.n_vert))
    # every interior face still has exactly one neighbour; the cut faces lie on the planes
    assert all(len(p) == 2 for p in _interior_pairs(part))
    nc = 2 ** part.dim
    for e, lf in zip(*np.nonzero(part.bface_tag == TAG_SYMMETRY)):
        r, s = divmod(int(lf), 2)
        pts = part.xyz[[part.elem_vert[e, k] for k in range(nc) if (k >> r) & 1 == s]]
        assert any(np.max(np.abs(pts[:, a])) == 0.0 for a in axes)
    # walls and far field carried over
    assert np.count_nonzero(part.bface_tag == TAG_WALL) == np.count_nonzero(mesh.bface_tag[keep] == TAG_WALL)
    if mesh.elem_geo is not None:
        assert np.array_equal(part.elem_geo, mesh.elem_geo[keep])
