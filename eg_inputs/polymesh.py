"""Synthetic tetrahedral / prismatic meshes standing in for the paper's
unstructured sphere grid (Section 5.2: tetrahedra with prisms in the layers
next to the body).

Conventions shared by every consumer (input format only, no method
arithmetic):

* ``xyz`` is ``float64[n_vert, 3]``.
* ``elem_type`` is ``int8[n_elem]``: 0 tetrahedron, 1 triangular prism.
* ``elem_vert`` is ``int32[n_elem, 6]``.  A tetrahedron uses the first four
  entries (the rest are -1) and is positively oriented:
  det(v1 - v0, v2 - v0, v3 - v0) > 0.  A prism lists its bottom triangle
  v0 v1 v2 and its top triangle v3 v4 v5 with v_{a+3} joined to v_a by a
  lateral edge; det(v1 - v0, v2 - v0, v3 - v0) > 0.
* Local faces.  Tetrahedron: face k is the triangle of the three vertices
  other than v_k.  Prism: face 0 = (v0 v1 v2), face 1 = (v3 v4 v5),
  face 2 = (v0 v1 v4 v3), face 3 = (v1 v2 v5 v4), face 4 = (v2 v0 v3 v5).
* ``bface_tag`` is ``int8[n_elem, 5]`` with the tags of the quad / hex
  meshes (0 interior, matched to the neighbour through the face's vertex
  set; 1 slip wall; 2 far-field; 3 exact-state ghost of the oracle's
  manufactured-solution tests; 4 symmetry plane).  Unused entries are 0.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .meshes import Mesh, box, cubed_sphere_shell

TET, PRISM = 0, 1
TET_FACES = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))
PRISM_FACES = ((0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5))


@dataclasses.dataclass
class PolyMesh:
    xyz: np.ndarray        # float64 [n_vert, 3]
    elem_type: np.ndarray  # int8 [n_elem]
    elem_vert: np.ndarray  # int32 [n_elem, 6]
    bface_tag: np.ndarray  # int8 [n_elem, 5]
    name: str = ""

    dim = 3

    @property
    def n_elem(self) -> int:
        return int(self.elem_type.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    def contiguous(self) -> "PolyMesh":
        return PolyMesh(np.ascontiguousarray(self.xyz, dtype=np.float64),
                        np.ascontiguousarray(self.elem_type, dtype=np.int8),
                        np.ascontiguousarray(self.elem_vert, dtype=np.int32),
                        np.ascontiguousarray(self.bface_tag, dtype=np.int8),
                        self.name)

    def counts(self):
        """(tetrahedra, prisms)."""
        n_tet = int(np.sum(self.elem_type == TET))
        return n_tet, self.n_elem - n_tet


def local_faces(kind: int):
    return TET_FACES if kind == TET else PRISM_FACES


def _det(xyz, a, b, c, d):
    return float(np.linalg.det(np.stack([xyz[b] - xyz[a], xyz[c] - xyz[a], xyz[d] - xyz[a]])))


def _prism_to_tets(pr, xyz):
    """Three tetrahedra filling the prism ``pr`` (6 global vertex ids) such
    that every lateral quadrilateral is cut along the diagonal through its
    lowest-numbered vertex, so that neighbouring prisms cut a shared face the
    same way (the rule of Dompierre et al., 1999, for prisms)."""
    pr = list(pr)
    k = int(np.argmin(pr))
    # bring the lowest vertex to slot 0: a rotation of the triangles, and a
    # swap of bottom and top when it sits on the top triangle
    rot = (k % 3, (k + 1) % 3, (k + 2) % 3)
    bot = [pr[r] for r in rot]
    top = [pr[r + 3] for r in rot]
    if k >= 3:
        bot, top = top, bot
    v = bot + top
    # the quad (v1 v2 v5 v4) is the only one not through v0
    if min(v[1], v[5]) < min(v[2], v[4]):
        tets = [(v[0], v[1], v[2], v[5]), (v[0], v[1], v[5], v[4]), (v[0], v[4], v[5], v[3])]
    else:
        tets = [(v[0], v[1], v[2], v[4]), (v[0], v[4], v[2], v[5]), (v[0], v[4], v[5], v[3])]
    out = []
    for t in tets:
        t = list(t)
        if _det(xyz, *t) < 0.0:
            t[2], t[3] = t[3], t[2]
        out.append(t)
    return out


def from_hexes(mesh: Mesh, axis: int, tet_elem=None, name: str = "") -> PolyMesh:
    """Split every hexahedron of ``mesh`` into two prisms whose lateral edges
    run along reference axis ``axis`` (the cut goes through the corners
    (0, 0) and (1, 1) of the two other axes, the same in every element), and
    the prisms of the hexahedra with ``tet_elem[e]`` true further into three
    tetrahedra each.  Boundary tags follow the hexahedron faces that contain
    the new faces.  Straight-sided meshes only."""
    if mesh.dim != 3 or mesh.elem_geo is not None:
        raise ValueError("from_hexes needs a straight-sided hexahedral mesh")
    xyz = mesh.xyz
    ne = mesh.n_elem
    tet_elem = np.zeros(ne, dtype=bool) if tet_elem is None else np.asarray(tet_elem, dtype=bool)
    t1, t2 = [r for r in range(3) if r != axis]
    types, verts, tags = [], [], []

    def corner(e, ca, c1, c2):
        k = (ca << axis) | (c1 << t1) | (c2 << t2)
        return int(mesh.elem_vert[e, k])

    for e in range(ne):
        hex_faces = []
        for lf in range(6):
            r, s = divmod(lf, 2)
            fv = frozenset(int(mesh.elem_vert[e, k]) for k in range(8) if (k >> r) & 1 == s)
            hex_faces.append((fv, int(mesh.bface_tag[e, lf])))

        def tag_of(vs):
            vs = set(vs)
            for fv, tg in hex_faces:
                if vs <= fv:
                    return tg
            return 0

        q = [(0, 0), (1, 0), (1, 1), (0, 1)]
        prisms = []
        for tri in ((0, 1, 2), (0, 2, 3)):
            bot = [corner(e, 0, *q[i]) for i in tri]
            top = [corner(e, 1, *q[i]) for i in tri]
            pr = bot + top
            if _det(xyz, pr[0], pr[1], pr[2], pr[3]) < 0.0:
                pr = [pr[0], pr[2], pr[1], pr[3], pr[5], pr[4]]
            prisms.append(pr)
        for pr in prisms:
            if tet_elem[e]:
                for t in _prism_to_tets(pr, xyz):
                    types.append(TET)
                    verts.append(t + [-1, -1])
                    tags.append([tag_of([t[i] for i in f]) for f in TET_FACES] + [0])
            else:
                types.append(PRISM)
                verts.append(pr)
                tags.append([tag_of([pr[i] for i in f]) for f in PRISM_FACES])
    return PolyMesh(xyz.copy(), np.array(types, dtype=np.int8), np.array(verts, dtype=np.int32),
                    np.array(tags, dtype=np.int8), name or (mesh.name + "+poly"))


def box_poly(n: int, kind: str = "mixed", tag: int = 3, skew: float = 0.0, seed: int | None = None,
             lo: float = 0.0, hi: float = 1.0) -> PolyMesh:
    """The n^3 box of ``meshes.box`` cut into prisms along z (``kind`` =
    "prism"), tetrahedra ("tet"), or prisms in the lower half of the layers
    and tetrahedra above ("mixed"); every boundary face tagged ``tag``."""
    hx = box(3, n, lo=lo, hi=hi, tag=tag, skew=skew, seed=seed)
    layer = np.arange(hx.n_elem) // (n * n)
    if kind == "prism":
        te = np.zeros(hx.n_elem, dtype=bool)
    elif kind == "tet":
        te = np.ones(hx.n_elem, dtype=bool)
    elif kind == "mixed":
        te = layer >= n // 2
    else:
        raise ValueError(kind)
    return from_hexes(hx, 2, te, f"box{n}{kind}")


def sphere_poly(n: int, n_prism: int, n_tet: int, r_in: float = 0.5, r_out: float = 20.0,
                stretch: float = 1.2, n_ref: int = 12) -> PolyMesh:
    """Sphere of radius ``r_in`` in a far field of radius ``r_out`` (Section
    5.2's geometry, straight-sided): the cubed-sphere hex shell with n x n
    columns per panel and n_prism + n_tet radial layers; the n_prism layers
    next to the body become prisms along r (12 n^2 per layer), the layers
    outside them tetrahedra (36 n^2 per layer).  n = 8, 6 + 4 layers: 4608
    prisms and 9216 tetrahedra (the paper's grid: 4248 prisms, 9778
    tetrahedra)."""
    n_r = n_prism + n_tet
    hx = cubed_sphere_shell(n, n_r, r_in, r_out, stretch, n_ref)
    layer = np.arange(hx.n_elem) // (6 * n * n)
    return from_hexes(hx, 0, layer >= n_prism, f"spherepoly{n}x{n_prism}p{n_tet}t")
