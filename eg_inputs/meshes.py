"""Synthetic quad / hex meshes standing in for the paper's cylinder
(Section 5.1, quadratic curved elements) and sphere (Section 5.2) grids.

Conventions shared by every consumer (they are the input format, not method
arithmetic):

* ``xyz`` is ``float64[n_vert, dim]``.
* ``elem_vert`` is ``int32[n_elem, 2**dim]``; local vertex ``a + 2 b (+ 4 c)``
  sits at reference corner ``xi = (2a-1, 2b-1[, 2c-1])`` of ``[-1, 1]^dim``.
  Elements are positively oriented (the trilinear map has positive Jacobian).
* ``bface_tag`` is ``int8[n_elem, 2*dim]``; local face ``2 r + s`` is the face
  ``xi_r = -1`` (s = 0) or ``xi_r = +1`` (s = 1).  Tags: 0 interior (matched
  to a neighbour through its shared vertices), 1 slip wall, 2 far-field,
  3 exact-state ghost (manufactured-solution tests of the oracle only),
  4 symmetry plane.
* ``elem_geo`` (optional) is ``float64[n_elem, 3**dim, dim]``: the nodes of a
  tensor quadratic element map; node ``a + 3 b (+ 9 c)`` sits at reference
  point ``(a - 1, b - 1[, c - 1])``, so the nodes whose digits are all 0 or 2
  are the vertices (``node_of_vertex``).  ``None`` means straight-sided
  (multilinear) elements.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

TAG_INTERIOR = 0
TAG_WALL = 1
TAG_FARFIELD = 2
TAG_EXACT = 3
TAG_SYMMETRY = 4


@dataclasses.dataclass
class Mesh:
    dim: int
    xyz: np.ndarray        # float64 [n_vert, dim]
    elem_vert: np.ndarray  # int32 [n_elem, 2**dim]
    bface_tag: np.ndarray  # int8 [n_elem, 2*dim]
    name: str = ""
    elem_geo: np.ndarray | None = None  # float64 [n_elem, 3**dim, dim] (curved) or None

    @property
    def n_elem(self) -> int:
        return int(self.elem_vert.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    def contiguous(self) -> "Mesh":
        return Mesh(self.dim,
                    np.ascontiguousarray(self.xyz, dtype=np.float64),
                    np.ascontiguousarray(self.elem_vert, dtype=np.int32),
                    np.ascontiguousarray(self.bface_tag, dtype=np.int8),
                    self.name,
                    None if self.elem_geo is None else np.ascontiguousarray(self.elem_geo, dtype=np.float64))


def node_ref(dim: int) -> np.ndarray:
    """int64[3**dim, dim]: reference position (digits - 1) of every node
    a + 3 b (+ 9 c) of a tensor quadratic element."""
    return np.array([[(k // 3 ** r) % 3 - 1 for r in range(dim)] for k in range(3 ** dim)], dtype=np.int64)


def node_of_vertex(dim: int) -> list:
    """Node index of every vertex a + 2 b (+ 4 c) (the node with digits 2a, 2b, 2c)."""
    return [sum(2 * ((k >> r) & 1) * 3 ** r for r in range(dim)) for k in range(2 ** dim)]


QUAD9_REF = node_ref(2)
QUAD9_CORNER = tuple(node_of_vertex(2))


def straight_nodes(mesh: Mesh) -> np.ndarray:
    """float64[n_elem, 3**dim, dim]: the nodes of each element's multilinear
    map (vertices at the corners, the other nodes at the multilinear
    positions of their reference points), i.e. the straight-sided element
    written as a quadratic one."""
    dim = mesh.dim
    X = mesh.xyz[mesh.elem_vert]  # [E, 2^dim, dim], vertex a + 2 b + 4 c
    ref = node_ref(dim) + 1
    geo = np.zeros((mesh.n_elem, 3 ** dim, dim))
    for k in range(3 ** dim):
        for v in range(2 ** dim):
            w = 1.0
            for r in range(dim):
                w *= 0.5 * ref[k, r] if (v >> r) & 1 else 1.0 - 0.5 * ref[k, r]
            if w != 0.0:
                geo[:, k] += w * X[:, v]
    return geo


def mapped(mesh: Mesh, fn, name: str = "") -> Mesh:
    """Curved mesh: every node of the mesh (vertices and the 3**dim nodes of
    each element, multilinear ones for a straight mesh) moved through the
    smooth map ``fn(float64[n, dim]) -> float64[n, dim]``.  Shared faces keep
    shared nodes because both neighbours evaluate ``fn`` at the same point."""
    dim = mesh.dim
    base = straight_nodes(mesh) if mesh.elem_geo is None else mesh.elem_geo
    geo = fn(base.reshape(-1, dim)).reshape(base.shape)
    xyz = fn(np.array(mesh.xyz, dtype=np.float64))
    for i, k in enumerate(node_of_vertex(dim)):
        geo[:, k] = xyz[mesh.elem_vert[:, i]]
    return Mesh(dim, xyz, mesh.elem_vert.copy(), mesh.bface_tag.copy(), name or mesh.name + "+mapped", geo)


def radial_map(n_r: int, r_in: float = 0.5, r_out: float = 20.0,
               stretch: float = 1.2, n_ref: int = 12) -> np.ndarray:
    """Radial node positions r_0..r_{n_r}.

    Geometric spacing with ratio ``stretch`` between consecutive cells when
    ``n_r == n_ref``; other ``n_r`` sample the same continuous map
    r(s) = r_in + (r_out - r_in) (stretch^(n_ref s) - 1) / (stretch^n_ref - 1).
    """
    s = np.arange(n_r + 1, dtype=np.float64) / n_r
    g = stretch ** n_ref
    r = r_in + (r_out - r_in) * (np.power(stretch, n_ref * s) - 1.0) / (g - 1.0)
    r[0] = r_in
    r[-1] = r_out
    return r


def ogrid(n_theta: int, n_r: int, r_in: float = 0.5, r_out: float = 20.0,
          stretch: float = 1.2, n_ref: int = 12, inner: int = TAG_WALL,
          outer: int = TAG_FARFIELD, curved: bool = False) -> Mesh:
    """Structured O-grid of quads around a circle of radius ``r_in``.

    Element (i, j), i circumferential (periodic), j radial (j = 0 touches the
    body) has index ``j * n_theta + i``.  Reference xi runs outward in r, eta
    counter-clockwise in theta, so the map is positively oriented; face 0 is
    the inner arc (``inner`` tag at j = 0), face 1 the outer arc (``outer`` tag
    at j = n_r - 1), faces 2/3 the two radial edges.

    ``curved`` adds biquadratic element nodes: the mid-arc nodes sit on the
    circles (angle halfway between the two vertices), the radial edges stay
    straight with their midpoints halfway in r.
    """
    if n_theta < 3 or n_r < 1:
        raise ValueError("ogrid needs n_theta >= 3 and n_r >= 1")
    r = radial_map(n_r, r_in, r_out, stretch, n_ref)
    th = 2.0 * math.pi * np.arange(n_theta, dtype=np.float64) / n_theta
    c, s = np.cos(th), np.sin(th)
    # exact axis points keep the mesh mirror-symmetric about y = 0
    for i in range(n_theta):
        if 4 * i == n_theta:
            c[i], s[i] = 0.0, 1.0
        elif 2 * i == n_theta:
            c[i], s[i] = -1.0, 0.0
        elif 4 * i == 3 * n_theta:
            c[i], s[i] = 0.0, -1.0
    c[0], s[0] = 1.0, 0.0
    # vertex (i, j) -> j * n_theta + i
    xyz = np.empty(((n_r + 1) * n_theta, 2))
    for j in range(n_r + 1):
        xyz[j * n_theta:(j + 1) * n_theta, 0] = r[j] * c
        xyz[j * n_theta:(j + 1) * n_theta, 1] = r[j] * s
    ev = np.empty((n_r * n_theta, 4), dtype=np.int32)
    tag = np.zeros((n_r * n_theta, 4), dtype=np.int8)
    for j in range(n_r):
        for i in range(n_theta):
            e = j * n_theta + i
            ip = (i + 1) % n_theta
            ev[e] = (j * n_theta + i, (j + 1) * n_theta + i,
                     j * n_theta + ip, (j + 1) * n_theta + ip)
            if j == 0:
                tag[e, 0] = inner
            if j == n_r - 1:
                tag[e, 1] = outer
    if not curved:
        return Mesh(2, xyz, ev, tag, f"ogrid{n_theta}x{n_r}")
    # node grid: 2 n_theta angles (vertex angles, then the mid angles) by
    # 2 n_r + 1 radii; every element reads its nine nodes from it, so shared
    # edges share bit-identical nodes
    thm = 2.0 * math.pi * (np.arange(n_theta, dtype=np.float64) + 0.5) / n_theta
    cm, sm = np.cos(thm), np.sin(thm)
    for i in range(n_theta):  # exact axis points, as for the vertices
        if 2 * (2 * i + 1) == n_theta:
            cm[i], sm[i] = 0.0, 1.0
        elif 2 * i + 1 == n_theta:
            cm[i], sm[i] = -1.0, 0.0
        elif 2 * (2 * i + 1) == 3 * n_theta:
            cm[i], sm[i] = 0.0, -1.0
    rr = np.empty(2 * n_r + 1)
    rr[0::2] = r
    rr[1::2] = 0.5 * (r[:-1] + r[1:])
    geo = np.empty((n_r * n_theta, 9, 2))
    for j in range(n_r):
        for i in range(n_theta):
            e = j * n_theta + i
            ip = (i + 1) % n_theta
            for k, (a, b) in enumerate(QUAD9_REF + 1):
                rad = rr[2 * j + a]
                cc, ss = ((c[i], s[i]), (cm[i], sm[i]), (c[ip], s[ip]))[b]
                geo[e, k] = (rad * cc, rad * ss)
    return Mesh(2, xyz, ev, tag, f"ogrid{n_theta}x{n_r}c", geo)


_PANELS = (
    # (normal, t1, t2) with normal = t1 x t2 (right handed)
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
)


def cubed_sphere_shell(n: int, n_r: int, r_in: float = 0.5, r_out: float = 20.0,
                       stretch: float = 1.2, n_ref: int = 12,
                       inner: int = TAG_WALL, outer: int = TAG_FARFIELD, curved: bool = False) -> Mesh:
    """Equiangular gnomonic cubed-sphere hex shell: 6 panels of n x n columns
    and ``n_r`` radial layers (6 n^2 n_r hexes).  Vertices on panel seams are
    shared.  xi runs outward in r; face 0 is on the body (``inner`` tag),
    face 1 on the outer sphere (``outer`` tag).

    ``curved`` adds triquadratic element nodes: the panel grid refined to
    half steps of the equiangular parameter, projected to the spheres of
    radius r_j, r_{j+1} and their mean (radial edges stay straight)."""
    if n < 1 or n_r < 1:
        raise ValueError("cubed_sphere_shell needs n >= 1 and n_r >= 1")
    r = radial_map(n_r, r_in, r_out, stretch, n_ref)
    t = np.tan(-math.pi / 4 + (math.pi / 2) * np.arange(n + 1) / n)
    t[0], t[-1] = -1.0, 1.0
    if n % 2 == 0:
        t[n // 2] = 0.0
    # unit directions per panel grid point, deduplicated across seams
    key_to_id: dict = {}
    dirs = []
    pid = np.empty((6, n + 1, n + 1), dtype=np.int64)
    for P, (nv, t1, t2) in enumerate(_PANELS):
        nv, t1, t2 = (np.array(a, dtype=np.float64) for a in (nv, t1, t2))
        for a in range(n + 1):
            for b in range(n + 1):
                v = nv + t[a] * t1 + t[b] * t2
                v = v / math.sqrt(float(v @ v))
                k = tuple(np.round(v * 1e9).astype(np.int64))
                if k not in key_to_id:
                    key_to_id[k] = len(dirs)
                    dirs.append(v)
                pid[P, a, b] = key_to_id[k]
    dirs = np.array(dirs)
    nd = dirs.shape[0]
    xyz = np.concatenate([r[j] * dirs for j in range(n_r + 1)], axis=0)
    ne = 6 * n * n * n_r
    ev = np.empty((ne, 8), dtype=np.int32)
    tag = np.zeros((ne, 6), dtype=np.int8)
    e = 0
    # element order: layer-major, then panel, then (b, a) so neighbours in a
    # panel are close in memory
    for j in range(n_r):
        for P in range(6):
            for b in range(n):
                for a in range(n):
                    for cz in range(2):
                        for cy in range(2):
                            for cx in range(2):
                                ev[e, cx + 2 * cy + 4 * cz] = (
                                    (j + cx) * nd + pid[P, a + cy, b + cz])
                    if j == 0:
                        tag[e, 0] = inner
                    if j == n_r - 1:
                        tag[e, 1] = outer
                    e += 1
    if not curved:
        return Mesh(3, xyz, ev, tag, f"cubedsphere6x{n}x{n}x{n_r}")
    # unit directions on the half-step panel grids, deduplicated across seams
    # so that neighbours on two panels read bit-identical nodes
    th = np.tan(-math.pi / 4 + (math.pi / 2) * np.arange(2 * n + 1) / (2 * n))
    th[0], th[-1], th[n] = -1.0, 1.0, 0.0
    hdirs: dict = {}
    hid = np.empty((6, 2 * n + 1, 2 * n + 1), dtype=np.int64)
    hlist = []
    for P, (nv, t1, t2) in enumerate(_PANELS):
        nv, t1, t2 = (np.array(a, dtype=np.float64) for a in (nv, t1, t2))
        for a in range(2 * n + 1):
            for b in range(2 * n + 1):
                v = nv + th[a] * t1 + th[b] * t2
                v = v / math.sqrt(float(v @ v))
                k = tuple(np.round(v * 1e9).astype(np.int64))
                if k not in hdirs:
                    hdirs[k] = len(hlist)
                    hlist.append(v)
                hid[P, a, b] = hdirs[k]
    hlist = np.array(hlist)
    rr = np.empty(2 * n_r + 1)
    rr[0::2] = r
    rr[1::2] = 0.5 * (r[:-1] + r[1:])
    geo = np.empty((ne, 27, 3))
    e = 0
    for j in range(n_r):
        for P in range(6):
            for b in range(n):
                for a in range(n):
                    for k, (dx, dy, dz) in enumerate(node_ref(3) + 1):
                        geo[e, k] = rr[2 * j + dx] * hlist[hid[P, 2 * a + dy, 2 * b + dz]]
                    e += 1
    # the corner nodes are the vertices themselves
    for i, k in enumerate(node_of_vertex(3)):
        geo[:, k] = xyz[ev[:, i]]
    return Mesh(3, xyz, ev, tag, f"cubedsphere6x{n}x{n}x{n_r}c", geo)


def box(dim: int, n: int, lo: float = 0.0, hi: float = 1.0, tag: int = TAG_EXACT,
        skew: float = 0.0, seed: int | None = None) -> Mesh:
    """Uniform n^dim box of quads/hexes with every boundary face tagged ``tag``.

    ``skew`` > 0 moves interior vertices by a seeded random offset of that
    fraction of the spacing (still straight-sided, positively oriented for
    skew < 0.25), so tests do not only see affine elements.
    """
    m = n + 1
    h = (hi - lo) / n
    grid = np.stack(np.meshgrid(*([lo + h * np.arange(m)] * dim), indexing="ij"),
                    axis=-1).reshape(-1, dim)
    # vertex id: lexicographic with the first axis fastest
    idx = np.arange(m ** dim).reshape([m] * dim, order="F")
    pts = np.empty((m ** dim, dim))
    it = np.ndindex(*([m] * dim))
    for mi in it:
        pts[idx[mi]] = lo + h * np.array(mi, dtype=np.float64)
    del grid
    if skew > 0.0:
        rng = np.random.Generator(np.random.PCG64(0 if seed is None else seed))
        off = rng.uniform(-skew * h, skew * h, size=pts.shape)
        interior = np.all((pts > lo + 0.5 * h) & (pts < hi - 0.5 * h), axis=1)
        pts[interior] += off[interior]
    ne = n ** dim
    ev = np.empty((ne, 2 ** dim), dtype=np.int32)
    tg = np.zeros((ne, 2 * dim), dtype=np.int8)
    e = 0
    for ei in np.ndindex(*([n] * dim)[::-1]):
        ei = ei[::-1]  # first axis fastest
        for c in range(2 ** dim):
            off = [(c >> r) & 1 for r in range(dim)]
            ev[e, c] = idx[tuple(ei[r] + off[r] for r in range(dim))]
        for r in range(dim):
            if ei[r] == 0:
                tg[e, 2 * r] = tag
            if ei[r] == n - 1:
                tg[e, 2 * r + 1] = tag
        e += 1
    return Mesh(dim, pts, ev, tg, f"box{dim}d{n}")


def wall_bumps(mesh: Mesh, amps, centers, sigma: float, r_in: float = 0.5,
               r_out: float = 20.0) -> Mesh:
    """Radial Gaussian bumps on the body of an O-grid or cubed-sphere shell.

    Vertex x at radius r moves radially by
        delta(x) = sum_k amps[k] exp(-theta_k(x)^2 / (2 sigma^2)) (r_out - r) / (r_out - r_in),
    theta_k the angle between x and the unit vector centers[k]: full
    amplitude on the wall, none on the far-field boundary, so the topology and
    the boundary tags are unchanged and small amplitudes keep every element
    positively oriented.
    """
    amps = np.asarray(amps, dtype=np.float64)
    centers = np.asarray(centers, dtype=np.float64).reshape(len(amps), mesh.dim)

    def move(x):
        x = np.array(x, dtype=np.float64)
        r = np.sqrt(np.sum(x * x, axis=1))
        xh = x / r[:, None]
        w = np.clip((r_out - r) / (r_out - r_in), 0.0, 1.0)
        delta = np.zeros_like(r)
        for a, c in zip(amps, centers):
            c = c / np.sqrt(float(c @ c))
            th = np.arccos(np.clip(xh @ c, -1.0, 1.0))
            delta += a * np.exp(-th * th / (2.0 * sigma * sigma))
        return xh * (r + delta * w)[:, None]

    xyz = move(mesh.xyz)
    geo = None
    if mesh.elem_geo is not None:  # curved nodes move with the same field
        geo = move(mesh.elem_geo.reshape(-1, mesh.dim)).reshape(mesh.elem_geo.shape)
        for i, k in enumerate(node_of_vertex(mesh.dim)):
            geo[:, k] = xyz[mesh.elem_vert[:, i]]
    return Mesh(mesh.dim, xyz, mesh.elem_vert.copy(), mesh.bface_tag.copy(), mesh.name + "+bumps", geo)


def _rotations(dim: int):
    """The orientation-preserving symmetries of the reference square / cube
    (signed permutation matrices with determinant +1): 4 in 2D, 24 in 3D."""
    import itertools
    out = []
    for perm in itertools.permutations(range(dim)):
        for signs in itertools.product((1, -1), repeat=dim):
            S = np.zeros((dim, dim), dtype=np.int64)
            for r in range(dim):
                S[r, perm[r]] = signs[r]
            if round(np.linalg.det(S)) == 1:
                out.append(S)
    return out


def reorient(mesh: Mesh, seed: int) -> Mesh:
    """Same elements and geometry, new local reference frames: each element's
    local vertex list is re-labelled by a seeded random rotation S of the
    reference square / cube (xi_old = S xi_new), and its boundary tags follow
    the faces they belong to.  Shared faces then meet with every combination
    of axis swap and flips, which the structured generators never produce."""
    dim = mesh.dim
    rots = _rotations(dim)
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.integers(0, len(rots), size=mesh.n_elem)
    nc = 2 ** dim
    corners = np.array([[2 * ((k >> r) & 1) - 1 for r in range(dim)] for k in range(nc)], dtype=np.int64)
    index_of = {tuple(c): k for k, c in enumerate(corners)}
    ev = np.empty_like(mesh.elem_vert)
    tg = np.empty_like(mesh.bface_tag)
    geo = None if mesh.elem_geo is None else np.empty_like(mesh.elem_geo)
    refs = node_ref(dim)
    node_of = {tuple(c): k for k, c in enumerate(refs)}
    for e in range(mesh.n_elem):
        S = rots[pick[e]]
        for k in range(nc):
            ev[e, k] = mesh.elem_vert[e, index_of[tuple(S @ corners[k])]]
        if geo is not None:
            for k in range(3 ** dim):
                geo[e, k] = mesh.elem_geo[e, node_of[tuple(S @ refs[k])]]
        for rn in range(dim):
            r = int(np.nonzero(S[:, rn])[0][0])
            for s in (-1, 1):
                so = S[r, rn] * s
                tg[e, 2 * rn + (s > 0)] = mesh.bface_tag[e, 2 * r + (so > 0)]
    return Mesh(dim, mesh.xyz.copy(), ev, tg, mesh.name + f"+reoriented{seed}", geo)


def clip(mesh: Mesh, keep, tag: int = TAG_SYMMETRY) -> Mesh:
    """The elements with ``keep[e]`` true, in their order, with unused
    vertices dropped; every interior face whose neighbour is dropped becomes
    a boundary face tagged ``tag``.  Cutting a mirror-symmetric mesh along
    its plane of symmetry gives the half (or, cut twice, the quarter) domain
    of Section 5.2's sphere, whose cut faces are symmetry planes."""
    keep = np.asarray(keep, dtype=bool)
    dim, nf = mesh.dim, 2 * mesh.dim
    nc = 2 ** dim
    owners: dict = {}
    for e in range(mesh.n_elem):
        for lf in range(nf):
            if mesh.bface_tag[e, lf] != TAG_INTERIOR:
                continue
            r, s = divmod(lf, 2)
            key = frozenset(int(mesh.elem_vert[e, k]) for k in range(nc) if (k >> r) & 1 == s)
            owners.setdefault(key, []).append((e, lf))
    tg = mesh.bface_tag.copy()
    for pair in owners.values():
        if len(pair) != 2:
            raise ValueError("interior face without exactly one neighbour")
        (e1, l1), (e2, l2) = pair
        if keep[e1] and not keep[e2]:
            tg[e1, l1] = tag
        elif keep[e2] and not keep[e1]:
            tg[e2, l2] = tag
    ev = mesh.elem_vert[keep]
    used = np.unique(ev)
    new_id = np.full(mesh.n_vert, -1, dtype=np.int64)
    new_id[used] = np.arange(len(used))
    geo = None if mesh.elem_geo is None else mesh.elem_geo[keep].copy()
    return Mesh(dim, mesh.xyz[used].copy(), new_id[ev].astype(np.int32), tg[keep], mesh.name + "+clip", geo)
