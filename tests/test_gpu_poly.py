"""GPU parity of the tetrahedron / prism path (Cartesian P_p basis
orthonormalised by MGS, Section 3.2) against the FP64 oracle, through the
C ABI (eg_poly_*).

Tolerances.  Both sides compute in FP64; the library contracts to FMA,
evaluates the state from monomial coefficients a = S^T u and forms the
residual as S times monomial moments, while the oracle evaluates psi = S chi
at every point.  The two orders of summation differ by a few ulps times the
size of S (entries up to ~1e2 on these elements) and the cancellation
between volume and face terms, so residuals are compared at 1e-11 of their
largest entry and the set-up (S, centroids, extents, volumes) at 1e-12."""

import numpy as np
import pytest

import oracle
from eg_inputs import box_poly, sphere_poly
from tests.gpu_util import to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu


def _tagged(m, seed):
    """Boundary faces re-tagged at random among wall, far-field and symmetry."""
    rng = np.random.default_rng(seed)
    t = m.bface_tag.copy()
    b = t != 0
    t[b] = rng.choice(np.array([1, 2, 4], dtype=np.int8), size=int(b.sum()))
    m.bface_tag = t
    return m


def _state(O, p, seed, amp=0.03):
    """Free stream plus a seeded perturbation scaled by sqrt|E| / 4^deg."""
    rng = np.random.default_rng(seed)
    u = O.freestream(p)
    vol, _, _ = O.geometry()
    deg = np.sum(oracle.poly_monomials(p), axis=1)
    u = u + amp * rng.uniform(-1, 1, u.shape) * (np.sqrt(vol)[:, None, None] * 0.25 ** deg[None, None, :])
    assert np.all(np.isfinite(O.residual(p, u)))
    return u


def _relabel(m, seed):
    """The same elements with re-labelled local vertices: a seeded even
    permutation of every tetrahedron's four vertices (orientation kept), a
    seeded cyclic rotation of every prism's triangles; boundary tags follow
    their faces.  The collapsed volume rules follow the element's vertex
    order, so this changes the quadrature points (both sides alike)."""
    import itertools
    rng = np.random.default_rng(seed)
    even = [pp for pp in itertools.permutations(range(4))
            if sum(1 for i in range(4) for j in range(i + 1, 4) if pp[i] > pp[j]) % 2 == 0]
    ev, tg = m.elem_vert.copy(), m.bface_tag.copy()
    for e in range(m.n_elem):
        if m.elem_type[e] == 0:
            pp = even[rng.integers(len(even))]
            ev[e, :4] = m.elem_vert[e, list(pp)]
            # face k omits vertex k: the new face k omits old vertex pp[k]
            tg[e, :4] = [m.bface_tag[e, pp[k]] for k in range(4)]
        else:
            r = int(rng.integers(3))
            rot = [(a + r) % 3 for a in range(3)]
            ev[e, :6] = m.elem_vert[e, rot + [a + 3 for a in rot]]
            tg[e, 2:5] = [m.bface_tag[e, 2 + (a + r) % 3] for a in range(3)]
    m.elem_vert, m.bface_tag = ev, tg
    m.name += f"+relabel{seed}"
    return m


MESHES = [
    ("box3-mixed-skew", lambda: _tagged(box_poly(3, "mixed", tag=2, skew=0.15, seed=1), 11)),
    ("box2-tet-skew", lambda: _tagged(box_poly(2, "tet", tag=2, skew=0.2, seed=4), 12)),
    ("box2-prism", lambda: _tagged(box_poly(2, "prism", tag=2), 13)),
    ("sphere2-1p1t", lambda: sphere_poly(2, 1, 1)),
    ("one-hex-6tets", lambda: box_poly(1, "tet", tag=2)),
    ("box3-mixed-relabelled", lambda: _relabel(_tagged(box_poly(3, "mixed", tag=2, skew=0.15, seed=1), 11), 5)),
]


@pytest.mark.parametrize("name,make", MESHES, ids=[m[0] for m in MESHES])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_poly_residual_parity(name, make, flux, p):
    import paper_1807_01151_amd as P
    m = make()
    O = oracle.PolyOracle(m, 3, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    S = P.PolySolver(m, 3, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    u = _state(O, p, seed=100 + p)
    r_o = O.residual(p, u)
    r_g = to_host(S.residual(p, to_dev(u)))
    err = rel_err(r_g, r_o)
    print(f"{name} {flux} p={p}: residual rel err {err:.2e}", flush=True)
    assert err < 1e-11, err


def test_poly_setup_matches_oracle():
    import paper_1807_01151_amd as P
    m = _tagged(box_poly(3, "mixed", tag=2, skew=0.15, seed=1), 11)
    O = oracle.PolyOracle(m, 3)
    S = P.PolySolver(m, 3)
    Sg, xg, Lg, vg = S.basis()
    vo, xo, Lo = O.geometry()
    assert rel_err(Sg, O.basis_S()) < 1e-12
    assert rel_err(xg, xo) < 1e-13 and rel_err(Lg, Lo) < 1e-15 and rel_err(vg, vo) < 1e-13


def test_poly_freestream_and_levels():
    """The library's free stream is the oracle's, preserved at every level;
    a level-p residual uses the leading block of the p_max basis."""
    import paper_1807_01151_amd as P
    m = box_poly(3, "mixed", tag=2, skew=0.15, seed=1)
    O = oracle.PolyOracle(m, 3, alpha_deg=10.0, beta_deg=5.0)
    S = P.PolySolver(m, 3, alpha_deg=10.0, beta_deg=5.0)
    for p in range(4):
        uf = S.freestream(p)
        assert rel_err(to_host(uf), O.freestream(p)) < 1e-14
        assert np.abs(to_host(S.residual(p, uf))).max() < 1e-12


def test_poly_sphere_fullsize_parity():
    """The 13 824-element sphere shell (9216 tetrahedra, 4608 prisms) at
    p = 3, Roe flux, every element compared."""
    import paper_1807_01151_amd as P
    m = sphere_poly(8, 6, 4)
    O = oracle.PolyOracle(m, 3, alpha_deg=2.0, flux="roe")
    S = P.PolySolver(m, 3, alpha_deg=2.0, flux="roe")
    u = _state(O, 3, seed=7)
    r_o = O.residual(3, u)
    r_g = to_host(S.residual(3, to_dev(u)))
    err = rel_err(r_g, r_o)
    print(f"sphere 13824 p=3 roe: residual rel err {err:.2e}", flush=True)
    assert err < 1e-11, err


def test_poly_errors():
    import torch
    import paper_1807_01151_amd as P
    m = box_poly(2, "tet", tag=2)
    bad = box_poly(2, "tet", tag=2)
    bad.bface_tag = bad.bface_tag.copy()
    bad.bface_tag[bad.bface_tag == 2] = 0  # boundary faces claimed interior: unmatched
    with pytest.raises(P.EgError, match="EG_ERR_MESH"):
        P.PolySolver(bad, 1)
    with pytest.raises(P.EgError, match="EG_ERR_ARG"):
        P.PolySolver(m, 4)
    S = P.PolySolver(m, 2)
    with pytest.raises(ValueError):
        S.residual(3, S.empty(2))
    with pytest.raises(ValueError):
        S.residual(1, torch.zeros(m.n_elem, 5, 10, dtype=torch.float64, device="cuda"))
    u = S.freestream(1)
    with pytest.raises(ValueError):
        S.residual(1, u, out=u)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_poly_timestep_parity(p):
    import paper_1807_01151_amd as P
    m = _tagged(box_poly(3, "mixed", tag=2, skew=0.15, seed=1), 11)
    O = oracle.PolyOracle(m, 3, alpha_deg=8.0, beta_deg=-4.0)
    S = P.PolySolver(m, 3, alpha_deg=8.0, beta_deg=-4.0)
    u = _state(O, p, seed=40 + p, amp=0.1)
    d_o = O.timestep(p, 37.0, u)
    d_g = to_host(S.timestep(p, 37.0, to_dev(u)))
    assert rel_err(d_g, d_o) < 1e-13


@pytest.mark.parametrize("p", [1, 3])
def test_poly_rnorm_parity(p):
    import paper_1807_01151_amd as P
    m = sphere_poly(2, 1, 1)
    O = oracle.PolyOracle(m, 3, flux="roe")
    S = P.PolySolver(m, 3, flux="roe")
    u = _state(O, p, seed=60 + p)
    r_o = O.residual(p, u)
    rn_o = O.rnorm(p, r_o)
    rn_g = S.rnorm(p, S.residual(p, to_dev(u)))
    assert abs(rn_g - rn_o) < 1e-12 * rn_o, (rn_g, rn_o)


def test_poly_transfers_are_truncation_and_padding():
    """Restriction keeps the leading N_pc modes, prolongation adds into them
    (exact copies: bit-identical)."""
    import paper_1807_01151_amd as P
    m = box_poly(2, "mixed", tag=2)
    S = P.PolySolver(m, 3)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (m.n_elem, 5, 20))
    y = rng.uniform(-1, 1, (m.n_elem, 5, 4))
    for pc, nc in ((0, 1), (1, 4), (2, 10), (3, 20)):
        yc = to_host(S.restrict(3, pc, to_dev(x)))
        assert np.array_equal(yc, x[:, :, :nc])
    xd = to_dev(x)
    S.prolong_add(1, 3, to_dev(y), xd)
    ref = x.copy()
    ref[:, :, :4] += y
    assert np.array_equal(to_host(xd), ref)
    with pytest.raises(ValueError):
        S.prolong_add(1, 3, xd, xd)


def _oracle_block(O, p, u, e):
    """D_E by its definition: the complex-step derivative of the oracle's
    residual of element e with respect to e's own coefficients."""
    N = O.N(p)
    n = 5 * N
    D = np.zeros((n, n))
    h = 1e-30
    for c in range(n):
        v, j = divmod(c, N)
        uc = u.astype(complex)
        uc[e, v, j] += 1j * h
        D[:, c] = O.residual_complex(p, uc)[e].imag.reshape(-1) / h
    return D


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_poly_element_block_parity(p, flux):
    """Every entry of D_E for a tetrahedron and a prism with wall / far-field
    / symmetry faces and for interior elements of a skewed mixed mesh."""
    import paper_1807_01151_amd as P
    m = _tagged(box_poly(2, "mixed", tag=2, skew=0.15, seed=3), 21)
    O = oracle.PolyOracle(m, 3, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    S = P.PolySolver(m, 3, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    u = _state(O, p, seed=80 + p)
    Dg = to_host(S.element_block(p, to_dev(u)))
    tets = np.nonzero(m.elem_type == 0)[0]
    prisms = np.nonzero(m.elem_type == 1)[0]
    for e in (int(prisms[0]), int(prisms[-1]), int(tets[0]), int(tets[len(tets) // 2])):
        Do = _oracle_block(O, p, u, e)
        err = rel_err(Dg[e], Do)
        print(f"{flux} p={p} element {e} (type {m.elem_type[e]}): block rel err {err:.2e}", flush=True)
        assert err < 1e-11, (e, err)


def _side_tags(m):
    """Unit-box boundary faces by position: slip walls on y = 0, 1, symmetry
    planes on z = 0, 1 (the flow is nearly tangential to both), far field on
    x = 0, 1.  (Walls facing the free stream head-on make the element blocks
    locally unstable, and a large PRK step then leaves the physical states.)"""
    from eg_inputs import TET_FACES, PRISM_FACES
    t = m.bface_tag.copy()
    for e in range(m.n_elem):
        faces = TET_FACES if m.elem_type[e] == 0 else PRISM_FACES
        for lf, f in enumerate(faces):
            if t[e, lf] == 0:
                continue
            X = m.xyz[[m.elem_vert[e, k] for k in f]]
            if np.all(X[:, 1] == X[0, 1]) and X[0, 1] in (0.0, 1.0):
                t[e, lf] = 1
            elif np.all(X[:, 2] == X[0, 2]) and X[0, 2] in (0.0, 1.0):
                t[e, lf] = 4
            else:
                t[e, lf] = 2
    m.bface_tag = t
    return m


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_poly_prk_step_parity(p, flux):
    """One 4-stage PRK step (CFL 20, with a forcing) on a skewed mixed mesh
    with wall / far-field / symmetry faces: the update u - u^n against the
    oracle's at 1e-10 of its largest entry (LU solves of blocks with
    condition numbers up to ~1e4 on top of the residual's rounding)."""
    import paper_1807_01151_amd as P
    m = _side_tags(box_poly(2, "mixed", tag=2, skew=0.15, seed=3))
    O = oracle.PolyOracle(m, 3, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    S = P.PolySolver(m, 3, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    u = _state(O, p, seed=90 + p)
    f = 0.1 * O.residual(p, _state(O, p, seed=190 + p))
    uo, st = O.prk(p, 4, 20.0, u, f)
    assert st == 0
    ug = to_dev(u)
    S.prk_step(p, 4, 20.0, ug, to_dev(f))
    du_g, du_o = to_host(ug) - u, uo - u
    err = rel_err(du_g, du_o)
    print(f"{flux} p={p}: PRK update rel err {err:.2e}", flush=True)
    assert err < 1e-10, err


def test_poly_prk_sphere_shell():
    """Three PRK steps (s = 4, CFL 100) on the 13 824-element shell at p = 1,
    Roe flux, from a perturbed free stream: parity of the state with the
    oracle's three steps."""
    import paper_1807_01151_amd as P
    m = sphere_poly(8, 6, 4)
    O = oracle.PolyOracle(m, 1, flux="roe")
    S = P.PolySolver(m, 1, flux="roe")
    u = _state(O, 1, seed=5)
    uo = u.copy()
    for _ in range(3):
        uo, st = O.prk(1, 4, 100.0, uo)
        assert st == 0
    ug = to_dev(u)
    for _ in range(3):
        S.prk_step(1, 4, 100.0, ug)
    err = rel_err(to_host(ug) - u, uo - u)
    print(f"sphere p=1, 3 PRK steps: rel err {err:.2e}", flush=True)
    assert err < 1e-10, err


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_poly_exp1_parity(flux):
    """EXP1 on the level-0 state (p_max = 2 time steps, CFL 20, m = 30, with a
    forcing): the update against the oracle's (CGS2 on the device vs twice
    swept MGS in the oracle, equal in exact arithmetic) at 1e-10."""
    import paper_1807_01151_amd as P
    m = _side_tags(box_poly(2, "mixed", tag=2, skew=0.15, seed=3))
    O = oracle.PolyOracle(m, 2, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    S = P.PolySolver(m, 2, alpha_deg=8.0, beta_deg=-4.0, flux=flux)
    u0 = _state(O, 0, seed=31)
    f0 = 0.1 * O.residual(0, _state(O, 0, seed=32))
    uo, st = O.exp1(30, 20.0, u0, f0)
    assert st == 0
    ug = to_dev(u0)
    S.exp1_step(20.0, ug, to_dev(f0))
    err = rel_err(to_host(ug) - u0, uo - u0)
    print(f"{flux}: EXP1 update rel err {err:.2e}", flush=True)
    assert err < 1e-10, err


@pytest.mark.parametrize("p", [1, 2, 3])
def test_poly_vcycle_map_parity(p):
    """Three V-cycles (s = 4, m = 30, CFL ramp to 100) from the free stream on
    the 48-element tetrahedron / prism sphere shell, Roe flux: entry norms
    and states after every cycle against the oracle's cycle map."""
    import paper_1807_01151_amd as P
    m = sphere_poly(1, 1, 1)
    O = oracle.PolyOracle(m, p, flux="roe")
    S = P.PolySolver(m, p, flux="roe")
    uo = O.freestream(p)
    ug = S.freestream(p)
    r1 = 0.0
    for n in range(1, 4):
        u_prev = uo.copy()
        uo, rn_o, cfl_o, st = O.vcycle(uo, n, rref=r1)
        assert st == 0
        rn_g, cfl_g = S.vcycle(ug, n, rref=r1)
        if n == 1:
            r1 = rn_o
        assert abs(rn_g - rn_o) <= 1e-12 * rn_o and abs(cfl_g - cfl_o) <= 1e-12 * cfl_o
        err = rel_err(to_host(ug) - u_prev, uo - u_prev)
        print(f"p={p} cycle {n}: rn {rn_o:.3e}, update rel err {err:.2e}", flush=True)
        assert err < 1e-9, (n, err)
        ug = to_dev(uo)  # next cycle from the common state


def test_poly_solve_reaches_the_drop():
    """The eMG steady solve on the 192-element tetrahedron / prism sphere
    shell at p = 1 (Roe flux, wall on the body) reaches the 1e-10 drop on the
    device; the history and the converged state agree with the oracle's."""
    import paper_1807_01151_amd as P
    m = sphere_poly(2, 1, 1)
    O = oracle.PolyOracle(m, 1, flux="roe")
    S = P.PolySolver(m, 1, flux="roe")
    uo, h_o, st_o = O.solve(O.freestream(1), s=4, m=30, cfl_max=100.0, drop=1e-10, max_cycles=600)
    assert st_o == 0
    ug = S.freestream(1)
    h_g, st = S.solve_steady(ug, drop_tol=1e-10, max_cycles=600)
    print(f"sphere p=1: oracle {len(h_o) - 1} cycles, device {len(h_g) - 1} cycles", flush=True)
    assert st == 0
    assert abs(len(h_g) - len(h_o)) <= 2
    k = min(len(h_g), len(h_o), 40)
    assert np.allclose(h_g[:k], h_o[:k], rtol=1e-6)
    assert rel_err(to_host(ug), uo) < 1e-8


def test_poly_prk_relabelled_mesh():
    """A PRK step and a V-cycle on a mesh with re-labelled local vertices
    (p = 2, Roe) against the oracle."""
    import paper_1807_01151_amd as P
    m = _relabel(_side_tags(box_poly(2, "mixed", tag=2, skew=0.15, seed=3)), 9)
    O = oracle.PolyOracle(m, 2, alpha_deg=8.0, beta_deg=-4.0, flux="roe")
    S = P.PolySolver(m, 2, alpha_deg=8.0, beta_deg=-4.0, flux="roe")
    u = _state(O, 2, seed=95)
    uo, st = O.prk(2, 4, 20.0, u)
    assert st == 0
    ug = to_dev(u)
    S.prk_step(2, 4, 20.0, ug)
    assert rel_err(to_host(ug) - u, uo - u) < 1e-10
    uo2, rn_o, _, st = O.vcycle(u, 1)
    assert st == 0
    ug = to_dev(u)
    rn_g, _ = S.vcycle(ug, 1)
    assert abs(rn_g - rn_o) <= 1e-12 * rn_o
    assert rel_err(to_host(ug) - u, uo2 - u) < 1e-9


def test_poly_vcycle_fullsize_map():
    """Two V-cycles on the 13 824-element shell at p = 1 (Roe): entry norms
    and states against the oracle's cycle map."""
    import paper_1807_01151_amd as P
    m = sphere_poly(8, 6, 4)
    O = oracle.PolyOracle(m, 1, flux="roe")
    S = P.PolySolver(m, 1, flux="roe")
    uo = O.freestream(1)
    ug = S.freestream(1)
    r1 = 0.0
    for n in (1, 2):
        u_prev = uo.copy()
        uo, rn_o, _, st = O.vcycle(uo, n, rref=r1)
        assert st == 0
        rn_g, _ = S.vcycle(ug, n, rref=r1)
        if n == 1:
            r1 = rn_o
        assert abs(rn_g - rn_o) <= 1e-12 * rn_o
        err = rel_err(to_host(ug) - u_prev, uo - u_prev)
        print(f"full shell p=1 cycle {n}: update rel err {err:.2e}", flush=True)
        assert err < 1e-9, (n, err)
        ug = to_dev(uo)
