"""Pins of the oracle's tetrahedra / prisms with the Cartesian P_p basis
(Section 3.2, eqs. (basis2) and (basis)) against facts fixed outside it:
closed-form simplex integrals, orthonormality under an independent, finer
rule with the basis evaluated here in numpy, finite-volume sums at p = 0,
free-stream preservation, conservation and the manufactured-solution rate."""

import math

import numpy as np
import pytest

import oracle
from eg_inputs import box_poly, sphere_poly, TET, PRISM, TET_FACES, PRISM_FACES


def _bary_integral(a):
    """int over the unit-volume-normalised simplex of prod lambda_k^a_k times
    6 (i.e. divided by 6 |T|): a0! a1! a2! a3! 3! / (|a| + 3)!."""
    num = math.prod(math.factorial(k) for k in a) * math.factorial(3)
    return num / math.factorial(sum(a) + 3)


def _exponents(n_var, deg):
    out = []

    def rec(prefix, left, k):
        if k == n_var - 1:
            out.append(prefix + [left])
            return
        for t in range(left + 1):
            rec(prefix + [t], left - t, k + 1)

    for d in range(deg + 1):
        rec([], d, 0)
    return out


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_tet_rule_exact_to_2p_plus_1(p):
    """The (p+2)-point collapsed rule integrates every polynomial of degree
    <= 2p+1 exactly on a skewed tetrahedron (barycentric monomials against
    the Dirichlet closed form)."""
    m = box_poly(2, "tet", skew=0.2, seed=4)
    O = oracle.PolyOracle(m, p)
    vol, _, _ = O.geometry()
    for e in (0, 7, 31):
        X, W = O.vol_rule(e, p + 2)
        V = m.xyz[m.elem_vert[e, :4]]
        # barycentric coordinates of the points
        A = np.vstack([V.T, np.ones(4)])
        lam = np.linalg.solve(A, np.vstack([X.T, np.ones(len(W))]))
        v6 = abs(np.linalg.det(np.stack([V[1] - V[0], V[2] - V[0], V[3] - V[0]])))
        assert abs(vol[e] - v6 / 6) < 1e-14 * v6
        for a in _exponents(4, 2 * p + 1):
            got = float(np.sum(W * np.prod(lam ** np.array(a)[:, None], axis=0)))
            assert abs(got - v6 * _bary_integral(a) / 6.0) < 1e-13 * v6, (e, a)


@pytest.mark.parametrize("p", [0, 2, 3])
def test_prism_rule_exact_on_right_prisms(p):
    """On the right prisms of an unskewed box the rule integrates
    x^a y^b z^c exactly for a + b <= 2p+2 (triangle part) and c <= 2p+3."""
    m = box_poly(2, "prism", lo=-0.3, hi=0.9)
    O = oracle.PolyOracle(m, p)
    for e in (0, 5, 11):
        X, W = O.vol_rule(e, p + 2)
        V = m.xyz[m.elem_vert[e, :6]]
        tri = V[:3, :2]
        z0, z1 = V[0, 2], V[3, 2]
        area = 0.5 * abs(np.linalg.det(np.stack([tri[1] - tri[0], tri[2] - tri[0]])))
        A = np.vstack([tri.T, np.ones(3)])
        lam = np.linalg.solve(A, np.vstack([X[:, :2].T, np.ones(len(W))]))
        for a in _exponents(3, 2 * p + 2):
            for c in range(2 * p + 4):
                tri_exact = 2 * area * math.prod(math.factorial(k) for k in a) / math.factorial(sum(a) + 2)
                z_exact = (z1 ** (c + 1) - z0 ** (c + 1)) / (c + 1)
                got = float(np.sum(W * np.prod(lam ** np.array(a)[:, None], axis=0) * X[:, 2] ** c))
                assert abs(got - tri_exact * z_exact) < 1e-13 * max(1.0, abs(tri_exact * z_exact)), (e, a, c)


def _psi_numpy(S, xc, L, mono, X):
    Xs = (X - xc) / L
    chi = np.prod(Xs[:, None, :] ** mono[None, :, :], axis=2)
    return chi @ S.T


@pytest.mark.parametrize("kind", ["tet", "prism", "mixed"])
def test_basis_orthonormal_hierarchical(kind):
    """psi = S chi evaluated here from S, xc and L is orthonormal under a
    finer rule (exact on affine elements); S is lower triangular with a
    positive diagonal (so psi_1..psi_N span P_p), xc is the centroid and L
    the half extents of the vertices; the p_max = 2 basis is the leading
    block of the p_max = 3 basis (hierarchy)."""
    m = box_poly(2, kind, skew=0.0 if kind != "tet" else 0.2, seed=2, lo=-1.0, hi=2.0)
    O3 = oracle.PolyOracle(m, 3)
    O2 = oracle.PolyOracle(m, 2)
    S3, S2 = O3.basis_S(), O2.basis_S()
    vol, xc, L = O3.geometry()
    mono = oracle.poly_monomials(3)
    assert np.array_equal(mono[:10], oracle.poly_monomials(2))
    assert sorted(map(tuple, mono)) == sorted((a, b, c) for a in range(4) for b in range(4) for c in range(4)
                                              if a + b + c <= 3)
    assert list(np.sum(mono, axis=1)) == sorted(np.sum(mono, axis=1))
    for e in range(m.n_elem):
        nv = 4 if m.elem_type[e] == TET else 6
        V = m.xyz[m.elem_vert[e, :nv]]
        assert np.allclose(L[e], 0.5 * (V.max(0) - V.min(0)), rtol=0, atol=1e-15)
        if m.elem_type[e] == TET:
            assert np.allclose(xc[e], V.mean(0), rtol=0, atol=1e-14)
        assert np.allclose(np.triu(S3[e], 1), 0.0)
        assert np.all(np.diag(S3[e]) > 0)
        assert np.allclose(S3[e][:10, :10], S2[e], rtol=1e-12, atol=1e-12 * np.abs(S2[e]).max())
    for e in (0, m.n_elem // 2, m.n_elem - 1):
        X, W = O3.vol_rule(e, 7)
        psi = _psi_numpy(S3[e], xc[e], L[e], mono, X)
        M = (psi * W[:, None]).T @ psi
        assert np.abs(M - np.eye(20)).max() < 1e-11, (e, np.abs(M - np.eye(20)).max())
        # the oracle's own evaluation agrees with this one
        ps, _ = O3.psi(e, 3, X[3])
        assert np.allclose(ps, psi[3], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_freestream_preserved(p, flux):
    m = box_poly(3, "mixed", tag=2, skew=0.15, seed=1)
    O = oracle.PolyOracle(m, p, alpha_deg=10.0, beta_deg=5.0, flux=flux)
    r = O.residual(p, O.freestream(p))
    assert np.abs(r).max() < 1e-13


def _face_table(m):
    """(e, lf) -> neighbour, from the vertex sets (built here, not by the oracle)."""
    own = {}
    for e in range(m.n_elem):
        fl = TET_FACES if m.elem_type[e] == TET else PRISM_FACES
        for lf, f in enumerate(fl):
            own.setdefault(frozenset(int(m.elem_vert[e, k]) for k in f), []).append((e, lf))
    nb = {}
    for l in own.values():
        if len(l) == 2:
            nb[l[0]] = l[1][0]
            nb[l[1]] = l[0][0]
    return nb


@pytest.mark.parametrize("kind,skew", [("tet", 0.2), ("mixed", 0.0)])
def test_p0_is_the_finite_volume_sum(kind, skew):
    """At p = 0 (psi_0 = |E|^-1/2, no volume term) the residual is
    -|E|^-1/2 sum_faces A_f F~(U_E, U_nb; n_f) on planar faces; areas,
    normals and neighbours are computed here from the vertices."""
    m = box_poly(3, kind, tag=2, skew=skew, seed=5)
    tags = m.bface_tag.copy()
    tags[tags == 2] = np.where(np.arange(np.sum(tags == 2)) % 3 == 0, 1, 2).astype(np.int8)
    m.bface_tag = tags
    O = oracle.PolyOracle(m, 0, alpha_deg=7.0, beta_deg=-3.0)
    H = oracle.Oracle(__import__("eg_inputs").box(3, 1, tag=2), 0, alpha_deg=7.0, beta_deg=-3.0)
    rng = np.random.default_rng(9)
    u = O.freestream(0) * (1.0 + 0.05 * rng.uniform(-1, 1, (m.n_elem, 5, 1)))
    r = O.residual(0, u)
    vol, _, _ = O.geometry()
    nb = _face_table(m)
    ref = np.zeros_like(r)
    for e in range(m.n_elem):
        Ue = u[e, :, 0] / math.sqrt(vol[e])
        nve = 4 if m.elem_type[e] == TET else 6
        ce = m.xyz[m.elem_vert[e, :nve]].mean(0)
        fl = TET_FACES if m.elem_type[e] == TET else PRISM_FACES
        for lf, f in enumerate(fl):
            P = m.xyz[[m.elem_vert[e, k] for k in f]]
            if len(f) == 3:
                nvec = 0.5 * np.cross(P[1] - P[0], P[2] - P[0])
            else:
                nvec = 0.5 * np.cross(P[2] - P[0], P[3] - P[1])
            A = np.linalg.norm(nvec)
            n = nvec / A
            if n @ (P.mean(0) - ce) < 0:
                n = -n
            if (e, lf) in nb:
                o = nb[(e, lf)]
                Uo = u[o, :, 0] / math.sqrt(vol[o])
            else:
                Uo = H.ghost(int(m.bface_tag[e, lf]), Ue, n, P.mean(0))
            ref[e, :, 0] -= A * oracle.rusanov(3, 1.4, Ue, Uo, n) / math.sqrt(vol[e])
    assert np.abs(r - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2])
def test_conservation_closed_walls(p):
    """All slip walls: the mass and energy residuals tested with the constant
    1 = |E|^1/2 psi_0 sum to zero over the mesh (interior fluxes cancel, the
    wall carries no mass or energy)."""
    m = box_poly(3, "mixed", tag=1, skew=0.1, seed=3)
    O = oracle.PolyOracle(m, p)
    vol, _, _ = O.geometry()
    rng = np.random.default_rng(1)
    u = O.freestream(p) + 0.02 * rng.uniform(-1, 1, (m.n_elem, 5, O.N(p))) * np.sqrt(vol)[:, None, None]
    r = O.residual(p, u)
    for v in (0, 4):
        s = float(np.sum(np.sqrt(vol) * r[:, v, 0]))
        assert abs(s) < 1e-13 * np.abs(r[:, v, 0]).sum(), (v, s)
    assert abs(float(np.sum(np.sqrt(vol) * r[:, 1, 0]))) > 1e-6  # pressure acts on the walls


def test_translation_invariance():
    """The basis is centred on each element: moving the mesh leaves R unchanged."""
    m = box_poly(2, "mixed", tag=2, skew=0.1, seed=6)
    O = oracle.PolyOracle(m, 2, alpha_deg=3.0)
    rng = np.random.default_rng(2)
    u = O.freestream(2) * (1 + 0.05 * rng.uniform(-1, 1, (m.n_elem, 5, 10)))
    r = O.residual(2, u)
    m2 = box_poly(2, "mixed", tag=2, skew=0.1, seed=6)
    m2.xyz = m2.xyz + np.array([3.0, -7.0, 11.0])
    r2 = oracle.PolyOracle(m2, 2, alpha_deg=3.0).residual(2, u)
    assert np.abs(r - r2).max() < 1e-11 * np.abs(r).max()


@pytest.mark.parametrize("p", [1, 2])
def test_mms_truncation_rate(p):
    """Manufactured solution with the exact-state ghost: the residual of its
    projection plus the source, ||R(Pi u_m) + f||, falls at rate >= p - 0.5
    with h (expected p).  A dropped term, a wrong sign or a wrong normal
    leaves an O(1) or O(1/h) defect."""
    errs = []
    for n in (2, 4):
        m = box_poly(n, "mixed", tag=3)
        O = oracle.PolyOracle(m, p)
        u = O.mms_project(p)
        f = O.mms_forcing(p)
        errs.append(np.linalg.norm(O.residual(p, u) + f))
    rate = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert rate >= p - 0.5, (errs, rate)


def test_complex_step_matches_central_difference():
    """The residual is analytic in u away from flux switches: the complex
    step of R along a direction matches a central difference."""
    m = box_poly(2, "tet", tag=2, skew=0.1, seed=8)
    O = oracle.PolyOracle(m, 1, mach=0.5, alpha_deg=30.0, beta_deg=20.0)
    rng = np.random.default_rng(3)
    u = O.freestream(1) * (1 + 0.03 * rng.uniform(-1, 1, (m.n_elem, 5, 4)))
    dv = rng.uniform(-1, 1, u.shape)
    h = 1e-30
    dcs = O.residual_complex(1, u + 1j * h * dv).imag / h
    eps = 1e-6
    dfd = (O.residual(1, u + eps * dv) - O.residual(1, u - eps * dv)) / (2 * eps)
    assert np.abs(dcs - dfd).max() < 1e-7 * np.abs(dcs).max()


def test_sphere_shell_counts_and_freestream():
    """The tetrahedron / prism sphere shell: element counts, closed surface
    (free stream preserved with wall and far-field ghosts at p = 1 is not
    exact, so far-field on both spheres here)."""
    m = sphere_poly(4, 2, 2)
    assert m.counts() == (2 * 36 * 16, 2 * 12 * 16)
    m.bface_tag[m.bface_tag == 1] = 2
    O = oracle.PolyOracle(m, 1, alpha_deg=4.0)
    assert np.abs(O.residual(1, O.freestream(1))).max() < 1e-12


def _numpy_volume_surface(m):
    """|E| and |dE| from the vertices (planar faces; straight prisms of an
    unskewed box are right prisms)."""
    vol, surf = np.zeros(m.n_elem), np.zeros(m.n_elem)
    for e in range(m.n_elem):
        X = m.xyz[m.elem_vert[e, :4 if m.elem_type[e] == TET else 6]]
        if m.elem_type[e] == TET:
            vol[e] = abs(np.linalg.det(np.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]]))) / 6.0
        else:
            vol[e] = 0.5 * np.linalg.norm(np.cross(X[1] - X[0], X[2] - X[0])) * abs(X[3, 2] - X[0, 2])
        for f in (TET_FACES if m.elem_type[e] == TET else PRISM_FACES):
            P = X[list(f)]
            if len(f) == 3:
                surf[e] += 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
            else:
                surf[e] += 0.5 * np.linalg.norm(np.cross(P[2] - P[0], P[3] - P[1]))
    return vol, surf


@pytest.mark.parametrize("kind,skew", [("tet", 0.2), ("mixed", 0.0)])
def test_timestep_length_scale_and_free_stream(kind, skew):
    """h_E = 6 |E| / |dE| from numpy volumes and face areas; on the free stream
    (rho = 1, c = 1) dtau_E = CFL h_E / ((2p+1)(Ma + 1))."""
    m = box_poly(3, kind, tag=2, skew=skew, seed=5)
    O = oracle.PolyOracle(m, 3, mach=0.3, alpha_deg=20.0, beta_deg=10.0)
    vol, surf = _numpy_volume_surface(m)
    vo, _, _ = O.geometry()
    so, ho = O.surface()
    assert np.allclose(vo, vol, rtol=1e-13) and np.allclose(so, surf, rtol=1e-13)
    assert np.allclose(ho, 6.0 * vol / surf, rtol=1e-13)
    for p in (0, 2, 3):
        dt = O.timestep(p, 7.0, O.freestream(p))
        assert np.allclose(dt, 7.0 * ho / ((2 * p + 1) * 1.3), rtol=1e-13)


def test_rnorm_definition():
    """(1/|Omega|) (sum of squared density coefficients)^(1/2), |Omega| = 1
    for the unit box."""
    m = box_poly(2, "mixed", tag=2)
    O = oracle.PolyOracle(m, 2)
    r = np.random.default_rng(4).uniform(-1, 1, (m.n_elem, 5, 10))
    assert abs(O.rnorm(2, r) - math.sqrt(np.sum(r[:, 0, :] ** 2)) / 1.0) < 1e-13 * math.sqrt(np.sum(r[:, 0, :] ** 2))


def _global_block(O, p, u, e):
    """D_E from the complex step of the whole-mesh residual (only element e
    perturbed): the definition, through a code path other than the
    element-local one that the oracle's blocks use."""
    N = O.N(p)
    n = 5 * N
    D = np.zeros((n, n))
    for c in range(n):
        v, j = divmod(c, N)
        uc = u.astype(complex)
        uc[e, v, j] += 1e-30j
        D[:, c] = O.residual_complex(p, uc)[e].imag.reshape(-1) / 1e-30
    return D


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("p", [1, 2])
def test_element_blocks_match_global_derivative(p, flux):
    m = box_poly(2, "mixed", tag=2, skew=0.15, seed=3)
    t = m.bface_tag.copy()
    t[t == 2] = np.where(np.arange(np.sum(t == 2)) % 3 == 0, 1, np.where(np.arange(np.sum(t == 2)) % 3 == 1, 4, 2))
    m.bface_tag = t
    O = oracle.PolyOracle(m, p, alpha_deg=8.0, flux=flux)
    rng = np.random.default_rng(5)
    vol, _, _ = O.geometry()
    u = O.freestream(p) + 0.02 * rng.uniform(-1, 1, (m.n_elem, 5, O.N(p))) * np.sqrt(vol)[:, None, None]
    D = O.element_blocks(p, u)
    for e in (0, 7, m.n_elem - 1):
        ref = _global_block(O, p, u, e)
        assert np.abs(D[e] - ref).max() < 1e-12 * np.abs(ref).max(), e


def test_prk_step_solves_the_block_systems_and_keeps_the_free_stream():
    """One stage: (I/dtau - D_E)(u^1 - u^n)_E = R_E(u^n) for every element
    (checked here with numpy on the oracle's blocks and time steps); s stages
    on the free stream leave it unchanged."""
    m = box_poly(2, "mixed", tag=2, skew=0.1, seed=6)
    O = oracle.PolyOracle(m, 2, alpha_deg=5.0, flux="roe")
    rng = np.random.default_rng(8)
    vol, _, _ = O.geometry()
    u = O.freestream(2) + 0.02 * rng.uniform(-1, 1, (m.n_elem, 5, 10)) * np.sqrt(vol)[:, None, None]
    u1, st = O.prk(2, 1, 20.0, u)
    assert st == 0
    D = O.element_blocks(2, u)
    dt = O.timestep(2, 20.0, u)
    R = O.residual(2, u)
    for e in range(m.n_elem):
        Pm = np.eye(50) / dt[e] - D[e]
        lhs = Pm @ (u1[e] - u[e]).reshape(-1)
        assert np.allclose(lhs, R[e].reshape(-1), rtol=1e-10, atol=1e-12 * np.abs(R).max())
    uf = O.freestream(2)
    u4, st = O.prk(2, 4, 100.0, uf)
    assert st == 0 and np.abs(u4 - uf).max() < 1e-13


def test_exp1_exhausted_krylov_equals_dense_phi1():
    """With m = K (the whole p = 0 space) the Krylov EXP1 is exact:
    u0 + phi_1(A) b with A = T J_0, b = T R_0, J_0 assembled here column by
    column from the complex-step residual, T = diag((p_max+1) dtau_E), and
    phi_1(A) b the last column of expm([[A, b], [0, 0]]) (scipy)."""
    import scipy.linalg
    m = box_poly(1, "tet", tag=2, skew=0.0)
    m.bface_tag[0, 0] = 1 if m.bface_tag[0, 0] else m.bface_tag[0, 0]
    O = oracle.PolyOracle(m, 2, alpha_deg=6.0, flux="roe")
    rng = np.random.default_rng(12)
    vol, _, _ = O.geometry()
    u0 = O.freestream(0) * (1.0 + 0.02 * rng.uniform(-1, 1, (m.n_elem, 5, 1)))
    K = m.n_elem * 5
    J = np.zeros((K, K))
    for c in range(K):
        uc = u0.astype(complex).reshape(-1)
        uc[c] += 1e-30j
        J[:, c] = O.residual_complex(0, uc.reshape(u0.shape)).imag.reshape(-1) / 1e-30
    dt = 3.0 * O.timestep(2, 40.0, np.concatenate([u0, np.zeros((m.n_elem, 5, 9))], axis=2))
    T = np.repeat(dt, 5)
    A = T[:, None] * J
    b = T * O.residual(0, u0).reshape(-1)
    Z = np.zeros((K + 1, K + 1))
    Z[:K, :K] = A
    Z[:K, K] = b
    ref = u0.reshape(-1) + scipy.linalg.expm(Z)[:K, K]
    got, st = O.exp1(K, 40.0, u0)
    assert st == 0
    assert np.abs(got.reshape(-1) - ref).max() < 1e-9 * np.abs(ref - u0.reshape(-1)).max()


def test_vcycle_free_stream_fixed_point_and_sphere_convergence():
    """The free stream is a fixed point of the V-cycle with far-field
    boundaries; on the smallest tetrahedron / prism sphere shell (wall inside)
    the eMG solve reaches the 1e-10 drop at p = 1."""
    m = box_poly(2, "mixed", tag=2, skew=0.1, seed=2)
    O = oracle.PolyOracle(m, 2, alpha_deg=4.0)
    u = O.freestream(2)
    u1, rn, cfl, st = O.vcycle(u, 1)
    assert st == 0 and np.abs(u1 - u).max() < 1e-13
    ms = sphere_poly(1, 1, 1)
    Os = oracle.PolyOracle(ms, 1, flux="roe")
    _, hist, st = Os.solve(Os.freestream(1), s=4, m=30, cfl_max=100.0, drop=1e-10, max_cycles=600)
    assert st == 0, (st, hist[-1] / hist[0], len(hist))
