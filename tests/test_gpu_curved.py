"""Quadratic curved elements on the GPU (nine-node biquadratic quads, the
cylinder grid of Section 5.1; 27-node triquadratic hexes, the sphere grid of
Section 5.2): mesh checks at the C ABI, the straight special case,
free-stream preservation, curved meshes inside a batch, and a curved steady
solve against the oracle.  Residual, time step, element blocks, PRK,
EXP1, V-cycle, J v, drag, adjoint and mixed precision on curved meshes are
compared with the oracle in the parity tests' curved rows."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell, straight_nodes, Mesh, TAG_FARFIELD
from tests.gpu_util import perturbed, to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu


def _solver(mesh, p, **kw):
    import paper_1807_01151_amd as P
    return P.Solver(mesh, p, **kw)


def test_curved_mesh_checks_at_the_abi():
    """Corner nodes off their vertices and faces whose two sides disagree on
    a face node (EG_ERR_MESH) are refused by eg_init_mesh (nodes inside an
    element or on a boundary face may move freely); node arrays of the wrong
    shape are refused by the binding."""
    import paper_1807_01151_amd as P
    m = ogrid(8, 2, curved=True)
    bad = m.elem_geo.copy()
    bad[3, 0, 0] += 1e-6
    with pytest.raises(P.EgError, match="corner") as ex:
        _solver(Mesh(2, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)
    assert ex.value.status == 2
    bad = m.elem_geo.copy()
    bad[3, 7, 1] += 1e-6
    with pytest.raises(P.EgError, match="non-conforming curved") as ex:
        _solver(Mesh(2, m.xyz, m.elem_vert, m.bface_tag, "", bad), 1)
    assert ex.value.status == 2
    s = cubed_sphere_shell(2, 1, curved=True)
    bad = s.elem_geo.copy()
    bad[5, 13, 2] += 1e-6  # the centre node: no face, so no check can see it
    _solver(Mesh(3, s.xyz, s.elem_vert, s.bface_tag, "", bad), 1)
    bad = s.elem_geo.copy()
    bad[5, 12, 0] += 1e-6  # the centre node of the inner face (body wall): no neighbour
    _solver(Mesh(3, s.xyz, s.elem_vert, s.bface_tag, "", bad), 1)
    bad = s.elem_geo.copy()
    bad[5, 4 + 9 * 2, 1] += 1e-6  # centre node of face 5 (zeta = +1), an interior face
    with pytest.raises(P.EgError, match="non-conforming curved") as ex:
        _solver(Mesh(3, s.xyz, s.elem_vert, s.bface_tag, "", bad), 1)
    assert ex.value.status == 2
    with pytest.raises(ValueError, match="elem_geo must have shape"):
        _solver(Mesh(3, s.xyz, s.elem_vert, s.bface_tag, "", np.zeros((s.n_elem, 9, 2))), 1)


def test_straight_nodes_match_vertex_only_mesh():
    """Nine nodes at the bilinear positions give the residual of the same
    mesh passed without nodes (the library derives those nodes itself)."""
    m = ogrid(16, 6)
    O = oracle.Oracle(m, 3, alpha_deg=2.0)
    u = to_dev(perturbed(O, 3, 41))
    r1 = to_host(_solver(m, 3, alpha_deg=2.0).residual(3, u))
    m9 = Mesh(2, m.xyz, m.elem_vert, m.bface_tag, "", straight_nodes(m))
    r2 = to_host(_solver(m9, 3, alpha_deg=2.0).residual(3, u))
    assert rel_err(r2, r1) < 1e-14


def test_straight_nodes_match_vertex_only_hexes():
    """27 nodes at the trilinear positions (the triquadratic instantiations)
    give the residual, PRK step and drag of the same shell passed without
    nodes (the trilinear ones)."""
    m = cubed_sphere_shell(2, 2)
    O = oracle.Oracle(m, 2, alpha_deg=2.0)
    u = perturbed(O, 2, 42)
    S1 = _solver(m, 2, alpha_deg=2.0)
    S2 = _solver(Mesh(3, m.xyz, m.elem_vert, m.bface_tag, "", straight_nodes(m)), 2, alpha_deg=2.0)
    assert rel_err(to_host(S2.residual(2, to_dev(u))), to_host(S1.residual(2, to_dev(u)))) < 1e-13
    u1, u2 = to_dev(u), to_dev(u)
    S1.prk_step(2, 10.0, u1)
    S2.prk_step(2, 10.0, u2)
    assert rel_err(to_host(u2) - u, to_host(u1) - u) < 1e-11
    assert abs(S2.drag(to_dev(u)) - S1.drag(to_dev(u))) <= 1e-13 * abs(S1.drag(to_dev(u)))


@pytest.mark.parametrize("mesh,p", [(ogrid(12, 5, inner=TAG_FARFIELD, curved=True), 1),
                                    (ogrid(12, 5, inner=TAG_FARFIELD, curved=True), 4),
                                    (cubed_sphere_shell(2, 2, inner=TAG_FARFIELD, curved=True), 1),
                                    (cubed_sphere_shell(2, 2, inner=TAG_FARFIELD, curved=True), 3)])
def test_freestream_preservation_curved_gpu(mesh, p):
    S = _solver(mesh, p, alpha_deg=4.0)
    r = to_host(S.residual(p, S.freestream(p)))
    assert np.max(np.abs(r)) < 1e-13 * max(1.0, float(np.max(np.abs(to_host(S.freestream(p))))))


@pytest.mark.parametrize("dim", [2, 3])
def test_batch_with_curved_and_straight_meshes(dim):
    """A batch of a curved, a straight and another curved grid: each solve's
    slice of the batch residual equals that solve's own residual bitwise
    (the straight one joins the batch through its multilinear nodes)."""
    import paper_1807_01151_amd as P
    if dim == 2:
        meshes = [ogrid(12, 4, curved=True), ogrid(10, 3), ogrid(16, 5, curved=True)]
    else:
        meshes = [cubed_sphere_shell(2, 2, curved=True), cubed_sphere_shell(2, 1),
                  cubed_sphere_shell(3, 2, curved=True)]
    machs, alphas, p = [0.3, 0.2, 0.35], [0.0, 3.0, -2.0], 2
    B = P.BatchSolver(meshes, p, machs, alphas)
    u = to_host(B.freestream(p))
    rng = np.random.default_rng(401)
    u[:, :, 1:] += 1e-3 * rng.uniform(-1, 1, u[:, :, 1:].shape)
    u = to_dev(u)
    r = B.residual(p, u)
    for i, (uv, rv) in enumerate(zip(B.views(u), B.views(r))):
        S = P.Solver(meshes[i], p, mach=machs[i], alpha_deg=alphas[i])
        r1 = to_host(S.residual(p, uv.contiguous()))
        if dim == 3 and meshes[i].elem_geo is None:
            # alone it takes the trilinear kernels, in the batch the triquadratic ones
            assert rel_err(to_host(rv), r1) < 1e-12, i
        else:
            assert np.array_equal(r1, to_host(rv)), i


def test_curved_c1_solve_against_oracle():
    """The c1 solve (O-grid 24 x 12, p = 1, s = 4, CFL_max 100, m = 30) on
    the curved mesh: the first 12 cycles of the history agree with the
    oracle's to 1e-12 r_1, the GPU reaches the 1e-10 drop, and the oracle's
    residual of the GPU's converged state is at the drop."""
    mesh = ogrid(24, 12, curved=True)
    O = oracle.Oracle(mesh, 1)
    S = _solver(mesh, 1, rk_stages=4, cfl_max=100.0, krylov_m=30)
    _, h_o, _ = O.solve(O.freestream(1), s=4, m=30, cfl_max=100.0, drop=1e-10, max_cycles=12)
    ud = S.freestream(1)
    h_g, st = S.solve_steady(ud, drop_tol=1e-10, max_cycles=4000)
    print("curved c1 cycles", len(h_g) - 1, "status", st, flush=True)
    assert st == 0
    dev = np.abs(h_g[:13] - h_o[:13]) / h_o[0]
    assert dev.max() < 1e-12, dev.max()
    assert O.rnorm(1, O.residual(1, to_host(ud))) <= 2e-10 * h_o[0]
