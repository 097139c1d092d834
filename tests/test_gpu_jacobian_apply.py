"""eg_jacobian_apply, the matrix-free (dR_p/du)(u) v of Section 3.3, eqs.
(jac1) and (jac2), against the oracle's assembled sparse Jacobian (its
blocks pinned to complex-step differentiation of the residual) at every
level, and the dot-product test <w, J v> = <J^T w, v> with the library's
transposed product eg_adjoint_apply.  FP64 on both sides; the sums differ
in order and the GPU contracts to FMA, so 1e-12 of the largest entry."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell, box, reorient, TAG_FARFIELD
from tests.gpu_util import perturbed, to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu

CASES = [
    ("ogrid12x4-p3", ogrid(12, 4), 3, 3.0, "rusanov"),
    ("ogrid10x3-p4-reoriented", reorient(ogrid(10, 3), 4), 4, -2.0, "rusanov"),
    ("box2d-far-p2", box(2, 4, skew=0.2, seed=2, tag=TAG_FARFIELD), 2, 7.0, "rusanov"),
    ("sphere6x2x2x2-p2-reoriented", reorient(cubed_sphere_shell(2, 2), 9), 2, 2.0, "rusanov"),
    ("ogrid12x4-p3-roe", ogrid(12, 4), 3, 3.0, "roe"),
    ("sphere6x2x2x2-p2-roe", cubed_sphere_shell(2, 2), 2, 2.0, "roe"),
    ("sphere6x2x2x2-p3", cubed_sphere_shell(2, 2), 3, 2.0, "rusanov"),
    ("ogrid12x4c-p3-curved-reoriented", reorient(ogrid(12, 4, curved=True), 6), 3, 3.0, "roe"),
    ("sphere6x2x2x2c-p2-curved-reoriented", reorient(cubed_sphere_shell(2, 2, curved=True), 7), 2, 2.0, "rusanov"),
]


@pytest.mark.parametrize("name,mesh,p,alpha,flux", CASES, ids=[c[0] for c in CASES])
def test_jacobian_apply_parity(name, mesh, p, alpha, flux):
    import paper_1807_01151_amd as P
    print("case", name, flush=True)
    O = oracle.Oracle(mesh, p, alpha_deg=alpha, flux=flux)
    S = P.Solver(mesh, p, alpha_deg=alpha, flux=flux)
    rng = np.random.default_rng(600)
    for lev in range(p + 1):
        u = perturbed(O, lev, 610 + lev)
        v = rng.standard_normal(u.shape)
        J = O.jacobian_sparse(lev, u)
        jv_o = (J @ v.ravel()).reshape(u.shape)
        jv_g = to_host(S.jacobian_apply(lev, to_dev(u), to_dev(v)))
        err = rel_err(jv_g, jv_o)
        print(f"  level {lev}: J v rel err {err:.2e}", flush=True)
        assert err < 1e-12, (lev, err)
        if lev >= 1:
            w = rng.standard_normal(u.shape)
            jtw = to_host(S.adjoint_apply(lev, to_dev(u), to_dev(w)))
            a, b = float(np.sum(w * jv_g)), float(np.sum(jtw * v))
            scale = float(np.sum(np.abs(w * jv_g)))
            print(f"  level {lev}: <w, Jv> {a:.15e} <J^T w, v> {b:.15e}", flush=True)
            assert abs(a - b) <= 1e-12 * scale
