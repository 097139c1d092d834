"""Parity at the full size of the 3D sphere adjoint workload (cubed-sphere hex
shell 6 x 12 x 12 x 16 = 13824 quadratic curved hexes, p = 3: 64 modes x 5 variables,
320 x 320 element blocks assembled and factorised in global memory, Ma 0.3)
in FP64 and in mixed precision: the residual at every level and the PRK step
on every element.  (The V-cycle, J v and the adjoint at p = 3 are compared
with the oracle on the small shell in test_gpu_parity, test_gpu_jacobian_apply
and test_gpu_adjoint.)"""

import pytest

import oracle
from eg_inputs import cubed_sphere_shell
from tests.gpu_util import perturbed, to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu

MESH = cubed_sphere_shell(12, 16, curved=True)  # the sphere grid is curved (Section 5.2)
KW = dict(rk_stages=4, cfl_max=100.0, krylov_m=30)  # the workload's smoother


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(MESH, 3)


@pytest.fixture(scope="module")
def prk_case(orc):
    """One perturbed state and the oracle's 4-stage PRK step from it (p = 3, CFL 10)."""
    u = perturbed(orc, 3, 913)
    return u, orc.prk(3, 4, 10.0, u)


def _solver(precision):
    import paper_1807_01151_amd as P
    return P.Solver(MESH, 3, precision=precision, **KW)


def test_c5_residual_full(orc):
    S = _solver("fp64")
    for lev in (3, 2, 1, 0):
        u = perturbed(orc, lev, 912 + 10 * lev, amp=0.01)
        e = rel_err(to_host(S.residual(lev, to_dev(u))), orc.residual(lev, u))
        print(f"c5 p={lev} residual error {e:.3e}", flush=True)
        assert e < 1e-12, (lev, e)


def test_c5_prk_full(prk_case):
    u, out_o = prk_case
    S = _solver("fp64")
    ud = to_dev(u)
    S.prk_step(3, 10.0, ud)
    e = rel_err(to_host(ud) - u, out_o - u)
    print(f"c5 FP64 PRK update error {e:.3e}", flush=True)
    assert e < 1e-11


def test_c5_mixed_residual_and_prk(orc, prk_case):
    """FP32 residual within 2e-5 and FP32 PRK step (FP32 blocks on the FP32
    matrix cores, LU and stage solves) within 2e-4 of the FP64 oracle."""
    S = _solver("mixed")
    u = perturbed(orc, 3, 914)
    e = rel_err(to_host(S.residual(3, to_dev(u))), orc.residual(3, u))
    print(f"c5 mixed residual error {e:.3e}", flush=True)
    assert e < 2e-5
    u, out_o = prk_case
    ud = to_dev(u)
    S.prk_step(3, 10.0, ud)
    e = rel_err(to_host(ud) - u, out_o - u)
    print(f"c5 mixed PRK update error {e:.3e}", flush=True)
    assert e < 2e-4
