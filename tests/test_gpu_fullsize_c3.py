"""Parity at the full size of the 3D sphere workload (cubed-sphere hex shell
6 x 16 x 16 x 24 = 36864 quadratic curved hexes, p = 2: 27 modes x 5 variables, 135 x 135
element blocks, Ma 0.3) in FP64 and in mixed precision: the residual and the
PRK step on every element, and the first V-cycle from the free stream
applied to the oracle's state."""

import numpy as np
import pytest

import oracle
from eg_inputs import cubed_sphere_shell
from tests.gpu_util import perturbed, to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu

MESH = cubed_sphere_shell(16, 24, curved=True)  # the sphere grid is curved (Section 5.2)
KW = dict(rk_stages=4, cfl_max=100.0, krylov_m=30)  # the workload's smoother


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(MESH, 2)


@pytest.fixture(scope="module")
def prk_case(orc):
    """One perturbed state and the oracle's 4-stage PRK step from it (p = 2, CFL 10)."""
    u = perturbed(orc, 2, 903)
    return u, orc.prk(2, 4, 10.0, u)


def _solver(precision):
    import paper_1807_01151_amd as P
    return P.Solver(MESH, 2, precision=precision, **KW)


def test_c3_residual_full(orc):
    S = _solver("fp64")
    for lev in (2, 1, 0):
        u = perturbed(orc, lev, 902 + 10 * lev, amp=0.01)
        e = rel_err(to_host(S.residual(lev, to_dev(u))), orc.residual(lev, u))
        print(f"c3 p={lev} residual error {e:.3e}", flush=True)
        assert e < 1e-12, (lev, e)


def test_c3_prk_full(prk_case):
    u, out_o = prk_case
    S = _solver("fp64")
    ud = to_dev(u)
    S.prk_step(2, 10.0, ud)
    e = rel_err(to_host(ud) - u, out_o - u)
    print(f"c3 FP64 PRK update error {e:.3e}", flush=True)
    assert e < 1e-11


def test_c3_mixed_residual_and_prk(orc, prk_case):
    """FP32 residual within 2e-5 and FP32 PRK step (FP32 blocks, LU and
    stage solves) within 2e-4 of the FP64 oracle, at the perturbation size
    of the small-mesh mixed tests (the FP32 error relative to the largest
    residual entry grows as the residual shrinks against the fluxes it
    sums)."""
    S = _solver("mixed")
    u = perturbed(orc, 2, 904)
    e = rel_err(to_host(S.residual(2, to_dev(u))), orc.residual(2, u))
    print(f"c3 mixed residual error {e:.3e}", flush=True)
    assert e < 2e-5
    u, out_o = prk_case
    ud = to_dev(u)
    S.prk_step(2, 10.0, ud)
    e = rel_err(to_host(ud) - u, out_o - u)
    print(f"c3 mixed PRK update error {e:.3e}", flush=True)
    assert e < 2e-4


def test_c3_first_cycle_map(orc):
    """The GPU V-cycle (p2 -> p1 -> p0, PCEXP with m = 30 on p0) applied to
    the free stream equals the oracle's cycle from that state."""
    S = _solver("fp64")
    u = orc.freestream(2)
    r1 = orc.rnorm(2, orc.residual(2, u))
    un, rn_o, _ = orc.vcycle(u, 1, s=4, m=30, cfl_max=100.0, rref=r1)
    g = to_dev(u)
    rn_g, _ = S.vcycle(g, 1, rref=r1)
    print(f"c3 cycle: r1 {r1:.6e} rn gpu {rn_g:.6e} oracle {rn_o:.6e}", flush=True)
    assert abs(rn_g - rn_o) <= 1e-13 * rn_o
    e = rel_err(to_host(g) - u, un - u)
    print(f"c3 cycle update error {e:.3e}", flush=True)
    assert np.isfinite(e) and e < 1e-10
