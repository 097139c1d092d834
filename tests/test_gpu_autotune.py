"""Residual tile autotuner (eg_autotune): the chosen tiles are among the
candidates, and every residual and V-cycle after tuning equals the untuned
one bitwise (each output of the residual is formed by one thread with the
same sums, whatever the number of elements per workgroup)."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid, cubed_sphere_shell
from tests.gpu_util import perturbed, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [("ogrid24x12-p3", ogrid(24, 12), 3), ("sphere6x2x2x2-p2", cubed_sphere_shell(2, 2), 2)]


@pytest.mark.parametrize("name,mesh,p", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotune_keeps_results(name, mesh, p, precision):
    import paper_1807_01151_amd as P
    O = oracle.Oracle(mesh, p)
    kw = dict(rk_stages=3, cfl_max=10.0, krylov_m=30, precision=precision)
    a, b = P.Solver(mesh, p, **kw), P.Solver(mesh, p, **kw)
    u = perturbed(O, p, 77, amp=0.01)
    ref = [to_host(a.residual(q, to_dev(perturbed(O, q, 78 + q, amp=0.01)))) for q in range(p + 1)]
    tiles = b.autotune(reps=3)
    print(name, precision, "tiles", tiles, flush=True)
    assert set(tiles) == {(q, k) for q in range(p + 1) for k in ("fp64", "fp32")}
    assert all(t >= 1 for t in tiles.values())
    for q in range(p + 1):
        got = to_host(b.residual(q, to_dev(perturbed(O, q, 78 + q, amp=0.01))))
        assert np.array_equal(got, ref[q])
    ua, ub = to_dev(u), to_dev(u)
    ha, _ = a.solve_steady(ua, drop_tol=0.0, max_cycles=6)
    hb, _ = b.solve_steady(ub, drop_tol=0.0, max_cycles=6)
    assert np.array_equal(ha, hb)
    assert np.array_equal(to_host(ua), to_host(ub))
