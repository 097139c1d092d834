"""Graph replay of the V-cycle (eg_set_graphs) against eager launches.

Every kernel is deterministic and the replayed graph launches the same
kernels in the same order on the same buffers, so the residual history (one
FP64 norm per replay, computed eagerly between replays) and the final state
must be bitwise equal to the eager solve, over many replays, across resumed
calls, across the mixed-precision phase switch and for batches."""

import numpy as np
import pytest

from eg_inputs import ogrid
from tests.gpu_util import to_host

pytestmark = pytest.mark.gpu

KW = dict(rk_stages=4, cfl_max=100.0, krylov_m=30)


def _pair(mesh, p, **kw):
    import paper_1807_01151_amd as P
    a = P.Solver(mesh, p, **KW, **kw)
    b = P.Solver(mesh, p, **KW, **kw)
    b.set_graphs(True)
    return a, b


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager_c1(precision):
    """O-grid 24 x 12, p = 1: 300 cycles, then resumed to the 1e-10 drop (the
    mixed solve switches phase, so both of its graphs are replayed)."""
    a, b = _pair(ogrid(24, 12), 1, precision=precision)
    ua, ub = a.freestream(1), b.freestream(1)
    ha, sa = a.solve_steady(ua, drop_tol=1e-10, max_cycles=300)
    hb, sb = b.solve_steady(ub, drop_tol=1e-10, max_cycles=300)
    assert sa == sb and np.array_equal(ha, hb)
    ha2, sa = a.solve_steady(ua, drop_tol=1e-10, max_cycles=4000, resume=True)
    hb2, sb = b.solve_steady(ub, drop_tol=1e-10, max_cycles=4000, resume=True)
    print(precision, "cycles", len(ha) - 1 + len(ha2) - 1, flush=True)
    assert sa == 0 and sb == 0
    assert np.array_equal(ha2, hb2)
    assert np.array_equal(to_host(ua), to_host(ub))


def test_graph_replay_equals_eager_benchmark_workload():
    """O-grid 128 x 64, p = 3, s = 3, CFL 10: 12 cycles."""
    import paper_1807_01151_amd as P
    mesh = ogrid(128, 64)
    a = P.Solver(mesh, 3, rk_stages=3, cfl_max=10.0, krylov_m=30)
    b = P.Solver(mesh, 3, rk_stages=3, cfl_max=10.0, krylov_m=30)
    b.set_graphs(True)
    ua, ub = a.freestream(3), b.freestream(3)
    ha, _ = a.solve_steady(ua, drop_tol=0.0, max_cycles=12)
    hb, _ = b.solve_steady(ub, drop_tol=0.0, max_cycles=12)
    assert np.array_equal(ha, hb)
    assert np.array_equal(to_host(ua), to_host(ub))


def test_graph_replay_equals_eager_batch():
    import paper_1807_01151_amd as P
    meshes = [ogrid(12, 4), ogrid(20, 6), ogrid(16, 5)]
    args = ([0.3, 0.2, 0.35], [0.0, 3.0, -2.0])
    a = P.BatchSolver(meshes, 1, *args, **KW)
    b = P.BatchSolver(meshes, 1, *args, **KW)
    b.set_graphs(True)
    ua, ub = a.freestream(1), b.freestream(1)
    ha, ca, sa = a.solve(ua, drop_tol=1e-10, max_cycles=4000)
    hb, cb, sb = b.solve(ub, drop_tol=1e-10, max_cycles=4000)
    assert sa == sb == 0 and ca == cb
    for x, y in zip(ha, hb):
        assert np.array_equal(x, y)
    assert np.array_equal(to_host(ua), to_host(ub))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager_p4(precision):
    """O-grid 10 x 3, p = 4 (column-split block factorisation, chunked stage
    kernels): 8 cycles replayed from the graph equal the eager cycles."""
    import paper_1807_01151_amd as P
    mesh = ogrid(10, 3)
    a = P.Solver(mesh, 4, rk_stages=3, cfl_max=10.0, krylov_m=30, precision=precision)
    b = P.Solver(mesh, 4, rk_stages=3, cfl_max=10.0, krylov_m=30, precision=precision)
    b.set_graphs(True)
    ua, ub = a.freestream(4), b.freestream(4)
    ha, _ = a.solve_steady(ua, drop_tol=0.0, max_cycles=8)
    hb, _ = b.solve_steady(ub, drop_tol=0.0, max_cycles=8)
    assert np.array_equal(ha, hb)
    assert np.array_equal(to_host(ua), to_host(ub))
