"""Batched independent solves (one handle, one launch per kernel for all
solves) against the same solves run one handle each and against the FP64
oracle.

The batch evaluates every element exactly as a single-solve handle does and
its Arnoldi blocks follow each solve's own row partition, so one batched
V-cycle equals the single-solve cycle to rounding (the residual norms are
summed in another order, 1e-14 relative); free-running histories are
compared over their first cycles (later cycles amplify rounding, as for the
single-solve histories) and at the converged states."""

import numpy as np
import pytest

import oracle
from eg_inputs import ogrid
from tests.gpu_util import to_dev, to_host, rel_err

pytestmark = pytest.mark.gpu

MESHES = [ogrid(12, 4), ogrid(20, 6), ogrid(16, 5)]
MACHS = [0.3, 0.2, 0.35]
ALPHAS = [0.0, 3.0, -2.0]
KW = dict(rk_stages=4, cfl_max=100.0, krylov_m=30)


def _batch(p, **kw):
    import paper_1807_01151_amd as P
    return P.BatchSolver(MESHES, p, MACHS, ALPHAS, **KW, **kw)


def _single(i, p, **kw):
    import paper_1807_01151_amd as P
    return P.Solver(MESHES[i], p, mach=MACHS[i], alpha_deg=ALPHAS[i], **KW, **kw)


def test_layout_and_freestream():
    B = _batch(2)
    u = B.freestream(2)
    e0 = 0
    for i, v in enumerate(B.views(u)):
        off, nm, ne = B.layout(i, 2)
        assert (off, nm, ne) == (e0 * 4 * 9, 9, MESHES[i].n_elem)
        e0 += ne
        S = _single(i, 2)
        assert rel_err(to_host(v), to_host(S.freestream(2))) == 0.0


def test_batch_residual_equals_single():
    """Per-solve free streams and far fields: the batch residual of a
    perturbed state equals each solve's own residual bitwise."""
    p = 2
    B = _batch(p)
    u = B.freestream(p)
    rng = np.random.default_rng(400)
    un = to_host(u)
    un[:, :, 1:] += 1e-3 * rng.uniform(-1, 1, un[:, :, 1:].shape)
    u = to_dev(un)
    r = B.residual(p, u)
    for i, (uv, rv) in enumerate(zip(B.views(u), B.views(r))):
        S = _single(i, p)
        assert np.array_equal(to_host(S.residual(p, uv.contiguous())), to_host(rv))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_solve_matches_single_solves(precision):
    """Batched solve from the free streams vs each solve alone: early
    histories to 1e-12 r_1, every solve reaches the 1e-10 drop, and the
    converged states agree to 1e-8 (FP64: also the oracle's residual of the
    batch state is at the drop)."""
    p = 1
    B = _batch(p, precision=precision)
    u = B.freestream(p)
    hists, cyc, st = B.solve(u, drop_tol=1e-10, max_cycles=6000)
    print(precision, "batch cycles", cyc, flush=True)
    assert st == 0
    for i, uv in enumerate(B.views(u)):
        S = _single(i, p, precision=precision)
        us = S.freestream(p)
        h, st_s = S.solve_steady(us, drop_tol=1e-10, max_cycles=6000)
        assert st_s == 0
        n = min(10, len(h), len(hists[i]))
        dev = np.max(np.abs(hists[i][:n] - h[:n])) / h[0]
        e = rel_err(to_host(uv), to_host(us))
        print(f"  solve {i}: cycles {cyc[i]} vs {len(h) - 1}, early history dev {dev:.2e}, state {e:.2e}",
              flush=True)
        assert dev < 1e-12
        assert e < 1e-8
        assert hists[i][-1] <= 1e-10 * hists[i][0]
        # the returned state is the one whose norm the history ends with,
        # although the batch kept cycling until its slowest solve converged
        # (near the drop the norm is round-off dominated, so the two
        # evaluations agree to 1e-12 r_1, not relative to r_n; further
        # cycles would move it by O(1e-10) r_1)
        S64 = _single(i, p)
        rn_ret = S64.rnorm(S64.residual(p, uv.contiguous()))
        print(f"  solve {i}: norm of the returned state {rn_ret:.6e}, recorded {hists[i][-1]:.6e}", flush=True)
        assert abs(rn_ret - hists[i][-1]) <= 1e-12 * hists[i][0]
        if precision == "fp64":
            O = oracle.Oracle(MESHES[i], p, mach=MACHS[i], alpha_deg=ALPHAS[i])
            ub = to_host(uv)
            assert O.rnorm(p, O.residual(p, ub)) <= 2e-10 * hists[i][0]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_p4_cycles_match_single(precision):
    """p = 4 (100 x 100 blocks: the LDS-resident assembly and LU and the
    chunked stage kernel) in a batch of two solves against each solve alone:
    five V-cycles from the free streams agree to 1e-12 r_1 (the batch sums
    its residual norms per solve in another order) and so do the states."""
    import paper_1807_01151_amd as P
    meshes, machs, alphas = MESHES[:2], MACHS[:2], ALPHAS[:2]
    kw = dict(rk_stages=3, cfl_max=10.0, krylov_m=30, precision=precision)
    B = P.BatchSolver(meshes, 4, machs, alphas, **kw)
    u = B.freestream(4)
    hists, cyc, st = B.solve(u, drop_tol=0.0, max_cycles=5)
    for i, uv in enumerate(B.views(u)):
        S = P.Solver(meshes[i], 4, mach=machs[i], alpha_deg=alphas[i], **kw)
        us = S.freestream(4)
        h, _ = S.solve_steady(us, drop_tol=0.0, max_cycles=5)
        n = min(len(h), len(hists[i]))
        dev = np.max(np.abs(hists[i][:n] - h[:n])) / h[0]
        e = rel_err(to_host(uv), to_host(us))
        print(f"  {precision} solve {i}: history dev {dev:.2e}, state {e:.2e}", flush=True)
        assert n == 6
        assert dev < 1e-12
        assert e < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("graphs", [False, True])
def test_solve_multi_matches_separate_batch_solves(precision, graphs):
    """Three batch handles of different orders (p = 1, 2, 3 over the same
    three meshes) advanced together by eg_solve_multi, eagerly and as one
    graph launch per cycle, against each handle's own eg_solve_batch: every
    handle runs the same arithmetic either way, so the histories, cycle
    counts, statuses and final states are bitwise equal (some solves reach
    the drop within the cap, others do not)."""
    import paper_1807_01151_amd as P
    orders = (1, 2, 3)
    Bs = [_batch(p, precision=precision) for p in orders]
    for B in Bs:
        B.set_graphs(graphs)
    us = [B.freestream(p) for B, p in zip(Bs, orders)]
    res = P.solve_multi(Bs, us, drop_tol=1e-5, max_cycles=400)
    for k, p in enumerate(orders):
        B = _batch(p, precision=precision)
        B.set_graphs(graphs)
        u = B.freestream(p)
        hists, cyc, st = B.solve(u, drop_tol=1e-5, max_cycles=400)
        hm, cm, sm = res[k]
        print(f"  {precision} graphs={graphs} p={p}: cycles {cm} status {sm}", flush=True)
        assert cm == cyc and sm == st
        for a, b in zip(hm, hists):
            assert np.array_equal(a, b)
        assert np.array_equal(to_host(us[k]), to_host(u))
