"""Benchmark of the eMG V-cycle on one MI355X.

Workload (the metric's configuration): 3D sphere, cubed-sphere hex shell
6 x 16 x 16 x 24 = 36864 hexes (radius 0.5 to 20, geometric radial stretch),
modal DG p = 2 (27 modes x 5 variables per element, 4,976,640 DOF), Rusanov
flux, slip wall + characteristic far field, Ma = 0.3 along +x, V-cycle
p2 -> p1 -> p0 with a 4-stage PRK smoother and the EXP1 step (Krylov
dimension 30) on p0, CFL_max = 100, free-stream start.

A step is one V-cycle (entry residual + norm, PRK on p = 2 and 1, EXP1 on
p = 0, transfers).  value = DOF-updates/s = DOF x cycles / wall time of the
timed FP64 cycles (inputs resident in HBM).  The run also reports the time to
a 1e-10 residual drop from the free stream in FP64 and in mixed precision,
the difference of the two converged states, the event-timed roofline of the
dominant kernel, measured achievable peaks, the 2D cylinder workload
(O-grid 128 x 64, p = 3), the batched workload, and the FP64 CPU oracle
timed on one V-cycle of the same workload on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector and FP64 matrix cores, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def work_model(d, p, fp32_blocks=False, nodes=None):
    """Algorithmic work per element of the three main kernel classes at order
    p, counted as the kernels execute it (no credit for avoided work):
    residual: the dense modal contractions (state at the volume points, the
    gradient projection, own and neighbour traces and the face projection);
    jacobian_lu: the block contraction with the D flux-Jacobian directions
    summed per volume point before the product with the basis (direction
    sums, volume products, face scalings, face products) plus the LU (2/3 n^3);
    prk_stage: bytes of one stage (factors, permutation, residual, base
    state, new state).  ``nodes``: geometry nodes per element (default 9 per
    quad, 8 per straight hex; 27 per curved hex)."""
    V, N, Q = d + 2, (p + 1) ** d, p + 2
    QV, QF, NF = Q ** d, Q ** (d - 1), 2 * d
    NC = nodes if nodes else (9 if d == 2 else 8)
    n = V * N
    NT = N * (N + 1) // 2
    fb = 4 if fp32_blocks else 8
    return {
        "residual": {"flop": 2 * V * N * (QV * (1 + d) + 3 * NF * QF),
                     "bytes": (2 * V * N + NC * d) * 8 + NF * 5},
        "jacobian_lu": {"flop": 2 * V * V * N * (QV * (d + N) + NF * QF * (1 + N)) + (2 * n ** 3) // 3,
                        "bytes": (V * N + NC * d + NT) * 8 + n * n * fb + n * 4},
        "prk_stage": {"flop": 2 * n * n, "bytes": n * n * fb + n * 4 + 3 * n * 8},
    }


# device functions behind each timed class, by source file (for the digest
# that ties a stored counter reading to the code it was taken on)
CLASS_SOURCES = {
    "jacobian_lu": [("eg_kernels.hip", ["k_jac_points"]), ("eg_jaclu_lds.hip", ["panel_wave", "k_jaclu_lds"])],
    "prk_stage": [("eg_kernels.hip", ["k_prk_stage_c", "k_prk_stage_t", "k_prk_stage"])],
    "residual": [("eg_kernels.hip", ["k_residual"])],
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vcycle_c3_pmc_traffic.md")


def kernel_source_digest(cls):
    """sha256 over the shared device headers and the text of the device
    functions of one kernel class (their definitions: lines that declare a
    __device__ or __global__ function of that name)."""
    csrc = os.path.join(ROOT, "paper_1807_01151_amd", "csrc")
    h = hashlib.sha256()
    for f in ("eg_common.h", "eg_physics.h", "eg_device.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    for fname, names in CLASS_SOURCES[cls]:
        src = open(os.path.join(csrc, fname)).read()
        for name in names:
            for m in re.finditer(r"\b" + name + r"\(", src):
                start = src.rfind("\n", 0, m.start())
                line = src[start + 1:src.find("\n", m.start())]
                if "__device__" not in line and "__global__" not in line:
                    continue  # a call, not the definition
                end = src.find("\n}\n", m.start())
                h.update(src[start:end].encode())
    return h.hexdigest()


def stored_traffic(cls, p):
    """HBM bytes per launch of a kernel class from the committed counter
    summary, or None if it is absent or was taken on other kernel code."""
    try:
        txt = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(re.findall(r"^- (.+?): (\S+)$", txt, re.M))
    if vals.get(f"source_digest[{cls}]") != kernel_source_digest(cls):
        return None
    v = vals.get(f"traffic_bytes_per_launch[{cls} p={p}]")
    return float(v) if v else None


def roofline_entry(cls, p, ms, launches, ne, d, peaks=None, nodes=None):
    w = work_model(d, p, nodes=nodes)[cls]
    avg_s = ms / launches / 1e3
    if cls == "prk_stage":
        ach = w["bytes"] * ne / avg_s / 1e9
        out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
               "traffic": stored_traffic(cls, p), "kernel": f"{cls} p={p}", "avg_launch_ms": ms / launches,
               "algorithmic_bytes_per_launch": w["bytes"] * ne}
        if peaks and peaks.get("hbm_gbs"):
            out["frac_of_measured_peak"] = ach / peaks["hbm_gbs"]
        return out
    ach = w["flop"] * ne / avg_s / 1e12
    bound = "mfma" if cls == "jacobian_lu" else "alu"
    out = {"bound": bound, "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": ach / FP64_PEAK_TFLOPS, "traffic": stored_traffic(cls, p), "kernel": f"{cls} p={p}",
           "avg_launch_ms": ms / launches, "algorithmic_flop_per_launch": w["flop"] * ne}
    key = "fp64_mfma_tflops" if bound == "mfma" else "fp64_fma_tflops"
    if peaks and peaks.get(key):
        out["frac_of_measured_peak"] = ach / peaks[key]
    return out


def profile_cycles(S, u, p, steps):
    """Event-timed pass over `steps` V-cycles continuing the solve of u:
    {class@p: (total ms, launches)}."""
    import paper_1807_01151_amd as P
    S.profile(True)
    S.solve_steady(u, drop_tol=0.0, max_cycles=steps, resume=True)
    prof = {}
    for cls in P.binding.KERNEL_CLASSES:
        for lev in range(p + 1):
            ms, n = S.profile_read(cls, lev)
            if n:
                prof[f"{cls}@p{lev}"] = (ms, n)
    S.profile(False)
    return prof


def drop_run(S, p, max_cycles, budget, tag, chunk=200):
    """Solve from the free stream to a 1e-10 drop in chunks (same ramp and
    cycle numbering), each chunk reporting its progress; stops at the drop,
    the cycle cap or the time budget.  Returns (summary, final state)."""
    import torch
    u2 = S.freestream(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hist, st = S.solve_steady(u2, drop_tol=1e-10, max_cycles=min(chunk, max_cycles))
    r1, done, last = hist[0], len(hist) - 1, hist[-1]
    while st == 5 and done < max_cycles and time.perf_counter() - t1 < budget:
        log(f"[bench] {tag} drop run: {done} cycles, r/r1 = {last / r1:.3e}, {time.perf_counter() - t1:.1f}s")
        h2, st = S.solve_steady(u2, drop_tol=1e-10, max_cycles=min(chunk, max_cycles - done), resume=True)
        done += len(h2) - 1
        last = h2[-1]
    torch.cuda.synchronize()
    t_drop = time.perf_counter() - t1
    out = {"cycles_to_1e-10": int(done) if st == 0 else None, "cycles_run": int(done),
           "time_to_1e-10_s": round(t_drop, 3) if st == 0 else None, "drop_run_s": round(t_drop, 3),
           "drop_reached": float(last / r1), "converged": st == 0}
    log(f"[bench] {tag} drop run: {out}")
    return out, u2


def c2_measurements(P, steps, warmup, drop_budget):
    """The 2D cylinder workload: O-grid 128 x 64 quadratic curved quads (the
    paper's cylinder grid is curved), p = 3, s = 3, CFL_max = 10, FP64:
    V-cycle throughput, dominant kernels, and the drop run to 1e-10."""
    import torch
    from eg_inputs import ogrid
    mesh = ogrid(128, 64, curved=True)
    S = P.Solver(mesh, 3, rk_stages=3, cfl_max=10.0, krylov_m=30, mach=0.3, alpha_deg=0.0)
    S.autotune()
    dof = mesh.n_elem * 4 * 16
    u = S.freestream(3)
    S.solve_steady(u, drop_tol=0.0, max_cycles=warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.solve_steady(u, drop_tol=0.0, max_cycles=steps, resume=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    prof = profile_cycles(S, u, 3, steps)
    out = {"workload": "2D cylinder O-grid 128x64 quadratic curved quads, DG p=3 (16 modes x 4 vars), "
                       "eMG V-cycle p3->p0, "
                       "3-stage PRK, EXP1 m=30, CFL_max 10, Ma 0.3, free-stream start, FP64",
           "dof": dof, "ms_per_cycle": round(ms, 4), "dof_updates_per_s": dof / ms * 1e3,
           "kernels_ms_per_cycle": {k: round(v[0] / steps, 5) for k, v in prof.items()}}
    for cls in ("residual", "jacobian_lu", "prk_stage"):
        k = f"{cls}@p3"
        if k in prof:
            e = roofline_entry(cls, 3, prof[k][0], prof[k][1], mesh.n_elem, 2)
            out[f"roofline_{cls}_p3"] = {"achieved": round(e["achieved"], 3), "unit": e["unit"],
                                         "frac": round(e["frac"], 4), "bound": e["bound"]}
    if drop_budget > 0:
        out["drop_run"], _ = drop_run(S, 3, 100000, drop_budget, "c2 fp64", chunk=1000)
    log(f"[bench] c2: {ms:.3f} ms/cycle")
    return out


def batched_measurements(P, steps, budget_s, precision="mixed"):
    """The batched workload: 64 independent cylinder solves (curved O-grids) drawn from seed
    1807 (N_theta ~ U{16..96}, N_r = N_theta / 2, p ~ U{1..4}, Ma ~ U[0.1,
    0.4], alpha ~ U[-5, 5] deg), s = 4, CFL_max = 100, one batch handle per
    order, all four advanced together (eg_solve_multi: per V-cycle one
    synchronisation and one graph launch holding every order group's
    V-cycle).  Reports the V-cycle throughput of the whole batch and, within
    a time budget, how many solves reach the 1e-10 drop, diverge or stall."""
    import numpy as np
    import torch
    from eg_inputs import batch_draws, ogrid
    draws = batch_draws(64, seed=1807)
    groups = {}
    for i, d in enumerate(draws):
        groups.setdefault(d["p"], []).append(i)
    t_init = time.perf_counter()
    handles = {}
    for p, idx in sorted(groups.items()):
        meshes = [ogrid(draws[i]["n_theta"], draws[i]["n_r"], curved=True) for i in idx]
        B = P.BatchSolver(meshes, p, [draws[i]["mach"] for i in idx], [draws[i]["alpha_deg"] for i in idx],
                          rk_stages=4, cfl_max=100.0, krylov_m=30, precision=precision)
        B.autotune()
        B.set_graphs(True)
        handles[p] = (B, idx)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    order = sorted(handles)
    Bs = [handles[p][0] for p in order]
    dof = sum(B.n_elem * B.V * B.N(B.p_max) for B in Bs)
    us = [B.freestream(B.p_max) for B in Bs]
    P.solve_multi(Bs, us, drop_tol=0.0, max_cycles=2)  # graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.solve_multi(Bs, us, drop_tol=0.0, max_cycles=steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_cycle = wall / steps * 1e3
    out = {"solves": 64, "elements": int(sum(B.n_elem for B in Bs)), "dof": int(dof),
           "groups": {str(p): len(handles[p][1]) for p in order}, "precision": precision,
           "rk_stages": 4, "cfl_max": 100.0, "setup_s": round(t_init, 3), "launch": "eg_solve_multi, one graph per cycle",
           "ms_per_batched_cycle": round(ms_cycle, 3), "dof_updates_per_s": dof * steps / wall}
    log(f"[bench] batched: {out}")
    us = [B.freestream(B.p_max) for B in Bs]
    cap = max(10, int(budget_s / (ms_cycle * 1e-3)))
    t1 = time.perf_counter()
    res = P.solve_multi(Bs, us, drop_tol=1e-10, max_cycles=cap)
    drops, conv, div, stall = [], 0, 0, 0
    per_group = {}
    for p, (hists, cyc, st) in zip(order, res):
        ok = sum(1 for h in hists if h[-1] <= 1e-10 * h[0])
        bad = sum(1 for h in hists if not np.isfinite(h[-1]))
        conv += ok
        div += bad
        stall += len(hists) - ok - bad
        per_group[str(p)] = {"converged": ok, "diverged": bad, "stalled": len(hists) - ok - bad,
                             "cycles_max": int(max(cyc))}
        drops += [float(h[-1] / h[0]) if np.isfinite(h[-1]) else float("inf") for h in hists]
    out["convergence_cap_cycles"] = cap
    out["converged_to_1e-10"] = conv
    out["diverged"] = div
    out["stalled"] = stall
    out["per_order"] = per_group
    fin = [d for d in drops if np.isfinite(d)]
    out["median_drop_reached"] = float(np.median(fin)) if fin else None
    out["per_solve_drop"] = [float(f"{d:.3g}") for d in drops]
    out["convergence_run_s"] = round(time.perf_counter() - t1, 2)
    out["ms_per_cycle_convergence_run"] = round(out["convergence_run_s"] * 1e3 / max(1, max(
        max(c) for _, c, _ in res)), 3)
    log(f"[bench] batched convergence: {per_group}, {out['convergence_run_s']} s")
    for B in Bs:
        B.close()
    return out


def c1_time_to_drop(P):
    """Time to a 1e-10 FP64 residual drop on the O-grid 24 x 12, p = 1 solve
    (s = 4, CFL_max = 100, m = 30), in FP64 and mixed."""
    import torch
    from eg_inputs import ogrid
    m1 = ogrid(24, 12)
    out = {}
    for prec in ("fp64", "mixed"):
        S = P.Solver(m1, 1, rk_stages=4, cfl_max=100.0, krylov_m=30, precision=prec)
        S.solve_steady(S.freestream(1), drop_tol=0.0, max_cycles=3)  # warm-up (kernel loading)
        u = S.freestream(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h, st = S.solve_steady(u, drop_tol=1e-10, max_cycles=6000)
        torch.cuda.synchronize()
        out[prec] = {"time_s": round(time.perf_counter() - t0, 4), "cycles": len(h) - 1, "converged": st == 0}
        log(f"[bench] c1 {prec}: {out[prec]}")
    out["speedup"] = round(out["fp64"]["time_s"] / out["mixed"]["time_s"], 3)
    return out


def c5_adjoint(P, budget):
    """The adjoint workload: cubed-sphere shell 6 x 12 x 12 x 16 = 13824 curved
    hexes at p = 3 (320 x 320 blocks), Ma 0.3, s = 4, CFL_max = 100: the mixed-
    precision solve from the free stream to the 1e-10 drop, then the adjoint
    solve (FP64) and dC_D/dtheta for theta = (Mach, two seeded 1e-3-scale
    Gaussian wall-bump amplitudes) from one paired residual and drag
    evaluation per parameter (eg_param_sensitivity, h = 1e-6)."""
    import math
    import torch
    from eg_inputs import cubed_sphere_shell, wall_bumps, bump_centers
    from paper_1807_01151_amd.binding import _freestream_direction
    mesh = cubed_sphere_shell(12, 16, curved=True)  # on straight hexes this solve stalls
    centers = bump_centers(3, 2, seed=1807)
    sref = math.pi * 0.25  # the unit-diameter sphere's frontal area
    kw = dict(rk_stages=4, cfl_max=100.0, krylov_m=30)
    S = P.Solver(mesh, 3, mach=0.3, precision="mixed", **kw)
    S.autotune()
    out = {"workload": "3D sphere shell 6x12x12x16 = 13824 curved hexes, DG p=3 (64 modes x 5 vars, "
                       "320 x 320 blocks), "
                       "mixed-precision steady state, FP64 adjoint, theta = (Ma, 2 wall bumps)"}
    out["steady"], u = drop_run(S, 3, 100000, budget, "c5 mixed", chunk=500)
    if not out["steady"]["converged"]:
        return out
    cd, g = S.drag(u, sref=sref, grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # in chunks of 250 cycles from the previous lambda, reporting progress;
    # the drop is relative to the first chunk's initial adjoint residual
    lam, r0, done, last, st = None, None, 0, None, 5
    while st == 5 and done < 4000:
        tol = 1e-10 if r0 is None else 1e-10 * r0 / last
        lam, hist, st = S.adjoint_solve(u, g, lam=lam, drop_tol=min(tol, 1.0), max_cycles=250, raise_on_fail=False)
        r0 = hist[0] if r0 is None else r0
        done += len(hist) - 1
        last = hist[-1]
        log(f"[bench] c5 adjoint: {done} cycles, drop {last / r0:.3e}, {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    out["adjoint"] = {"cycles": done, "drop": float(last / r0), "status": int(st),
                      "time_s": round(time.perf_counter() - t0, 3)}
    log(f"[bench] c5 adjoint: {out['adjoint']}")
    h = 1e-6
    theta = [0.3, 0.0, 0.0]
    direction = _freestream_direction(3, 0.0, 0.0)
    grad = []
    t0 = time.perf_counter()
    for i in range(3):
        tp, tm = list(theta), list(theta)
        tp[i] += h
        tm[i] -= h
        Sp = P.Solver(wall_bumps(mesh, tp[1:], centers, 0.4), 3, mach=tp[0], **kw)
        Sm = P.Solver(wall_bumps(mesh, tm[1:], centers, 0.4), 3, mach=tm[0], **kw)
        grad.append(Sp.param_sensitivity(Sm, h, u, lam, direction=direction, sref=sref))
        Sp.close()
        Sm.close()
    out["C_D"] = cd
    out["dCD_dtheta"] = grad
    out["sensitivity_s"] = round(time.perf_counter() - t0, 3)
    log(f"[bench] c5: C_D {cd:.8e} gradient {grad}")
    S.close()
    return out


def poly_work(p, n_tet, n_prism):
    """Algorithmic FP64 flops of one tetrahedron / prism residual at order p
    (the contractions only; the pointwise flux arithmetic is not counted):
    monomial coefficients S^T u and R = S m (V N (N+1) each), the state at
    every volume point (2 V N) and face point (own and neighbour: 4 V N), the
    flux moments (2 * 15 N_{p-1} per volume point) and the face moments
    (2 V N per face point).  Bytes: state in, coefficients written and read,
    the lower triangle of S, residual out."""
    V, N, NL, Q = 5, (p + 1) * (p + 2) * (p + 3) // 6, p * (p + 1) * (p + 2) // 6, p + 2
    def one(nf):
        nfp = nf * Q * Q
        return 2 * V * N * (N + 1) + Q ** 3 * (2 * V * N + 30 * NL) + nfp * (4 * V * N + 2 * V * N)
    flops = n_tet * one(4) + n_prism * one(5)
    byts = (n_tet + n_prism) * 8 * (4 * V * N + N * (N + 1) // 2)
    return flops, byts


def poly_measurements(P, steps, solve=True):
    """The DG residual with the paper's Cartesian P_p basis on the
    tetrahedron / prism sphere shell (9216 tetrahedra, 4608 prisms; Section
    3.2, Section 5.2's element types), p = 1..3, Roe flux: event-timed
    launches on the solver's stream."""
    import torch
    from eg_inputs import sphere_poly
    m = sphere_poly(8, 6, 4)
    n_tet, n_pr = m.counts()
    S = P.PolySolver(m, 3, mach=0.3, flux="roe")
    out = {"mesh": f"sphere shell r 0.5..20, {n_tet} tetrahedra + {n_pr} prisms (straight-sided)", "levels": {}}
    for p in (1, 2, 3):
        u = S.freestream(p)
        u.mul_(1.0 + 0.01 * torch.rand_like(u))
        r = S.residual(p, u)
        for _ in range(3):
            S.residual(p, u, out=r)
        st = S.stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n = max(steps, 10)
        e0.record(st)
        for _ in range(n):
            S.residual(p, u, out=r)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        fl, by = poly_work(p, n_tet, n_pr)
        out["levels"][f"p{p}"] = {"ms_per_residual": round(ms, 4), "dof": m.n_elem * 5 * P.PolySolver.N(p),
                                  "algorithmic_gflop": round(fl / 1e9, 4), "achieved_tflops": round(fl / ms / 1e9, 3),
                                  "frac_fp64_vector_peak": round(fl / ms / 1e9 / 78.6, 4),
                                  "algorithmic_bytes": by, "achieved_GBps": round(by / ms / 1e6, 1)}
        log(f"[bench] tet/prism residual p={p}: {ms * 1e3:.1f} us, {fl / ms / 1e9:.2f} TFLOP/s")
        # one 4-stage PRK smoother step at CFL 100 (time step, element blocks,
        # block LU, four residuals and stage solves) from a free stream
        # perturbed by 0.1 %
        up = S.freestream(p)
        up.mul_(1.0 + 0.001 * (2.0 * torch.rand_like(up) - 1.0))
        try:
            S.prk_step(p, 4, 100.0, up)
            e0.record(st)
            for _ in range(3):
                S.prk_step(p, 4, 100.0, up)
            e1.record(st)
            torch.cuda.synchronize()
            ms_prk = e0.elapsed_time(e1) / 3
            out["levels"][f"p{p}"]["ms_per_prk_step_s4"] = round(ms_prk, 3)
            log(f"[bench] tet/prism PRK step p={p}: {ms_prk:.3f} ms")
        except P.EgError as err:
            out["levels"][f"p{p}"]["prk_step_error"] = str(err)
            log(f"[bench] tet/prism PRK step p={p} failed: {err}")
        del up
    # the eMG steady solve on the same shell (s = 4, m = 30, CFL_max 100):
    # seconds per V-cycle at every order, time to the 1e-10 drop at p = 1, 2
    out["solve"] = {}
    for p in (1, 2, 3):
        Sv = P.PolySolver(m, p, rk_stages=4, cfl_max=100.0, krylov_m=30, mach=0.3, flux="roe")
        u = Sv.freestream(p)
        Sv.vcycle(u, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(2, 7):
            Sv.vcycle(u, n)
        torch.cuda.synchronize()
        ent = {"ms_per_vcycle": round((time.perf_counter() - t0) / 5 * 1e3, 3)}
        if p <= 2 and solve:
            u = Sv.freestream(p)
            t0 = time.perf_counter()
            hist, st = Sv.solve_steady(u, drop_tol=1e-10, max_cycles=1500)
            ent.update({"converged": st == 0, "cycles": len(hist) - 1, "drop_reached": float(hist[-1] / hist[0]),
                        "time_s": round(time.perf_counter() - t0, 2)})
        out["solve"][f"p{p}"] = ent
        log(f"[bench] tet/prism eMG solve p={p}: {ent}")
        del Sv, u
    return out


def cpu_baseline(mesh, p):
    """The FP64 oracle on the host cores (all of them): one V-cycle of the
    benchmark workload from the free stream (a bounded sample, ~20 s)."""
    import oracle
    threads = int(oracle.lib().orc_get_threads())
    O = oracle.Oracle(mesh, p)
    u = O.freestream(p)
    t0 = time.perf_counter()
    u, rn, cfl = O.vcycle(u, 1, s=4, m=30, cfl_max=100.0, rref=0.0)
    el = time.perf_counter() - t0
    log(f"[bench] oracle: one V-cycle in {el:.1f}s on {threads} threads")
    return {"value": u.size / el, "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"1 V-cycle of the same workload from the free stream ({el:.1f} s, OpenMP threads = cores)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--drop-cycles", type=int, default=20000, help="cycle cap of the time-to-1e-10 runs")
    ap.add_argument("--drop-budget", type=float, default=150.0,
                    help="seconds cap of each (FP64, mixed) time-to-1e-10 run on the benchmark mesh")
    ap.add_argument("--no-drop", action="store_true", help="skip the time-to-1e-10 runs")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision measurements")
    ap.add_argument("--no-c2", action="store_true", help="skip the 2D cylinder workload")
    ap.add_argument("--c2-drop-budget", type=float, default=60.0, help="seconds of the c2 drop run (0: none)")
    ap.add_argument("--no-c1", action="store_true", help="skip the c1 time-to-1e-10 runs")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-solve batched workload")
    ap.add_argument("--batch-budget", type=float, default=30.0, help="seconds cap of the batched convergence run")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured-peak kernels")
    ap.add_argument("--no-poly", action="store_true", help="skip the tetrahedron / prism residual timing")
    ap.add_argument("--no-poly-solve", action="store_true",
                    help="tetrahedron / prism section: time V-cycles but skip the runs to the drop (profiling runs)")
    ap.add_argument("--poly-only", action="store_true",
                    help="only the tetrahedron / prism residual timing (profiling runs); prints its JSON")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--c5", action="store_true",
                    help="also run the 3D p = 3 adjoint workload (minutes: a converged 13824-hex p = 3 solve)")
    ap.add_argument("--c5-budget", type=float, default=600.0, help="seconds cap of the c5 steady solve")
    ap.add_argument("--straight", action="store_true",
                    help="straight-sided (trilinear) hexes instead of the curved (triquadratic) sphere shell")
    ap.add_argument("--calibrate", action="store_true",
                    help="end with a 256 MiB device-to-device copy (the reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(its element-domain sharding over several GPUs is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_01151_amd as P
    from eg_inputs import cubed_sphere_shell

    torch.cuda.set_device(0)
    if args.poly_only:
        res = poly_measurements(P, args.steps, solve=not args.no_poly_solve)
        if args.calibrate:
            nb = 256 << 20
            x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
            y = torch.empty_like(x)
            torch.cuda.synchronize()
            y.copy_(x)
            torch.cuda.synchronize()
            res["calibration_copy_bytes"] = nb
        print(json.dumps({"tet_prism_residual": res}), flush=True)
        return
    # the sphere grid is built from quadratic curved elements (Section 5.2)
    mesh = cubed_sphere_shell(16, 24, curved=not args.straight)
    nodes = 8 if args.straight else 27
    d, p = 3, 2
    dof = mesh.n_elem * 5 * 27
    kw = dict(rk_stages=4, cfl_max=100.0, krylov_m=30, mach=0.3, alpha_deg=0.0)
    log("[bench] init")
    S = P.Solver(mesh, p, **kw)
    tiles = S.autotune()  # residual tiles per order and precision (outside the timed region)
    log(f"[bench] residual tiles (elements per workgroup): {tiles}")
    u = S.freestream(p)
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.steps, resume=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    log(f"[bench] timed {args.steps} cycles: {ms_per_step:.3f} ms/cycle")
    peaks = {}
    if not args.no_peaks:
        peaks = {"hbm_gbs": P.binding.measure_peak("hbm"), "fp64_mfma_tflops": P.binding.measure_peak("fp64_mfma"),
                 "fp64_fma_tflops": P.binding.measure_peak("fp64_fma")}
        log(f"[bench] measured peaks: {peaks}")
    # event-timed pass over the same number of cycles for the per-kernel roofline
    prof = profile_cycles(S, u, p, args.steps)
    tot = sum(v[0] for v in prof.values())
    log("[bench] kernel time per cycle (ms):",
        ", ".join(f"{k}={v[0] / args.steps:.4f}" for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])))
    cands = [(v[0], k) for k, v in prof.items() if k.split("@")[0] in ("residual", "jacobian_lu", "prk_stage")]
    ms_dom, key = max(cands)
    cls, lev = key.split("@")[0], int(key.split("@p")[1])
    roof = roofline_entry(cls, lev, prof[key][0], prof[key][1], mesh.n_elem, d, peaks, nodes)
    roof["share_of_kernel_time"] = ms_dom / tot
    extras = {"kernels_ms_per_cycle": {k: round(v[0] / args.steps, 5) for k, v in prof.items()},
              "kernel_time_per_cycle_ms": round(tot / args.steps, 4),
              "residual_tiles": {f"p{q}/{k}": t for (q, k), t in tiles.items()}, "measured_peaks": peaks}
    for c2 in ("residual", "jacobian_lu", "prk_stage"):
        k2 = f"{c2}@p{p}"
        if k2 in prof:
            e2 = roofline_entry(c2, p, prof[k2][0], prof[k2][1], mesh.n_elem, d, peaks, nodes)
            extras[f"roofline_{c2}_p{p}"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in e2.items()}
    arn = prof.get("arnoldi@p0")
    if arn:
        # Arnoldi traffic model: per step one product over J0 (diagonal and
        # neighbour V x V blocks, neighbour values) plus the CGS2 passes over the
        # basis (about 4 (j + 1) K0-vector passes at step j), 8 bytes per value
        K0 = mesh.n_elem * 5
        m = 30
        byts = m * (K0 * 5 * (1 + 6) * 8 + K0 * 8 * 7) + sum(4 * (j + 1) * K0 * 8 for j in range(m))
        extras["arnoldi"] = {"ms_per_cycle": round(arn[0] / args.steps, 4), "model_bytes_per_exp1": byts,
                             "model_GBps": byts / (arn[0] / args.steps * 1e-3) / 1e9}
    config = {"workload": "3D sphere, cubed-sphere hex shell 6x16x16x24 = 36864 "
                          + ("straight-sided (trilinear)" if args.straight else "quadratic curved (27-node)")
                          + " hexes, DG p=2 (27 modes x 5 vars), "
                          "eMG V-cycle p2->p1->p0, 4-stage PRK, EXP1 Krylov m=30, CFL_max 100, Ma 0.3, "
                          "free-stream start, FP64",
              "n_elem": mesh.n_elem, "dof": dof, "p_max": p, "rk_stages": 4, "krylov_m": 30, "cfl_max": 100.0}
    u64 = None
    if not args.no_drop:
        config["fp64_drop"], u64 = drop_run(S, p, args.drop_cycles, args.drop_budget, "c3 fp64")
    del S
    torch.cuda.empty_cache()
    if not args.straight:
        # the same shell with straight-sided hexes: per-cycle cost of the
        # triquadratic geometry (the trilinear kernel instantiations)
        Ss = P.Solver(cubed_sphere_shell(16, 24), p, **kw)
        Ss.autotune()
        us = Ss.freestream(p)
        Ss.solve_steady(us, drop_tol=0.0, max_cycles=args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Ss.solve_steady(us, drop_tol=0.0, max_cycles=args.steps, resume=True)
        torch.cuda.synchronize()
        extras["straight_sided_hexes_ms_per_cycle"] = round((time.perf_counter() - t0) / args.steps * 1e3, 4)
        log(f"[bench] straight-sided hexes: {extras['straight_sided_hexes_ms_per_cycle']} ms/cycle")
        del Ss, us
        torch.cuda.empty_cache()
    if not args.no_mixed:
        Sm = P.Solver(mesh, p, precision="mixed", **kw)
        Sm.autotune()
        um = Sm.freestream(p)
        Sm.solve_steady(um, drop_tol=0.0, max_cycles=args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sm.solve_steady(um, drop_tol=0.0, max_cycles=args.steps, resume=True)
        torch.cuda.synchronize()
        ms_m = (time.perf_counter() - t0) / args.steps * 1e3
        mixed = {"ms_per_cycle_from_free_stream": round(ms_m, 4), "dof_updates_per_s": dof / ms_m * 1e3,
                 "speedup_per_cycle_vs_fp64": round(ms_per_step / ms_m, 3)}
        log(f"[bench] mixed: {ms_m:.3f} ms/cycle")
        if not args.no_drop:
            mixed["drop"], umx = drop_run(Sm, p, args.drop_cycles, args.drop_budget, "c3 mixed")
            fd, md = config.get("fp64_drop", {}), mixed["drop"]
            if fd.get("converged") and md["converged"]:
                diff = float(torch.max(torch.abs(umx - u64)) / torch.max(torch.abs(u64)))
                mixed["final_state_rel_diff_vs_fp64"] = diff
                mixed["time_to_1e-10_speedup_vs_fp64"] = round(fd["time_to_1e-10_s"] / md["time_to_1e-10_s"], 3)
                log(f"[bench] mixed vs fp64 final state: {diff:.3e}")
            del umx
        config["mixed"] = mixed
        del Sm, um
        torch.cuda.empty_cache()
    del u64
    if not args.no_c2:
        extras["c2"] = c2_measurements(P, args.steps, args.warmup, args.c2_drop_budget)
        if not args.no_c1:
            extras["c1_time_to_1e-10"] = c1_time_to_drop(P)
    if not args.no_batched:
        extras["batched"] = batched_measurements(P, 10, args.batch_budget)
    if not args.no_poly:
        extras["tet_prism_residual"] = poly_measurements(P, args.steps, solve=not args.no_poly_solve)
    if args.c5:
        extras["c5_adjoint"] = c5_adjoint(P, args.c5_budget)
    if args.calibrate:
        nb = 256 << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        extras["calibration_copy_bytes"] = nb
        log(f"[bench] calibration copy of {nb} bytes done")
    cpu = None if args.no_cpu_baseline else cpu_baseline(mesh, p)
    fd = config.get("fp64_drop") or {}
    if cpu and fd.get("converged"):
        # labelled extrapolation: the GPU FP64 solve's cycle count times the
        # oracle's measured seconds per cycle (the oracle is not run to the drop)
        per_cycle = mesh.n_elem * 5 * 27 / cpu["value"]
        cpu["time_to_1e-10_extrapolated_s"] = round(fd["cycles_to_1e-10"] * per_cycle, 1)
        cpu["extrapolation"] = "cycles_to_1e-10 of the FP64 GPU solve x the oracle's seconds per V-cycle"
    line = {
        "metric": "V-cycle DOF-updates/s & time to 1e-10 residual drop, FP64 vs mixed precision",
        "value": dof * args.steps / wall,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
