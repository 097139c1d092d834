"""Benchmark of the eMG V-cycle on one MI355X.

Workload: 2D cylinder, O-grid 128 x 64 quads (radius 0.5 to 20, geometric
radial stretch), modal DG p = 3 (16 modes x 4 variables per element, 524,288
DOF), Rusanov flux, slip wall + characteristic far field, Ma = 0.3, FP64,
V-cycle p3 -> p2 -> p1 -> p0 with a 3-stage PRK smoother and the EXP1 step
(Krylov dimension 30) on p0, CFL_max = 10, free-stream start.

A step is one V-cycle (entry residual + norm, PRK on p = 3, 2, 1, EXP1 on
p = 0, transfers).  value = DOF-updates/s = DOF x cycles / wall time of the
timed cycles.  The run also reports the time to a 1e-10 residual drop from
the free stream, the event-timed roofline of the dominant kernel, and the
FP64 CPU oracle timed on a bounded sample on the host.

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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_VALU_TFLOPS = 78.6      # MI355X FP64 vector peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def work_model(d, p):
    """Algorithmic work per element of the three main kernels at order p."""
    V, N, Q = d + 2, (p + 1) ** d, p + 2
    QV, QF, NF, NC = Q ** d, Q ** (d - 1), 2 * d, 2 ** d
    n = V * N
    return {
        # dense modal contractions: state at volume points, gradient projection,
        # own and neighbour traces and face projection (2 FLOP per FMA)
        "residual": {"flop": 2 * V * N * (QV * (1 + d) + 3 * NF * QF),
                     "bytes": (2 * V * N + NC * d) * 8 + NF * 5},
        # block assembly contraction + LU (2/3 n^3) of the n x n PRK block
        "jacobian_lu": {"flop": 2 * N * N * V * V * (QV * d + NF * QF) + (2 * n ** 3) // 3,
                        "bytes": (V * N + NC * d + N * (N + 1) // 2) * 8 + n * n * 8 + n * 4},
        # LU solve: read the factors, permutation, residual, base state; write the stage
        "prk_stage": {"flop": 2 * n * n, "bytes": n * n * 8 + n * 4 + 3 * n * 8},
    }


# kernels behind each timed class (bench time classes -> device functions)
CLASS_KERNELS = {"jacobian_lu": ["k_jac_points", "k_jaclu_wave", "wave_max_u32", "readlane_d", "bperm_d"],
                 "prk_stage": ["k_prk_stage_t", "k_prk_stage"],
                 "residual": ["k_residual", "stage"]}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobian_lu_c2_pmc_traffic.md")


def kernel_source_digest(cls):
    """sha256 over the shared device headers and the text of the device
    functions of one kernel class (their definitions: lines that declare a
    __device__ or __global__ function of that name), so that a stored counter
    reading can be matched to the code it was taken on."""
    csrc = os.path.join(ROOT, "paper_1807_01151_amd", "csrc")
    h = hashlib.sha256()
    for f in ("eg_common.h", "eg_physics.h"):
        h.update(open(os.path.join(csrc, f), "rb").read())
    src = open(os.path.join(csrc, "eg_kernels.hip")).read()
    for name in CLASS_KERNELS[cls]:
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


def roofline_entry(cls, p, ms, launches, ne, d):
    w = work_model(d, p)[cls]
    avg_s = ms / launches / 1e3
    if cls == "prk_stage":
        ach = w["bytes"] * ne / avg_s / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": stored_traffic(cls, p), "kernel": f"{cls} p={p}", "avg_launch_ms": ms / launches,
                "algorithmic_bytes_per_launch": w["bytes"] * ne}
    ach = w["flop"] * ne / avg_s / 1e12
    return {"bound": "alu", "achieved": ach, "peak": FP64_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP64_VALU_TFLOPS, "traffic": stored_traffic(cls, p), "kernel": f"{cls} p={p}",
            "avg_launch_ms": ms / launches, "algorithmic_flop_per_launch": w["flop"] * ne}


def cpu_baseline(mesh, budget_s=12.0):
    """The FP64 oracle on the host cores: V-cycles of the same workload from the
    free stream until about budget_s seconds of work (at least one cycle)."""
    import oracle
    O = oracle.Oracle(mesh, 3)
    u = O.freestream(3)
    dof = u.size
    t0 = time.perf_counter()
    cycles = 0
    rref = None
    while True:
        u, rn, cfl = O.vcycle(u, cycles + 1, s=3, m=30, cfl_max=10.0, rref=rref if rref else 0.0)
        if rref is None:
            rref = rn
        cycles += 1
        el = time.perf_counter() - t0
        log(f"[bench] oracle cycle {cycles}: {el:.1f}s")
        if el > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": dof * cycles / el, "unit": "DOF-updates/s", "cores": int(oracle.lib().orc_get_threads()),
            "kind": "oracle", "sample": f"{cycles} V-cycles of the same workload from the free stream "
                                        f"({el:.1f} s, OpenMP threads = cores)"}


def drop_run(S, p, max_cycles, budget, tag):
    """Solve from the free stream to a 1e-10 drop in chunks of 500 cycles (same
    ramp and cycle numbering), each chunk reporting its progress; stops at the
    drop, the cycle cap or the time budget."""
    import torch
    u2 = S.freestream(p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    chunk = 500
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
           "time_to_1e-10_s": round(t_drop, 4) if st == 0 else None, "drop_run_s": round(t_drop, 3),
           "drop_reached": float(last / r1), "converged": st == 0}
    log(f"[bench] {tag} drop run: {out}")
    return out


def mixed_measurements(P, mesh, p, dof, args, fp64_ms):
    """Mixed precision on the benchmark workload: V-cycle cost in phase A
    (FP32 residuals, blocks and stage solves) from the free stream, and in
    phase B (FP64 residuals, FP32 blocks and stage solves) once the solve has
    switched (r <= 1e-4 r_1)."""
    import torch
    S = P.Solver(mesh, p, rk_stages=3, cfl_max=10.0, krylov_m=30, mach=0.3, alpha_deg=0.0, precision="mixed")
    S.autotune()
    u = S.freestream(p)
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h, _ = S.solve_steady(u, drop_tol=0.0, max_cycles=args.steps)
    torch.cuda.synchronize()
    ms_a = (time.perf_counter() - t0) / args.steps * 1e3
    # run on (phase A) until the switch, then time phase-B cycles
    r1 = h[0]
    done = 0
    while h[-1] > 1e-4 * r1 and done < 5000:
        h, _ = S.solve_steady(u, drop_tol=0.0, max_cycles=250, resume=True)
        done += 250
    S.solve_steady(u, drop_tol=0.0, max_cycles=2, resume=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.steps, resume=True)
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) / args.steps * 1e3
    log(f"[bench] mixed: phase A {ms_a:.3f} ms/cycle, phase B {ms_b:.3f} ms/cycle (FP64 {fp64_ms:.3f})")
    return {"phase_a_ms_per_cycle": round(ms_a, 4), "phase_b_ms_per_cycle": round(ms_b, 4),
            "phase_a_dof_updates_per_s": dof / ms_a * 1e3, "phase_b_dof_updates_per_s": dof / ms_b * 1e3,
            "phase_a_speedup_vs_fp64": round(fp64_ms / ms_a, 3), "phase_b_speedup_vs_fp64": round(fp64_ms / ms_b, 3)}


def sphere_measurements(P, warmup=2, steps=10):
    """FP64 against mixed precision on the 3D sphere workload (cubed-sphere
    hex shell 6 x 16 x 16 x 24 = 36864 hexes, p = 2, 135 x 135 blocks): V-cycle
    cost from the free stream (the mixed solve is in phase A there)."""
    import torch
    from eg_inputs import cubed_sphere_shell
    mesh = cubed_sphere_shell(16, 24)
    dof = mesh.n_elem * 27 * 5
    out = {"workload": "3D sphere, cubed-sphere hex shell 6x16x16x24 = 36864 hexes, DG p=2 (27 modes x 5 vars), "
                       "eMG V-cycle p2->p0, 3-stage PRK, EXP1 m=30, CFL 10, Ma 0.3, free-stream start",
           "dof": dof}
    for prec in ("fp64", "mixed"):
        S = P.Solver(mesh, 2, rk_stages=3, cfl_max=10.0, krylov_m=30, mach=0.3, alpha_deg=0.0, precision=prec)
        S.autotune()
        u = S.freestream(2)
        S.solve_steady(u, drop_tol=0.0, max_cycles=warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.solve_steady(u, drop_tol=0.0, max_cycles=steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[f"{prec}_ms_per_cycle"] = round(ms, 3)
        out[f"{prec}_dof_updates_per_s"] = dof / ms * 1e3
        log(f"[bench] sphere {prec}: {ms:.3f} ms/cycle")
        del S, u
        torch.cuda.empty_cache()
    out["mixed_speedup_vs_fp64"] = round(out["fp64_ms_per_cycle"] / out["mixed_ms_per_cycle"], 3)
    return out


def batched_measurements(P, steps, budget_s, precision="mixed"):
    """The batched workload: 64 independent cylinder solves drawn from seed
    1807 (N_theta ~ U{16..96}, N_r = N_theta / 2, p ~ U{1..4}, Ma ~ U[0.1,
    0.4], alpha ~ U[-5, 5] deg), one batch handle per order (every kernel
    launch covers all solves of that order).  Reports the V-cycle
    throughput of the whole batch and, within a time budget, how many solves
    reach the 1e-10 drop."""
    import torch
    from eg_inputs import batch_draws, ogrid
    draws = batch_draws(64, seed=1807)
    groups = {}
    for i, d in enumerate(draws):
        groups.setdefault(d["p"], []).append(i)
    t_init = time.perf_counter()
    handles = {}
    for p, idx in sorted(groups.items()):
        meshes = [ogrid(draws[i]["n_theta"], draws[i]["n_r"]) for i in idx]
        B = P.BatchSolver(meshes, p, [draws[i]["mach"] for i in idx], [draws[i]["alpha_deg"] for i in idx],
                          rk_stages=3, cfl_max=10.0, krylov_m=30, precision=precision)
        B.autotune()  # residual tiles of this order group
        handles[p] = (B, B.freestream(p), idx)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t_init
    dof = sum(B.n_elem * B.V * B.N(p) for p, (B, _, _) in handles.items())
    for p, (B, u, _) in handles.items():
        B.solve(u, drop_tol=0.0, max_cycles=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, (B, u, _) in handles.items():
        B.solve(u, drop_tol=0.0, max_cycles=steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"solves": 64, "elements": int(sum(B.n_elem for B, _, _ in handles.values())), "dof": int(dof),
           "groups": {str(p): len(idx) for p, (_, _, idx) in handles.items()}, "precision": precision,
           "setup_s": round(t_init, 3), "ms_per_batched_cycle": round(wall / steps * 1e3, 3),
           "dof_updates_per_s": dof * steps / wall}
    log(f"[bench] batched: {out}")
    # convergence within the budget: each order group from its free streams
    import numpy as np
    conv, div, drops = 0, 0, []
    t1 = time.perf_counter()
    for p, (B, _, idx) in sorted(handles.items()):
        left = budget_s - (time.perf_counter() - t1)
        if left <= 0:
            break
        u = B.freestream(p)
        # cycle cap from the measured cost so the group fits its share of the budget
        cap = max(10, int(left / len(handles) / max(wall / steps / len(handles), 1e-4)))
        hists, cyc, st = B.solve(u, drop_tol=1e-10, max_cycles=cap)
        ok = sum(1 for h in hists if h[-1] <= 1e-10 * h[0])
        bad = sum(1 for h in hists if not np.isfinite(h[-1]))
        conv += ok
        div += bad
        drops += [float(h[-1] / h[0]) for h in hists if np.isfinite(h[-1])]
        log(f"[bench] batched p={p}: {ok}/{len(hists)} converged, {bad} diverged, cap {cap} cycles, "
            f"{time.perf_counter() - t1:.1f}s")
    out["converged_to_1e-10"] = conv
    out["diverged"] = div
    out["median_drop_reached"] = float(np.median(drops)) if drops else None
    out["convergence_run_s"] = round(time.perf_counter() - t1, 2)
    for B, _, _ in handles.values():
        B.close()
    return out


def c1_time_to_drop(P):
    """Time to a 1e-10 FP64 residual drop on the O-grid 24 x 12, p = 1 solve
    (s = 4, CFL_max = 100, m = 30), which converges, in FP64 and mixed."""
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--drop-cycles", type=int, default=100000, help="cycle cap of the time-to-1e-10 run")
    ap.add_argument("--drop-budget", type=float, default=60.0,
                    help="seconds cap of each (FP64, mixed) time-to-1e-10 run on the benchmark mesh")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision measurements")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-solve batched workload")
    ap.add_argument("--no-sphere", action="store_true",
                    help="skip the FP64 / mixed V-cycle timing on the 3D sphere (also skipped by --no-mixed)")
    ap.add_argument("--batch-budget", type=float, default=30.0, help="seconds cap of the batched convergence run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-drop", action="store_true", help="skip the time-to-1e-10 run")
    ap.add_argument("--calibrate", action="store_true",
                    help="end with a 256 MiB device-to-device copy (the reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(its element-domain sharding over several GPUs is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1807_01151_amd as P
    from eg_inputs import ogrid

    torch.cuda.set_device(0)
    mesh = ogrid(128, 64)
    d, p = 2, 3
    log("[bench] init")
    S = P.Solver(mesh, p, rk_stages=3, cfl_max=10.0, krylov_m=30, mach=0.3, alpha_deg=0.0)
    tiles = S.autotune()  # residual tiles per order and precision (outside the timed region)
    log(f"[bench] residual tiles (elements per workgroup): {tiles}")
    dof = mesh.n_elem * 4 * 16
    u = S.freestream(p)
    # warm-up cycles
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} done")
    # timed cycles
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    log(f"[bench] timed {args.steps} cycles: {ms_per_step:.3f} ms/cycle")
    # event-timed pass over the same number of cycles for the per-kernel roofline
    S.profile(True)
    S.solve_steady(u, drop_tol=0.0, max_cycles=args.steps)
    prof = {}
    for cls in P.binding.KERNEL_CLASSES:
        for lev in range(p + 1):
            ms, n = S.profile_read(cls, lev)
            if n:
                prof[f"{cls}@p{lev}"] = (ms, n)
    S.profile(False)
    tot = sum(v[0] for v in prof.values())
    log("[bench] kernel time per cycle (ms):",
        ", ".join(f"{k}={v[0] / args.steps:.4f}" for k, v in sorted(prof.items(), key=lambda kv: -kv[1][0])))
    cands = [(v[0], k) for k, v in prof.items() if k.split("@")[0] in ("residual", "jacobian_lu", "prk_stage")]
    ms_dom, key = max(cands)
    cls, lev = key.split("@")[0], int(key.split("@p")[1])
    roof = roofline_entry(cls, lev, prof[key][0], prof[key][1], mesh.n_elem, d)
    roof["share_of_kernel_time"] = ms_dom / tot
    extras = {"kernels_ms_per_cycle": {k: round(v[0] / args.steps, 5) for k, v in prof.items()},
              "residual_tiles": {f"p{q}/{k}": t for (q, k), t in tiles.items()}}
    for c2 in ("residual", "jacobian_lu", "prk_stage"):
        k2 = f"{c2}@p{p}"
        if k2 in prof:
            e2 = roofline_entry(c2, p, prof[k2][0], prof[k2][1], mesh.n_elem, d)
            extras[f"roofline_{c2}_p{p}"] = {"achieved": round(e2["achieved"], 3), "unit": e2["unit"],
                                             "frac": round(e2["frac"], 4), "bound": e2["bound"]}
    # time to a 1e-10 residual drop from the free stream
    drop = {}
    if not args.no_drop:
        drop = drop_run(S, p, args.drop_cycles, args.drop_budget, "fp64")
    mixed = None
    if not args.no_mixed:
        mixed = mixed_measurements(P, mesh, p, dof, args, ms_per_step)
        if not args.no_drop:
            Sm = P.Solver(mesh, p, rk_stages=3, cfl_max=10.0, krylov_m=30, mach=0.3, alpha_deg=0.0,
                          precision="mixed")
            mixed["drop_run"] = drop_run(Sm, p, args.drop_cycles, args.drop_budget, "mixed")
            del Sm
        mixed["c1_time_to_1e-10"] = c1_time_to_drop(P)
        extras["mixed"] = mixed
        if not args.no_sphere:
            extras["sphere"] = sphere_measurements(P)
    if not args.no_batched:
        extras["batched"] = batched_measurements(P, 10, args.batch_budget)
    if args.calibrate:
        nb = 256 << 20
        x = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        extras["calibration_copy_bytes"] = nb
        log(f"[bench] calibration copy of {nb} bytes done")
    cpu = None if args.no_cpu_baseline else cpu_baseline(mesh)
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
        "config": {"workload": "2D cylinder O-grid 128x64 quads, DG p=3 (16 modes x 4 vars), eMG V-cycle "
                               "p3->p0, 3-stage PRK, EXP1 Krylov m=30, CFL 10, Ma 0.3, free-stream start, FP64",
                   "n_elem": mesh.n_elem, "dof": dof, "p_max": p, "rk_stages": 3, "krylov_m": 30,
                   "cfl_max": 10.0, **drop},
        "roofline": roof,
        "cpu_baseline": cpu,
        "detail": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
