#!/usr/bin/env python
"""Full-solve benchmark of the MI355X octree multigrid PCG solver.

One step = one complete solve A p = rhs from p = 0 to relative residual 1e-10
(PCG, Algorithm 1, preconditioned by one FAS-style cycle, Algorithm 4) on
the large adaptive cut-cell workload: leaf levels 7..10 refined where 4^3
nodes touch 8 seeded spheres or the surface of a solid box, beta = fluid face
fraction with 1% jitter, Neumann walls and solid, Dirichlet top wall, seeded
zero-mean random right-hand side (synthetic inputs, about 26.3M leaves).
Inputs are resident in HBM before the timed region; octree, coefficients and
hierarchy are built beforehand.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Counter passes for the HBM traffic of the finest half-sweep (each under its
own `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` run):

    python bench.py --traffic-pass [--traffic-fp64]   # half-sweeps + a plain copy
    python bench.py --summarize-pmc FETCH.csv WRITE.csv  # mixed or fp64 record

Prints one JSON line.  `value` is the mixed-precision solve rate (FP32
cycle with FP16 inner coefficients inside FP64 PCG) in million active leaf
cells per second; the FP64 solve rate is reported beside it.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("PCG+MG full-solve Mcells/s to 1e-10 rel resid (FP64 vs mixed); "
          "V-cycle HBM GB/s")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources that define the kernels and their launches (the
    dominant kernel, everything it calls, the Krylov kernels and the host
    code that sets grids and cache policies)."""
    h = hashlib.sha256()
    for f in ("kernels.hpp", "device.hpp", "pcg_kernels.hpp", "mfmg.hip"):
        with open(os.path.join(ROOT, "paper_2604_18886_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision_name, level, key="hbm_bytes_per_launch"):
    """HBM bytes per launch of the dominant kernel (or, with key, per whole
    cycle) from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_smooth_large_workload.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    rec = t.get(precision_name)
    if not rec or rec.get("source_hash") != kernel_source_hash() or rec.get("level") != level:
        return None
    return rec.get(key)


def traced_launch_us(kernel):
    """Average duration (us) of a kernel in the committed rocprofv3 kernel
    statistics of the benchmark, if taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "kernel_trace_large_workload.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_hash") != kernel_source_hash():
        return None
    rec = t.get("kernels", {}).get(kernel)
    return rec["avg_us"] if rec else None


def summarize_trace(stats_csv):
    """Per-kernel calls and average duration from a rocprofv3 --stats
    kernel_stats.csv, stored with the kernel source hash."""
    import csv
    kernels = {}
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            # "void mfmg::k_smooth<float, float, __half, 256, 0>(mfmg::LevelArgs<...>, int)"
            # -> "mfmg::k_smooth<float, float, __half, 256, 0>"
            name = r["Name"].strip()
            if name.startswith("void "):
                name = name[5:]
            name = name.split("(", 1)[0]
            kernels[name] = {"calls": int(r["Calls"]),
                             "avg_us": float(r["AverageNs"]) / 1e3,
                             "total_ms": float(r["TotalDurationNs"]) / 1e6}
    rec = {"source_hash": kernel_source_hash(), "kernels": kernels}
    path = os.path.join(ROOT, "profiles", "kernel_trace_large_workload.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


COPY_BYTES = 1 << 30      # plain copy used to scale the counters
TRAFFIC_REPS = 4


def smooth_precision(kernel_name):
    """Hierarchy a half-sweep dispatch belongs to, from its kernel name:
    FP32 values (the mixed cycle) or FP64 values."""
    if "k_smooth<float" in kernel_name:
        return "mixed"
    if "k_smooth<double" in kernel_name:
        return "fp64"
    return None


CYCLE_KERNELS = ("k_fill", "k_smooth", "k_restrict", "k_fas_rhs", "k_bottom", "k_prolong",
                 "k_coarsest")


def summarize_pmc(fetch_csv, write_csv, level):
    """HBM bytes per launch of the finest half-sweep (mixed or FP64, from the
    kernel name) and per whole cycle, from two rocprofv3 counter_collection.csv
    files (FETCH_SIZE, WRITE_SIZE in KiB per dispatch) of a --traffic-pass
    run, each scaled by what the same counter reads for a plain copy of
    COPY_BYTES bytes.  The half-sweeps are the k_smooth dispatches before the
    first cycle's k_fill; the cycles are every cycle kernel after it, per
    k_bottom dispatch (one per V-cycle).  Returns (precision, record)."""
    import csv

    def dispatches(path, counter):
        """(dispatch id, kernel name, bytes) in dispatch order; a counter
        summed over its instances."""
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r.get("Counter_Name") != counter:
                    continue
                key = int(r["Dispatch_Id"])
                name, v = acc.get(key, (r["Kernel_Name"], 0.0))
                acc[key] = (name, v + float(r["Counter_Value"]) * 1024.0)
        return [(k, n, v) for k, (n, v) in sorted(acc.items())]

    out = {}
    precisions = set()
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = dispatches(path, counter)
        first_fill = min((d for d, n, _ in rows if "k_fill" in n), default=None)
        smooth = [v for d, n, v in rows if "k_smooth<" in n
                  and (first_fill is None or d < first_fill)]
        precisions |= {smooth_precision(n) for _, n, _ in rows if "k_smooth<" in n}
        cyc = [(d, n, v) for d, n, v in rows if first_fill is not None and d >= first_fill
               and any(k in n for k in CYCLE_KERNELS)]
        ncyc = sum(1 for _, n, _ in cyc if "k_bottom" in n)
        last = max((d for d, n, _ in rows if any(k in n for k in CYCLE_KERNELS)), default=None)
        # the TRAFFIC_REPS device copies of COPY_BYTES that follow the
        # half-sweeps and cycles (earlier copy dispatches move other buffers)
        copy = [v for d, n, v in rows
                if last is not None and d > last and "copy" in n.lower()]
        if not smooth or len(copy) != TRAFFIC_REPS or not ncyc:
            raise SystemExit(f"{path}: expected k_smooth dispatches, cycles and "
                             f"{TRAFFIC_REPS} copies for {counter}")
        factor = (sum(copy) / len(copy)) / COPY_BYTES
        out[counter] = {"per_launch_bytes_raw": sum(smooth) / len(smooth),
                        "launches": len(smooth), "copy_raw_bytes": sum(copy) / len(copy),
                        "copy_factor": factor,
                        "per_launch_bytes": sum(smooth) / len(smooth) / factor,
                        "cycles": ncyc,
                        "per_cycle_bytes": sum(v for _, _, v in cyc) / ncyc / factor}
    if len(precisions) != 1 or None in precisions:
        raise SystemExit("expected the half-sweeps of one hierarchy, found "
                         f"{sorted(map(str, precisions))}")
    rec = {"source_hash": kernel_source_hash(), "level": level,
           "fetch_bytes_per_launch": out["FETCH_SIZE"]["per_launch_bytes"],
           "write_bytes_per_launch": out["WRITE_SIZE"]["per_launch_bytes"],
           "hbm_bytes_per_launch": (out["FETCH_SIZE"]["per_launch_bytes"]
                                    + out["WRITE_SIZE"]["per_launch_bytes"]),
           "cycle_fetch_bytes": out["FETCH_SIZE"]["per_cycle_bytes"],
           "cycle_write_bytes": out["WRITE_SIZE"]["per_cycle_bytes"],
           "cycle_hbm_bytes": (out["FETCH_SIZE"]["per_cycle_bytes"]
                               + out["WRITE_SIZE"]["per_cycle_bytes"]),
           "counters": out}
    return precisions.pop(), rec


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, iters_full, n_iter=2):
    """The oracle (test infrastructure) timed on the host, one thread, on the
    benchmark's own workload: its octree, discretisation and hierarchy are
    built (not timed), then PCG is run for n_iter iterations (n_iter + 1
    cycles and operator applications with the initial cycle and the final
    true residual); the full solve's time is that scaled to the iters_full
    iterations the solve to 1e-10 takes, i.e. (iters_full + 1) / (n_iter + 1)
    times the measured time."""
    from threadpoolctl import threadpool_limits

    import problems
    from oracle import discretize as D
    from oracle import krylov as K
    from oracle import multigrid as M
    from oracle import octree as O

    t0 = time.perf_counter()
    spec = problems.config_spec(cfg)
    T = O.Octree(spec)
    bc, th = problems.config_bc(cfg)
    disc = D.Discretization(T, None, bc, th)
    disc.set_beta(problems.face_beta(cfg, disc.face_level, disc.face_ijk, disc.face_dir))
    rhs = problems.rhs_random(cfg, T.level, T.ijk)
    H = M.Hierarchy(disc)
    setup = time.perf_counter() - t0
    log(f"[bench] oracle set up in {setup:.0f} s; timing {n_iter} PCG iterations")
    with threadpool_limits(1):
        t0 = time.perf_counter()
        K.pcg(disc.A, rhs, H.vcycle, 1e-10, n_iter, active=disc.active)
        dt = time.perf_counter() - t0
    nact = int(disc.active.sum())
    full = dt * (iters_full + 1) / (n_iter + 1)
    return {"value": nact / full / 1e6, "unit": "Mcells/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": (f"the benchmark's workload ({T.n} leaves, {nact} active): {n_iter} PCG "
                       f"iterations of the oracle ({n_iter + 1} cycles and operator "
                       f"applications) in {dt:.1f} s, scaled to the {iters_full} iterations of "
                       f"the solve to 1e-10 ({full:.0f} s); NumPy/SciPy FP64, 1 thread of "
                       f"{os.cpu_count()} ({cpu_model()}); octree, discretisation and "
                       f"hierarchy built beforehand in {setup:.0f} s")}


def oracle_sample(cfg):
    """The oracle's solution of the workload at relative residual 1e-13,
    sampled at seeded active leaves (written by
    tests/golden/make_large_workload_sample.py), or None."""
    if cfg != 4:
        return None
    path = os.path.join(ROOT, "tests", "golden", "large_workload_solution_sample.npz")
    if not os.path.exists(path):
        return None
    import numpy as np
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def error_vs_oracle(p, sample):
    """Relative L2 error of the solution p (device tensor, canonical order)
    against the oracle's p* over the sampled leaves, and the relative
    difference of the full 2-norms."""
    import numpy as np
    import torch
    idx = torch.as_tensor(sample["idx"], device=p.device)
    got = p[idx].cpu().numpy()
    want = sample["val"]
    return {"rel_l2_sampled": float(np.linalg.norm(got - want) / np.linalg.norm(want)),
            "rel_norm_diff": float(abs(torch.linalg.norm(p).item() - float(sample["norm"]))
                                   / float(sample["norm"])),
            "samples": int(len(want)), "oracle_rtol": float(sample["rtol"])}


def projection_timing(mfmg, torch, h, beta_d, fdir, kind, bc, reps=5):
    """The projection wrapper on the workload with the static test's field
    u = (0, -1, 0) (zero on solid walls): wall time of the divergence and
    of the velocity update (best of reps), one projection end to end, and
    the volume-weighted RMS divergence before and after."""
    import numpy as np
    d = np.asarray(fdir)
    u = np.where((d >> 1) == 1, -1.0, 0.0)
    u[(np.asarray(kind) == 0) & (np.asarray(bc)[d] == 0)] = 0.0
    u0 = torch.as_tensor(u, dtype=torch.float64, device="cuda")
    del u
    uw = u0.clone()

    def best(fn):
        fn()
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append(time.perf_counter() - t0)
        return min(t) * 1e3

    div = mfmg.divergence(h, beta_d, u0)
    pz = torch.zeros_like(div)
    ms_div = best(lambda: mfmg.divergence(h, beta_d, u0))
    ms_upd = best(lambda: mfmg.project_velocity(h, beta_d, pz, uw))
    uw.copy_(u0)
    mfmg.project(h, beta_d, uw)
    uw.copy_(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st, rms0, rms1 = mfmg.project(h, beta_d, uw)
    torch.cuda.synchronize()
    total = (time.perf_counter() - t0) * 1e3
    return {"divergence_ms": ms_div, "update_ms": ms_upd, "projection_ms": total,
            "iters": st["iters"], "rms_div_before": rms0, "rms_div_after": rms1,
            "field": "u = (0, -1, 0), zero on solid walls", "rtol": 1e-10}


def fit_slope(x, y):
    """Least-squares slope of log2(y) against x."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    ly = np.log2(np.asarray(y, dtype=np.float64))
    return float(np.polyfit(x, ly, 1)[0])


def static_projection(mfmg, torch, obstacle, root_level, rtol=1e-6, mu=2, sweep_iters=8):
    """The static projection test (Section 4.4) on one grid: tank with solid
    floor and sides and an open top, a solid sphere or star at the centre,
    u = (0, -1, 0); mixed-precision hierarchy with the mu-cycle, PCG to rtol.
    The discrete solution is p = y - 1 exactly (the discretisation
    reproduces linear fields), so the pressure error and the velocity left
    after the update measure the solve alone.  RMS_V of the divergence in
    two readings: of div_i / V_i (the divergence density) and of the
    integrated divergence div_i (a flux)."""
    import numpy as np
    import problems
    spec = problems.tank_spec(root_level, obstacle)
    bc, theta = problems.tank_bc()
    t0 = time.perf_counter()
    tree = mfmg.build_octree(spec, device=True)
    lev, ijk = tree.leaves()
    owner, fdir, other, kind = tree.faces()
    beta = problems.tank_beta(obstacle, lev[owner], ijk[owner], fdir)
    u0 = problems.tank_velocity(fdir, kind, bc)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    beta_d, u0_d = dev(beta), dev(u0)
    del beta, u0, owner, other, kind
    co = mfmg.assemble_coeffs(tree, beta_d, bc, theta)
    h = mfmg.build_hierarchy(co, precision=mfmg.MIXED, mu=mu)
    act = (co.leaf_coeffs()[0] != 0)
    hl = torch.as_tensor(np.ldexp(1.0, -lev.astype(np.int64)), device="cuda")
    V = hl ** 3
    y = torch.as_tensor((ijk[:, 1] + 0.5), dtype=torch.float64, device="cuda") * hl
    setup = time.perf_counter() - t0

    def rms_flux(div):
        return float(torch.sqrt((V * div * div)[act].sum() / V[act].sum()))

    div0 = mfmg.divergence(h, beta_d, u0_d)
    rms0 = mfmg.divergence_rms(h, div0)
    rms0_flux = rms_flux(div0)
    mfmg.pcg_solve(h, div0, rtol=rtol)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p, st, hist = mfmg.pcg_solve(h, div0, rtol=rtol, history=True)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    u = u0_d.clone()
    mfmg.project_velocity(h, beta_d, p, u)
    div1 = mfmg.divergence(h, beta_d, u)
    fluid = beta_d > 0

    def perr_rms(x):
        e = (x - (y - 1.0))[act]
        return float(torch.sqrt((V[act] * e * e).sum() / V[act].sum()))

    perr = float(torch.abs(p - (y - 1.0))[act].max())
    out = {"obstacle": obstacle, "root_level": root_level, "levels": [root_level, root_level + 2],
           "leaves": tree.n_leaves, "active": int(act.sum()), "setup_s": setup,
           "iters": st["iters"], "status": st["status"], "solve_ms": t_solve * 1e3,
           "residual_history": [float(v) for v in hist],
           "reduction_factor": 2.0 ** -fit_slope(range(1, len(hist)), hist[1:]),
           "rms_div_before": rms0, "rms_div_after": mfmg.divergence_rms(h, div1),
           "rms_flux_before": rms0_flux, "rms_flux_after": rms_flux(div1),
           "p_max_err_vs_exact": perr, "p_rms_err_vs_exact": perr_rms(p),
           "u_max_after": float(torch.abs(u[fluid]).max())}
    if sweep_iters:
        # RMS of the divergence left after a projection with k iterations
        per = []
        for k in range(1, sweep_iters + 1):
            pk, _ = mfmg.pcg_solve(h, div0, rtol=0.0, max_iter=k)
            uk = u0_d.clone()
            mfmg.project_velocity(h, beta_d, pk, uk)
            dk = mfmg.divergence(h, beta_d, uk)
            per.append({"iters": k, "rms_div": mfmg.divergence_rms(h, dk),
                        "rms_flux": rms_flux(dk),
                        "p_max_err_vs_exact": float(torch.abs(pk - (y - 1.0))[act].max()),
                        "p_rms_err_vs_exact": perr_rms(pk)})
        out["per_iteration"] = per
    del h, co, tree
    return out


def projection_study(mfmg, torch, roots=None):
    """The static projection test over root cell sizes 1/16 .. 1/256 (sphere)
    and 1/16 .. 1/128 (star, whose refined shell is larger), with fitted
    orders of the RMS divergence left at rtol 1e-6 and the residual
    reduction factors, next to the paper's figures (context)."""
    import warnings
    roots = roots or {"sphere": [4, 5, 6, 7, 8], "star": [4, 5, 6, 7]}
    res = {"paper": {"rms_div_order": {"sphere": 2.54, "star": 2.27},
                     "reduction_factor": {"sphere 256~1024": 7.16, "star 64~256": 5.17,
                                          "star 256~1024": 5.88},
                     "precision": "FP32 with FP64 dot products, rtol 1e-6, mu = 2"},
           "runs": []}
    for obstacle, levels in roots.items():
        for l0 in levels:
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                r = static_projection(mfmg, torch, obstacle, l0)
            log(f"[bench] static projection {obstacle} root 1/{2 ** l0} (levels {l0}..{l0 + 2}, "
                f"{r['leaves']} leaves): {r['iters']} iterations, reduction factor "
                f"{r['reduction_factor']:.2f}, RMS_V div {r['rms_div_before']:.3e} -> "
                f"{r['rms_div_after']:.3e} (flux {r['rms_flux_before']:.3e} -> "
                f"{r['rms_flux_after']:.3e}), |p - (y - 1)| max {r['p_max_err_vs_exact']:.2e} "
                f"RMS_V {r['p_rms_err_vs_exact']:.2e}, "
                f"max |u| {r['u_max_after']:.2e}, solve {r['solve_ms']:.1f} ms")
            res["runs"].append(r)
        runs = [r for r in res["runs"] if r["obstacle"] == obstacle]
        x = [-r["root_level"] for r in runs]  # log2 of the root cell size
        res.setdefault("rms_div_order", {})[obstacle] = fit_slope(
            x, [r["rms_div_after"] for r in runs])
        res.setdefault("rms_flux_order", {})[obstacle] = fit_slope(
            x, [r["rms_flux_after"] for r in runs])
    return res


def rebuild_timing(mfmg, torch, spec, beta_d, bc, theta, reps=3):
    """Wall time of the steps that rebuild the solver for a changed octree
    on the device (octree, canonical face list, assembly, Algorithm 3
    coarsening of the mixed hierarchy), best of reps, against the host
    octree build."""
    t0 = time.perf_counter()
    mfmg.build_octree(spec)
    host = time.perf_counter() - t0
    best = None
    for _ in range(reps + 1):  # the first pass warms the allocator
        torch.cuda.synchronize()
        t = [time.perf_counter()]
        td = mfmg.build_octree(spec, device=True)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        faces = td.faces_device()
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        co = mfmg.assemble_coeffs(td, beta_d, bc, theta)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        h = mfmg.build_hierarchy(co, precision=mfmg.MIXED)
        torch.cuda.synchronize()
        t.append(time.perf_counter())
        steps = [1e3 * (b - a) for a, b in zip(t[:-1], t[1:])]
        if best is None or sum(steps) < sum(best):
            best = steps
        del h, co, faces, td
    return {"host_octree_ms": host * 1e3, "octree_ms": best[0], "faces_ms": best[1],
            "assemble_ms": best[2], "hierarchy_ms": best[3], "total_ms": sum(best),
            "best_of": reps + 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", type=int, default=4, choices=[1, 2, 3, 4])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-pass", action="store_true",
                    help="only the finest mixed half-sweep and a plain copy (counter runs)")
    ap.add_argument("--traffic-fp64", action="store_true",
                    help="with --traffic-pass: the FP64 hierarchy's half-sweep instead")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--projection-study", action="store_true",
                    help="only the static projection test over root cell sizes (one JSON line)")
    ap.add_argument("--summarize-trace", metavar="KERNEL_STATS_CSV",
                    help="store per-kernel averages of a rocprofv3 --stats run of bench.py")
    args = ap.parse_args()
    if args.summarize_trace:
        rec = summarize_trace(args.summarize_trace)
        print(json.dumps({"kernels": len(rec["kernels"]), "source_hash": rec["source_hash"]}))
        return
    if args.summarize_pmc:
        spec = __import__("problems").config_spec(args.workload)
        prec, rec = summarize_pmc(*args.summarize_pmc, spec["max_level"])
        if args.workload == 4:  # the benchmark's workload: the record bench.py reads
            path = os.path.join(ROOT, "profiles", "traffic_smooth_large_workload.json")
            store = {}
            if os.path.exists(path):
                with open(path) as fh:
                    store = json.load(fh)
            store[prec] = rec
            with open(path, "w") as fh:
                json.dump(store, fh, indent=1)
        print(json.dumps({prec: rec}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the solver is "
              "single-GPU; how it would shard is described with the design", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import problems
    from paper_2604_18886_amd import mfmg

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.projection_study:
        print(json.dumps({"static_projection": projection_study(mfmg, torch)}), flush=True)
        return
    cfg = args.workload
    spec = problems.config_spec(cfg)
    bc, theta = problems.config_bc(cfg)
    t0 = time.perf_counter()
    tree = mfmg.build_octree(spec)
    lev, ijk = tree.leaves()
    owner, fdir, other, kind = tree.faces()
    beta = problems.face_beta(cfg, lev[owner], ijk[owner], fdir)
    if cfg in (1, 2):
        rhs = problems.rhs_manufactured(cfg, lev, ijk, owner, lev[owner], ijk[owner], fdir,
                                        other, beta, bc, theta)
    else:
        rhs = problems.rhs_random(cfg, lev, ijk)
    log(f"[bench] workload {cfg}: {tree.n_leaves} leaves, {tree.n_faces} faces, "
        f"inputs in {time.perf_counter() - t0:.1f} s")
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                                    device="cuda")
    beta_d = dev(beta)
    rhs_d = dev(rhs)
    del beta
    t0 = time.perf_counter()
    co = mfmg.assemble_coeffs(tree, beta_d, bc, theta)
    act_d = co.leaf_coeffs()[0] != 0
    nact = int(act_d.sum().item())
    act = act_d.cpu().numpy()
    L = spec["max_level"]
    if args.traffic_pass:
        h = mfmg.build_hierarchy(co, precision=mfmg.FP64 if args.traffic_fp64 else mfmg.MIXED)
        ms, by = mfmg.profile(h, mfmg.PROFILE_SMOOTH, L, reps=TRAFFIC_REPS)
        mfmg.profile(h, mfmg.PROFILE_CYCLE, 0, reps=TRAFFIC_REPS)
        src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(TRAFFIC_REPS):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] traffic pass: {TRAFFIC_REPS + 1} half-sweeps at level {L} "
            f"({by:.3e} algorithmic bytes each), {TRAFFIC_REPS + 1} cycles, "
            f"{TRAFFIC_REPS} copies of {COPY_BYTES} bytes")
        return
    hiers = {"mixed": mfmg.build_hierarchy(co, precision=mfmg.MIXED),
             "fp64": mfmg.build_hierarchy(co, precision=mfmg.FP64)}
    torch.cuda.synchronize()
    log(f"[bench] {nact} active leaves; coefficients + hierarchies in "
        f"{time.perf_counter() - t0:.1f} s")
    out = {}
    sols = {}
    errs = {}
    sample = oracle_sample(cfg)
    p = torch.empty_like(rhs_d)
    for name, h in hiers.items():
        for _ in range(args.warmup):
            mfmg.pcg_solve(h, rhs_d, p, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for _ in range(args.steps):
            _, st = mfmg.pcg_solve(h, rhs_d, p, rtol=1e-10)
            stats.append(st)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = stats[-1]
        ms_s, by_s = mfmg.profile(h, mfmg.PROFILE_SMOOTH, L, reps=50)
        ms_c, by_c = mfmg.profile(h, mfmg.PROFILE_CYCLE, 0, reps=10)
        ms_cp, by_cp = mfmg.profile(h, mfmg.PROFILE_COPY, 0, reps=20)
        sols[name] = p.clone()
        if sample is not None:
            errs[name] = error_vs_oracle(p, sample)
            log(f"[bench] {name}: relative L2 error against the oracle's p* (1e-13) over "
                f"{errs[name]['samples']} sampled leaves {errs[name]['rel_l2_sampled']:.2e}")
        # adjoint of L = ||p - p_t||^2 at this solution (outside the timed region)
        pn = p.cpu().numpy()
        pt = problems.adjoint_target(lev, ijk, np.abs(pn).max())
        g_d = dev(np.where(act, 2.0 * (pn - pt), 0.0))
        mfmg.pcg_solve_adjoint(h, p, g_d, rtol=1e-10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, ast = mfmg.pcg_solve_adjoint(h, p, g_d, rtol=1e-10)
        torch.cuda.synchronize()
        dt_adj = time.perf_counter() - t0
        out[name] = {"ms_per_solve": dt * 1e3, "mcells_per_s": nact / dt / 1e6,
                     "iters": st["iters"], "rel_resid_true": st["rel_resid_true"],
                     "device_ms_per_solve": st["seconds"] * 1e3,
                     "smooth_ms": ms_s, "smooth_bytes": by_s,
                     "smooth_gbs": by_s / ms_s / 1e6,
                     "cycle_ms": ms_c, "cycle_bytes": by_c, "cycle_gbs": by_c / ms_c / 1e6,
                     "copy_gbs": by_cp / ms_cp / 1e6,
                     "adjoint_ms": dt_adj * 1e3, "adjoint_iters": ast["iters"],
                     "adjoint_rel_resid_true": ast["rel_resid_true"]}
        log(f"[bench] {name}: {dt * 1e3:.2f} ms/solve, {st['iters']} iterations, "
            f"true residual {st['rel_resid_true']:.2e}, {nact / dt / 1e6:.1f} Mcells/s; "
            f"finest half-sweep {ms_s * 1e3:.1f} us = {by_s / ms_s / 1e6:.0f} GB/s; "
            f"cycle {ms_c:.3f} ms = {by_c / ms_c / 1e6:.0f} GB/s; "
            f"streaming copy {by_cp / ms_cp / 1e6:.0f} GB/s; adjoint solve + gradient "
            f"{dt_adj * 1e3:.1f} ms ({ast['iters']} iterations)")
    # the mu = 2 cycle (W-cycle) with the mixed hierarchy, outside the timed region
    hw = mfmg.build_hierarchy(co, precision=mfmg.MIXED, mu=2)
    mfmg.pcg_solve(hw, rhs_d, p, rtol=1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, stw = mfmg.pcg_solve(hw, rhs_d, p, rtol=1e-10)
    torch.cuda.synchronize()
    dt_w = time.perf_counter() - t0
    del hw
    log(f"[bench] mixed W-cycle (mu=2): {dt_w * 1e3:.2f} ms/solve, {stw['iters']} iterations, "
        f"true residual {stw['rel_resid_true']:.2e}")
    proj = projection_timing(mfmg, torch, hiers["mixed"], beta_d, fdir, kind, bc)
    log(f"[bench] projection (mixed): divergence {proj['divergence_ms']:.2f} ms, velocity "
        f"update {proj['update_ms']:.2f} ms, whole projection {proj['projection_ms']:.1f} ms "
        f"({proj['iters']} iterations); RMS_V of the divergence {proj['rms_div_before']:.3e} -> "
        f"{proj['rms_div_after']:.3e}")
    rebuild = rebuild_timing(mfmg, torch, spec, beta_d, bc, theta)
    log(f"[bench] rebuild on the device: octree {rebuild['octree_ms']:.1f} ms (host build "
        f"{rebuild['host_octree_ms']:.0f} ms), face list {rebuild['faces_ms']:.1f} ms, "
        f"assembly {rebuild['assemble_ms']:.1f} ms, mixed hierarchy "
        f"{rebuild['hierarchy_ms']:.1f} ms; total {rebuild['total_ms']:.1f} ms")
    head = out["mixed"]
    mixed_vs_fp64 = float(torch.linalg.norm(sols["mixed"] - sols["fp64"]) /
                          torch.linalg.norm(sols["fp64"]))
    log(f"[bench] mixed vs FP64 solution: relative L2 difference {mixed_vs_fp64:.2e}")
    del sols
    traffic = measured_traffic("mixed", L)
    roof = {"bound": "hbm", "achieved": head["smooth_gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": head["smooth_gbs"] / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"k_smooth<float,float,__half> colour half-sweep, level {L}",
            "algorithmic_bytes_per_launch": head["smooth_bytes"],
            "avg_launch_us": head["smooth_ms"] * 1e3,
            "rocprof_avg_launch_us": traced_launch_us("mfmg::k_smooth<float, float, __half, 256, 0>"),
            "stream_copy_gbs": head["copy_gbs"],
            "frac_of_stream_copy": head["smooth_gbs"] / head["copy_gbs"]}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(cfg, out["fp64"]["iters"])
        log(f"[bench] cpu baseline {cpu['value']:.3f} Mcells/s")
    res = {
        "metric": METRIC,
        "value": head["mcells_per_s"],
        "unit": "Mcells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": ("large adaptive cut-cell octree, leaf levels "
                         f"{spec['min_level']}..{spec['max_level']}, 8 seeded refinement "
                         "spheres + solid box, Dirichlet top wall" if cfg == 4 else
                         f"workload {cfg}"),
            "leaves": tree.n_leaves, "active_leaves": nact, "faces": tree.n_faces,
            "rtol": 1e-10, "cycle": "FAS-style V-cycle, RBGS 2+2, coarsest 10 at level 3",
            "precision": "FP64 PCG; cycle FP32 with FP32 leaf / FP16 inner coefficients",
        },
        "T_iter": head["mcells_per_s"] * head["iters"],
        "rel_l2_vs_oracle": errs.get("mixed"),
        "fp64": {"value": out["fp64"]["mcells_per_s"], "ms_per_step": out["fp64"]["ms_per_solve"],
                 "T_iter": out["fp64"]["mcells_per_s"] * out["fp64"]["iters"],
                 "rel_l2_vs_oracle": errs.get("fp64"),
                 "iters": out["fp64"]["iters"], "rel_resid_true": out["fp64"]["rel_resid_true"],
                 "vcycle_gbs": out["fp64"]["cycle_gbs"], "vcycle_ms": out["fp64"]["cycle_ms"],
                 "vcycle_frac_of_peak": out["fp64"]["cycle_gbs"] / HBM_PEAK_GBS,
                 "vcycle_algorithmic_bytes": out["fp64"]["cycle_bytes"],
                 "vcycle_traffic": measured_traffic("fp64", L, "cycle_hbm_bytes"),
                 "smooth_us": out["fp64"]["smooth_ms"] * 1e3,
                 "smooth_algorithmic_bytes": out["fp64"]["smooth_bytes"],
                 "smooth_frac_of_peak": out["fp64"]["smooth_gbs"] / HBM_PEAK_GBS,
                 "smooth_traffic": measured_traffic("fp64", L),
                 "adjoint_ms": out["fp64"]["adjoint_ms"],
                 "adjoint_iters": out["fp64"]["adjoint_iters"]},
        "mixed": {"iters": head["iters"], "rel_resid_true": head["rel_resid_true"],
                  "rel_l2_diff_vs_fp64": mixed_vs_fp64,
                  "vcycle_gbs": head["cycle_gbs"], "vcycle_ms": head["cycle_ms"],
                  "vcycle_frac_of_peak": head["cycle_gbs"] / HBM_PEAK_GBS,
                  "vcycle_algorithmic_bytes": head["cycle_bytes"],
                  "vcycle_traffic": measured_traffic("mixed", L, "cycle_hbm_bytes"),
                  "adjoint_ms": head["adjoint_ms"], "adjoint_iters": head["adjoint_iters"],
                  "wcycle_ms_per_solve": dt_w * 1e3, "wcycle_iters": stw["iters"]},
        "rebuild": rebuild,
        "projection": proj,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
