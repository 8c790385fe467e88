"""Benchmark: constraints solved per second at <= 1e-12 relative violation.

Workload (default): 4,096 random-tree molecules with log-uniform atom counts
8..2,048, 5% ring closures, all bonds constrained, sigma = 0.002 nm.  Inputs
(r, masses and a pool of perturbed r_u sets) are resident in HBM before the
timed region.  One step = one full constraint solve of the whole system.

Prints one JSON line.  Run `python bench.py` (defaults: 1 GPU, 20 timed
steps after 3 warm-up steps).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
AT_DEFAULT_STORE = os.path.join(os.path.expanduser("~"), ".cache", "ilves_tuning_new.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name, seed):
    from paper_2503_13075_amd import synth as S
    if name == "batch4096":
        sm = S.random_tree_batch(4096, seed=seed)
        return sm, 0.002, {"workload": "4096 random-tree molecules, 8-2048 atoms log-uniform, 5% rings, all bonds",
                           "molecules": 4096}
    if name == "protein300":
        sm = S.protein_system(seed=seed, n_res=300)
        return sm, 0.002, {"workload": "one protein-like molecule, 300 residues, all bonds", "molecules": 1}
    if name == "giant":
        sm = S.protein_system(seed=seed, n_res=1650)
        return sm, 0.002, {"workload": "one protein-like molecule of 1650 residues (~26,600 bond constraints, "
                                       "the size of the paper's largest single molecule), all bonds", "molecules": 1}
    if name == "angles":
        sm = S.angles_system(seed=seed)
        return sm, 0.006, {"workload": "20 proteins + 1000 lipid chains, bonds + H-X-H/H-X-Y angles",
                           "molecules": 1020}
    if name == "water":
        sm = S.water_box(500_000, seed=seed)
        return sm, 0.002, {"workload": "500,000 rigid waters (O-H, O-H, H-H), small-molecule path",
                           "molecules": 500_000}
    if name == "chain64":
        sm = S.chain64(seed)
        return sm, 0.002, {"workload": "64-atom chain, bonds + 1-3 angles", "molecules": 1}
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(sm, plan_stats):
    """Minimal HBM traffic of one solve: per constrained atom r, r_u, mass
    read and r' written (80 B); per constraint its pair and d^2 read and
    lambda written (24 B); the factor pattern read once (4 B per stored
    off-diagonal entry of L plus 8 B per row)."""
    s = plan_stats["atoms"]
    n = plan_stats["constraints"]
    nnz_l = (plan_stats["factor_entries"] - n) // 2
    return 80 * s + 24 * n + 4 * nnz_l + 8 * n


def copy_bandwidth_gbs(dev, mib=1024, reps=10):
    """Bandwidth of a plain device-to-device copy (bytes read + written per
    second), the practical HBM ceiling to set beside the published peak."""
    import torch
    src = torch.empty(mib * (1 << 20) // 8, dtype=torch.float64, device=dev).uniform_()
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * 8 * reps / (ev0.elapsed_time(ev1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def measured_traffic(workload, variant, tuning):
    """HBM bytes per solve from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs, if they were taken from the current kernel sources with
    the same launch tuning (otherwise None)."""
    path = os.path.join(ROOT, "profiles", f"solve_kernel_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    from paper_2503_13075_amd.build import kernel_source_hash
    with open(path) as f:
        rec = json.load(f)
    if rec.get("variant", "mixed") != variant or rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    t = rec.get("tuning")
    if t is None or tuning is None or t["band_block"] != list(tuning["band_block"]) or \
            t["lds_limit"] != tuning["lds_limit"]:
        return None
    return rec["traffic_bytes_per_solve"]


def _oracle_molecule(task):
    """One molecule through the CPU oracle (a worker of cpu_baseline's pool)."""
    from oracle import newton_dense as O
    r, ru, lp, d, inv_m = task
    _, _, it, st, _ = O.solve_molecule(r, ru, lp, d, inv_m, 1e-12, 20)
    return len(d) if st == O.OK else 0, it


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sm, ru, budget_s=20.0, max_workers=16):
    """The CPU oracle on a bounded sample of the same workload's molecules:
    molecules in a seeded random order are spread over a pool of worker
    processes, one per available core (at most max_workers), each with its
    BLAS held to one thread; the pool stops taking molecules once budget_s
    has passed.  The rate is the constraints of the molecules it solved to
    1e-12 divided by the wall time of the sample (start of the first
    molecule to the end of the last)."""
    import multiprocessing as mp
    from oracle import newton_dense as O
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(max_workers, avail))
    mols = O.molecules(sm.n_atoms, sm.pairs)
    rng = np.random.default_rng(0)
    order = rng.permutation(len(mols))

    def tasks():
        for i in order:
            atoms, cons = mols[i]
            local = np.full(sm.n_atoms, -1, np.int64)
            local[atoms] = np.arange(atoms.size)
            yield sm.r[atoms], ru[atoms], local[sm.pairs[cons]], sm.d[cons], 1.0 / sm.mass[atoms]

    # spawned workers import numpy afresh and inherit these limits (one BLAS thread each)
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    solved = done = 0
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(workers) as pool:
            pool.map(abs, range(workers))  # workers up before the clock starts
            t0 = time.perf_counter()
            for n_ok, _ in pool.imap_unordered(_oracle_molecule, tasks(), chunksize=1):
                solved += n_ok
                done += 1
                if time.perf_counter() - t0 > budget_s:
                    break
            dt = time.perf_counter() - t0
            pool.terminate()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {"value": solved / dt, "unit": "constraints/s", "cores": workers, "kind": "oracle",
            "workers": workers, "os_cpu_count": os.cpu_count(), "cpu_model": _cpu_model(),
            "sample": f"{done} of {len(mols)} molecules (seeded random order) on {workers} worker processes "
                      f"(one BLAS thread each), {solved} constraints solved in {dt:.1f} s of wall time; the rate "
                      f"is that sample's constraints / wall time, taken as the rate of the whole workload; "
                      f"dense FP64 Newton per molecule, tol 1e-12"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch4096")
    ap.add_argument("--split-rows", type=int, default=0,
                    help="split molecules above this many constraints across workgroups (0 automatic, <0 never)")
    ap.add_argument("--split-part-rows", type=int, default=0, help="constraints per part of a split molecule")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--pool", type=int, default=8, help="distinct r_u sets resident in HBM")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--variants", default="fp64,mixed,decoupled,learned",
                    help="comma list of fp64, mixed, decoupled (mixed, each constraint's decoupled solution as "
                         "lambda_0), learned (mixed, network lambda_0), and the chord method (A(r, r) factored "
                         "once per solve): chord64, chord_mixed, chord_decoupled")
    ap.add_argument("--ordering", type=int, default=0,
                    help="fill-reducing ordering: 0 automatic, 1 minimum deficiency, 2 nested dissection")
    ap.add_argument("--eager", action="store_true", help="launch every step instead of replaying HIP graphs")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch tuning")
    ap.add_argument("--tuning", default=None,
                    help='apply this launch tuning instead of autotuning, JSON: {"band_block": [5 ints], "lds_limit": n}')
    ap.add_argument("--tuning-file", default=os.path.join(ROOT, "paper_2503_13075_amd", "tuning.json"),
                    help="launch tunings recorded per device and workload; a miss autotunes and records the result "
                         "in --tuning-store")
    ap.add_argument("--tuning-store", default=AT_DEFAULT_STORE,
                    help="file that receives tunings found by autotuning (the recorded file is left unchanged)")
    ap.add_argument("--retune", action="store_true",
                    help="autotune even when the tuning file has an entry (the entry seeds the search); the result "
                         "goes to --tuning-store")
    ap.add_argument("--rng-steps", type=int, default=1000,
                    help="also replay a graph of [device Philox inputs, solve, step += 1] this many times (0: skip)")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="MiB of a plain device copy run once before timing (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the solve works on one GPU's share of molecules and "
              "this library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    t0 = time.perf_counter()
    sm, sigma, cfg = make_workload(args.workload, args.seed)
    from paper_2503_13075_amd import synth as S
    pool_np = [S.perturb(sm.r, sigma, 10_000 + i) for i in range(args.pool)]
    log(f"workload {args.workload}: {sm.n_atoms} atoms, {sm.n_constraints} constraints, "
        f"generated in {time.perf_counter() - t0:.1f} s")

    import torch
    from paper_2503_13075_amd import _lib as L
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t1 = time.perf_counter()
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d, split_rows=args.split_rows, split_part_rows=args.split_part_rows,
                  ordering=args.ordering)
    st = plan.stats()
    log(f"plan: {time.perf_counter() - t1:.1f} s, {st}")
    r = torch.from_numpy(S.soa(sm.r)).to(dev)
    mass = torch.from_numpy(sm.mass.copy()).to(dev)
    pool = [torch.from_numpy(S.soa(x)).to(dev) for x in pool_np]
    r_out = torch.empty_like(r)
    lam = torch.zeros(sm.n_constraints, dtype=torch.float64, device=dev)
    nm = plan.n_molecules
    mol = plan.molecules()
    ncon_mol = torch.from_numpy(mol["n_con"].astype(np.int64)).to(dev)
    stream = torch.cuda.current_stream()

    def run(precision, steps, warmup, learned=False, warm=L.WARM_ZERO, variant=L.VARIANT_NEWTON):
        iters = torch.zeros((steps, nm), dtype=torch.int32, device=dev)
        status = torch.full((steps, nm), -1, dtype=torch.int32, device=dev)
        fallback = torch.zeros((steps, nm), dtype=torch.int32, device=dev)
        wi = torch.zeros(nm, dtype=torch.int32, device=dev)
        ws = torch.zeros(nm, dtype=torch.int32, device=dev)

        def one(k, it, stt, fb):
            if learned:
                plan.solve_learned(r, pool[k % len(pool)], mass, 1e-12, r_out, lam, it, stt, fb, precision=precision,
                                   variant=variant)
            else:
                plan.solve(r, pool[k % len(pool)], mass, 1e-12, r_out, lam, it, stt, precision=precision,
                           warm_start=warm, variant=variant)

        for w in range(warmup):
            one(w, wi, ws, None)
        torch.cuda.synchronize()
        graphs = []
        if not args.eager:
            # one graph per resident r_u set; each writes its own status row
            n_g = min(len(pool), steps)
            for p in range(n_g):
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    one(p, iters[p], status[p], fallback[p])
                graphs.append(g)
            torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t_start = time.perf_counter()
        ev0.record(stream)
        for k in range(steps):
            if graphs:
                graphs[k % len(graphs)].replay()
            else:
                one(k, iters[k], status[k], fallback[k])
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        gpu_ms = ev0.elapsed_time(ev1)
        if graphs:
            # replays of one graph repeat the same deterministic solve: step k
            # has the status row of graph k % len(graphs)
            rows = torch.tensor([k % len(graphs) for k in range(steps)], device=dev)
            status = status.index_select(0, rows)
            iters = iters.index_select(0, rows)
            fallback = fallback.index_select(0, rows)
        ok = (status == 0)
        solved = int((ok.to(torch.int64) * ncon_mol[None, :]).sum().item())
        it = iters.to(torch.float64)
        q = np.percentile(iters.cpu().numpy().ravel(), [50, 99]).tolist()
        return {"gpu_ms": gpu_ms, "wall_s": wall, "solved": solved, "all_ok": bool(ok.all().item()),
                "iters_mean": float(it.mean().item()), "iters_max": int(iters.max().item()),
                "iters_p50": q[0], "iters_p99": q[1],
                "fallback_rate": float(fallback.to(torch.float64).mean().item()),
                "last_index": (steps - 1) % len(pool)}

    def check_last(res):
        from oracle import newton_dense as O  # violation check of the final result only
        rp = r_out.cpu().numpy().T
        viol = float(np.max(O.relative_violation(rp, sm.pairs, sm.d)))
        return viol

    def rng_graph(steps, precision, learned, warm=L.WARM_ZERO, variant=L.VARIANT_NEWTON):
        """Many solves without the host: one captured graph draws the step's
        r_u on the device (Philox4x32-10 + Box-Muller, step index in device
        memory), solves, folds status and iterations into device
        accumulators and advances the step; it is replayed `steps` times.
        A graph of the generator alone gives its share of the step time."""
        step = torch.tensor([0], dtype=torch.int64, device=dev)
        ru = torch.empty_like(r)
        it = torch.zeros(nm, dtype=torch.int32, device=dev)
        stt = torch.zeros(nm, dtype=torch.int32, device=dev)
        worst = torch.zeros(nm, dtype=torch.int32, device=dev)
        it_sum = torch.zeros(nm, dtype=torch.int64, device=dev)

        def gen():
            L.perturb_normal(r, sigma, 1, step, ru)

        def one():
            gen()
            if learned:
                plan.solve_learned(r, ru, mass, 1e-12, r_out, lam, it, stt, precision=precision, variant=variant)
            else:
                plan.solve(r, ru, mass, 1e-12, r_out, lam, it, stt, precision=precision, warm_start=warm,
                           variant=variant)
            torch.maximum(worst, stt, out=worst)
            it_sum.add_(it)
            L.counter_add(step, 1)

        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            one()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g_all, g_gen = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(g_all):
            one()
        with torch.cuda.graph(g_gen):
            gen()
        worst.zero_()
        it_sum.zero_()
        step.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g_all.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ok = bool((worst == 0).all().item())
        iters = float(it_sum.sum().item()) / (steps * nm)
        viol = check_last(None)
        e0.record()
        for _ in range(steps):
            g_gen.replay()
        e1.record()
        torch.cuda.synchronize()
        gen_ms = e0.elapsed_time(e1) / steps
        solve_ms = ms - gen_ms
        return {"steps": steps, "ms_per_step_with_inputs": ms, "input_generation_ms": gen_ms,
                "ms_per_step_solve": solve_ms,
                "constraints_per_s_solve": (sm.n_constraints / (solve_ms / 1e3)) if ok else 0.0,
                "all_ok": ok, "newton_iters_mean_per_molecule": iters, "max_rel_violation_last": viol,
                "variant": ("chord_" if variant == L.VARIANT_CHORD else "") +
                           ("learned" if learned else ("decoupled" if warm == L.WARM_DECOUPLED else "mixed")),
                "seed": 1, "sigma_nm": sigma}

    if args.calibrate_copy > 0:
        nb = args.calibrate_copy * (1 << 20)
        src = torch.empty(nb // 8, dtype=torch.float64, device=dev).uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb} bytes read, {nb} bytes written")
        del src, dst

    results = {}
    wanted = set(args.variants.split(","))
    from paper_2503_13075_amd import warmstart as WS
    weights = WS.WEIGHTS["angles" if args.workload == "angles" else "trees"]
    if "learned" in wanted:
        params, norm, meta = WS.load(weights)
        plan.load_mlp(params, norm)
    tunings = {}

    def tune(prec, warm=L.WARM_ZERO, variant=L.VARIANT_NEWTON):
        """Autotunes the launch of this precision and start once (untimed):
        the fastest launch depends on the iteration counts the start gives."""
        if args.tuning or args.no_autotune:
            t = json.loads(args.tuning) if args.tuning else {"band_block": [64, 128, 256, 512, 1024], "lds_limit": 0}
            plan.tune(band_block=t["band_block"], lds_limit=t["lds_limit"])
            return {"band_block": t["band_block"], "lds_limit": t["lds_limit"], "autotuned": False}
        if (prec, warm, variant) in tunings:
            t = tunings[(prec, warm, variant)]
            plan.tune(band_block=t["band_block"], lds_limit=t["lds_limit"])
            return t
        from paper_2503_13075_amd import autotune as AT
        it = torch.zeros(nm, dtype=torch.int32, device=dev)
        stt = torch.zeros(nm, dtype=torch.int32, device=dev)
        key = AT.plan_key(plan, prec, variant, "decoupled" if warm == L.WARM_DECOUPLED else "zero")
        run_one = lambda: plan.solve(r, pool[0], mass, 1e-12, r_out, lam, it, stt, precision=prec,  # noqa: E731
                                     warm_start=warm, variant=variant)
        if args.retune:
            hit = AT.load_cached(key, args.tuning_file)
            t = AT.autotune(plan, run_one, reps=10, seeds=[hit] if hit else [])
            AT.store(key, t, args.tuning_store)
            t = dict(t, cached=False)
        else:
            t = AT.tuned(plan, run_one, key, path=args.tuning_file, reps=10,
                         store_path=args.tuning_store)
        log(f"tuning precision {prec} start {warm} variant {variant} (key {key}): {t}")
        tunings[(prec, warm, variant)] = t
        return t

    VARIANTS = (("fp64", L.PREC_FP64, L.WARM_ZERO, L.VARIANT_NEWTON),
                ("mixed", L.PREC_MIXED, L.WARM_ZERO, L.VARIANT_NEWTON),
                ("decoupled", L.PREC_MIXED, L.WARM_DECOUPLED, L.VARIANT_NEWTON),
                ("learned", L.PREC_MIXED, L.WARM_ZERO, L.VARIANT_NEWTON),
                ("chord64", L.PREC_FP64, L.WARM_ZERO, L.VARIANT_CHORD),
                ("chord_mixed", L.PREC_MIXED, L.WARM_ZERO, L.VARIANT_CHORD),
                ("chord_decoupled", L.PREC_MIXED, L.WARM_DECOUPLED, L.VARIANT_CHORD))
    for name, prec, warm, variant in VARIANTS:
        if name not in wanted:
            continue
        tuning = tune(prec, warm, variant)
        res = run(prec, args.steps, args.warmup, learned=(name == "learned"), warm=warm, variant=variant)
        res["tuning"] = tuning
        res["max_rel_violation_last"] = check_last(res)
        ms = res["gpu_ms"] / args.steps
        res["ms_per_step"] = ms
        res["constraints_per_s"] = res["solved"] / (res["gpu_ms"] / 1e3)
        results[name] = res
        log(f"{name}: {ms:.3f} ms/step, {res['constraints_per_s']:.3e} constraints/s, all ok {res['all_ok']}, "
            f"iters mean {res['iters_mean']:.2f} max {res['iters_max']}, last violation {res['max_rel_violation_last']:.2e}")

    heads = [k for k in ("mixed", "decoupled", "learned", "chord_mixed", "chord_decoupled")
             if k in results and results[k]["all_ok"]]
    if "fp64" not in results or not heads:
        print(json.dumps(results), flush=True)
        return
    head_name = max(heads, key=lambda k: results[k]["constraints_per_s"])
    head = results[head_name]
    abytes = algorithmic_bytes(sm, st)
    achieved = abytes / (head["ms_per_step"] / 1e3) / 1e9
    traffic = measured_traffic(args.workload, head_name, head["tuning"])
    variants = {k: {"value": v["constraints_per_s"], "ms_per_step": v["ms_per_step"], "all_ok": v["all_ok"],
                    "newton_iters_mean": v["iters_mean"], "newton_iters_max": v["iters_max"],
                    "newton_iters_p50": v["iters_p50"], "newton_iters_p99": v["iters_p99"],
                    "fallback_rate": v["fallback_rate"] if k == "learned" else None,
                    "max_rel_violation_last": v["max_rel_violation_last"],
                    "tuning": v["tuning"]} for k, v in results.items()}
    out = {
        "metric": "constraints solved/s at <=1e-12 rel violation",
        "value": head["constraints_per_s"],
        "unit": "constraints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 residual/lambda/positions, f32 factor; bf16 network (learned start)",
        "data": "synthetic",
        "graph_replay": not args.eager,
        "config": dict(cfg, atoms=sm.n_atoms, constraints=sm.n_constraints,
                       variant={"learned": "mixed precision Newton, learned lambda_0",
                                "decoupled": "mixed precision Newton, lambda_0 = each constraint's decoupled solution",
                                "mixed": "mixed precision Newton, lambda_0 = 0",
                                "chord_mixed": "mixed precision chord (A(r, r) factored once), lambda_0 = 0",
                                "chord_decoupled": "mixed precision chord (A(r, r) factored once), lambda_0 = each "
                                                   "constraint's decoupled solution"}[head_name],
                       sigma_nm=sigma, tol=1e-12, split_molecules=st["split_molecules"],
                       split_parts=st["split_parts"]),
        "newton_iters": {k: v["iters_mean"] for k, v in results.items()},
        "variants": variants,
        "speedup_vs_fp64": head["constraints_per_s"] / results["fp64"]["constraints_per_s"],
        "all_ok": head["all_ok"],
        "max_rel_violation_last": head["max_rel_violation_last"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_step": abytes, "kernel": "solve_kernel (all launch groups of one solve)"},
    }
    copy_gbs = copy_bandwidth_gbs(dev)
    out["roofline"]["copy_gbs"] = copy_gbs                      # measured 1 GiB device copy
    out["roofline"]["frac_of_copy"] = achieved / copy_gbs
    if traffic is not None:
        out["roofline"]["traffic_gbs"] = traffic / (head["ms_per_step"] / 1e3) / 1e9
    log(f"roofline: {achieved:.0f} GB/s algorithmic, copy {copy_gbs:.0f} GB/s, peak {HBM_PEAK_GBS:.0f} GB/s")
    if args.rng_steps > 0:
        head_warm = L.WARM_DECOUPLED if head_name in ("decoupled", "chord_decoupled") else L.WARM_ZERO
        head_variant = L.VARIANT_CHORD if head_name.startswith("chord") else L.VARIANT_NEWTON
        tune(L.PREC_MIXED, head_warm, head_variant)  # the head variant's launch tuning
        out["rng_graph"] = rng_graph(args.rng_steps, L.PREC_MIXED, head_name == "learned", head_warm, head_variant)
        log(f"rng graph: {out['rng_graph']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(sm, pool_np[0], args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
