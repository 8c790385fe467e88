"""Learned warm start: harvest (features, lambda*) pairs from the solver,
train the network on the GPU with the library's own kernels, evaluate it.

    python -m paper_2503_13075_amd.warmstart train            # harvest + train + save
    python -m paper_2503_13075_amd.warmstart evaluate         # held-out seeds

Training systems are small versions of the angle-constrained workload
(one protein-like molecule with H-X-H / H-X-Y angles plus united-atom lipid
chains, sigma = 0.006 nm), seeds 0-999; evaluation uses seeds 1000-1099.
The labels lambda* come from the FP64 Newton solve of the GPU library.
All arithmetic of the network (forward, backward, Adam, inference) runs in
the library's HIP kernels; torch only holds device memory.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import _lib as L
from . import synth as S

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = {"angles": os.path.join(HERE, "weights", "warmstart_c3like.npz"),
           "trees": os.path.join(HERE, "weights", "warmstart_trees.npz")}
DEFAULT_WEIGHTS = WEIGHTS["angles"]
SIGMA = {"angles": 0.006, "trees": 0.002}
N_FEAT, N_HID = 16, 64


def c3like_system(seed: int, n_res: int = 40, n_lipid: int = 20) -> S.System:
    """One protein-like molecule with h-angles plus lipid chains."""
    mols = [S.add_h_angles(S.protein(n_res=n_res, seed=7919 * seed + 1))]
    mols += [S.lipid_chain(104729 * seed + j) for j in range(n_lipid)]
    return S.concat(mols, spacing=3.0, name=f"c3like{seed}")


def trees_system(seed: int, n_mol: int = 6) -> S.System:
    """A few random-tree molecules of log-uniform size (batch workload)."""
    sizes = S.batch_sizes(n_mol, 31337 + seed)
    return S.concat([S.random_tree(int(n), 9_000_000 + 97 * seed + i) for i, n in enumerate(sizes)], spacing=3.0,
                    name=f"trees{seed}")


def make_system(kind: str, seed: int) -> S.System:
    return c3like_system(seed) if kind == "angles" else trees_system(seed)


def perturbed(sm: S.System, seed: int, kind: str = "angles") -> np.ndarray:
    return S.perturb(sm.r, SIGMA[kind], 500_000 + seed)


def _device_inputs(sm, ru, dev):
    import torch
    r = torch.from_numpy(S.soa(sm.r)).to(dev)
    rut = torch.from_numpy(S.soa(ru)).to(dev)
    mass = torch.from_numpy(np.ascontiguousarray(sm.mass)).to(dev)
    return r, rut, mass


def harvest(seeds, dev="cuda", log=print, kind="angles"):
    """(features [N, 16] float32, t* = lambda* w [N] float64) over the seeds,
    from converged FP64 solves."""
    import torch
    feats, targets = [], []
    t0 = time.perf_counter()
    for i, seed in enumerate(seeds):
        sm = make_system(kind, seed)
        ru = perturbed(sm, seed, kind)
        plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
        r, rut, mass = _device_inputs(sm, ru, dev)
        n = sm.n_constraints
        nm = plan.n_molecules
        r_out = torch.empty_like(r)
        lam = torch.zeros(n, dtype=torch.float64, device=dev)
        iters = torch.zeros(nm, dtype=torch.int32, device=dev)
        status = torch.zeros(nm, dtype=torch.int32, device=dev)
        plan.solve(r, rut, mass, 1e-14, r_out, lam, iters, status, precision=L.PREC_FP64, max_iter=30)
        feat = torch.empty((n, N_FEAT), dtype=torch.float32, device=dev)
        w = torch.empty(n, dtype=torch.float32, device=dev)
        plan.features(r, rut, mass, feat, w)
        torch.cuda.synchronize()
        cid = plan.row_constraints()
        st = status.cpu().numpy()
        # rows of converged molecules only
        ok_rows = np.ones(n, bool)
        mol = plan.molecules()
        row = 0
        for m in range(nm):
            k = int(mol["n_con"][m])
            if st[m] != L.OK:
                ok_rows[row:row + k] = False
            row += k
        lam_rows = lam.cpu().numpy()[cid]
        w_rows = w.cpu().numpy().astype(np.float64)
        # w in float32 would bias the target: recompute in FP64 from masses
        w64 = (1.0 / sm.mass[sm.pairs[cid, 0]] + 1.0 / sm.mass[sm.pairs[cid, 1]])
        del w_rows
        feats.append(feat.cpu().numpy()[ok_rows])
        targets.append((lam_rows * w64)[ok_rows])
        plan.close()
        if (i + 1) % 100 == 0:
            log(f"harvest: {i + 1}/{len(seeds)} seeds, {sum(len(t) for t in targets)} pairs, "
                f"{time.perf_counter() - t0:.1f} s")
    return np.concatenate(feats), np.concatenate(targets)


def fit_normalisation(X, t):
    mean = X.mean(0).astype(np.float64)
    std = X.std(0).astype(np.float64)
    std = np.where(std > 1e-8, std, 1.0)
    y = t - X[:, 0].astype(np.float64)
    scale = float(max(np.std(y), 1e-12))
    return np.concatenate([mean, std, [scale]]).astype(np.float32)


def init_params(seed=0):
    """He initialisation; zero output layer (the untrained network returns
    the decoupled solution t0)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, math.sqrt(2.0 / N_FEAT), (N_FEAT, N_HID))
    W2 = rng.normal(0, math.sqrt(2.0 / N_HID), (N_HID, N_HID))
    p = np.concatenate([W1.ravel(), np.zeros(N_HID), W2.ravel(), np.zeros(N_HID), np.zeros(N_HID), np.zeros(1)])
    assert p.size == L.mlp_param_count()
    return p.astype(np.float32)


def train(X, t, epochs=30, batch=4096, lr=2e-3, seed=0, dev="cuda", log=print):
    """Adam on 1/(2n) sum (MLP(norm x) - (t - t0) / scale)^2 with the
    library's FP32 kernels.  Returns (params, norm, history)."""
    import torch
    norm = fit_normalisation(X, t)
    mean, std, scale = norm[:N_FEAT], norm[N_FEAT:2 * N_FEAT], float(norm[-1])
    Xn = ((X - mean) / std).astype(np.float32)
    y = ((t - X[:, 0]) / scale).astype(np.float32)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(y))
    n_val = max(1, len(y) // 20)
    val, tr = perm[:n_val], perm[n_val:]
    Xt = torch.from_numpy(Xn[tr]).to(dev)
    yt = torch.from_numpy(y[tr]).to(dev)
    Xv = torch.from_numpy(Xn[val]).to(dev)
    yv = torch.from_numpy(y[val]).to(dev)
    params = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    work = torch.zeros(L.mlp_grad_workspace(batch), dtype=torch.float32, device=dev)
    vout = torch.zeros(len(val), dtype=torch.float32, device=dev)
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    step = 0
    hist = []
    n_tr = len(tr)
    for ep in range(epochs):
        order = torch.randperm(n_tr, generator=g).to(dev)
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))   # cosine schedule
        tot = 0.0
        for b0 in range(0, n_tr - batch + 1, batch):
            idx = order[b0:b0 + batch]
            xb = Xt.index_select(0, idx).contiguous()
            yb = yt.index_select(0, idx).contiguous()
            L.mlp_grad_f32(params, xb, yb, grad, loss, work)
            step += 1
            L.mlp_adam(params, grad, m, v, lr_ep, step)
            tot += float(loss.item()) if b0 == 0 else 0.0
        L.mlp_forward_f32(params, Xv, vout)
        torch.cuda.synchronize()
        vm = float(((vout - yv) ** 2).mean().item())
        base = float((yv ** 2).mean().item())
        hist.append({"epoch": ep, "val_mse": vm, "val_mse_zero_net": base})
        log(f"epoch {ep}: val mse {vm:.4e} (network off: {base:.4e}), lr {lr_ep:.2e}")
    return params.cpu().numpy(), norm, hist


def save(path, params, norm, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), norm=norm.astype(np.float32),
             meta=np.array(json.dumps(meta)))


def load(path=DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), z["norm"].astype(np.float32), json.loads(str(z["meta"]))


def evaluate(seeds, params, norm, precision=L.PREC_MIXED, dev="cuda", tol=1e-12, kind="angles"):
    """Per molecule of the given seeds: Newton iterations from lambda_0 = 0,
    from the decoupled start (the untrained network's output) and from the
    network, the fallback rates, convergence, and the error of both starts
    against the converged multipliers lambda* (FP64 solve to 1e-14):
    |lambda_0 - lambda*| / |lambda*| over each molecule's constraints (RMS
    over molecules) and the maximum relative violation at lambda_0."""
    import torch
    it = {"zero": [], "decoupled": [], "learned": []}
    ok = {"zero": [], "decoupled": [], "learned": []}
    fb = {"decoupled": [], "learned": []}
    err = {"decoupled": [], "learned": []}
    v0 = {"zero": [], "decoupled": [], "learned": []}
    for seed in seeds:
        sm = make_system(kind, seed)
        ru = perturbed(sm, seed, kind)
        plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
        plan.load_mlp(params, norm)
        r, rut, mass = _device_inputs(sm, ru, dev)
        n, nm = sm.n_constraints, plan.n_molecules
        r_out = torch.empty_like(r)
        lam = torch.zeros(n, dtype=torch.float64, device=dev)
        iters = torch.zeros(nm, dtype=torch.int32, device=dev)
        status = torch.zeros(nm, dtype=torch.int32, device=dev)
        fallback = torch.zeros(nm, dtype=torch.int32, device=dev)
        hist = torch.zeros((nm, 2), dtype=torch.float64, device=dev)
        # converged multipliers
        plan.solve(r, rut, mass, 1e-14, r_out, lam, iters, status, precision=L.PREC_FP64, max_iter=30)
        torch.cuda.synchronize()
        lam_star = lam.cpu().numpy().copy()
        # the two starts themselves
        lam0 = torch.zeros_like(lam)
        plan.predict(r, rut, mass, lam0)
        torch.cuda.synchronize()
        starts = {"learned": lam0.cpu().numpy().copy()}
        feat = torch.empty((n, N_FEAT), dtype=torch.float32, device=dev)
        wf = torch.empty(n, dtype=torch.float32, device=dev)
        plan.features(r, rut, mass, feat, wf)
        torch.cuda.synchronize()
        cid = plan.row_constraints()
        w64 = 1.0 / sm.mass[sm.pairs[:, 0]] + 1.0 / sm.mass[sm.pairs[:, 1]]
        dec = np.zeros(n)
        dec[cid] = feat.cpu().numpy()[:, 0].astype(np.float64)
        starts["decoupled"] = dec / w64
        mol = plan.molecules()
        row = 0
        for m in range(nm):
            k = int(mol["n_con"][m])
            cons = cid[row:row + k]
            row += k
            den = np.linalg.norm(lam_star[cons])
            for name in ("decoupled", "learned"):
                err[name].append(np.linalg.norm(starts[name][cons] - lam_star[cons]) / max(den, 1e-300))
        # the solves from each start (with the per-molecule fallback rule)
        for name, warm in (("zero", L.WARM_ZERO), ("decoupled", L.WARM_DECOUPLED), ("learned", L.WARM_MLP)):
            fallback.zero_()
            if name == "learned":
                plan.solve_learned(r, rut, mass, tol, r_out, lam, iters, status, fallback, precision=precision)
                plan.solve(r, rut, mass, tol, r_out, lam, iters, status, precision=precision, warm_start=warm,
                           history=hist)
            else:
                plan.solve(r, rut, mass, tol, r_out, lam, iters, status, precision=precision, warm_start=warm,
                           history=hist)
            torch.cuda.synchronize()
            it[name].append(iters.cpu().numpy().copy())
            ok[name].append(status.cpu().numpy() == L.OK)
            v0[name].append(hist.cpu().numpy()[:, 0].copy())
            if name == "learned":
                fb[name].append(fallback.cpu().numpy().copy())
            elif name == "decoupled":
                # the decoupled start falls back where its violation is not below that at 0
                fb[name].append((v0[name][-1] >= v0["zero"][-1]).astype(np.int32))
        plan.close()
    cat = {k: np.concatenate(v) for k, v in it.items()}
    res = {"molecules": int(cat["zero"].size)}
    for k in ("zero", "decoupled", "learned"):
        res[f"iters_{k}_mean"] = float(cat[k].mean())
        res[f"iters_{k}_max"] = int(cat[k].max())
        res[f"converged_{k}"] = float(np.concatenate(ok[k]).mean())
        res[f"violation0_{k}_median"] = float(np.median(np.concatenate(v0[k])))
    for k in ("decoupled", "learned"):
        res[f"fallback_rate_{k}"] = float(np.concatenate(fb[k]).mean())
        e = np.asarray(err[k])
        res[f"start_error_{k}_rms"] = float(np.sqrt(np.mean(e * e)))
        res[f"start_error_{k}_median"] = float(np.median(e))
    res["fallback_rate"] = res["fallback_rate_learned"]
    return res


def heldout_benchmark(seeds, params, norm, kind="angles", steps=20, dev="cuda", log=print):
    """Constraints solved per second at 1e-12 on the held-out systems
    concatenated into one system (one solve of all of them), for lambda_0 =
    0, the decoupled start and the learned start, mixed precision, each
    step replayed from a captured HIP graph; iterations and fallback too."""
    import torch
    systems = [make_system(kind, s) for s in seeds]
    sm = S.concat(systems, spacing=3.0, name=f"heldout-{kind}")
    ru = np.concatenate([perturbed(x, s, kind) + (sm.r[o:o + x.n_atoms] - x.r)
                         for x, s, o in zip(systems, seeds, np.cumsum([0] + [x.n_atoms for x in systems[:-1]]))])
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    plan.load_mlp(params, norm)
    r, rut, mass = _device_inputs(sm, ru, dev)
    nm = plan.n_molecules
    ncon = torch.from_numpy(plan.molecules()["n_con"].astype(np.int64)).to(dev)
    out = {"systems": len(seeds), "constraints": int(sm.n_constraints), "molecules": int(nm)}
    for name in ("zero", "decoupled", "learned"):
        r_out = torch.empty_like(r)
        lam = torch.zeros(sm.n_constraints, dtype=torch.float64, device=dev)
        iters = torch.zeros(nm, dtype=torch.int32, device=dev)
        status = torch.zeros(nm, dtype=torch.int32, device=dev)
        fallback = torch.zeros(nm, dtype=torch.int32, device=dev)

        def one():
            if name == "learned":
                plan.solve_learned(r, rut, mass, 1e-12, r_out, lam, iters, status, fallback, precision=L.PREC_MIXED)
            else:
                plan.solve(r, rut, mass, 1e-12, r_out, lam, iters, status, precision=L.PREC_MIXED,
                           warm_start=L.WARM_DECOUPLED if name == "decoupled" else L.WARM_ZERO)
        for _ in range(3):
            one()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            one()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        okm = status == L.OK
        solved = int((okm.to(torch.int64) * ncon).sum().item())
        out[name] = {"ms_per_solve": ms, "constraints_per_s": solved / (ms / 1e3),
                     "all_ok": bool(okm.all().item()), "iters_mean": float(iters.double().mean().item()),
                     "iters_max": int(iters.max().item()),
                     "fallback_rate": float(fallback.double().mean().item()) if name == "learned" else None}
        log(f"held-out benchmark {name}: {out[name]}")
    plan.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate", "benchmark"])
    ap.add_argument("--kind", choices=["angles", "trees"], default="angles")
    ap.add_argument("--out", default=None)
    ap.add_argument("--seeds", type=int, default=1000)
    ap.add_argument("--pairs", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--eval-seeds", type=int, default=100)
    args = ap.parse_args(argv)

    def log(*a):
        print(*a, flush=True)

    out = args.out or WEIGHTS[args.kind]
    if args.cmd == "train":
        X, t = harvest(range(args.seeds), log=log, kind=args.kind)
        rng = np.random.default_rng(0)
        if len(t) > args.pairs:
            sel = rng.choice(len(t), args.pairs, replace=False)
            X, t = X[sel], t[sel]
        log(f"training on {len(t)} pairs")
        params, norm, hist = train(X, t, epochs=args.epochs, log=log)
        res = evaluate(range(1000, 1000 + args.eval_seeds), params, norm, kind=args.kind)
        log(f"held-out evaluation: {res}")
        meta = {"kind": args.kind, "pairs": int(len(t)), "train_seeds": [0, args.seeds - 1], "epochs": args.epochs,
                "history": hist[-3:], "heldout": res, "sigma_nm": SIGMA[args.kind]}
        save(out, params, norm, meta)
        log(f"saved {out}")
    elif args.cmd == "evaluate":
        params, norm, meta = load(out)
        res = evaluate(range(1000, 1000 + args.eval_seeds), params, norm, kind=args.kind)
        log(json.dumps(res))
    else:
        params, norm, meta = load(out)
        res = heldout_benchmark(list(range(1000, 1000 + args.eval_seeds)), params, norm, kind=args.kind, log=log)
        log(json.dumps(res))


if __name__ == "__main__":
    main()
