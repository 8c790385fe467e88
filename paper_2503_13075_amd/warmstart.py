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
    """Newton iterations with lambda_0 = 0 vs the learned start on the
    given seeds (per molecule), fallback rate and convergence."""
    import torch
    it0, it1, fb, ok0, ok1 = [], [], [], [], []
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
        plan.solve(r, rut, mass, tol, r_out, lam, iters, status, precision=precision)
        torch.cuda.synchronize()
        it0.append(iters.cpu().numpy().copy())
        ok0.append(status.cpu().numpy() == L.OK)
        plan.solve_learned(r, rut, mass, tol, r_out, lam, iters, status, fallback, precision=precision)
        torch.cuda.synchronize()
        it1.append(iters.cpu().numpy().copy())
        ok1.append(status.cpu().numpy() == L.OK)
        fb.append(fallback.cpu().numpy().copy())
        plan.close()
    it0, it1, fb = np.concatenate(it0), np.concatenate(it1), np.concatenate(fb)
    return {"molecules": int(it0.size), "iters_zero_mean": float(it0.mean()), "iters_learned_mean": float(it1.mean()),
            "iters_zero_max": int(it0.max()), "iters_learned_max": int(it1.max()),
            "fallback_rate": float(fb.mean()), "converged_zero": float(np.concatenate(ok0).mean()),
            "converged_learned": float(np.concatenate(ok1).mean())}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate"])
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
    else:
        params, norm, meta = load(out)
        res = evaluate(range(1000, 1000 + args.eval_seeds), params, norm, kind=args.kind)
        # ablation: the untrained network (zero output layer) returns the
        # decoupled solution t0 alone
        res0 = evaluate(range(1000, 1000 + args.eval_seeds), init_params(0), norm, kind=args.kind)
        res["iters_decoupled_start_mean"] = res0["iters_learned_mean"]
        res["fallback_rate_decoupled_start"] = res0["fallback_rate"]
        log(json.dumps(res))


if __name__ == "__main__":
    main()
