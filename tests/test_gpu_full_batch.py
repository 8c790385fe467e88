"""The headline configuration at full size: the 4,096-molecule tree batch
(1,599,718 constraints) that bench.py times, with bench's seed, its first
perturbed input and its recorded launch tuning for the mixed-precision
decoupled start, the mixed-precision learned start with the shipped tree
network, and FP64 from lambda_0 = 0.  Every constraint is checked
(violation <= 1e-12 after rounding to the returned positions; the correction
conserves momentum), and sampled molecules -- the smallest, the largest and
random ones -- are compared with the oracle one by one."""
import json
import os

import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import DeviceSystem, solve_once

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _recorded_tuning(key):
    with open(os.path.join(HERE, "..", "paper_2503_13075_amd", "tuning.json")) as f:
        return json.load(f).get(key)


def _solve_learned(sm, ru, plan, prec):
    import torch
    from paper_2503_13075_amd import warmstart as WS
    params, norm, _ = WS.load(WS.WEIGHTS["trees"])
    plan.load_mlp(params, norm)
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    rut = ds.upload_ru(ru)
    fb = torch.zeros(plan.n_molecules, dtype=torch.int32, device="cuda")
    plan.solve_learned(ds.r, rut, ds.mass, 1e-12, ds.r_out, ds.lam, ds.iters, ds.status, fb, precision=prec)
    torch.cuda.synchronize()
    return {"r_out": ds.r_out.cpu().numpy().T.copy(), "lam": ds.lam.cpu().numpy().copy(),
            "iters": ds.iters[:plan.n_molecules].cpu().numpy().copy(),
            "status": ds.status[:plan.n_molecules].cpu().numpy().copy(), "fallback": fb.cpu().numpy()}


@pytest.mark.parametrize("name,prec,warm", [("mixed decoupled", L.PREC_MIXED, L.WARM_DECOUPLED),
                                            ("mixed learned", L.PREC_MIXED, None),
                                            ("fp64 zero", L.PREC_FP64, L.WARM_ZERO)])
def test_batch4096_full_size(name, prec, warm):
    from paper_2503_13075_amd import autotune as AT
    print(f"== batch4096 full size, {name}", flush=True)
    sm = S.random_tree_batch(4096, seed=2)          # bench.py --seed default
    ru = S.perturb(sm.r, 0.002, 10_000)             # bench.py's first resident input
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    # the learned start runs with the lambda_0 = 0 launch tuning, as in bench.py
    key = AT.plan_key(plan, prec, L.VARIANT_NEWTON, "decoupled" if warm == L.WARM_DECOUPLED else "zero")
    t = _recorded_tuning(key)
    if t is not None:
        plan.tune(band_block=t["band_block"], lds_limit=t["lds_limit"])
    if warm is None:
        out = _solve_learned(sm, ru, plan, prec)
        print(f"   fallback rate {out['fallback'].mean():.3f}", flush=True)
    else:
        out = solve_once(sm, ru, 1e-12, prec, L.VARIANT_NEWTON, plan=plan, warm=warm)
    assert np.all(out["status"] == L.OK)
    viol = np.max(O.relative_violation(out["r_out"], sm.pairs, sm.d))
    corr = sm.mass[:, None] * (out["r_out"] - ru)
    dp = np.abs(corr.sum(0)).max() / np.abs(corr).sum()
    print(f"   tuning {t}, violation {viol:.2e}, momentum {dp:.1e}, iterations mean {out['iters'].mean():.2f}",
          flush=True)
    assert viol <= 1e-12 and dp <= 1e-12
    mols = O.molecules(sm.n_atoms, sm.pairs)
    sizes = np.array([len(c) for _, c in mols])
    rng = np.random.default_rng(0)
    pick = sorted(set([int(np.argmin(sizes)), int(np.argmax(sizes))] + rng.choice(len(mols), 4, replace=False).tolist()))
    for i in pick:
        atoms, cons = mols[i]
        local = np.full(sm.n_atoms, -1, np.int64)
        local[atoms] = np.arange(atoms.size)
        rp, lam, it, st, _ = O.solve_molecule(sm.r[atoms], ru[atoms], local[sm.pairs[cons]], sm.d[cons],
                                               1.0 / sm.mass[atoms], 1e-15, 40, until_stagnation=True)
        # the oracle runs to stagnation (its own violation ~1e-15, whether or
        # not that meets its 1e-15 target)
        ref_viol = np.max(O.relative_violation(rp, local[sm.pairs[cons]], sm.d[cons]))
        dr = np.max(np.abs(out["r_out"][atoms] - rp))
        dl = np.max(np.abs(out["lam"][cons] - lam)) / np.max(np.abs(lam))
        print(f"   molecule {i} ({len(cons)} constraints): oracle violation {ref_viol:.1e}, |dr'| {dr:.1e} nm, "
              f"|dlambda| rel {dl:.1e}", flush=True)
        assert ref_viol <= 1e-13 and dr <= 1e-10 and dl <= 1e-9
