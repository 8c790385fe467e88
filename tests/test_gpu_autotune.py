"""The launch autotuner: it leaves the plan on a valid tuning that still
solves to the oracle's bar, and its cache returns what was stored."""
import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import autotune as AT
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import DeviceSystem, solve_once


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert AT.load_cached("k", path) is None
    t = {"band_block": [64, 64, 256, 512, 1024], "lds_limit": 0, "ms_default": 1.0, "ms_tuned": 0.9}
    AT.store("k", t, path)
    AT.store("j", dict(t, lds_limit=4096), path)
    assert AT.load_cached("k", path) == t
    assert AT.load_cached("j", path)["lds_limit"] == 4096


@pytest.mark.gpu
def test_autotune_keeps_parity(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sizes = [5, 12, 30, 64, 90, 200, 600, 1500]
    sm = S.concat([S.random_tree(n, seed=300 + i) for i, n in enumerate(sizes)])
    ru = S.perturb(sm.r, 0.002, 8)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    rut = ds.upload_ru(ru)

    def run():
        plan.solve(ds.r, rut, ds.mass, 1e-12, ds.r_out, ds.lam, ds.iters, ds.status, precision=L.PREC_MIXED)

    key = AT.plan_key(plan, L.PREC_MIXED, L.VARIANT_NEWTON)
    path = str(tmp_path / "tune.json")
    res = AT.tuned(plan, run, key, path=path, reps=3)
    print("autotune:", res, flush=True)
    assert not res["cached"] and res["ms_tuned"] <= res["ms_default"]
    assert plan.get_tuning()["band_block"] == res["band_block"]
    again = AT.tuned(plan, run, key, path=path)
    assert again["cached"] and again["band_block"] == res["band_block"]
    seeded = AT.autotune(plan, run, reps=3, passes=1,
                         seeds=[{"band_block": [1024, 1024, 1024, 512, 1024], "lds_limit": 32 * 1024}])
    print("seeded autotune:", seeded, flush=True)
    assert plan.get_tuning()["band_block"] == seeded["band_block"]
    out = solve_once(sm, ru, 1e-12, L.PREC_MIXED, plan=plan)
    ref = O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=1e-15, until_stagnation=True, max_iter=40)
    assert np.all(out["status"] == L.OK)
    assert np.max(O.relative_violation(out["r_out"], sm.pairs, sm.d)) <= 1e-12
    assert np.max(np.abs(out["r_out"] - ref["r_new"])) <= 1e-10
