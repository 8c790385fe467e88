"""The angle-constrained configuration at full size: 20 protein-like
molecules with bonds and H-X-H / H-X-Y angle constraints (each split across
workgroups) plus 1,000 lipid chains, 253,926 constraints, with bench.py's
seed, first perturbed input (sigma 0.006 nm) and default launch.  Every
constraint is checked (violation <= 1e-12; the correction conserves linear
and angular momentum and is the sum of pair forces along the old bond
vectors).  The first protein (10,519 constraints, split across workgroups)
is compared element by element with the dense CPU oracle's solution stored
in tests/golden/angles_protein0.npz (written by
tests/golden/make_angles_protein.py, which calls only the oracle); sampled
lipids are solved by the oracle in the test; the split proteins are also
compared with the same system solved with every molecule whole on one
workgroup."""
import os

import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import solve_once

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "angles_protein0.npz")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


@pytest.fixture(scope="module")
def system():
    sm = S.angles_system(seed=2)                # bench.py --workload angles, --seed default
    ru = S.perturb(sm.r, 0.006, 10_000)         # bench.py's first resident input
    return sm, ru


@pytest.mark.parametrize("name,prec,warm", [("mixed decoupled", L.PREC_MIXED, L.WARM_DECOUPLED),
                                            ("fp64 zero", L.PREC_FP64, L.WARM_ZERO)])
def test_angles_full_size(system, name, prec, warm):
    sm, ru = system
    print(f"== angles full size, {name}", flush=True)
    out = solve_once(sm, ru, 1e-12, prec, L.VARIANT_NEWTON, warm=warm)
    st = out["plan"].stats()
    assert st["split_molecules"] == 20 and st["split_shared_lane_levels"] > 0, st
    assert np.all(out["status"] == L.OK)
    viol = np.max(O.relative_violation(out["r_out"], sm.pairs, sm.d))
    corr = sm.mass[:, None] * (out["r_out"] - ru)
    dp = np.abs(corr.sum(0)).max() / np.abs(corr).sum()
    e = sm.r[sm.pairs[:, 0]] - sm.r[sm.pairs[:, 1]]
    f = np.zeros_like(sm.r)
    np.add.at(f, sm.pairs[:, 0], -out["lam"][:, None] * e)
    np.add.at(f, sm.pairs[:, 1], out["lam"][:, None] * e)
    df = np.max(np.abs(f - corr)) / np.abs(corr).max()
    torque = np.cross(sm.r, f)
    dl = np.abs(torque.sum(0)).max() / np.abs(torque).sum()
    print(f"   parts {st['split_parts']}, violation {viol:.2e}, momentum {dp:.1e}, pair forces {df:.1e}, "
          f"moment {dl:.1e}, iterations mean {out['iters'].mean():.2f} max {out['iters'].max()}", flush=True)
    assert viol <= 1e-12 and dp <= 1e-12 and df <= 1e-12 and dl <= 1e-12

    mols = O.molecules(sm.n_atoms, sm.pairs)
    # the first protein against the dense oracle's stored solution
    gold = np.load(GOLDEN)
    atoms, cons = mols[0]
    assert np.array_equal(atoms, gold["atoms"]) and np.array_equal(cons, gold["cons"])
    dr = np.max(np.abs(out["r_out"][atoms] - gold["r_new"]))
    dlam = np.max(np.abs(out["lam"][cons] - gold["lam"])) / np.max(np.abs(gold["lam"]))
    vmol = np.max(O.relative_violation(out["r_out"], sm.pairs[cons], sm.d[cons]))
    print(f"   protein 0 ({len(cons)} constraints) vs dense oracle: |dr'| {dr:.1e} nm, |dlambda| rel {dlam:.1e}, "
          f"violation {vmol:.1e} (oracle {float(gold['violation']):.1e}, {int(gold['iters'])} iterations)", flush=True)
    assert dr <= 1e-10 and dlam <= 1e-9 and vmol <= 1e-12

    sizes = np.array([len(c) for _, c in mols])
    small = np.flatnonzero(sizes < 1000)
    rng = np.random.default_rng(0)
    pick = sorted(set([int(np.argmin(sizes))] + rng.choice(small, 5, replace=False).tolist()))
    for i in pick:
        atoms, cons = mols[i]
        local = np.full(sm.n_atoms, -1, np.int64)
        local[atoms] = np.arange(atoms.size)
        rp, lam, _, _, _ = O.solve_molecule(sm.r[atoms], ru[atoms], local[sm.pairs[cons]], sm.d[cons],
                                             1.0 / sm.mass[atoms], 1e-15, 40, until_stagnation=True)
        dr = np.max(np.abs(out["r_out"][atoms] - rp))
        dlam = np.max(np.abs(out["lam"][cons] - lam)) / np.max(np.abs(lam))
        print(f"   molecule {i} ({len(cons)} constraints): |dr'| {dr:.1e} nm, |dlambda| rel {dlam:.1e}", flush=True)
        assert dr <= 1e-10 and dlam <= 1e-9

    whole = solve_once(sm, ru, 1e-12, prec, L.VARIANT_NEWTON, warm=warm, split_rows=-1)
    assert whole["plan"].stats()["split_molecules"] == 0
    assert np.all(whole["status"] == L.OK)
    big = np.concatenate([atoms for atoms, cons in mols if len(cons) >= 1000])
    dw = np.max(np.abs(out["r_out"][big] - whole["r_out"][big]))
    print(f"   split proteins vs whole-molecule solves: |dr'| {dw:.1e} nm", flush=True)
    assert dw <= 1e-10
