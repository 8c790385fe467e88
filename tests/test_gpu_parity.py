"""GPU parity of the HIP solve path against the CPU oracle.

Bar (per result): max relative constraint violation <= 1e-12 and max
position difference to the oracle <= 1e-10 nm, for the FP64 Newton path,
the mixed-precision path and the chord variant.  The oracle runs to
stagnation (its own violation ~1e-16), so the difference measures the GPU
result.  All calls go through the C ABI (ctypes binding).
"""
import os

import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import solve_once

pytestmark = pytest.mark.gpu

TOL = 1e-12
POS_TOL = 1e-10
# lambda against the oracle, relative to the largest |lambda| (observed <= 1.5e-11)
LAM_TOL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _oracle(sm, ru, **kw):
    return O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=1e-15, until_stagnation=True, max_iter=40, **kw)


def _check(sm, ru, out, ref, label):
    assert np.all(out["status"] == L.OK), (label, np.unique(out["status"], return_counts=True))
    viol = np.max(O.relative_violation(out["r_out"], sm.pairs, sm.d))
    dpos = np.max(np.abs(out["r_out"] - ref["r_new"]))
    lam_scale = np.max(np.abs(ref["lam"]))
    dlam = np.max(np.abs(out["lam"] - ref["lam"])) / lam_scale
    print(f"{label}: max rel violation {viol:.2e}, max |dr'| {dpos:.2e} nm, max |dlambda|/max|lambda| {dlam:.2e}, "
          f"iters {np.unique(out['iters'], return_counts=True)}", flush=True)
    assert viol <= TOL, (label, viol)
    assert dpos <= POS_TOL, (label, dpos)
    assert dlam <= LAM_TOL, (label, dlam)


VARIANTS = [("fp64", L.PREC_FP64, L.VARIANT_NEWTON), ("mixed", L.PREC_MIXED, L.VARIANT_NEWTON),
            ("chord64", L.PREC_FP64, L.VARIANT_CHORD), ("chord_mixed", L.PREC_MIXED, L.VARIANT_CHORD)]


@pytest.mark.parametrize("name,prec,variant", VARIANTS)
def test_chain64(name, prec, variant):
    sm = S.chain64(0)
    ru = S.perturb(sm.r, 0.002, 1)
    out = solve_once(sm, ru, TOL, prec, variant)
    _check(sm, ru, out, _oracle(sm, ru), f"chain64/{name}")


@pytest.fixture(scope="module")
def protein_case():
    sm = S.protein_system(seed=1, n_res=300)
    ru = S.perturb(sm.r, 0.002, 1000)
    return sm, ru, _oracle(sm, ru)


@pytest.mark.parametrize("name,prec,variant", VARIANTS[:2])
def test_protein_full_size(protein_case, name, prec, variant):
    sm, ru, ref = protein_case
    out = solve_once(sm, ru, TOL, prec, variant)
    _check(sm, ru, out, ref, f"protein300/{name}")


@pytest.fixture(scope="module")
def batch_case():
    sizes = [8, 9, 11, 16, 23, 40, 64, 65, 100, 128, 200, 300, 513, 900, 1400, 2048]
    sm = S.concat([S.random_tree(n, seed=100 + i) for i, n in enumerate(sizes)])
    ru = S.perturb(sm.r, 0.002, 5)
    return sm, ru, _oracle(sm, ru)


@pytest.mark.parametrize("name,prec,variant", VARIANTS)
def test_batch_of_trees(batch_case, name, prec, variant):
    sm, ru, ref = batch_case
    out = solve_once(sm, ru, TOL, prec, variant)
    _check(sm, ru, out, ref, f"batch16/{name}")


@pytest.fixture(scope="module")
def angles_case():
    mols = [S.add_h_angles(S.protein(40, seed=70 + i)) for i in range(2)]
    mols += [S.lipid_chain(900 + j) for j in range(20)]
    sm = S.concat(mols)
    ru = S.perturb(sm.r, 0.006, 9)
    return sm, ru, _oracle(sm, ru)


@pytest.mark.parametrize("name,prec,variant", VARIANTS[:2])
def test_angles(angles_case, name, prec, variant):
    sm, ru, ref = angles_case
    out = solve_once(sm, ru, TOL, prec, variant)
    _check(sm, ru, out, ref, f"angles/{name}")


@pytest.fixture(scope="module")
def small_case():
    mols = [S.small_molecules(6, seed=41), S.water_box(300, seed=42), S.random_tree(60, seed=43)]
    sm = S.concat(mols, spacing=3.0)
    ru = S.perturb(sm.r, 0.003, 44)
    return sm, ru, _oracle(sm, ru)


@pytest.mark.parametrize("name,prec,variant", VARIANTS)
def test_small_molecules(small_case, name, prec, variant):
    """Molecules of one to three constraints on at most four atoms take the
    one-thread-per-molecule path (register Newton, FP64 whatever the
    precision); the tree in the same plan takes the general path."""
    sm, ru, ref = small_case
    out = solve_once(sm, ru, TOL, prec, variant)
    _check(sm, ru, out, ref, f"small/{name}")


@pytest.mark.parametrize("warm", [L.WARM_ZERO, L.WARM_DECOUPLED])
def test_small_molecules_orientation(small_case, warm):
    """Reversing the atom pair of every constraint leaves G(r), and so lambda
    and r', unchanged (e_k and the signs of row k flip together).  The small
    molecules are renumbered in their shape's canonical order at plan time,
    so the reversed topology must give the oracle's result as well, and the
    same numbers as the original one to rounding."""
    import dataclasses
    sm, ru, ref = small_case
    flipped = dataclasses.replace(sm, pairs=np.ascontiguousarray(sm.pairs[:, ::-1]))
    print(f"== small orientation warm {warm}", flush=True)
    a = solve_once(sm, ru, TOL, L.PREC_FP64, warm=warm)
    b = solve_once(flipped, ru, TOL, L.PREC_FP64, warm=warm)
    _check(flipped, ru, b, ref, f"small/flipped/{warm}")
    assert np.array_equal(a["iters"], b["iters"])
    assert np.max(np.abs(a["r_out"] - b["r_out"])) <= 1e-13
    assert np.max(np.abs(a["lam"] - b["lam"])) <= 1e-12 * np.max(np.abs(a["lam"]))


def test_small_molecules_warm_start_and_failures(small_case):
    sm, ru, ref = small_case
    out = solve_once(sm, ru, TOL, L.PREC_FP64, lam0=ref["lam"])
    assert np.all(out["status"] == L.OK) and np.all(out["iters"] <= 1)
    out = solve_once(sm, ru, TOL, L.PREC_FP64, max_iter=1)
    assert np.all(out["status"] == L.ERR_NOT_CONVERGED)
    bad = ru.copy()
    bad[0, 0] = np.inf
    out = solve_once(sm, bad, TOL, L.PREC_FP64)
    assert out["status"][0] == L.ERR_NONFINITE and np.all(out["status"][1:] == L.OK)


def test_placements_and_lane_mappings_agree(batch_case):
    """Global-memory placement and a different lane mapping (other kernel
    instantiations) agree with the default schedule to rounding: the
    compiler may contract multiply-adds differently per instantiation."""
    sm, ru, _ = batch_case
    a = solve_once(sm, ru, TOL, L.PREC_FP64)
    b = solve_once(sm, ru, TOL, L.PREC_FP64, lds_limit=1)          # everything in the global workspace
    c = solve_once(sm, ru, TOL, L.PREC_FP64, block_threads=64)      # other lane mapping
    assert b["plan"].stats()["mol_workspace"] == len(b["iters"])
    scale = np.max(np.abs(a["lam"]))
    for other in (b, c):
        assert np.all(other["status"] == L.OK)
        assert np.max(np.abs(a["r_out"] - other["r_out"])) <= 1e-13
        assert np.max(np.abs(a["lam"] - other["lam"])) <= 1e-10 * scale


def test_retuned_plan_agrees(batch_case):
    """Re-tuning a plan (block size per band, LDS limit) moves molecules
    between kernels and lane mappings; results stay at the oracle's bar and
    agree with the untuned plan to rounding.  Bad tunings are rejected."""
    sm, ru, ref = batch_case
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    base = solve_once(sm, ru, TOL, L.PREC_MIXED, plan=plan)
    assert plan.get_tuning()["band_block"] == [64, 128, 256, 512, 1024]
    scale = np.max(np.abs(base["lam"]))
    for bb, lim in (([1024, 1024, 1024, 1024, 1024], 0), ([128, 64, 512, 512, 512], 0),
                    ([256, 256, 256, 512, 1024], 4096), ([64, 128, 256, 512, 1024], 1)):
        plan.tune(band_block=bb, lds_limit=lim)
        t = plan.get_tuning()
        assert t["band_block"] == bb
        out = solve_once(sm, ru, TOL, L.PREC_MIXED, plan=plan)
        _check(sm, ru, out, ref, f"batch16/tuned {bb} {lim}")
        assert np.max(np.abs(base["r_out"] - out["r_out"])) <= 1e-13
        assert np.max(np.abs(base["lam"] - out["lam"])) <= 1e-10 * scale
    assert plan.stats()["mol_workspace"] == plan.n_molecules      # lds_limit 1: nothing in LDS
    for bad in (dict(band_block=[32, 128, 256, 512, 1024]), dict(band_block=[64, 128, 256, 512, 100]),
                dict(lds_limit=-1)):
        with pytest.raises(L.IlvesError) as e:
            plan.tune(**bad)
        assert e.value.code == L.ERR_ARG
    out = solve_once(sm, ru, TOL, L.PREC_MIXED, plan=plan)        # a rejected tuning leaves the plan usable
    _check(sm, ru, out, ref, "batch16/after rejected tuning")


def test_deterministic_repeat(batch_case):
    sm, ru, _ = batch_case
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    a = solve_once(sm, ru, TOL, L.PREC_MIXED, plan=plan)
    b = solve_once(sm, ru, TOL, L.PREC_MIXED, plan=plan)
    assert np.array_equal(a["r_out"], b["r_out"]) and np.array_equal(a["lam"], b["lam"])


def test_free_atoms_and_empty_topology():
    sm = S.chain64(0)
    r = np.concatenate([sm.r, np.ones((3, 3))])
    ru = np.concatenate([S.perturb(sm.r, 0.002, 1), 2 * np.ones((3, 3))])
    ext = S.System(pairs=sm.pairs, d=sm.d, mass=np.concatenate([sm.mass, np.ones(3)]), r=r, kind=sm.kind)
    out = solve_once(ext, ru, TOL)
    assert np.array_equal(out["r_out"][64:], ru[64:])
    empty = S.System(pairs=np.zeros((0, 2), np.int32), d=np.zeros(0), mass=np.ones(5), r=np.zeros((5, 3)),
                     kind=np.zeros(0, np.int8))
    ru5 = np.arange(15.0).reshape(5, 3)
    out = solve_once(empty, ru5, TOL)
    assert np.array_equal(out["r_out"], ru5) and out["plan"].n_molecules == 0


def test_failure_statuses():
    sm = S.chain64(0)
    ru = S.perturb(sm.r, 0.002, 1)
    out = solve_once(sm, ru, TOL, max_iter=1)
    assert out["status"][0] == L.ERR_NOT_CONVERGED and out["iters"][0] == 1
    bad = ru.copy()
    bad[7, 2] = np.nan
    out = solve_once(sm, bad, TOL)
    assert out["status"][0] == L.ERR_NONFINITE
    pts = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [0.1, 0.1, 0]], float)
    pairs = np.array([(i, j) for i in range(4) for j in range(i + 1, 4)], np.int32)
    d = np.array([np.linalg.norm(pts[i] - pts[j]) for i, j in pairs])
    red = S.System(pairs=pairs, d=d, mass=np.ones(4), r=pts, kind=np.zeros(6, np.int8))
    out = solve_once(red, S.perturb(pts, 0.001, 2), TOL)
    assert out["status"][0] == L.ERR_SINGULAR


def test_caller_warm_start_from_solution():
    sm = S.chain64(0)
    ru = S.perturb(sm.r, 0.002, 1)
    ref = _oracle(sm, ru)
    out = solve_once(sm, ru, TOL, lam0=ref["lam"])
    assert out["status"][0] == L.OK and out["iters"][0] <= 1
    assert np.max(np.abs(out["r_out"] - ref["r_new"])) <= POS_TOL


def test_native_library_is_loaded_once():
    maps = open(f"/proc/{os.getpid()}/maps").read()
    assert "libilves.so" in maps
    hip = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(hip) == 1, hip


def test_plain_entry_point_takes_the_plan_options(batch_case):
    """ilves_solve (no per-call options) runs with the precision, variant and
    start the plan was created with: same result as the explicit call."""
    import ctypes

    import torch

    from paper_2503_13075_amd.device import DeviceSystem
    sm, ru, ref = batch_case
    for prec, warm in ((L.PREC_FP64, L.WARM_ZERO), (L.PREC_MIXED, L.WARM_DECOUPLED)):
        plan = L.Plan(sm.n_atoms, sm.pairs, sm.d, precision=prec, warm_start=warm)
        ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
        rud = ds.upload_ru(ru)
        code = plan._L.ilves_solve(plan._h, ds.r.data_ptr(), rud.data_ptr(), ds.mass.data_ptr(), TOL,
                                   ds.r_out.data_ptr(), ds.lam.data_ptr(), ds.iters.data_ptr(), ds.status.data_ptr(),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert code == L.OK
        torch.cuda.synchronize()
        out = {"r_out": ds.r_out.cpu().numpy().T.copy(), "lam": ds.lam.cpu().numpy().copy(),
               "iters": ds.iters[:plan.n_molecules].cpu().numpy().copy(),
               "status": ds.status[:plan.n_molecules].cpu().numpy().copy()}
        _check(sm, ru, out, ref, f"batch16/ilves_solve prec {prec} warm {warm}")
        ex = solve_once(sm, ru, TOL, prec, L.VARIANT_NEWTON, plan=plan, warm=warm)
        assert np.array_equal(out["r_out"], ex["r_out"]) and np.array_equal(out["iters"], ex["iters"])
