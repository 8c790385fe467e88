"""Convergence shape of the GPU solve (Supplement section 2.3: Newton's
iteration converges quadratically near the root; the chord method of
Supplement section 3 linearly; with the factor in FP32 the Newton step is
inexact and the iteration contracts linearly once the FP32 error of the
step dominates, still down to FP64 accuracy).  The solve returns, per
molecule, the maximum relative violation at every iterate (the quantity of
Supplement section 4's stopping rule); it is compared with the oracle's
history of the same quantity on the 64-atom chain and a batch of 16 trees
(8 to 2,048 atoms)."""
import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import DeviceSystem

pytestmark = pytest.mark.gpu

TOL = 1e-12
HLEN = 41


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _gpu_history(torch, sm, ru, prec, variant):
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    nm = plan.n_molecules
    ds = DeviceSystem(sm).alloc_status(nm)
    rud = ds.upload_ru(ru)
    hist = torch.full((nm, HLEN), float("nan"), dtype=torch.float64, device=ds.r.device)
    plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status, precision=prec, variant=variant,
               history=hist)
    torch.cuda.synchronize()
    first = plan.molecules()["first_constraint"]
    return (ds.iters.cpu().numpy()[:nm], ds.status.cpu().numpy()[:nm], hist.cpu().numpy(), first)


def _oracle_histories(sm, ru, variant="newton"):
    ref = O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=TOL, max_iter=40, variant=variant)
    return {int(cons[0]): (int(ref["iters"][m]), np.asarray(ref["history"][m]))
            for m, (_, cons) in enumerate(ref["molecules"])}


def _systems():
    chain = S.chain64(0)
    sizes = [8, 9, 11, 16, 23, 40, 64, 65, 100, 128, 200, 300, 513, 900, 1400, 2048]
    trees = S.concat([S.random_tree(n, seed=100 + i) for i, n in enumerate(sizes)])
    return {"chain64": (chain, S.perturb(chain.r, 0.002, 1)), "batch16": (trees, S.perturb(trees.r, 0.002, 5))}


@pytest.mark.parametrize("case", ["chain64", "batch16"])
def test_fp64_newton_history_matches_oracle_and_is_quadratic(torch, case):
    sm, ru = _systems()[case]
    print(f"== FP64 Newton history, {case}", flush=True)
    iters, status, hist, first = _gpu_history(torch, sm, ru, L.PREC_FP64, L.VARIANT_NEWTON)
    ref = _oracle_histories(sm, ru)
    assert np.all(status == L.OK)
    orders = []
    for m in range(len(iters)):
        it_ref, h_ref = ref[int(first[m])]
        h = hist[m, :iters[m] + 1]
        assert iters[m] == it_ref, (m, iters[m], it_ref)
        # the same iterates up to rounding: the same violations
        assert np.all(np.abs(h - h_ref) <= 1e-6 * h_ref + 1e-13), (m, h, h_ref)
        assert h[-1] <= TOL and np.all(h[:-1] > TOL)
        # quadratic: log rho_{l+1} / log rho_l near 2 once rho_l < 1e-2 (the
        # last step, into the rounding floor of the coordinates, is left out)
        for l in range(len(h) - 1):
            if h[l] < 1e-2 and h[l + 1] > TOL:
                orders.append(np.log(h[l + 1]) / np.log(h[l]))
    print(f"   {len(iters)} molecules, iterations {np.unique(iters, return_counts=True)}, "
          f"convergence orders min {min(orders):.2f} median {np.median(orders):.2f}", flush=True)
    assert min(orders) >= 1.8


@pytest.mark.parametrize("case", ["chain64", "batch16"])
def test_mixed_history_contracts_to_fp64_accuracy(torch, case):
    """The FP32 factor: the early iterates follow the FP64 Newton history
    (their error is far above the FP32 step error), every step contracts the
    violation at least tenfold, and the last iterate is within 1e-12."""
    sm, ru = _systems()[case]
    print(f"== mixed-precision Newton history, {case}", flush=True)
    iters, status, hist, first = _gpu_history(torch, sm, ru, L.PREC_MIXED, L.VARIANT_NEWTON)
    ref = _oracle_histories(sm, ru)
    assert np.all(status == L.OK)
    worst = 0.0
    for m in range(len(iters)):
        _, h_ref = ref[int(first[m])]
        h = hist[m, :iters[m] + 1]
        assert h[-1] <= TOL
        ratio = h[1:] / h[:-1]
        worst = max(worst, float(ratio.max()) if ratio.size else 0.0)
        assert np.all(ratio <= 0.1), (m, h)
        k = min(len(h), len(h_ref))
        big = h_ref[:k] >= 1e-6
        assert np.all(np.abs(h[:k][big] - h_ref[:k][big]) <= 1e-2 * h_ref[:k][big]), (m, h, h_ref)
    print(f"   iterations {np.unique(iters, return_counts=True)}, largest step ratio {worst:.2e}", flush=True)


def test_chord_history_is_linear(torch):
    """The chord method (A(r, r) factored once): linear contraction, the
    same iterates as the oracle's chord iteration."""
    sm, ru = _systems()["chain64"]
    print("== FP64 chord history, chain64", flush=True)
    iters, status, hist, first = _gpu_history(torch, sm, ru, L.PREC_FP64, L.VARIANT_CHORD)
    ref = _oracle_histories(sm, ru, variant="chord")
    assert np.all(status == L.OK)
    it_ref, h_ref = ref[int(first[0])]
    h = hist[0, :iters[0] + 1]
    assert iters[0] == it_ref and np.all(np.abs(h - h_ref) <= 1e-6 * h_ref + 1e-13)
    ratio = h[1:] / h[:-1]
    orders = np.log(h[1:]) / np.log(h[:-1])
    print(f"   iterations {iters[0]}, step ratios {np.array2string(ratio, precision=2)}, orders "
          f"{np.array2string(orders, precision=2)}", flush=True)
    assert np.all(ratio < 1.0) and np.median(orders[1:]) < 1.5
