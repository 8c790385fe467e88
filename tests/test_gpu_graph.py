"""The solve (fork/join over the plan's streams, every launch group, and the
learned start's feature and network kernels) captured in a HIP graph:
each replay, interleaved with eager work and synchronisations, must equal
the eager solve bit for bit."""
import numpy as np
import pytest

from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd import warmstart as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("learned", [False, True])
def test_graph_replays_match_eager(learned):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sizes = [9, 40, 130, 700, 2000]
    sm = S.concat([S.random_tree(n, seed=300 + i) for i, n in enumerate(sizes)])
    ru = S.perturb(sm.r, 0.002, 8)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    if learned:
        params, norm, _ = W.load(W.WEIGHTS["trees"])
        plan.load_mlp(params, norm)
    r, rut, mass = W._device_inputs(sm, ru, "cuda")
    nm = plan.n_molecules

    def buffers():
        return (torch.empty_like(r), torch.zeros(sm.n_constraints, dtype=torch.float64, device="cuda"),
                torch.zeros(nm, dtype=torch.int32, device="cuda"), torch.zeros(nm, dtype=torch.int32, device="cuda"))

    def solve(bufs):
        ro, lam, it, st = bufs
        if learned:
            plan.solve_learned(r, rut, mass, 1e-12, ro, lam, it, st, precision=L.PREC_MIXED)
        else:
            plan.solve(r, rut, mass, 1e-12, ro, lam, it, st, precision=L.PREC_MIXED)

    eager = buffers()
    solve(eager)
    torch.cuda.synchronize()
    gb = buffers()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        solve(gb)                      # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        solve(gb)
    for rep in range(4):
        for t in gb:
            t.fill_(-7)                # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, gb):
            assert torch.equal(a, b), f"replay {rep} differs"
        assert int((gb[3] == L.OK).sum()) == nm


def test_device_inputs_match_host_generator_and_advance_in_a_graph():
    """ilves_perturb_normal against the host Philox/Box-Muller generator,
    then a captured graph [perturb, solve, step += 1]: every replay draws
    the next step's inputs and solves them to the tolerance."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import newton_dense as O
    sizes = [12, 90, 400]
    sm = S.concat([S.random_tree(n, seed=500 + i) for i, n in enumerate(sizes)])
    sigma, seed = 0.002, 2025
    r = torch.from_numpy(S.soa(sm.r)).cuda()
    mass = torch.from_numpy(sm.mass.copy()).cuda()
    step = torch.tensor([3], dtype=torch.int64, device="cuda")
    ru = torch.empty_like(r)
    for st in (3, 4):
        L.perturb_normal(r, sigma, seed, step, ru)
        torch.cuda.synchronize()
        host = S.perturb_philox(sm.r, sigma, seed, st)
        got = ru.cpu().numpy().T
        assert np.max(np.abs(got - host)) <= 1e-15 * 8 + 1e-14 * sigma
        L.counter_add(step, 1)
    torch.cuda.synchronize()
    assert int(step.item()) == 5
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    nm = plan.n_molecules
    ro = torch.empty_like(r)
    lam = torch.zeros(sm.n_constraints, dtype=torch.float64, device="cuda")
    it = torch.zeros(nm, dtype=torch.int32, device="cuda")
    stt = torch.zeros(nm, dtype=torch.int32, device="cuda")

    def step_fn():
        L.perturb_normal(r, sigma, seed, step, ru)
        plan.solve(r, ru, mass, 1e-12, ro, lam, it, stt, precision=L.PREC_MIXED)
        L.counter_add(step, 1)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step_fn()                       # warm-up outside the capture (step 5)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step_fn()
    torch.cuda.synchronize()
    step.fill_(10)
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert int(step.item()) == 11 + k
        assert int((stt == L.OK).sum()) == nm
        rp = ro.cpu().numpy().T
        host_ru = S.perturb_philox(sm.r, sigma, seed, 10 + k)
        assert np.max(np.abs(ru.cpu().numpy().T - host_ru)) <= 1e-14
        assert np.max(O.relative_violation(rp, sm.pairs, sm.d)) <= 1e-12
