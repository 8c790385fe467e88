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
