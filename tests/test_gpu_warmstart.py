"""GPU tests of the learned warm start against the CPU oracle: features,
FP32 forward / gradient / Adam kernels, BF16 MFMA inference, the
warm-started solve and its fallback, and (with the shipped weights) the gain
over lambda_0 = 0 on held-out seeds."""
import os

import numpy as np
import pytest

from oracle import mlp as M
from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd import warmstart as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return t


def _case(seed=5):
    sm = W.c3like_system(seed, n_res=12, n_lipid=4)
    return sm, W.perturbed(sm, seed)


def test_features_match_oracle(torch):
    sm, ru = _case()
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    r, rut, mass = W._device_inputs(sm, ru, "cuda")
    feat = torch.empty((sm.n_constraints, 16), dtype=torch.float32, device="cuda")
    w = torch.empty(sm.n_constraints, dtype=torch.float32, device="cuda")
    plan.features(r, rut, mass, feat, w)
    torch.cuda.synchronize()
    cid = plan.row_constraints()
    ref, wref = M.features(sm.pairs, sm.d, sm.mass, sm.r, ru)
    got = feat.cpu().numpy()
    exp = ref[cid]
    scale = np.maximum(np.abs(exp).max(0), 1e-6)
    err = np.abs(got - exp) / scale
    print("max feature error / column scale:", err.max(0), flush=True)
    assert err.max() < 1e-5
    assert np.allclose(w.cpu().numpy(), wref[cid], rtol=1e-6)


def _net(seed):
    rng = np.random.default_rng(seed)
    p = M.init_params(seed) + rng.normal(0, 0.05, M.N_PARAMS)
    return p


def test_fp32_forward_and_gradient_match_oracle(torch):
    rng = np.random.default_rng(1)
    n = 200                                   # several 64-sample blocks and a ragged tail
    x = rng.normal(size=(n, 16))
    y = rng.normal(size=n)
    p = _net(2)
    pt = torch.from_numpy(p.astype(np.float32)).cuda()
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    yt = torch.from_numpy(y.astype(np.float32)).cuda()
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    L.mlp_forward_f32(pt, xt, out)
    grad = torch.empty_like(pt)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    work = torch.empty(L.mlp_grad_workspace(n), dtype=torch.float32, device="cuda")
    L.mlp_grad_f32(pt, xt, yt, grad, loss, work)
    torch.cuda.synchronize()
    p32 = p.astype(np.float32).astype(np.float64)
    x32 = x.astype(np.float32).astype(np.float64)
    y32 = y.astype(np.float32).astype(np.float64)
    ref_out = M.forward(p32, x32)
    ref_loss, ref_g = M.loss_and_grad(p32, x32, y32)
    assert np.max(np.abs(out.cpu().numpy() - ref_out)) <= 1e-5 * max(1.0, np.max(np.abs(ref_out)))
    assert abs(loss.item() - ref_loss) <= 1e-5 * ref_loss
    g = grad.cpu().numpy()
    rel = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    print("gradient relative error", rel, flush=True)
    assert rel < 1e-4
    # deterministic: same gradient bit for bit on a repeat
    grad2 = torch.empty_like(pt)
    L.mlp_grad_f32(pt, xt, yt, grad2, loss, work)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)


def test_adam_matches_oracle(torch):
    rng = np.random.default_rng(3)
    p = rng.normal(size=300)
    gs = [rng.normal(size=300) for _ in range(3)]
    pt = torch.from_numpy(p.astype(np.float32)).cuda()
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    pr, mr, vr = p.copy(), np.zeros(300), np.zeros(300)
    for step, g in enumerate(gs, start=1):
        L.mlp_adam(pt, torch.from_numpy(g.astype(np.float32)).cuda(), m, v, 1e-2, step)
        pr, mr, vr = M.adam_step(pr, g, mr, vr, step, lr=1e-2)
    torch.cuda.synchronize()
    assert np.max(np.abs(pt.cpu().numpy() - pr)) < 1e-5


def test_bf16_inference_matches_oracle(torch):
    sm, ru = _case(7)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    f, w = M.features(sm.pairs, sm.d, sm.mass, sm.r, ru)
    mean, std = f.mean(0), np.maximum(f.std(0), 1e-6)
    scale = 0.05
    p = _net(4)
    norm = np.concatenate([mean, std, [scale]])
    plan.load_mlp(p.astype(np.float32), norm.astype(np.float32))
    r, rut, mass = W._device_inputs(sm, ru, "cuda")
    lam = torch.zeros(sm.n_constraints, dtype=torch.float64, device="cuda")
    plan.predict(r, rut, mass, lam)
    torch.cuda.synchronize()
    got_t = lam.cpu().numpy() * w
    ref_t = M.predict_lambda(p.astype(np.float32).astype(np.float64), mean.astype(np.float32),
                             std.astype(np.float32), scale, f, w) * w
    net_ref = (ref_t - f[:, 0]) / scale
    err = np.abs(got_t - ref_t) / scale
    print("BF16 network output error (units of the output):", err.max(), "output range", np.abs(net_ref).max(),
          flush=True)
    assert err.max() < 2e-2 * max(1.0, np.abs(net_ref).max())


def _solve_learned(torch, sm, ru, plan, precision=L.PREC_MIXED):
    r, rut, mass = W._device_inputs(sm, ru, "cuda")
    nm = plan.n_molecules
    r_out = torch.empty_like(r)
    lam = torch.zeros(sm.n_constraints, dtype=torch.float64, device="cuda")
    iters = torch.zeros(nm, dtype=torch.int32, device="cuda")
    status = torch.zeros(nm, dtype=torch.int32, device="cuda")
    fb = torch.zeros(nm, dtype=torch.int32, device="cuda")
    plan.solve_learned(r, rut, mass, 1e-12, r_out, lam, iters, status, fb, precision=precision)
    torch.cuda.synchronize()
    return (r_out.cpu().numpy().T, lam.cpu().numpy(), iters.cpu().numpy(), status.cpu().numpy(),
            fb.cpu().numpy())


@pytest.mark.parametrize("precision", [L.PREC_FP64, L.PREC_MIXED])
def test_learned_start_solve_matches_oracle(torch, precision):
    sm, ru = _case(9)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    f, w = M.features(sm.pairs, sm.d, sm.mass, sm.r, ru)
    norm = np.concatenate([f.mean(0), np.maximum(f.std(0), 1e-6), [0.01]]).astype(np.float32)
    plan.load_mlp(_net(5).astype(np.float32), norm)
    rp, lam, iters, status, fb = _solve_learned(torch, sm, ru, plan, precision)
    ref = O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=1e-15, until_stagnation=True, max_iter=40)
    viol = np.max(O.relative_violation(rp, sm.pairs, sm.d))
    dpos = np.max(np.abs(rp - ref["r_new"]))
    dlam = np.max(np.abs(lam - ref["lam"])) / np.max(np.abs(ref["lam"]))
    print(f"learned start, precision {precision}: max rel violation {viol:.2e}, max |dr'| {dpos:.2e} nm, "
          f"max |dlambda|/max|lambda| {dlam:.2e}, iterations mean {iters.mean():.2f}, fallback {fb.mean():.2f}",
          flush=True)
    assert np.all(status == L.OK)
    assert viol <= 1e-12
    assert dpos <= 1e-10
    assert dlam <= 1e-9


def test_corrupted_network_falls_back_and_converges(torch):
    sm, ru = _case(11)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d)
    p = np.zeros(M.N_PARAMS, np.float32)
    p[-1] = 1e3                                   # b3: a huge constant output
    norm = np.concatenate([np.zeros(16), np.ones(16), [1.0]]).astype(np.float32)
    plan.load_mlp(p, norm)
    rp, lam, iters, status, fb = _solve_learned(torch, sm, ru, plan)
    assert np.all(fb == 1)
    assert np.all(status == L.OK)
    assert np.max(O.relative_violation(rp, sm.pairs, sm.d)) <= 1e-12


@pytest.mark.skipif(not os.path.exists(W.DEFAULT_WEIGHTS), reason="no trained weights shipped")
def test_trained_network_beats_the_untrained_one_on_heldout_seeds(torch):
    """What training buys over the same network untrained (zero output
    layer: the decoupled start, each constraint's own solution, which the
    network corrects).  On held-out seeds 1000-1011 of the angle-constrained
    training distribution the trained network's lambda_0 is closer to the
    converged multipliers, the violation at lambda_0 is lower, Newton takes no
    more iterations, and every molecule converges from both starts; lambda_0
    = 0 is reported beside them."""
    params, norm, meta = W.load()
    res = W.evaluate(range(1000, 1012), params, norm)
    print("held-out (12 seeds):", res, flush=True)
    assert res["converged_learned"] == 1.0 and res["converged_decoupled"] == 1.0
    assert res["start_error_learned_rms"] <= 0.9 * res["start_error_decoupled_rms"]
    assert res["violation0_learned_median"] < res["violation0_decoupled_median"]
    assert res["iters_learned_mean"] <= res["iters_decoupled_mean"] + 0.02
    assert res["iters_learned_mean"] < res["iters_zero_mean"]
