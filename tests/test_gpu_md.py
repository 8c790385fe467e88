"""Constrained leapfrog around the device solve: the supplement's simple
pendulum (energy error bounded and second order in h at Tol = 1e-12, drift
at loose tolerance with the simplified Newton method, the sign of the energy
error at Tol = 1e-4 opposite for Newton and chord), a multi-link pendulum
on the general path, and a few steps of a mixed system against the same
integration done on the CPU with the oracle."""
import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import md as MD
from paper_2503_13075_amd import synth as S

pytestmark = pytest.mark.gpu

G, LEN, V0 = 9.82, 1.0, 1.0


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _period():
    th = np.arccos(1.0 - 0.5 * V0 ** 2 / (G * LEN))
    return 2 * np.pi * np.sqrt(LEN / G) * (1 + th ** 2 / 16 + 11 * th ** 4 / 3072)


def _pendulum_run(steps_per_period, periods, tol, variant):
    """Relative energy error R_k = (E_k - E_0) / E_0 with E_k from r_k and
    v_k = (v_{k-1/2} + v_{k+1/2}) / 2, and the bob's x coordinate."""
    import torch
    T = _period()
    h = T / steps_per_period
    sm, v = MD.pendulum(LEN, 1.0, 1e20, V0)
    v = v.copy()
    v[1] = [V0, -0.5 * h * V0 ** 2 / LEN, 0.0]      # v_{-1/2}: second-order start (centripetal)
    ig = MD.ConstrainedLeapfrog(sm, v, h, tol=tol, variant=variant)
    f = torch.from_numpy(S.soa(MD.gravity(sm, G, fixed=(0,)))).cuda()
    e0 = 0.5 * V0 ** 2
    rp, vp = ig.state()
    R, xs = [], []
    for _ in range(steps_per_period * periods):
        ig.step(f)
        r, vv = ig.state()
        vk = 0.5 * (vp[1] + vv[1])
        R.append((0.5 * vk @ vk + G * rp[1, 1] - e0) / e0)
        xs.append(r[1, 0])
        rp, vp = r, vv
    assert np.all(ig.worst.cpu().numpy() == L.OK)
    return np.array(R), np.array(xs), h, rp


def test_pendulum_energy_is_bounded_and_second_order():
    """The supplement's simple pendulum at Tol = 1e-12: the maximum relative
    energy error is about 2^-10 at 100 steps per period and falls four-fold
    per halving of h (2^-12 at 200), with no drift; the period matches the
    large-amplitude series 2 pi sqrt(l/g) (1 + th^2/16 + 11 th^4/3072)."""
    R1, x1, h1, rp = _pendulum_run(100, 100, 1e-12, L.VARIANT_NEWTON)
    R2, x2, h2, _ = _pendulum_run(200, 100, 1e-12, L.VARIANT_NEWTON)
    m1, m2 = np.abs(R1).max(), np.abs(R2).max()
    print(f"max |R|: 100 steps/period {m1:.3e} (2^{np.log2(m1):.2f}), 200 {m2:.3e} (2^{np.log2(m2):.2f})", flush=True)
    assert 2.0 ** -10.5 < m1 < 2.0 ** -9.5
    assert 3.5 < m1 / m2 < 4.5
    for R, spp in ((R1, 100), (R2, 200)):
        n5 = 5 * spp
        assert abs(R[-n5:].mean() - R[:n5].mean()) < 0.01 * np.abs(R).max()
    cross = np.where((x2[:-1] < 0) & (x2[1:] >= 0))[0]
    period = np.diff(cross).mean() * h2
    assert abs(period / _period() - 1.0) < 2e-3
    assert abs(np.linalg.norm(rp[1] - rp[0]) - LEN) < 1e-12 * 4


def test_pendulum_loose_tolerance_drifts():
    """Simplified Newton (chord) at loose tolerance: the energy drifts for
    Tol = 1e-3 and stays bounded for Tol = 1e-6 (supplement, second set of
    pendulum runs)."""
    Rl, _, _, _ = _pendulum_run(100, 100, 1e-3, L.VARIANT_CHORD)
    Rt, _, _, _ = _pendulum_run(100, 100, 1e-6, L.VARIANT_CHORD)
    n5 = 500
    drift_l = Rl[-n5:].mean() - Rl[:n5].mean()
    drift_t = Rt[-n5:].mean() - Rt[:n5].mean()
    print(f"drift of the 5-period mean energy error: Tol 1e-3 {drift_l:.3e}, Tol 1e-6 {drift_t:.3e}", flush=True)
    assert drift_l > 0.05 * np.abs(Rl).max()
    assert abs(drift_t) < 0.01 * np.abs(Rt).max()


def _pendulum_sign_run(periods, variant, tol=1e-4, steps_per_period=100, every=10):
    """Relative energy error of the pendulum every ``every`` steps over
    ``periods`` periods; ten steps and the energy sample are captured in one
    HIP graph and replayed, so that a million steps take seconds."""
    import torch
    T = _period()
    h = T / steps_per_period
    sm, v = MD.pendulum(LEN, 1.0, 1e20, V0)
    v = v.copy()
    v[1] = [V0, -0.5 * h * V0 ** 2 / LEN, 0.0]
    ig = MD.ConstrainedLeapfrog(sm, v, h, tol=tol, variant=variant)
    f = torch.from_numpy(S.soa(MD.gravity(sm, G, fixed=(0,)))).cuda()
    e0 = 0.5 * V0 ** 2
    n_rec = periods * steps_per_period // every
    R = torch.zeros(n_rec + 1, dtype=torch.float64, device="cuda")
    idx = torch.zeros(1, dtype=torch.int64, device="cuda")
    one = torch.ones(1, dtype=torch.int64, device="cuda")
    vp = torch.empty(3, dtype=torch.float64, device="cuda")
    yp = torch.empty(1, dtype=torch.float64, device="cuda")

    def block():
        for _ in range(every - 1):
            ig.step(f)
        vp.copy_(ig.v[:, 1])
        yp.copy_(ig.r[1, 1:2])
        ig.step(f)
        vk = 0.5 * (vp + ig.v[:, 1])
        R.index_put_((idx,), (0.5 * (vk * vk).sum() + G * yp - e0) / e0)
        idx.add_(one)

    block()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        block()
    torch.cuda.synchronize()
    idx.zero_()
    for _ in range(n_rec):
        g.replay()
    torch.cuda.synchronize()
    assert np.all(ig.worst.cpu().numpy() == L.OK)
    return R[:n_rec].cpu().numpy()


def test_pendulum_energy_error_sign_depends_on_the_solver():
    """The supplement's third set of pendulum runs: 10,000 periods at 100
    steps per period with Tol = 1e-4.  With Newton's method the relative
    energy error settles below zero (the pendulum appears to lose energy);
    with the simplified Newton (chord) method it stays above zero (it appears
    to gain energy): the sign of the computed drift depends on the solver."""
    rn = _pendulum_sign_run(10_000, L.VARIANT_NEWTON)
    rc = _pendulum_sign_run(10_000, L.VARIANT_CHORD)
    half = len(rn) // 2
    print(f"Newton: negative in {100 * (rn < 0).mean():.1f}% of the samples ({100 * (rn[half:] < 0).mean():.1f}% "
          f"of the second half), mean {rn.mean():.2e}; chord: positive in {100 * (rc > 0).mean():.1f}%, "
          f"mean {rc.mean():.2e}", flush=True)
    assert (rn[half:] < 0).mean() >= 0.9 and rn[half:].mean() < 0
    assert (rc > 0).mean() >= 0.99 and rc[half:].mean() > 0


def test_chain_pendulum_on_general_path():
    """A 12-link pendulum (more than three constraints: general path): the
    energy error stays bounded and every link keeps its length."""
    import torch
    n = 12
    link = 0.25
    r = np.zeros((n + 1, 3))
    r[:, 1] = -link * np.arange(n + 1)
    r[0, 1] = 0.0
    pairs = np.stack([np.arange(n), np.arange(1, n + 1)], 1).astype(np.int32)
    mass = np.concatenate([[1e20], np.ones(n)])
    sm = S.System(pairs=pairs, d=np.full(n, link), mass=mass, r=r, kind=np.zeros(n, np.int8))
    v = np.zeros((n + 1, 3))
    v[1:, 0] = 0.3 * np.arange(1, n + 1) / n
    h = 1e-3
    ig = MD.ConstrainedLeapfrog(sm, v, h, tol=1e-12, precision=L.PREC_MIXED)
    assert ig.plan.n_molecules == 1
    f = torch.from_numpy(S.soa(MD.gravity(sm, G, fixed=(0,)))).cuda()

    def energy(rr, vk):
        return 0.5 * float((mass[1:, None] * vk[1:] ** 2).sum()) + G * float((mass[1:] * rr[1:, 1]).sum())

    rp, vp = ig.state()
    E = []
    for _ in range(3000):
        ig.step(f)
        rr, vv = ig.state()
        E.append(energy(rp, 0.5 * (vp + vv)))
        rp, vp = rr, vv
    assert np.all(ig.worst.cpu().numpy() == L.OK)
    E = np.array(E)
    scale = np.abs(E).max()
    assert (E.max() - E.min()) / scale < 1e-3
    lens = np.linalg.norm(rp[pairs[:, 0]] - rp[pairs[:, 1]], axis=1)
    assert np.max(np.abs(lens - link)) < 1e-12 * 4 * link


def test_leapfrog_matches_cpu_integration():
    """Five steps of a mixed system (small molecules, a tree, free atoms)
    under a harmonic trap: device leapfrog + solve against the same scheme
    on the CPU with the oracle's solve."""
    import torch
    sm = S.concat([S.small_molecules(2, seed=61), S.random_tree(40, seed=62), S.water_box(3, seed=63)], spacing=2.0)
    free = np.array([[5.0, 5.0, 5.0], [-4.0, 2.0, 1.0]])
    sm = S.System(pairs=sm.pairs, d=sm.d, mass=np.concatenate([sm.mass, [12.0, 1.0]]),
                  r=np.concatenate([sm.r, free]), kind=sm.kind)
    rng = np.random.default_rng(64)
    v0 = rng.normal(0.0, 0.3, size=(sm.n_atoms, 3))
    h, k_trap = 2e-3, 50.0
    ig = MD.ConstrainedLeapfrog(sm, v0, h, tol=1e-12)
    r_cpu, v_cpu = sm.r.copy(), v0.copy()
    for step in range(5):
        f_cpu = -k_trap * r_cpu
        ig.step(torch.from_numpy(S.soa(f_cpu)).cuda())
        v_cpu = v_cpu + h * f_cpu / sm.mass[:, None]
        ru = r_cpu + h * v_cpu
        ref = O.solve(sm.pairs, sm.d, sm.mass, r_cpu, ru, tol=1e-15, until_stagnation=True, max_iter=40)
        v_cpu = (ref["r_new"] - r_cpu) / h
        r_cpu = ref["r_new"]
        r_gpu, v_gpu = ig.state()
        assert np.max(np.abs(r_gpu - r_cpu)) <= 1e-10, step
        assert np.max(np.abs(v_gpu - v_cpu)) <= 1e-10 / h, step
        r_cpu, v_cpu = r_gpu, v_gpu      # continue from the device state (compare one step at a time)
    assert np.all(ig.worst.cpu().numpy() == L.OK)


def test_leapfrog_warm_starts_agree_and_save_iterations():
    """The same trajectory (to the solve tolerance) from lambda_0 = 0, from
    the decoupled start and from the previous step's multipliers; the
    previous step's multipliers need fewer Newton iterations."""
    import torch
    sm = S.concat([S.random_tree(60, seed=71), S.protein(20, seed=72)], spacing=2.0)
    rng = np.random.default_rng(73)
    v0 = rng.normal(0.0, 0.3, size=(sm.n_atoms, 3))
    h, k_trap = 2e-3, 50.0
    runs = {}
    for warm in ("zero", "decoupled", "previous"):
        ig = MD.ConstrainedLeapfrog(sm, v0, h, tol=1e-12, warm=warm)
        its = []
        for step in range(20):
            r, _ = ig.state()
            ig.step(torch.from_numpy(S.soa(-k_trap * r)).cuda())
            its.append(ig.iters[:ig.plan.n_molecules].cpu().numpy().mean())
        assert np.all(ig.worst.cpu().numpy() == L.OK)
        runs[warm] = (ig.state()[0], np.mean(its[1:]))
        print(f"warm {warm}: mean Newton iterations (steps 2-20) {runs[warm][1]:.2f}", flush=True)
    for warm in ("decoupled", "previous"):
        assert np.max(np.abs(runs[warm][0] - runs["zero"][0])) <= 1e-9
    assert runs["previous"][1] < runs["zero"][1]
