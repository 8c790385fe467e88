"""Velocity constraints on the GPU (ilves_project_velocities, the velocity
half of RATTLE): parity with the oracle's projection on the per-molecule,
small-molecule and split paths, FP64 and mixed precision; tangency to
rounding; and the projected velocity of the simple pendulum is
perpendicular to its rod."""
import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import md as MD
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import DeviceSystem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _project(sm, v, prec, **plan_kw):
    import torch
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d, **plan_kw)
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    vd = torch.from_numpy(S.soa(v)).cuda()
    vo = torch.empty_like(vd)
    mu = torch.zeros(sm.n_constraints, dtype=torch.float64, device="cuda")
    plan.project_velocities(ds.r, vd, ds.mass, 1e-12, vo, mu, ds.iters, ds.status, precision=prec)
    torch.cuda.synchronize()
    return (vo.cpu().numpy().T.copy(), mu.cpu().numpy(), ds.iters[:plan.n_molecules].cpu().numpy(),
            ds.status[:plan.n_molecules].cpu().numpy(), plan)


@pytest.mark.parametrize("name", ["batch", "split"])
def test_projection_matches_oracle(name):
    if name == "batch":
        sm = S.concat([S.random_tree(n, seed=400 + i) for i, n in enumerate([8, 40, 300, 1500])] +
                      [S.small_molecules(20, seed=5)], spacing=2.0)
        free = np.array([[9.0, 9.0, 9.0]])
        sm = S.System(pairs=sm.pairs, d=sm.d, mass=np.concatenate([sm.mass, [3.0]]), r=np.concatenate([sm.r, free]),
                      kind=sm.kind)
        kw = {}
    else:
        sm = S.protein(60, seed=3)
        kw = {"split_rows": 100, "split_part_rows": 50}
    rng = np.random.default_rng(11)
    v = rng.normal(0.0, 0.5, size=(sm.n_atoms, 3))
    ref, mu_ref = O.project_velocities(sm.pairs, sm.mass, sm.r, v)
    G = O.jacobian(sm.r, sm.pairs, sm.n_atoms)
    print(f"== velocity projection {name}", flush=True)
    for prec in (L.PREC_FP64, L.PREC_MIXED):
        vo, mu, iters, status, plan = _project(sm, v, prec, **kw)
        if name == "split":
            assert plan.stats()["split_molecules"] == 1
        assert np.all(status == L.OK), status
        assert np.max(iters) <= 2
        dv = np.max(np.abs(vo - ref)) / np.max(np.abs(v))
        dmu = np.max(np.abs(mu - mu_ref)) / np.max(np.abs(mu_ref))
        tan = np.max(np.abs(G @ vo.ravel())) / np.max(np.abs(G @ v.ravel()))
        print(f"   prec {prec}: |dv| rel {dv:.2e}, |dmu| rel {dmu:.2e}, |G v_out| rel {tan:.2e}, iters {np.unique(iters)}",
              flush=True)
        assert dv <= 1e-10 and dmu <= 1e-8 and tan <= 1e-12
        if name == "batch":
            assert np.array_equal(vo[-1], v[-1])


def test_pendulum_tangent_velocity():
    import torch
    sm, v0 = MD.pendulum(1.0, 1.0, 1e20, 1.0)
    ig = MD.ConstrainedLeapfrog(sm, v0, 0.01, tol=1e-12)
    f = torch.from_numpy(S.soa(MD.gravity(sm, 9.82, fixed=(0,)))).cuda()
    for _ in range(30):
        ig.step(f)
    vt, st = ig.tangent_velocities()
    torch.cuda.synchronize()
    r, v = ig.state()
    vt = vt.cpu().numpy().T
    rod = r[1] - r[0]
    assert np.all(st.cpu().numpy()[:ig.plan.n_molecules] == L.OK)
    assert abs(vt[1] @ rod) <= 1e-13 * np.linalg.norm(vt[1]) * np.linalg.norm(rod)
    assert np.linalg.norm(vt[1] - v[1]) <= 0.05 * np.linalg.norm(v[1])   # a small correction of the chord velocity
