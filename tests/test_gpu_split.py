"""Molecules split across workgroups on the GPU (block-bordered LU with a
Schur complement on the separator rows, one workgroup per part, device-wide
barriers between the phases of a Newton iteration): parity with the oracle
and with the host replay of the same schedule, for FP64 / mixed precision,
Newton / chord, caller's warm start, the learned start (and its features,
computed over the whole molecule); repeated solves on one plan (the
barrier state carries over), graph replay, status reporting, and a system
that mixes split, whole and small molecules with free atoms."""
import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S
from paper_2503_13075_amd.device import DeviceSystem, solve_once

pytestmark = pytest.mark.gpu

TOL = 1e-12
POS_TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()
    return torch


def _oracle(sm, ru):
    return O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=1e-15, until_stagnation=True, max_iter=40)


def _check(sm, out, ref, label):
    assert np.all(out["status"] == L.OK), (label, out["status"])
    viol = np.max(O.relative_violation(out["r_out"], sm.pairs, sm.d))
    dpos = np.max(np.abs(out["r_out"] - ref["r_new"]))
    dlam = np.max(np.abs(out["lam"] - ref["lam"])) / np.max(np.abs(ref["lam"]))
    print(f"{label}: violation {viol:.2e}, |dr'| {dpos:.2e} nm, |dlambda| rel {dlam:.2e}, iters {out['iters']}",
          flush=True)
    assert viol <= TOL and dpos <= POS_TOL and dlam <= 1e-9, label


CASES = {
    "protein": lambda: (S.protein(60, seed=3), 0.002, 100, 50),
    "tree_rings": lambda: (S.random_tree(1500, seed=11, ring_frac=0.08), 0.002, 200, 64),
    "h_angles": lambda: (S.add_h_angles(S.protein(50, seed=9)), 0.004, 300, 100),
}
VARIANTS = [("fp64", L.PREC_FP64, L.VARIANT_NEWTON), ("mixed", L.PREC_MIXED, L.VARIANT_NEWTON),
            ("chord64", L.PREC_FP64, L.VARIANT_CHORD), ("chord_mixed", L.PREC_MIXED, L.VARIANT_CHORD)]


@pytest.fixture(scope="module")
def cases():
    out = {}
    for name, make in CASES.items():
        sm, sigma, rows, part = make()
        ru = S.perturb(sm.r, sigma, 5)
        out[name] = (sm, ru, rows, part, _oracle(sm, ru))
    return out


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("name,prec,variant", VARIANTS)
def test_split_matches_oracle_and_replay(cases, case, name, prec, variant):
    sm, ru, rows, part, ref = cases[case]
    print(f"== split {case}/{name}", flush=True)
    out = solve_once(sm, ru, TOL, prec, variant, split_rows=rows, split_part_rows=part)
    st = out["plan"].stats()
    assert st["split_molecules"] == 1 and st["split_parts"] >= 2, st
    if case == "h_angles":  # its parts' long chains take the shared-lane levels (every variant, chord included)
        assert st["split_shared_lane_levels"] > 0, st
    print(f"   parts {st['split_parts']}, separator rows {st['max_separator']}", flush=True)
    _check(sm, out, ref, f"{case}/{name}")
    rep = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru), TOL, precision=prec,
                        variant=variant, split_rows=rows, split_part_rows=part)
    assert np.max(np.abs(out["r_out"] - rep["r_out"].T)) <= POS_TOL
    if variant == L.VARIANT_NEWTON:
        assert abs(int(out["iters"][0]) - int(rep["iters"][0])) <= 1


def test_split_learned_start_and_features(cases):
    """The learned start on a split molecule: the feature passes run over the
    whole molecule (a border row's neighbours in other parts included), so
    its features equal the oracle's; the warm-started split solve matches
    the oracle in both precisions."""
    import torch
    from oracle import mlp as M
    from paper_2503_13075_amd import warmstart as WS
    sm, ru, rows, part, ref = cases["protein"]
    print("== split learned start", flush=True)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d, split_rows=rows, split_part_rows=part)
    assert plan.stats()["split_molecules"] == 1
    params, norm, _ = WS.load(WS.WEIGHTS["trees"])
    plan.load_mlp(params, norm)
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    rud = ds.upload_ru(ru)
    feat = torch.empty((sm.n_constraints, 16), dtype=torch.float32, device="cuda")
    w = torch.empty(sm.n_constraints, dtype=torch.float32, device="cuda")
    plan.features(ds.r, rud, ds.mass, feat, w)
    torch.cuda.synchronize()
    fref, wref = M.features(sm.pairs, sm.d, sm.mass, sm.r, ru)
    exp = fref[plan.row_constraints()]
    err = np.abs(feat.cpu().numpy() - exp) / np.maximum(np.abs(exp).max(0), 1e-6)
    print(f"   max feature error / column scale {err.max():.1e}", flush=True)
    assert err.max() < 1e-5
    fb = torch.zeros(plan.n_molecules, dtype=torch.int32, device="cuda")
    for prec in (L.PREC_FP64, L.PREC_MIXED):
        plan.solve_learned(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status, fb, precision=prec)
        torch.cuda.synchronize()
        out = {"r_out": ds.r_out.cpu().numpy().T, "lam": ds.lam.cpu().numpy(),
               "iters": ds.iters.cpu().numpy()[:plan.n_molecules], "status": ds.status.cpu().numpy()[:plan.n_molecules]}
        _check(sm, out, ref, f"protein/learned/{prec} (fallback {int(fb[0].item())})")


def test_split_warm_start_and_repeated_solves(cases):
    """Caller's lambda_0 near the answer converges in at most one step; ten
    solves in a row on one plan (the barrier counters carry over between
    launches) give bitwise the same result."""
    import torch
    sm, ru, rows, part, ref = cases["protein"]
    print("== split warm start / repeats", flush=True)
    lam0 = ref["lam"] * (1.0 + 1e-9)
    out = solve_once(sm, ru, TOL, L.PREC_FP64, L.VARIANT_NEWTON, lam0=lam0, split_rows=rows, split_part_rows=part)
    _check(sm, out, ref, "protein/warm")
    assert out["iters"][0] <= 1
    plan = out["plan"]
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    rud = ds.upload_ru(ru)
    first = None
    for rep in range(10):
        plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status, precision=L.PREC_MIXED)
        torch.cuda.synchronize()
        r = ds.r_out.cpu().numpy().copy()
        assert np.all(ds.status.cpu().numpy()[:plan.n_molecules] == L.OK)
        if first is None:
            first = r
        else:
            assert np.array_equal(r, first), rep


def test_split_in_graph_replay(cases):
    """A captured solve of a split molecule replayed five times, with eager
    work and synchronisation between replays: every replay matches the
    eager solve bitwise."""
    import torch
    sm, ru, rows, part, ref = cases["tree_rings"]
    print("== split graph replay", flush=True)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d, split_rows=rows, split_part_rows=part)
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    rud = ds.upload_ru(ru)
    plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status, precision=L.PREC_MIXED)
    torch.cuda.synchronize()
    eager = ds.r_out.cpu().numpy().copy()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status, precision=L.PREC_MIXED, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status, precision=L.PREC_MIXED,
                       stream=s)
    for rep in range(5):
        ds.r_out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ds.r_out.cpu().numpy(), eager), rep
        assert np.all(ds.status.cpu().numpy()[:plan.n_molecules] == L.OK)


def test_split_status_paths(cases):
    """Iteration cap and a non-finite input reach every part's decision
    alike (the solve returns with the status of the molecule)."""
    sm, ru, rows, part, ref = cases["protein"]
    print("== split status paths", flush=True)
    out = solve_once(sm, ru, TOL, L.PREC_FP64, L.VARIANT_NEWTON, max_iter=1, split_rows=rows, split_part_rows=part)
    assert out["status"][0] == L.ERR_NOT_CONVERGED and out["iters"][0] == 1
    bad = ru.copy()
    bad[sm.pairs[len(sm.pairs) // 2, 0], 1] = np.nan
    out = solve_once(sm, bad, TOL, L.PREC_FP64, L.VARIANT_NEWTON, split_rows=rows, split_part_rows=part)
    assert out["status"][0] == L.ERR_NONFINITE


def test_mixed_system_with_split_molecules():
    """Two split proteins next to whole trees, small molecules and free
    atoms, FP64 and mixed, against the oracle."""
    print("== split mixed system", flush=True)
    sm = S.concat([S.random_tree(30, seed=1), S.protein(50, seed=2), S.water_box(2, seed=3), S.random_tree(200, seed=4),
                   S.protein(40, seed=5)], spacing=2.0)
    free = np.array([[9.0, 9.0, 9.0]])
    sm = S.System(pairs=sm.pairs, d=sm.d, mass=np.concatenate([sm.mass, [12.0]]), r=np.concatenate([sm.r, free]),
                  kind=sm.kind)
    ru = S.perturb(sm.r, 0.002, 7)
    ref = _oracle(sm, ru)
    for prec in (L.PREC_FP64, L.PREC_MIXED):
        out = solve_once(sm, ru, TOL, prec, L.VARIANT_NEWTON, split_rows=300, split_part_rows=80)
        assert out["plan"].stats()["split_molecules"] == 2
        _check(sm, out, ref, f"mixed system/{prec}")
        assert np.array_equal(out["r_out"][-1], ru[-1])


def test_split_with_values_only_in_lds():
    """Angle-constrained protein whose parts' update lists do not fit in
    LDS next to their factor values: in FP64 the parts keep only the values
    in LDS and read their structure through L2; with the FP32 factor they
    keep the values and the per-row structure in LDS and read only the pair
    tasks and update lists from global memory; both against the oracle."""
    print("== split values-only placement", flush=True)
    sm = S.add_h_angles(S.protein(80, seed=9))
    ru = S.perturb(sm.r, 0.004, 5)
    ref = _oracle(sm, ru)
    for prec in (L.PREC_FP64, L.PREC_MIXED):
        out = solve_once(sm, ru, TOL, prec, L.VARIANT_NEWTON, split_rows=1000, split_part_rows=1000)
        st = out["plan"].stats()
        print(f"   {sm.n_constraints} constraints, parts {st['split_parts']}, separator {st['max_separator']}, "
              f"values-only {st['split_values_lds']}, pairs-global {st['split_pairs_global']}", flush=True)
        assert st["split_molecules"] == 1 and st["split_values_lds"] == 1 and st["split_pairs_global"] == 1, st
        assert st["split_shared_lane_levels"] > 0, st  # the angle fill gives levels whose items share lanes
        _check(sm, out, ref, f"h-angle protein values-only/{prec}")


def test_split_molecules_of_different_placements_interleaved():
    """Three split molecules whose parts take different placements, the one
    that does not fit in LDS between the two that do: the split launches
    take the parts grouped by placement (one launch per placement, not one
    per run of consecutive molecules), and every molecule matches the
    oracle."""
    print("== split placements interleaved", flush=True)
    sm = S.concat([S.protein(120, seed=21), S.add_h_angles(S.protein(80, seed=9)), S.protein(110, seed=22)],
                  spacing=2.0)
    ru = S.perturb(sm.r, 0.003, 7)
    ref = _oracle(sm, ru)
    for prec in (L.PREC_FP64, L.PREC_MIXED):
        out = solve_once(sm, ru, TOL, prec, L.VARIANT_NEWTON, split_rows=1000, split_part_rows=1000)
        st = out["plan"].stats()
        print(f"   {sm.n_constraints} constraints, split {st['split_molecules']}, parts {st['split_parts']}, "
              f"values-only {st['split_values_lds']}, pairs-global {st['split_pairs_global']}", flush=True)
        assert st["split_molecules"] == 3 and st["split_values_lds"] == 1 and st["split_pairs_global"] == 1, st
        _check(sm, out, ref, f"interleaved placements/{prec}")


def test_split_wait_limit_reports_timeout_and_reset_recovers():
    """Failure handling of the split barriers, forced from the host: with a
    wait limit of zero polls a workgroup that has to wait gives up at once,
    marks the molecule poisoned and every part leaves; the split molecule
    reports ILVES_ERR_TIMEOUT (the whole molecules of the system still solve),
    and so does every later solve of that plan, whatever the limit, until
    the host clears the barriers (ilves_plan_reset_barriers); the plan then
    solves the split molecule again, against the oracle."""
    import torch
    print("== split wait limit", flush=True)
    sm = S.concat([S.protein(60, seed=3), S.random_tree(200, seed=4)], spacing=2.0)
    ru = S.perturb(sm.r, 0.002, 5)
    plan = L.Plan(sm.n_atoms, sm.pairs, sm.d, split_rows=500, split_part_rows=50)
    assert plan.stats()["split_molecules"] == 1
    mol = plan.molecules()
    split_idx = int(np.argmax(mol["n_con"]))
    ds = DeviceSystem(sm).alloc_status(plan.n_molecules)
    rud = ds.upload_ru(ru)
    plan.set_wait_limit(0)
    for rep in range(2):
        plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status)
        torch.cuda.synchronize()
        st = ds.status.cpu().numpy()[:plan.n_molecules]
        assert st[split_idx] == L.ERR_TIMEOUT, (rep, st)
        assert np.all(np.delete(st, split_idx) == L.OK), (rep, st)
        plan.set_wait_limit(1 << 22)
    plan.reset_barriers()
    plan.solve(ds.r, rud, ds.mass, TOL, ds.r_out, ds.lam, ds.iters, ds.status)
    torch.cuda.synchronize()
    st = ds.status.cpu().numpy()[:plan.n_molecules]
    assert np.all(st == L.OK), st
    out = {"r_out": ds.r_out.cpu().numpy().T.copy(), "lam": ds.lam.cpu().numpy().copy(), "status": st,
           "iters": ds.iters.cpu().numpy()[:plan.n_molecules]}
    _check(sm, out, _oracle(sm, ru), "split after reset")
    with pytest.raises(L.IlvesError):
        plan.set_wait_limit(-1)


def test_giant_molecule_full_size_properties():
    """One 26,389-constraint molecule (the size of the paper's largest single
    molecule) at the bench's automatic split, where the oracle's dense LU is
    out of reach: properties that hold at any size -- every constraint within
    1e-12; the correction m_i (r'_i - r_u,i) sums to zero and has no moment
    about the origin when taken at the old positions (the multiplier forces
    are central pair forces along the old bond vectors); and the same result
    as the molecule solved whole by one workgroup."""
    print("== giant molecule full size", flush=True)
    sm = S.protein_system(seed=1, n_res=1650)
    ru = S.perturb(sm.r, 0.002, 3)
    for prec in (L.PREC_FP64, L.PREC_MIXED):
        out = solve_once(sm, ru, TOL, prec, L.VARIANT_NEWTON)
        st = out["plan"].stats()
        assert st["split_molecules"] == 1 and st["split_parts"] >= 8, st
        assert np.all(out["status"] == L.OK)
        viol = np.max(O.relative_violation(out["r_out"], sm.pairs, sm.d))
        corr = sm.mass[:, None] * (out["r_out"] - ru)
        scale = np.abs(corr).sum()
        dp = np.abs(corr.sum(0)).max() / scale
        # moment of the multiplier forces about the origin, taken at the old positions
        lam = out["lam"]
        e = sm.r[sm.pairs[:, 0]] - sm.r[sm.pairs[:, 1]]
        f = np.zeros_like(sm.r)
        np.add.at(f, sm.pairs[:, 0], -lam[:, None] * e)
        np.add.at(f, sm.pairs[:, 1], lam[:, None] * e)
        assert np.max(np.abs(f - corr)) <= 1e-12 * np.abs(corr).max()
        dl = np.abs(np.cross(sm.r, f).sum(0)).max() / (np.abs(np.cross(sm.r, f)).sum())
        whole = solve_once(sm, ru, TOL, prec, L.VARIANT_NEWTON, split_rows=-1)
        dw = np.max(np.abs(out["r_out"] - whole["r_out"]))
        print(f"   prec {prec}: parts {st['split_parts']}, violation {viol:.2e}, momentum {dp:.1e}, "
              f"moment {dl:.1e}, |split - whole| {dw:.1e} nm, iters {out['iters']} / {whole['iters']}", flush=True)
        assert viol <= TOL and dp <= 1e-12 and dl <= 1e-12 and dw <= 1e-10
