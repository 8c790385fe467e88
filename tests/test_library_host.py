"""Host-side checks of the C-ABI library (no GPU): it loads, exports every
function include/ilves.h declares, validates topologies, and its planner's
schedule, replayed on the host, reproduces the oracle."""

import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import _lib as L
from paper_2503_13075_amd import synth as S


def test_exports_every_header_symbol():
    lib = L.lib()
    names = L.header_functions()
    assert "ilves_solve" in names and "ilves_plan_create" in names
    for n in names:
        assert hasattr(lib, n), n
    assert b"gfx950" in lib.ilves_version()


def test_status_strings():
    lib = L.lib()
    for code in range(10):
        assert lib.ilves_status_string(code)


@pytest.mark.parametrize("bad", [
    ([[0, 0]], [0.1], "same"),
    ([[0, 5]], [0.1], "range"),
    ([[0, 1], [1, 0]], [0.1, 0.1], "duplicate"),
    ([[0, 1]], [-0.1], "positive"),
])
def test_topology_validation(bad):
    pairs, d, word = bad
    with pytest.raises(L.IlvesError) as ei:
        L.replay_host(3, pairs, d, np.ones(3), np.zeros((3, 3)), np.zeros((3, 3)), 1e-12)
    assert ei.value.code == L.ERR_TOPOLOGY


CASES = {
    "chain64": lambda: (S.chain64(0), 0.002),
    "tree": lambda: (S.random_tree(400, seed=3), 0.002),
    "protein40": lambda: (S.protein(40, seed=1), 0.002),
    "protein_hangles": lambda: (S.add_h_angles(S.protein(25, seed=2)), 0.006),
    "batch": lambda: (S.concat([S.random_tree(int(n), seed=i) for i, n in enumerate([8, 9, 30, 120, 64])]), 0.002),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision", [L.PREC_FP64, L.PREC_MIXED])
@pytest.mark.parametrize("ordering", [1, 2])
def test_replayed_schedule_matches_oracle(case, precision, ordering):
    sm, sigma = CASES[case]()
    ru = S.perturb(sm.r, sigma, 11)
    ref = O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=1e-15, until_stagnation=True, max_iter=40)
    h = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru), 1e-12,
                      precision=precision, ordering=ordering)
    assert np.all(h["status"] == L.OK)
    rp = h["r_out"].T
    assert np.max(O.relative_violation(rp, sm.pairs, sm.d)) <= 1e-12
    assert np.max(np.abs(rp - ref["r_new"])) <= 1e-10
    assert np.allclose(h["lam"], ref["lam"], rtol=1e-6, atol=1e-9 * np.max(np.abs(ref["lam"])))


def test_replay_chord_variant():
    sm = S.chain64(0)
    ru = S.perturb(sm.r, 0.002, 1)
    ref = O.solve(sm.pairs, sm.d, sm.mass, sm.r, ru, tol=1e-12, variant="chord", max_iter=60)
    h = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru), 1e-12,
                      variant=L.VARIANT_CHORD)
    assert h["status"][0] == L.OK
    # same linear iteration as the oracle's chord method, same count
    assert abs(int(h["iters"][0]) - int(ref["iters"][0])) <= 1
    assert np.max(np.abs(h["r_out"].T - ref["r_new"])) < 1e-10


def test_replay_edge_cases():
    # free atoms keep r_u; redundant constraints are singular; cap reports
    sm = S.chain64(0)
    ru = S.perturb(sm.r, 0.002, 1)
    h = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru), 1e-12, max_iter=1)
    assert h["status"][0] == L.ERR_NOT_CONVERGED and h["iters"][0] == 1
    # atoms 64.. are free
    r = np.concatenate([sm.r, np.ones((3, 3))])
    ru2 = np.concatenate([ru, 2 * np.ones((3, 3))])
    m = np.concatenate([sm.mass, np.ones(3)])
    h = L.replay_host(67, sm.pairs, sm.d, m, S.soa(r), S.soa(ru2), 1e-12)
    assert np.array_equal(h["r_out"][:, 64:], S.soa(ru2)[:, 64:])
    # a rigid triangle plus a fourth planar point with all distances: redundant
    pts = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0], [0.1, 0.1, 0]], float)
    pairs = [(i, j) for i in range(4) for j in range(i + 1, 4)]
    d = [np.linalg.norm(pts[i] - pts[j]) for i, j in pairs]
    h = L.replay_host(4, pairs, d, np.ones(4), S.soa(pts), S.soa(S.perturb(pts, 0.001, 2)), 1e-12)
    assert h["status"][0] == L.ERR_SINGULAR
    # non-finite input
    ru3 = ru.copy()
    ru3[5, 1] = np.nan
    h = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru3), 1e-12)
    assert h["status"][0] == L.ERR_NONFINITE


def test_nested_dissection_shortens_chains():
    sm = S.protein(60, seed=4)
    ru = S.perturb(sm.r, 0.002, 3)
    md = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru), 1e-12, ordering=1)
    nd = L.replay_host(sm.n_atoms, sm.pairs, sm.d, sm.mass, S.soa(sm.r), S.soa(ru), 1e-12, ordering=2)
    assert nd["stats"]["max_levels"] * 4 < md["stats"]["max_levels"]
    # minimum degree on a tree: zero fill (leaf stripping is a perfect elimination order)
    t = S.random_tree(300, seed=1, ring_frac=0.0)
    h = L.replay_host(t.n_atoms, t.pairs, t.d, t.mass, S.soa(t.r), S.soa(t.r), 1e-12, ordering=1)
    assert h["stats"]["fill"] == 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library nothing falls back to a CPU path: loading
    it, and planning through it, raise."""
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "libilves.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()
    with pytest.raises(ImportError):
        L.Plan(2, np.array([[0, 1]], np.int32), np.array([0.1]))


def test_stat_names_cover_the_header_count():
    """ilves_plan_stats writes ILVES_STAT_COUNT int64 values into the buffer
    the binding sizes from its list of names: the two must agree."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ilves.h")).read()
    count = int(re.search(r"#define ILVES_STAT_COUNT (\d+)", hdr).group(1))
    assert len(L.STAT_NAMES) == count
