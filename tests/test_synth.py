"""Synthetic workload generators: sizes, masses, exact reference geometry,
valence limits, reproducibility and full rank of the constraint set."""
import math

import numpy as np
import pytest

from paper_2503_13075_amd import synth as S


def _violation(sysm):
    e = sysm.r[sysm.pairs[:, 0]] - sysm.r[sysm.pairs[:, 1]]
    return np.max(np.abs(np.linalg.norm(e, axis=1) - sysm.d) / sysm.d)


def test_chain64_layout():
    c = S.chain64(0)
    assert c.n_atoms == 64 and c.n_constraints == 125
    assert np.sum(c.kind == 0) == 63 and np.sum(c.kind == 1) == 62
    assert np.allclose(c.d[c.kind == 0], 0.153) and np.allclose(c.d[c.kind == 1], 0.250)
    assert np.allclose(c.mass[::2], 12.011) and np.allclose(c.mass[1::2], 14.027)
    assert _violation(c) < 1e-14
    # angle implied by the two distances
    e1 = c.r[1] - c.r[0]
    e2 = c.r[1] - c.r[2]
    ang = math.degrees(math.acos(e1 @ e2 / np.linalg.norm(e1) / np.linalg.norm(e2)))
    assert abs(ang - 109.57) < 0.01


def test_protein_size_and_chemistry():
    p = S.protein(300, seed=1)
    assert abs(p.n_atoms - 4700) / 4700 < 0.05
    assert p.n_constraints > p.n_atoms - 1          # ring closures add bonds
    assert _violation(p) < 1e-13
    deg = np.bincount(p.pairs.ravel(), minlength=p.n_atoms)
    assert deg.max() <= 4
    h = np.array([e == "H" for e in p.elem])
    assert np.all(deg[h] == 1)
    assert set(np.round(p.mass, 3)) <= {1.008, 12.011, 14.007, 15.999, 32.06}
    assert np.all((p.d >= 0.0999) & (p.d <= 0.1531))


def test_random_tree_exact_size_and_rings():
    for n in (8, 37, 500, 2048):
        t = S.random_tree(n, seed=n)
        assert t.n_atoms == n
        rings = t.n_constraints - (n - 1)
        assert rings == int(round(0.05 * n)) or n < 40
        assert _violation(t) < 1e-13
        assert np.bincount(t.pairs.ravel(), minlength=n).max() <= 4


def test_batch_sizes_log_uniform():
    s = S.batch_sizes(4096, seed=2)
    assert s.min() >= 8 and s.max() <= 2048
    # log-uniform: mean of log size is the midpoint
    assert abs(np.mean(np.log(s)) - 0.5 * (math.log(8) + math.log(2048))) < 0.1


def test_reproducible():
    a = S.random_tree(300, seed=5)
    b = S.random_tree(300, seed=5)
    assert np.array_equal(a.pairs, b.pairs) and np.array_equal(a.r, b.r)
    assert np.array_equal(S.perturb(a.r, 0.002, 3), S.perturb(b.r, 0.002, 3))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_h_angles_full_rank(seed):
    p = S.add_h_angles(S.protein(10, seed=seed))
    assert np.sum(p.kind == 1) > 0 and _violation(p) < 1e-13
    assert len(set(map(tuple, np.sort(p.pairs, axis=1)))) == p.n_constraints
    # rank of G(r): the constraint gradients are independent
    n = p.n_constraints
    G = np.zeros((n, 3 * p.n_atoms))
    for k, (a, b) in enumerate(p.pairs):
        e = p.r[a] - p.r[b]
        G[k, 3 * a:3 * a + 3] = e
        G[k, 3 * b:3 * b + 3] = -e
    sv = np.linalg.svd(G, compute_uv=False)
    assert sv[-1] / sv[0] > 1e-4


def test_concat_keeps_molecules_apart():
    m = [S.random_tree(20, seed=i) for i in range(5)]
    c = S.concat(m)
    assert c.n_atoms == 100 and c.n_constraints == sum(x.n_constraints for x in m)
    assert _violation(c) < 1e-13
    assert list(c.mol_start) == [0, 20, 40, 60, 80]


def test_philox_known_answers():
    """Known-answer vectors of Philox4x32-10 published with the generator
    (Random123 distribution): counter / key -> output words."""
    cases = [([0, 0, 0, 0], (0, 0), [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
             ([0xffffffff] * 4, (0xffffffff, 0xffffffff), [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
             ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], (0xa4093822, 0x299f31d0),
              [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1])]
    for ctr, key, want in cases:
        got = S.philox4x32_10(np.array([ctr], np.uint32), key)[0]
        assert [int(x) for x in got] == want


def test_philox_normals_statistics_and_streams():
    z = S.philox_normals(200_000, seed=11, step=5)
    assert np.all(np.abs(z.mean(0)) < 0.01)
    assert np.all(np.abs(z.std(0) - 1.0) < 0.01)
    kurt = ((z - z.mean(0)) ** 4).mean(0) / z.var(0) ** 2
    assert np.all(np.abs(kurt - 3.0) < 0.05)
    # different steps, seeds and atoms give different draws
    assert not np.allclose(S.philox_normals(10, 11, 5), S.philox_normals(10, 11, 6))
    assert not np.allclose(S.philox_normals(10, 11, 5), S.philox_normals(10, 12, 5))
    assert np.array_equal(S.philox_normals(10, 11, 5), S.philox_normals(20, 11, 5)[:10])
    assert abs(np.corrcoef(z[:, 0], z[:, 2])[0, 1]) < 0.01
