"""Pins of the CPU oracle against facts that do not come from the oracle.

Closed forms (diatomic, symmetric triatomic), SHAKE to stagnation in
extended precision, a 50-digit root find, finite-difference Jacobians,
conservation of linear and angular momentum, symmetries, matrix structure
(Eq. defA and Supplement section 3), and Newton's quadratic convergence.
A last group plants mistakes in the oracle and checks that a pin fails.
"""
import numpy as np
import pytest

from oracle import newton_dense as O
from paper_2503_13075_amd import synth as S
from tests import pins as P


def _solve(sysm, r_u, **kw):
    kw.setdefault("tol", 1e-15)
    kw.setdefault("until_stagnation", True)
    kw.setdefault("max_iter", 50)
    return O.solve(sysm.pairs, sysm.d, sysm.mass, sysm.r, r_u, **kw)


def _diatomic(rng, sigma=0.01):
    m = rng.uniform(1.0, 32.0, size=2)
    d = rng.uniform(0.1, 0.153)
    e = P.random_rotation(rng)[:, 0] * d
    r = np.array([[0.3, -0.2, 0.1], [0.3, -0.2, 0.1]]) + np.array([e / 2, -e / 2])
    ru = r + rng.normal(0, sigma, size=r.shape)
    return r, ru, m, d


# --------------------------------------------------------------------------- closed forms

def diatomic_pin_error(solver=None):
    """Largest relative lambda error and position error of the oracle on 50
    random diatomics against the closed form."""
    rng = np.random.default_rng(11)
    worst_l, worst_r = 0.0, 0.0
    for _ in range(50):
        r, ru, m, d = _diatomic(rng)
        out = O.solve([[0, 1]], [d], m, r, ru, tol=1e-15, until_stagnation=True, max_iter=50)
        lam = P.diatomic_lambda(r[0], r[1], ru[0], ru[1], m[0], m[1], d)
        e = r[0] - r[1]
        rp = ru.copy()
        rp[0] -= lam / m[0] * e
        rp[1] += lam / m[1] * e
        worst_l = max(worst_l, abs(out["lam"][0] - lam) / abs(lam))
        worst_r = max(worst_r, float(np.max(np.abs(out["r_new"] - rp))))
    return worst_l, worst_r


def test_diatomic_closed_form():
    el, er = diatomic_pin_error()
    assert el < 1e-12 and er < 1e-15, (el, er)


def _sym_triatomic(rng):
    m1, m2 = rng.uniform(1.0, 16.0), rng.uniform(1.0, 16.0)
    d = 0.12
    half = np.radians(rng.uniform(50, 60))
    # atom 2 at the origin, mirror plane x = 0 swaps atoms 1 and 3
    r2 = np.array([0.0, 0.0, 0.0])
    r1 = np.array([-d * np.sin(half), d * np.cos(half), 0.0])
    r3 = np.array([d * np.sin(half), d * np.cos(half), 0.0])
    n1 = rng.normal(0, 0.004, 3)
    n2 = rng.normal(0, 0.004, 3)
    n2[0] = 0.0                          # atom 2 stays on the mirror plane
    mirror = np.array([-1.0, 1.0, 1.0])
    ru = np.array([r1 + n1, r2 + n2, r3 + n1 * mirror])
    return np.array([r1, r2, r3]), ru, np.array([m1, m2, m1]), d


def test_symmetric_triatomic_closed_form():
    rng = np.random.default_rng(5)
    for _ in range(20):
        r, ru, m, d = _sym_triatomic(rng)
        out = O.solve([[0, 1], [2, 1]], [d, d], m, r, ru, tol=1e-15, until_stagnation=True)
        lam = P.symmetric_triatomic_lambda(r[0], r[1], r[2], ru[0], ru[1], m[0], m[1], d)
        assert np.allclose(out["lam"], lam, rtol=1e-11, atol=0), (out["lam"], lam)


# --------------------------------------------------------------------------- brute force

def _tiny_molecules():
    rng = np.random.default_rng(3)
    # triangle: two bonds and the 1-3 distance
    ch = S.united_chain(3, seed=4, angles=True)
    yield "triangle", ch, S.perturb(ch.r, 0.005, 1)
    # four-atom chain with both 1-3 distances (5 constraints)
    ch4 = S.united_chain(4, seed=5, angles=True)
    yield "chain4", ch4, S.perturb(ch4.r, 0.005, 2)
    # methyl-like star: C bonded to 3 H and 1 C (4 constraints) plus 2 H-C-H (6)
    b = S._Builder(S._Rand(9))
    c0 = b.root("C")
    for _ in range(3):
        b.child(c0, "H")
    c1 = b.child(c0, "C")
    b.hydrogens(c1, 1)
    star = b.to_system("star")
    star = S.add_h_angles(star)
    keep = min(6, star.n_constraints)
    star = S.System(pairs=star.pairs[:keep], d=star.d[:keep], mass=star.mass, r=star.r,
                    kind=star.kind[:keep], elem=star.elem)
    yield "star", star, S.perturb(star.r, 0.004, 3)
    del rng


@pytest.mark.parametrize("case", list(range(3)))
def test_mpmath_root(case):
    name, sysm, ru = list(_tiny_molecules())[case]
    out = _solve(sysm, ru)
    lam, rp = P.mp_root(sysm.pairs, sysm.d, sysm.mass, sysm.r, ru)
    assert np.allclose(out["lam"], lam, rtol=1e-12, atol=0), name
    assert np.max(np.abs(out["r_new"] - rp)) < 1e-15, name


@pytest.mark.slow
def test_shake_extended_chain64():
    c = S.chain64(0)
    ru = S.perturb(c.r, 0.002, 1)
    out = _solve(c, ru)
    rp, lam, sweeps = P.shake_extended(c.pairs, c.d, c.mass, c.r, ru, max_sweeps=20000)
    assert np.max(np.abs(out["r_new"] - rp)) < 1e-14
    assert np.max(np.abs(out["lam"] - lam) / np.max(np.abs(lam))) < 1e-11


def test_shake_extended_tree():
    t = S.random_tree(40, seed=7)
    ru = S.perturb(t.r, 0.002, 2)
    out = _solve(t, ru)
    rp, lam, sweeps = P.shake_extended(t.pairs, t.d, t.mass, t.r, ru, max_sweeps=5000)
    assert np.max(np.abs(out["r_new"] - rp)) < 1e-14
    assert np.max(np.abs(out["lam"] - lam) / np.max(np.abs(lam))) < 1e-11


# --------------------------------------------------------------------------- Jacobian

def jacobian_pin_error(sysm, ru, seed=0):
    """Relative difference between A(r'(lambda), r) and minus the
    finite-difference Jacobian of lambda -> g(r'(lambda)) (Eq. defA)."""
    rng = np.random.default_rng(seed)
    inv = 1.0 / sysm.mass
    lam = rng.normal(0, 0.01, sysm.n_constraints)

    def F(l):
        return O.constraint_values(O.position_map(sysm.r, ru, sysm.pairs, inv, l), sysm.pairs, sysm.d)

    J = P.finite_difference_jacobian(F, lam, h=1e-5)
    A = O.newton_matrix(O.position_map(sysm.r, ru, sysm.pairs, inv, lam), sysm.r, sysm.pairs, inv)
    return float(np.max(np.abs(A + J)) / np.max(np.abs(A)))


def test_newton_matrix_is_the_jacobian():
    c = S.united_chain(10, seed=2, angles=True)
    ru = S.perturb(c.r, 0.01, 3)
    assert jacobian_pin_error(c, ru) < 1e-8


def test_structure_line_graph_and_symmetry():
    t = S.add_h_angles(S.random_tree(60, seed=3))
    ru = S.perturb(t.r, 0.01, 4)
    inv = 1.0 / t.mass
    A = O.newton_matrix(ru, t.r, t.pairs, inv)
    n = t.n_constraints
    share = np.zeros((n, n), bool)
    for i in range(n):
        for j in range(n):
            share[i, j] = len(set(t.pairs[i]) & set(t.pairs[j])) > 0
    assert np.array_equal(np.abs(A) > 0, share)
    Ars = O.newton_matrix(t.r, t.r, t.pairs, inv)
    assert np.allclose(Ars, Ars.T, rtol=0, atol=1e-15)
    assert not np.allclose(A, A.T, rtol=0, atol=1e-9)


# --------------------------------------------------------------------------- invariants

@pytest.mark.parametrize("maker", [lambda: S.chain64(0), lambda: S.random_tree(200, seed=8),
                                   lambda: S.add_h_angles(S.protein(8, seed=2))])
def test_momentum_conservation(maker):
    sysm = maker()
    ru = S.perturb(sysm.r, 0.004, 9)
    out = _solve(sysm, ru)
    dr = out["r_new"] - ru
    m = sysm.mass[:, None]
    lin = np.sum(m * dr, axis=0)
    ang = np.sum(np.cross(sysm.r, m * dr), axis=0)
    scale = np.sum(np.abs(m * dr))
    assert np.max(np.abs(lin)) < 1e-14 * max(1.0, scale)
    assert np.max(np.abs(ang)) < 1e-13 * max(1.0, scale)


def test_symmetries():
    rng = np.random.default_rng(21)
    t = S.random_tree(80, seed=12)
    ru = S.perturb(t.r, 0.003, 13)
    base = _solve(t, ru)
    # common rotation
    Q = P.random_rotation(rng)
    rot = O.solve(t.pairs, t.d, t.mass, t.r @ Q.T, ru @ Q.T, tol=1e-15, until_stagnation=True)
    assert np.allclose(rot["lam"], base["lam"], rtol=1e-10, atol=1e-14)
    assert np.allclose(rot["r_new"], base["r_new"] @ Q.T, rtol=0, atol=1e-13)
    # independent translations of r and r_u
    tr = O.solve(t.pairs, t.d, t.mass, t.r + 1.7, ru - 0.9, tol=1e-15, until_stagnation=True)
    assert np.allclose(tr["lam"], base["lam"], rtol=1e-9, atol=1e-13)
    assert np.allclose(tr["r_new"], base["r_new"] - 0.9, rtol=0, atol=1e-12)
    # mass scaling: lambda scales, positions do not move
    ms = O.solve(t.pairs, t.d, 3.0 * t.mass, t.r, ru, tol=1e-15, until_stagnation=True)
    assert np.allclose(ms["lam"], 3.0 * base["lam"], rtol=1e-10, atol=1e-14)
    assert np.allclose(ms["r_new"], base["r_new"], rtol=0, atol=1e-14)
    # relabel atoms and constraints, reverse some constraint orientations
    pa = rng.permutation(t.n_atoms)
    inv_pa = np.argsort(pa)
    pc = rng.permutation(t.n_constraints)
    pairs = inv_pa[t.pairs[pc]]
    flip = rng.random(len(pc)) < 0.5
    pairs[flip] = pairs[flip][:, ::-1]
    rl = O.solve(pairs, t.d[pc], t.mass[pa], t.r[pa], ru[pa], tol=1e-15, until_stagnation=True)
    assert np.allclose(rl["lam"], base["lam"][pc], rtol=1e-10, atol=1e-14)
    assert np.allclose(rl["r_new"], base["r_new"][pa], rtol=0, atol=1e-14)


# --------------------------------------------------------------------------- convergence

def test_newton_quadratic_and_chord_linear():
    c = S.chain64(0)
    ru = S.perturb(c.r, 0.002, 1)
    h = _solve(c, ru, tol=1e-12, until_stagnation=False)["history"][0]
    # quadratic: log rho_{l+1} / log rho_l approaches 2 (above roundoff)
    ratios = [np.log(h[i + 1]) / np.log(h[i]) for i in range(1, len(h) - 1) if h[i + 1] > 1e-14]
    assert ratios and ratios[-1] > 1.7, h
    hc = _solve(c, ru, tol=1e-12, until_stagnation=False, variant="chord", max_iter=60)["history"][0]
    q = [hc[i + 1] / hc[i] for i in range(2, len(hc) - 1)]
    assert max(q) < 0.2 and min(q) > 1e-4, hc        # linear rate, not quadratic
    assert len(hc) > len(h)


def test_already_converged_takes_zero_iterations():
    c = S.chain64(0)
    out = O.solve(c.pairs, c.d, c.mass, c.r, c.r.copy(), tol=1e-12)
    assert out["iters"][0] == 0 and out["status"][0] == O.OK


def test_iteration_cap_reports_not_converged():
    c = S.chain64(0)
    out = O.solve(c.pairs, c.d, c.mass, c.r, S.perturb(c.r, 0.002, 1), tol=1e-12, max_iter=1)
    assert out["status"][0] == O.NOT_CONVERGED and out["iters"][0] == 1


def test_decoupled_constraints_are_independent():
    """H-bond-only benzene-like case: constraints share no atom, A is
    diagonal, and every constraint obeys the diatomic closed form."""
    rng = np.random.default_rng(4)
    rs, rus, ms, ds = [], [], [], []
    for _ in range(6):
        r, ru, m, d = _diatomic(rng, sigma=0.005)
        rs.append(r + rng.normal(0, 1, 3))
        rus.append(ru + (rs[-1] - r))
        ms.append(m)
        ds.append(d)
    r = np.concatenate(rs)
    ru = np.concatenate(rus)
    m = np.concatenate(ms)
    pairs = np.arange(12).reshape(6, 2)
    A = O.newton_matrix(ru, r, pairs, 1.0 / m)
    assert np.count_nonzero(A - np.diag(np.diag(A))) == 0
    out = O.solve(pairs, ds, m, r, ru, tol=1e-15, until_stagnation=True)
    assert len(out["molecules"]) == 6
    for k in range(6):
        lam = P.diatomic_lambda(r[2 * k], r[2 * k + 1], ru[2 * k], ru[2 * k + 1], m[2 * k], m[2 * k + 1], ds[k])
        assert abs(out["lam"][k] - lam) <= 1e-12 * abs(lam)


# --------------------------------------------------------------------------- planted mistakes

def test_planted_mistakes_are_caught(monkeypatch):
    """Each plausible mistake planted in the oracle makes a pin fail."""
    good_pm = O.position_map
    good_nm = O.newton_matrix
    c = S.united_chain(10, seed=2, angles=True)
    ru = S.perturb(c.r, 0.01, 3)

    # 1. position map built on G(r_u) instead of G(r)
    monkeypatch.setattr(O, "position_map", lambda r, r_u, pairs, inv, lam: good_pm(r_u, r_u, pairs, inv, lam))
    assert diatomic_pin_error()[0] > 1e-6
    monkeypatch.setattr(O, "position_map", good_pm)

    # 2. Newton matrix with transposed operands, A(r, r') instead of A(r', r)
    monkeypatch.setattr(O, "newton_matrix", lambda x, y, p, inv: good_nm(y, x, p, inv))
    assert jacobian_pin_error(c, ru) > 1e-4
    # 3. Newton matrix without the off-diagonal couplings
    monkeypatch.setattr(O, "newton_matrix", lambda x, y, p, inv: np.diag(np.diag(good_nm(x, y, p, inv))))
    assert jacobian_pin_error(c, ru) > 1e-2
    # 4. wrong inverse-mass factor (mass instead of 1/mass) on one side
    monkeypatch.setattr(O, "newton_matrix", lambda x, y, p, inv: good_nm(x, y, p, 1.0 / inv))
    assert jacobian_pin_error(c, ru) > 1e-2
    monkeypatch.setattr(O, "newton_matrix", good_nm)

    # 5. dropped factor 1/2 in g: the triatomic closed form no longer holds
    good_cv = O.constraint_values
    monkeypatch.setattr(O, "constraint_values", lambda x, p, d: 2.0 * good_cv(x, p, d))
    rng = np.random.default_rng(5)
    r, ru3, m, d = _sym_triatomic(rng)
    out = O.solve([[0, 1], [2, 1]], [d, d], m, r, ru3, tol=1e-15, until_stagnation=True, max_iter=8)
    lam = P.symmetric_triatomic_lambda(r[0], r[1], r[2], ru3[0], ru3[1], m[0], m[1], d)
    assert np.max(np.abs(out["lam"] - lam)) > 1e-6 * abs(lam)


# --------------------------------------------------------------------------- the violation measure

# Two atoms a distance L apart under a constraint of length d: the constraint
# value is (L^2 - d^2) / 2 and the relative violation that the stopping rule
# bounds (Supplement section 4, read with an absolute value) is
# |L^2 - d^2| / (2 d^2).  Values worked out by hand:
#   (L, d, g, relative violation)
VIOLATION_CASES = [
    (2.0, 1.0, 1.5, 1.5),
    (0.5, 1.0, -0.375, 0.375),
    (0.11, 0.1, 0.00105, 0.105),
    (0.09, 0.1, -0.00095, 0.095),
    (0.0, 0.25, -0.03125, 0.5),
    (0.153, 0.153, 0.0, 0.0),
]


def violation_pin_error():
    """Largest deviation of the oracle's constraint values and relative
    violations from the hand-computed cases.  Each pair sits at an arbitrary
    centre and orientation; all pairs are in one system so that the output
    order is checked too."""
    rng = np.random.default_rng(21)
    k = len(VIOLATION_CASES)
    x = np.zeros((2 * k, 3))
    pairs = np.zeros((k, 2), np.int64)
    d = np.zeros(k)
    for i, (L, dd, _, _) in enumerate(VIOLATION_CASES):
        c = rng.uniform(-5, 5, 3)
        u = P.random_rotation(rng)[:, 0]
        x[2 * i], x[2 * i + 1] = c + 0.5 * L * u, c - 0.5 * L * u
        pairs[i] = (2 * i + 1, 2 * i) if i % 2 else (2 * i, 2 * i + 1)
        d[i] = dd
    g = O.constraint_values(x, pairs, d)
    rel = O.relative_violation(x, pairs, d)
    err = 0.0
    for i, (L, dd, gv, rv) in enumerate(VIOLATION_CASES):
        err = max(err, abs(g[i] - gv) / max(abs(gv), dd * dd), abs(rel[i] - rv) / max(rv, 1.0))
    return err


def test_relative_violation_hand_computed():
    assert violation_pin_error() <= 1e-12


def test_planted_violation_mistakes_are_caught(monkeypatch):
    """Dividing by d instead of d^2 (0.0105 instead of 0.105), dropping the
    factor 1/2 (0.21) or the absolute value (-0.375) fails the pin."""
    good_cv = O.constraint_values
    for bad in (lambda x, p, d: np.abs(good_cv(x, p, d)) / d,
                lambda x, p, d: 2.0 * np.abs(good_cv(x, p, d)) / (d * d),
                lambda x, p, d: good_cv(x, p, d) / (d * d)):
        monkeypatch.setattr(O, "relative_violation", bad)
        assert violation_pin_error() > 1e-3


def test_relative_violation_of_a_stretched_chain():
    """Every bond of a straight 5-atom chain stretched by 1%: each bond's
    relative violation is (1.01^2 - 1) / 2 = 0.01005; the 1-3 distance of a
    straight chain is exactly twice the bond, so a 1-3 constraint of length
    2 d also reads 0.01005."""
    d = 0.153
    x = np.zeros((5, 3))
    x[:, 0] = np.arange(5) * 1.01 * d
    pairs = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [0, 2]])
    dd = np.array([d, d, d, d, 2 * d])
    rel = O.relative_violation(x, pairs, dd)
    assert np.allclose(rel, 0.01005, rtol=1e-12, atol=0.0), rel
