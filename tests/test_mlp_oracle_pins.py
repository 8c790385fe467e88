"""Pins of the warm-start oracle: gradients against central finite
differences, Adam against its closed-form first step, GELU against its
definition by quadrature, and the features against invariances and the
diatomic closed form."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import mlp as M
from oracle import newton_dense as O
from paper_2503_13075_amd import synth as S
from tests import pins as P


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = M.init_params(1) + rng.normal(0, 0.05, M.N_PARAMS)   # non-zero output layer
    x = rng.normal(size=(7, M.N_FEAT))
    y = rng.normal(size=7)
    loss, g = M.loss_and_grad(p, x, y)
    idx = rng.choice(M.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [M.N_PARAMS - 1, M.N_PARAMS - 2, 0, M.N_FEAT * M.N_HID]])
    h = 1e-6
    for i in idx:
        dp = np.zeros(M.N_PARAMS)
        dp[i] = h
        fd = (M.loss_and_grad(p + dp, x, y)[0] - M.loss_and_grad(p - dp, x, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_gelu_is_x_times_normal_cdf():
    for xv in (-3.0, -0.7, 0.0, 0.4, 2.5):
        phi = quad(lambda t: math.exp(-t * t / 2) / math.sqrt(2 * math.pi), -np.inf, xv)[0]
        assert abs(M.gelu(np.array([xv]))[0] - xv * phi) < 1e-12
        fd = (M.gelu(np.array([xv + 1e-6]))[0] - M.gelu(np.array([xv - 1e-6]))[0]) / 2e-6
        assert abs(M.gelu_grad(np.array([xv]))[0] - fd) < 1e-8


def test_adam_first_step_is_sign_times_lr():
    rng = np.random.default_rng(2)
    p = rng.normal(size=10)
    g = rng.normal(size=10)
    p1, m, v = M.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-15)


def test_untrained_network_returns_decoupled_solution():
    rng = np.random.default_rng(3)
    pts = np.array([[0.0, 0, 0], [0.11, 0, 0]])
    ru = pts + rng.normal(0, 0.005, pts.shape)
    m = np.array([1.008, 12.011])
    f, w = M.features([[0, 1]], [0.11], m, pts, ru)
    lam = M.predict_lambda(M.init_params(0), np.zeros(16), np.ones(16), 0.1, f, w)
    ref = P.diatomic_lambda(pts[0], pts[1], ru[0], ru[1], m[0], m[1], 0.11)
    assert abs(lam[0] - ref) <= 1e-12 * abs(ref)
    # a decoupled constraint's exact multiplier is the same root
    out = O.solve([[0, 1]], [0.11], m, pts, ru, tol=1e-15, until_stagnation=True)
    assert abs(out["lam"][0] - lam[0]) <= 1e-12 * abs(ref)


def test_untrained_network_without_a_root_takes_one_newton_step():
    """Where the decoupled quadratic has no usable root (u.e <= 0: the
    unconstrained bond turned away from the old one), the untrained network
    returns the decoupled start's fallback, the first Newton step from
    lambda = 0 of the constraint alone: the oracle's Newton solve of the
    diatomic stopped after one iteration."""
    pts = np.array([[0.0, 0, 0], [0.11, 0, 0]])
    m = np.array([1.008, 12.011])
    for ru in (np.array([[0.0, 0, 0], [-0.02, 0.105, 0.0]]),     # u.e < 0, real root
               np.array([[0.0, 0, 0], [-0.05, 0.01, 0.0]])):     # u.e < 0, no real root
        f, w = M.features([[0, 1]], [0.11], m, pts, ru)
        lam = M.predict_lambda(M.init_params(0), np.zeros(16), np.ones(16), 0.1, f, w)
        one = O.solve([[0, 1]], [0.11], m, pts, ru, tol=1e-300, max_iter=1)
        assert one["iters"][0] == 1
        assert abs(lam[0] - one["lam"][0]) <= 1e-12 * abs(one["lam"][0])


def test_features_invariances():
    rng = np.random.default_rng(4)
    sm = S.add_h_angles(S.protein(6, seed=3))
    ru = S.perturb(sm.r, 0.006, 5)
    f, w = M.features(sm.pairs, sm.d, sm.mass, sm.r, ru)
    Q = P.random_rotation(rng)
    f2, _ = M.features(sm.pairs, sm.d, sm.mass, sm.r @ Q.T + 1.3, ru @ Q.T + 1.3)
    assert np.allclose(f, f2, rtol=1e-9, atol=1e-12)
    f3, w3 = M.features(sm.pairs, sm.d, 2.5 * sm.mass, sm.r, ru)
    assert np.allclose(f, f3, rtol=1e-12, atol=1e-14) and np.allclose(w3, w / 2.5)
    # reversing a constraint's orientation changes nothing
    pr = sm.pairs.copy()
    pr[::3] = pr[::3, ::-1]
    f4, _ = M.features(pr, sm.d, sm.mass, sm.r, ru)
    assert np.allclose(f, f4, rtol=1e-12, atol=1e-14)
    assert np.all(np.isfinite(f)) and f.shape == (sm.n_constraints, 16)


@pytest.mark.parametrize("seed", [0, 1])
def test_neighbour_ratio_is_newton_matrix_ratio(seed):
    """rho_kj in the features is A_kj(r, r) / A_kk(r, r) (Eq. defA): f8 is
    the row sum of |A_kj| / A_kk over the off-diagonal entries."""
    sm = S.random_tree(30, seed=seed)
    ru = S.perturb(sm.r, 0.002, 1)
    f, _ = M.features(sm.pairs, sm.d, sm.mass, sm.r, ru)
    A = O.newton_matrix(sm.r, sm.r, sm.pairs, 1.0 / sm.mass)
    off = np.abs(A - np.diag(np.diag(A))).sum(1) / np.diag(A)
    assert np.allclose(f[:, 8], off, rtol=1e-12, atol=1e-15)


# --------------------------------------------------------------------------- forward pass

def _gelu_by_quadrature(x):
    """x Phi(x) with Phi integrated numerically (independent of the oracle's
    erf-based GELU)."""
    return x * quad(lambda t: math.exp(-t * t / 2) / math.sqrt(2 * math.pi), -np.inf, x)[0]


def _routing_network():
    """A network with a handful of non-zero weights placed by the documented
    flat layout (W1 [16, 64] row-major, b1 [64], W2 [64, 64] row-major, b2,
    W3 [64], b3), so that each output is a known composition of GELUs:
      h1_0 = G(1.5 x_2),  h1_1 = G(0.3 - x_7)
      h2_4 = G(h1_0 + 2 h1_1 - 0.1),  h2_9 = G(h1_1)
      out  = 3 h2_4 - 0.5 h2_9 + 0.25
    (every other hidden unit is G(0) = 0)."""
    F, H = M.N_FEAT, M.N_HID
    o_b1 = F * H
    o_W2 = o_b1 + H
    o_b2 = o_W2 + H * H
    o_W3 = o_b2 + H
    o_b3 = o_W3 + H
    p = np.zeros(M.N_PARAMS)
    p[2 * H + 0] = 1.5
    p[7 * H + 1] = -1.0
    p[o_b1 + 1] = 0.3
    p[o_W2 + 0 * H + 4] = 1.0
    p[o_W2 + 1 * H + 4] = 2.0
    p[o_b2 + 4] = -0.1
    p[o_W2 + 1 * H + 9] = 1.0
    p[o_W3 + 4] = 3.0
    p[o_W3 + 9] = -0.5
    p[o_b3] = 0.25
    assert o_b3 + 1 == M.N_PARAMS
    return p


def _routing_expected(x):
    G = _gelu_by_quadrature
    out = []
    for row in x:
        h0, h1 = G(1.5 * row[2]), G(0.3 - row[7])
        out.append(3.0 * G(h0 + 2.0 * h1 - 0.1) - 0.5 * G(h1) + 0.25)
    return np.array(out)


def test_forward_pass_of_a_routing_network():
    """The forward pass against a hand-built network evaluated with a
    quadrature GELU.  Transposed weight matrices, a dropped bias or a
    missing activation route or shift the output and fail."""
    rng = np.random.default_rng(8)
    x = rng.normal(0, 1.5, size=(9, M.N_FEAT))
    p = _routing_network()
    got = M.forward(p, x)
    exp = _routing_expected(x)
    assert np.allclose(got, exp, rtol=1e-12, atol=1e-13), np.abs(got - exp).max()
    # inputs the network does not read leave the output unchanged
    x2 = x.copy()
    x2[:, [0, 1, 3, 4, 5, 6, 8, 15]] += 3.0
    assert np.array_equal(M.forward(p, x2), got)
    # the training path's own forward pass: its loss at y = 0 is mean(out^2) / 2
    loss, _ = M.loss_and_grad(p, x, np.zeros(x.shape[0]))
    assert abs(loss - 0.5 * np.mean(exp ** 2)) <= 1e-12 * loss


def test_predict_lambda_composition():
    """lambda_0 = (t0 + scale * MLP((f - mean) / std)) / w with the routing
    network: normalisation, scale, the decoupled base term f_0 and the
    division by w each enter as stated."""
    rng = np.random.default_rng(9)
    f = rng.normal(0, 1.0, size=(6, M.N_FEAT))
    mean = rng.normal(0, 0.3, M.N_FEAT)
    std = rng.uniform(0.5, 2.0, M.N_FEAT)
    w = rng.uniform(0.05, 1.0, 6)
    scale = 0.037
    lam = M.predict_lambda(_routing_network(), mean, std, scale, f, w)
    exp = (f[:, 0] + scale * _routing_expected((f - mean) / std)) / w
    assert np.allclose(lam, exp, rtol=1e-12, atol=1e-14), np.abs(lam - exp).max()
