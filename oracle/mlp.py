"""CPU oracle for the learned warm start (test infrastructure only).

Plain FP64 NumPy reference of the per-constraint features, the multilayer
perceptron [16 -> 64 -> 64 -> 1] with exact GELU, its mean-squared-error
gradient and one Adam step.  Only the tests, the smoke entry point and the
benchmark's CPU-baseline leg may use it.  It shares no code with the GPU
path.

The warm start predicts the initial multipliers lambda_0 of the Newton
iteration (whose own starting point is lambda_0 = 0, Supplement section
2.3).  With w_k = 1/m_a + 1/m_b the network works on the dimensionless
quantity t_k = lambda_k w_k, and predicts it as a correction of the
decoupled (diatomic) solution t0_k:  t_k = t0_k + scale * MLP(norm(f_k)).

Features (all invariant under rotations and translations of r and r_u and
under a common scaling of the masses, like lambda w itself):
  e = r_a - r_b, u = r_u,a - r_u,b, c = |u|^2 - d^2, b = u.e
  f0  t0 = c / (b + sqrt(b^2 - |e|^2 c))        decoupled solution
  f1  c / (2 d^2)                              initial relative violation
  f2  b / d^2 - 1
  f3  |u x e| / d^2
  f4  |1/m_a - 1/m_b| / w
  f5  (deg_a + deg_b - 2) / 4                  deg = constraints at the atom
  f6  |deg_a - deg_b| / 4
  over the constraints j sharing atom x with k, with
  rho_kj = s_kx s_jx (1/m_x) (e_k . e_j) / (w_k |e_k|^2)  and  q_kj = w_k / w_j:
  f7  sum rho q t0_j     f8  sum |rho|     f9  max |rho|     f10 sum rho q f1_j
  f11 sum rho^2          f12 mean s s cos(e_k, e_j)          f13 count / 6
  f14 sum rho q f2_j     f15 sum rho q f3_j
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_FEAT, N_HID = 16, 64
N_PARAMS = N_FEAT * N_HID + N_HID + N_HID * N_HID + N_HID + N_HID + 1


def features(pairs, d, mass, r, r_u):
    """Per-constraint features [n, 16] and w_k [n] (FP64)."""
    pairs = np.asarray(pairs, np.int64).reshape(-1, 2)
    n = pairs.shape[0]
    a, b = pairs[:, 0], pairs[:, 1]
    inv = 1.0 / np.asarray(mass, np.float64)
    e = r[a] - r[b]
    u = r_u[a] - r_u[b]
    d2 = np.asarray(d, np.float64) ** 2
    w = inv[a] + inv[b]
    ee = np.einsum("ij,ij->i", e, e)
    bb = np.einsum("ij,ij->i", u, e)
    c = np.einsum("ij,ij->i", u, u) - d2
    # t0 = w * (the decoupled start of constraint k): the root nearest 0 of
    # |u - t e|^2 = d^2 when u.e > 0 and a real root exists, else the Newton
    # step from t = 0, c / (2 u.e) (0 when u.e = 0)
    disc = bb * bb - ee * c
    root = (bb > 0) & (disc >= 0)
    safe_bb = np.where(bb != 0, bb, 1.0)
    t0 = np.where(root, c / np.where(root, bb + np.sqrt(np.maximum(disc, 0.0)), 1.0),
                  np.where(bb != 0, c / (2 * safe_bb), 0.0))
    f = np.zeros((n, N_FEAT))
    f[:, 0] = t0
    f[:, 1] = c / (2 * d2)
    f[:, 2] = bb / d2 - 1
    f[:, 3] = np.linalg.norm(np.cross(u, e), axis=1) / d2
    f[:, 4] = np.abs(inv[a] - inv[b]) / w
    deg = np.bincount(pairs.ravel(), minlength=len(mass))
    f[:, 5] = (deg[a] + deg[b] - 2) / 4.0
    f[:, 6] = np.abs(deg[a] - deg[b]) / 4.0
    # neighbour sums: constraints sharing an atom
    inc = [[] for _ in range(len(mass))]
    for k in range(n):
        inc[a[k]].append((k, 1.0))
        inc[b[k]].append((k, -1.0))
    nb_sum = np.zeros((n, 7))
    nb_max = np.zeros(n)
    nb_cnt = np.zeros(n)
    norm_e = np.sqrt(ee)
    for x in range(len(mass)):
        lst = inc[x]
        for k, sk in lst:
            for j, sj in lst:
                if j == k:
                    continue
                dot = e[k] @ e[j]
                rho = sk * sj * inv[x] * dot / (w[k] * ee[k])
                q = w[k] / w[j]
                nb_sum[k, 0] += rho * q * t0[j]
                nb_sum[k, 1] += abs(rho)
                nb_sum[k, 2] += rho * q * f[j, 1]
                nb_sum[k, 3] += rho * rho
                nb_sum[k, 4] += sk * sj * dot / (norm_e[k] * norm_e[j])
                nb_sum[k, 5] += rho * q * f[j, 2]
                nb_sum[k, 6] += rho * q * f[j, 3]
                nb_max[k] = max(nb_max[k], abs(rho))
                nb_cnt[k] += 1
    f[:, 7] = nb_sum[:, 0]
    f[:, 8] = nb_sum[:, 1]
    f[:, 9] = nb_max
    f[:, 10] = nb_sum[:, 2]
    f[:, 11] = nb_sum[:, 3]
    f[:, 12] = nb_sum[:, 4] / np.maximum(nb_cnt, 1.0)
    f[:, 13] = nb_cnt / 6.0
    f[:, 14] = nb_sum[:, 5]
    f[:, 15] = nb_sum[:, 6]
    return f, w


# --------------------------------------------------------------------------- network

def unpack(p):
    """Flat parameter vector -> (W1 [16,64], b1, W2 [64,64], b2, W3 [64], b3)."""
    p = np.asarray(p, np.float64)
    o = 0
    W1 = p[o:o + N_FEAT * N_HID].reshape(N_FEAT, N_HID); o += N_FEAT * N_HID
    b1 = p[o:o + N_HID]; o += N_HID
    W2 = p[o:o + N_HID * N_HID].reshape(N_HID, N_HID); o += N_HID * N_HID
    b2 = p[o:o + N_HID]; o += N_HID
    W3 = p[o:o + N_HID]; o += N_HID
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def gelu(x):
    """Exact GELU, x Phi(x)."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(p, x):
    """Network output for normalised inputs x [B, 16] -> [B]."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = gelu(x @ W1 + b1)
    h2 = gelu(h1 @ W2 + b2)
    return h2 @ W3 + b3[0]


def loss_and_grad(p, x, y):
    """L = 1/(2B) sum (out - y)^2 and dL/dp (flat, same layout as p)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    B = x.shape[0]
    z1 = x @ W1 + b1
    h1 = gelu(z1)
    z2 = h1 @ W2 + b2
    h2 = gelu(z2)
    out = h2 @ W3 + b3[0]
    r = out - y
    loss = 0.5 * np.mean(r * r)
    do = r / B
    gW3 = h2.T @ do
    gb3 = np.array([do.sum()])
    dz2 = np.outer(do, W3) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * gelu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
    return loss, g


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation (the output layer starts at zero so that the
    untrained network returns the decoupled solution)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, math.sqrt(2.0 / N_FEAT), (N_FEAT, N_HID))
    W2 = rng.normal(0, math.sqrt(2.0 / N_HID), (N_HID, N_HID))
    return np.concatenate([W1.ravel(), np.zeros(N_HID), W2.ravel(), np.zeros(N_HID), np.zeros(N_HID), np.zeros(1)])


def predict_lambda(p, mean, std, scale, f, w):
    """lambda_0 from features: (t0 + scale * MLP((f - mean) / std)) / w."""
    x = (f - mean) / std
    return (f[:, 0] + scale * forward(p, x)) / w
