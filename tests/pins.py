"""Independent references that pin the oracle (no code shared with it).

* closed forms for a diatomic and for a mirror-symmetric triatomic;
* SHAKE (nonlinear Gauss-Seidel, Supplement section 2.3) run to stagnation in
  extended precision;
* a 50-digit multidimensional root find (mpmath, numerical Jacobian) of
  g(r'(lambda)) = 0 started from lambda = 0.

Convention: g_k = 1/2 (|x_a - x_b|^2 - d_k^2), r' = r_u - M^{-1} G(r)^T lambda.
"""
from __future__ import annotations

import math

import numpy as np


def diatomic_lambda(r_a, r_b, u_a, u_b, m_a, m_b, d):
    """Root of |u - lambda w e|^2 = d^2 reached from lambda = 0.

    e = r_a - r_b, u = u_a - u_b, w = 1/m_a + 1/m_b.  The quadratic
    w^2 |e|^2 l^2 - 2 w (u.e) l + (|u|^2 - d^2) = 0 has the small root
    c / (w (b + sqrt(b^2 - |e|^2 c))) with b = u.e, c = |u|^2 - d^2
    (written without cancellation).
    """
    e = np.asarray(r_a, float) - np.asarray(r_b, float)
    u = np.asarray(u_a, float) - np.asarray(u_b, float)
    w = 1.0 / m_a + 1.0 / m_b
    b = float(u @ e)
    c = float(u @ u) - d * d
    return c / (w * (b + math.sqrt(b * b - float(e @ e) * c)))


def symmetric_triatomic_lambda(r1, r2, r3, u1, u2, m1, m2, d):
    """Mirror-symmetric 1-2-3 with constraints (1,2) and (3,2), m1 = m3.

    By symmetry both multipliers equal lambda; with e1 = r1 - r2,
    e2 = r3 - r2 and p = (1/m1 + 1/m2) e1 + (1/m2) e2 the bond vector becomes
    u1 - lambda p, so |u1 - lambda p|^2 = d^2 with u1 the unconstrained
    1-2 vector.  Small root: c / (b + sqrt(b^2 - a c)).
    """
    e1 = np.asarray(r1, float) - np.asarray(r2, float)
    e2 = np.asarray(r3, float) - np.asarray(r2, float)
    u = np.asarray(u1, float) - np.asarray(u2, float)
    p = (1.0 / m1 + 1.0 / m2) * e1 + (1.0 / m2) * e2
    a = float(p @ p)
    b = float(u @ p)
    c = float(u @ u) - d * d
    return c / (b + math.sqrt(b * b - a * c))


def shake_extended(pairs, d, mass, r, r_u, max_sweeps=200000, tol=None):
    """SHAKE in numpy.longdouble: sweep the constraints in order, correcting
    each one along its old bond vector with a one-dimensional Newton step,
    until the maximum relative violation stops decreasing.

    Returns (r' as float64, lambda as float64, sweeps).
    """
    ld = np.longdouble
    pairs = np.asarray(pairs, np.int64)
    x = np.asarray(r_u, ld).copy()
    rr = np.asarray(r, ld)
    inv = ld(1) / np.asarray(mass, ld)
    dd = np.asarray(d, ld) ** 2
    e = rr[pairs[:, 0]] - rr[pairs[:, 1]]
    lam = np.zeros(len(pairs), ld)
    best = None
    prev = None
    stall = 0
    eps = np.finfo(ld).eps
    if tol is None:
        tol = 4 * eps
    for sweep in range(max_sweeps):
        for k in range(len(pairs)):
            a, b = pairs[k]
            ek = e[k]
            v = x[a] - x[b]
            g = (v @ v - dd[k]) / 2
            w = inv[a] + inv[b]
            delta = g / (w * (v @ ek))
            lam[k] += delta
            x[a] -= inv[a] * delta * ek
            x[b] += inv[b] * delta * ek
        v = x[pairs[:, 0]] - x[pairs[:, 1]]
        rho = np.max(np.abs((np.einsum("ij,ij->i", v, v) - dd) / 2 / dd))
        if best is None or rho < best[0]:
            best = (rho, x.copy(), lam.copy())
        if rho <= tol:
            break
        if prev is not None and rho >= prev:
            stall += 1
            if stall > 20:
                break
        else:
            stall = 0
        prev = rho
    return np.asarray(best[1], np.float64), np.asarray(best[2], np.float64), sweep + 1


def mp_root(pairs, d, mass, r, r_u, dps=50):
    """50-digit root of F(lambda) = g(r'(lambda)) from lambda = 0 with
    mpmath's multidimensional Newton (numerical Jacobian).  Small systems
    only."""
    import mpmath as mp

    mp.mp.dps = dps
    pairs = [tuple(int(v) for v in p) for p in pairs]
    R = [[mp.mpf(float(v)) for v in row] for row in np.asarray(r)]
    U = [[mp.mpf(float(v)) for v in row] for row in np.asarray(r_u)]
    inv = [1 / mp.mpf(float(m)) for m in mass]
    D2 = [mp.mpf(float(v)) ** 2 for v in d]
    E = [[R[a][c] - R[b][c] for c in range(3)] for a, b in pairs]

    def F(*lam):
        X = [row[:] for row in U]
        for k, (a, b) in enumerate(pairs):
            for c in range(3):
                X[a][c] -= inv[a] * lam[k] * E[k][c]
                X[b][c] += inv[b] * lam[k] * E[k][c]
        out = []
        for k, (a, b) in enumerate(pairs):
            v = [X[a][c] - X[b][c] for c in range(3)]
            out.append((v[0] ** 2 + v[1] ** 2 + v[2] ** 2 - D2[k]) / 2)
        return out

    x0 = [mp.mpf(0)] * len(pairs)
    root = mp.findroot(F, x0, tol=mp.mpf(10) ** (-2 * dps + 10), maxsteps=100)
    if len(pairs) == 1:
        root = [root]
    lam = np.array([float(root[k]) for k in range(len(pairs))])
    X = [row[:] for row in U]
    for k, (a, b) in enumerate(pairs):
        for c in range(3):
            X[a][c] -= inv[a] * root[k] * E[k][c]
            X[b][c] += inv[b] * root[k] * E[k][c]
    return lam, np.array([[float(v) for v in row] for row in X])


def finite_difference_jacobian(F, lam, h=1e-6):
    """Central differences of a vector function F at lam."""
    n = lam.size
    J = np.zeros((n, n))
    for j in range(n):
        dl = np.zeros(n)
        dl[j] = h
        J[:, j] = (F(lam + dl) - F(lam - dl)) / (2 * h)
    return J


def random_rotation(rng):
    q, rmat = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(rmat))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q
