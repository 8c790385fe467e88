"""CPU oracle for the per-timestep constraint solve (test infrastructure only).

Plain, slow, FP64 reference of what the solver computes.  Only the tests, the
smoke entry point and the benchmark's CPU-baseline leg may use it; the GPU
product path never calls it.  It shares no code with the GPU path.

Problem (Supplement section 2.3; written with the sign convention
g_k(x) = 1/2 (|x_a - x_b|^2 - d_k^2) and lambda scaled so that no time step
appears: lambda_here = -h^2 lambda_paper):

  r'(lambda) = r_u - M^{-1} G(r)^T lambda                (Eq. 6, phi_k)
  find lambda with g(r'(lambda)) = 0                    (Eq. nonlinear:1c)

Newton (Eqs. defA and newton-constraint-equation):
  A(x, y) = G(x) M^{-1} G(y)^T
  A(r'_l, r) z_l = g(r'_l),   lambda_{l+1} = lambda_l + z_l,   lambda_0 = 0

Chord / simplified Newton (Supplement section 3, ILVES-F): the same with the
constant matrix A(r, r).

Stopping rule (Supplement section 4): stop when every relative violation
|g_k| / d_k^2 is at most Tol, or at the iteration cap.

Each molecule (connected component of the constraint graph, Supplement
section 3) is an independent block and is solved on its own with a dense
LAPACK solve (partial pivoting).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

OK, NOT_CONVERGED, SINGULAR, NONFINITE = 0, 1, 2, 3


def molecules(n_atoms: int, pairs: np.ndarray):
    """Connected components of the constraint graph G (Supplement section 3).

    Returns a list of (atom indices, constraint indices), both sorted, one
    entry per component that has at least one constraint.
    """
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    n = pairs.shape[0]
    if n == 0:
        return []
    adj = sp.coo_matrix((np.ones(n), (pairs[:, 0], pairs[:, 1])), shape=(n_atoms, n_atoms))
    _, label = connected_components(adj, directed=False)
    con_label = label[pairs[:, 0]]
    out = []
    order = np.argsort(con_label, kind="stable")
    bounds = np.flatnonzero(np.diff(con_label[order])) + 1
    for cons in np.split(order, bounds):
        atoms = np.unique(pairs[cons].ravel())
        out.append((atoms, np.sort(cons)))
    return out


def constraint_values(x: np.ndarray, pairs: np.ndarray, d: np.ndarray) -> np.ndarray:
    """g_k(x) = 1/2 (|x_a - x_b|^2 - d_k^2)  (Eq. ecconstr, opposite sign)."""
    e = x[pairs[:, 0]] - x[pairs[:, 1]]
    return 0.5 * (np.einsum("ij,ij->i", e, e) - d * d)


def relative_violation(x: np.ndarray, pairs: np.ndarray, d: np.ndarray) -> np.ndarray:
    """|g_k(x)| / d_k^2, the quantity bounded by Tol (Supplement section 4)."""
    return np.abs(constraint_values(x, pairs, d)) / (d * d)


def jacobian(x: np.ndarray, pairs: np.ndarray, n_atoms: int) -> sp.csr_matrix:
    """G(x), the n x 3s Jacobian of g: row k holds +e_k on atom a_k and
    -e_k on atom b_k, e_k = x_a - x_b (Supplement section 2.2)."""
    n = pairs.shape[0]
    e = x[pairs[:, 0]] - x[pairs[:, 1]]
    rows = np.repeat(np.arange(n), 6)
    cols = np.concatenate([3 * pairs[:, [0]] + np.arange(3), 3 * pairs[:, [1]] + np.arange(3)], axis=1).ravel()
    vals = np.concatenate([e, -e], axis=1).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, 3 * n_atoms))


def position_map(r: np.ndarray, r_u: np.ndarray, pairs: np.ndarray, inv_mass: np.ndarray,
                 lam: np.ndarray) -> np.ndarray:
    """r'(lambda) = r_u - M^{-1} G(r)^T lambda  (Eq. 6)."""
    s = r.shape[0]
    G = jacobian(r, pairs, s)
    minv = np.repeat(inv_mass, 3)
    return r_u - (minv * (G.T @ lam)).reshape(s, 3)


def newton_matrix(x: np.ndarray, y: np.ndarray, pairs: np.ndarray, inv_mass: np.ndarray) -> np.ndarray:
    """Dense A(x, y) = G(x) M^{-1} G(y)^T  (Eq. defA without the -h^2)."""
    s = x.shape[0]
    Gx = jacobian(x, pairs, s)
    Gy = jacobian(y, pairs, s)
    Minv = sp.diags(np.repeat(inv_mass, 3))
    return (Gx @ Minv @ Gy.T).toarray()


def solve_molecule(r, r_u, pairs, d, inv_mass, tol, max_iter, lam0=None, variant="newton",
                   until_stagnation=False):
    """Newton (or chord) iteration on one molecule; all arrays local to it.

    Returns (r', lambda, iterations, status, history of max relative
    violation).  ``iterations`` counts linear solves.  With
    ``until_stagnation`` the iteration continues past ``tol`` while the
    maximum violation keeps decreasing and returns the best iterate.
    """
    n = pairs.shape[0]
    lam = np.zeros(n) if lam0 is None else np.array(lam0, dtype=np.float64)
    A_fixed = newton_matrix(r, r, pairs, inv_mass) if variant == "chord" else None
    hist = []
    best = None                      # (r', lambda, iterations, rho) with the smallest rho
    it = 0
    status = NOT_CONVERGED
    while True:
        rp = position_map(r, r_u, pairs, inv_mass, lam)
        g = constraint_values(rp, pairs, d)
        rho = float(np.max(np.abs(g) / (d * d)))
        hist.append(rho)
        if not np.isfinite(rho):
            status = NONFINITE
            return rp, lam, it, status, hist
        if best is None or rho < best[3]:
            best = (rp, lam.copy(), it, rho)
        if rho <= tol:
            status = OK
            if not until_stagnation or (len(hist) > 1 and rho >= hist[-2]):
                break
        if it >= max_iter:
            break
        A = A_fixed if A_fixed is not None else newton_matrix(rp, r, pairs, inv_mass)
        try:
            z = np.linalg.solve(A, g)
        except np.linalg.LinAlgError:
            return rp, lam, it, SINGULAR, hist
        lam = lam + z
        it += 1
    if status == OK:
        return best[0], best[1], best[2], status, hist
    return rp, lam, it, status, hist


def solve(pairs, d, mass, r, r_u, tol=1e-12, max_iter=20, lam0=None, variant="newton",
          until_stagnation=False):
    """Solves every molecule of a system independently.

    pairs [n,2] int, d [n], mass [s], r and r_u [s,3] (nm, amu).  Atoms in no
    constraint keep r_u.  Returns a dict with r_new [s,3], lam [n] (input
    constraint order), and per-molecule iters, status, max relative
    violation, plus the molecule list.
    """
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    d = np.asarray(d, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    r_u = np.asarray(r_u, dtype=np.float64)
    s = mass.shape[0]
    inv_mass = 1.0 / mass
    r_new = r_u.copy()
    lam = np.zeros(pairs.shape[0])
    mols = molecules(s, pairs)
    iters = np.zeros(len(mols), np.int64)
    status = np.zeros(len(mols), np.int64)
    viol = np.zeros(len(mols))
    hists = []
    for m, (atoms, cons) in enumerate(mols):
        local = np.full(s, -1, np.int64)
        local[atoms] = np.arange(atoms.size)
        lp = local[pairs[cons]]
        l0 = None if lam0 is None else np.asarray(lam0)[cons]
        rp, lm, it, st, h = solve_molecule(r[atoms], r_u[atoms], lp, d[cons], inv_mass[atoms], tol,
                                           max_iter, l0, variant, until_stagnation)
        r_new[atoms] = rp
        lam[cons] = lm
        iters[m] = it
        status[m] = st
        viol[m] = float(np.max(relative_violation(rp, lp, d[cons])))
        hists.append(h)
    return {"r_new": r_new, "lam": lam, "iters": iters, "status": status, "max_rel": viol,
            "molecules": mols, "history": hists}


def project_velocities(pairs, mass, r, v):
    """Velocity constraints (the velocity half of RATTLE; the derivative of
    g(r) = 0 along the motion, G(r) v = 0, with the multiplier term of the
    equations of motion, Supplement section 2): the velocity closest to v in
    the kinetic metric among those tangent to the constraints,

      v_out = v - M^{-1} G(r)^T mu,   G(r) M^{-1} G(r)^T mu = G(r) v,

    solved per molecule with a dense LAPACK solve.  Atoms in no constraint
    keep v.  Returns (v_out [s, 3], mu [n])."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    mass = np.asarray(mass, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    v_out = v.copy()
    mu = np.zeros(pairs.shape[0])
    for atoms, cons in molecules(r.shape[0], pairs):
        local = np.full(r.shape[0], -1, np.int64)
        local[atoms] = np.arange(atoms.size)
        lp = local[pairs[cons]]
        inv_m = 1.0 / mass[atoms]
        G = jacobian(r[atoms], lp, atoms.size)
        A = newton_matrix(r[atoms], r[atoms], lp, inv_m)
        m_loc = np.linalg.solve(A, G @ v[atoms].ravel())
        v_out[atoms] = v[atoms] - (np.repeat(inv_m, 3) * (G.T @ m_loc)).reshape(-1, 3)
        mu[cons] = m_loc
    return v_out, mu
