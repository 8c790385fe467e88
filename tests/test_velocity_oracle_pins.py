"""Pins of the oracle's velocity projection (velocity constraints of
RATTLE) by properties the definition fixes, not by retyping it: the result
is tangent to the constraints, the removed part is orthogonal in the
kinetic metric to every tangent velocity (a basis of the null space of G
from an SVD), projecting twice changes nothing, linear and angular momentum
are conserved (the multiplier forces are central pair forces), a single
bond keeps its centre-of-mass velocity and loses its relative velocity
along the bond, and atoms in no constraint keep their velocity."""
import numpy as np
import scipy.linalg as sla

from oracle import newton_dense as O
from paper_2503_13075_amd import synth as S


def _system(seed):
    sm = S.concat([S.random_tree(12, seed=seed), S.protein(3, seed=seed + 1), S.small_molecules(2, seed=seed + 2)],
                  spacing=2.0)
    rng = np.random.default_rng(seed)
    v = rng.normal(0.0, 0.5, size=(sm.n_atoms, 3))
    return sm, v


def test_projection_is_tangent_and_kinetic_orthogonal():
    for seed in range(3):
        sm, v = _system(seed)
        vo, mu = O.project_velocities(sm.pairs, sm.mass, sm.r, v)
        G = O.jacobian(sm.r, sm.pairs, sm.n_atoms).toarray()
        assert np.max(np.abs(G @ vo.ravel())) <= 1e-12 * np.max(np.abs(G @ v.ravel()))
        N = sla.null_space(G)                       # tangent velocities
        M = np.repeat(sm.mass, 3)
        assert np.max(np.abs(N.T @ (M * (v - vo).ravel()))) <= 1e-10 * np.max(np.abs(M * v.ravel()))
        vo2, mu2 = O.project_velocities(sm.pairs, sm.mass, sm.r, vo)
        assert np.max(np.abs(vo2 - vo)) <= 1e-13 and np.max(np.abs(mu2)) <= 1e-11 * np.max(np.abs(mu))


def test_projection_conserves_momenta():
    sm, v = _system(7)
    vo, _ = O.project_velocities(sm.pairs, sm.mass, sm.r, v)
    p0, p1 = (sm.mass[:, None] * v).sum(0), (sm.mass[:, None] * vo).sum(0)
    l0, l1 = np.cross(sm.r, sm.mass[:, None] * v).sum(0), np.cross(sm.r, sm.mass[:, None] * vo).sum(0)
    assert np.max(np.abs(p1 - p0)) <= 1e-11 * np.abs(p0).max()
    assert np.max(np.abs(l1 - l0)) <= 1e-11 * np.abs(l0).max()


def test_single_bond_and_free_atoms():
    r = np.array([[0.0, 0.0, 0.0], [0.1, 0.02, 0.0], [3.0, 3.0, 3.0]])
    mass = np.array([12.0, 1.0, 5.0])
    v = np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, 0.2], [1.0, 2.0, 3.0]])
    vo, _ = O.project_velocities(np.array([[0, 1]]), mass, r, v)
    e = r[0] - r[1]
    assert abs((vo[0] - vo[1]) @ e) <= 1e-15
    com0 = (mass[:2, None] * v[:2]).sum(0) / mass[:2].sum()
    com1 = (mass[:2, None] * vo[:2]).sum(0) / mass[:2].sum()
    assert np.allclose(com0, com1, atol=1e-15)
    # the relative velocity keeps its component across the bond
    perp = lambda x: x - (x @ e) / (e @ e) * e  # noqa: E731
    assert np.allclose(perp(vo[0] - vo[1]), perp(v[0] - v[1]), atol=1e-15)
    assert np.array_equal(vo[2], v[2])
