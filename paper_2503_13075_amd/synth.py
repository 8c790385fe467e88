"""Seeded synthetic molecular systems for the constraint solve.

This module only builds inputs: topologies (which atom pairs are held at a
fixed distance), masses, a reference geometry that satisfies every
constraint, and perturbed "unconstrained" positions.  It contains none of the
solver's arithmetic and is shared by the GPU path, the CPU oracle, the tests
and the benchmark.

Workloads (stand-ins for the paper's GROMACS systems, which are not
available; sizes follow Supp. section 6, systems table):

* ``chain64``      64-atom united-atom chain, bonds + 1-3 angle distances.
* ``protein``      protein-like molecule: backbone N-CA-C(=O), branched side
                   chains of 1-10 heavy atoms, valence-limited hydrogens,
                   5-/6-ring closures in 10% of residues (COVID main protease
                   stand-in: ~4,700 atoms, ~4,700 bond constraints).
* ``random_tree``  random recursive tree, valence <= 4, H only at leaves,
                   5% of atoms rings (many-molecule systems stand-in).
* ``lipid_chain``  united-atom chain of 50 atoms, bonds only.
* ``add_h_angles`` adds H-X-H and H-X-Y angles as 1-3 distance constraints
                   (GROMACS ``h-angles`` style, main text and Supp. section 6).

Units are nm and amu throughout.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# element table: mass (amu), maximum number of bonds
MASS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "S": 32.06,
        "CH2": 14.027, "CH3": 15.035}
VALENCE = {"H": 1, "C": 4, "N": 3, "O": 2, "S": 2}

# bond lengths by element pair, all inside [0.100, 0.153] nm
_BOND = {
    ("C", "H"): 0.109, ("H", "N"): 0.101, ("H", "O"): 0.100, ("H", "S"): 0.134,
    ("C", "C"): 0.153, ("C", "N"): 0.147, ("C", "O"): 0.143, ("C", "S"): 0.153,
    ("N", "N"): 0.145, ("N", "O"): 0.140, ("O", "O"): 0.148, ("N", "S"): 0.153,
    ("O", "S"): 0.153, ("S", "S"): 0.153,
}
RING_BOND = 0.140           # regular 5-/6-ring edge length (nm)
TETRA_COS = -1.0 / 3.0      # cos of the tetrahedral angle
CHAIN_BOND = 0.153          # united-atom chain bond (nm)
CHAIN_13 = 0.250            # united-atom chain 1-3 distance (nm)


def bond_length(e1: str, e2: str) -> float:
    return _BOND[tuple(sorted((e1, e2)))]


@dataclass
class System:
    """A set of atoms with distance constraints.

    pairs[k] = (a_k, b_k), d[k] = target distance, kind[k] = 0 for a bond,
    1 for an angle written as a 1-3 distance.  ``r`` satisfies every
    constraint of the reference geometry to rounding.
    """
    pairs: np.ndarray            # int32  [n, 2]
    d: np.ndarray                # float64 [n]
    mass: np.ndarray             # float64 [s]
    r: np.ndarray                # float64 [s, 3]
    kind: np.ndarray             # int8 [n]
    elem: list = field(default_factory=list)
    mol_start: np.ndarray | None = None   # atom offset of each generated molecule
    name: str = ""

    @property
    def n_atoms(self) -> int:
        return int(self.mass.shape[0])

    @property
    def n_constraints(self) -> int:
        return int(self.pairs.shape[0])


# ----------------------------------------------------------------------------
# small 3-vector helpers on tuples (faster than numpy for per-atom work)

def _add(a, b):
    return (a[0] + b[0], a[1] + b[1], a[2] + b[2])


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _scale(a, s):
    return (a[0] * s, a[1] * s, a[2] * s)


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _norm(a):
    return math.sqrt(_dot(a, a))


def _unit(a):
    n = _norm(a)
    return (a[0] / n, a[1] / n, a[2] / n)


def _perp(b, rng):
    """A random unit vector perpendicular to unit vector b."""
    while True:
        v = (rng.normal(), rng.normal(), rng.normal())
        v = _sub(v, _scale(b, _dot(v, b)))
        if _norm(v) > 1e-3:
            return _unit(v)


class _Rand:
    """Pre-drawn buffers of standard normals and uniforms from one seeded
    numpy Generator, consumed in order (scalar draws from numpy are slow)."""

    def __init__(self, seed, chunk=4096):
        self.g = np.random.default_rng(seed)
        self.chunk = chunk
        self._n = self.g.standard_normal(chunk).tolist()
        self._u = self.g.random(chunk).tolist()
        self._in = 0
        self._iu = 0

    def normal(self):
        if self._in == len(self._n):
            self._n = self.g.standard_normal(self.chunk).tolist()
            self._in = 0
        v = self._n[self._in]
        self._in += 1
        return v

    def random(self):
        if self._iu == len(self._u):
            self._u = self.g.random(self.chunk).tolist()
            self._iu = 0
        v = self._u[self._iu]
        self._iu += 1
        return v

    def uniform(self, lo, hi):
        return lo + (hi - lo) * self.random()

    def integers(self, n):
        return min(int(self.random() * n), n - 1)


def _random_unit(rng):
    while True:
        v = (rng.normal(), rng.normal(), rng.normal())
        n = _norm(v)
        if n > 1e-3:
            return _scale(v, 1.0 / n)


class _Builder:
    """Grows one molecule atom by atom with near-tetrahedral geometry."""

    def __init__(self, rng, origin=(0.0, 0.0, 0.0)):
        self.rng = rng
        self.pos: list = []
        self.elem: list = []
        self.maxval: list = []
        self.dirs: list = []          # unit bond directions per atom
        self.nbrs: list = []
        self.bonds: list = []         # (i, j, length)
        self.origin = origin

    @property
    def n(self):
        return len(self.pos)

    def free(self, i):
        return self.maxval[i] - len(self.nbrs[i])

    def _new(self, p, el, maxval):
        self.pos.append(p)
        self.elem.append(el)
        self.maxval.append(maxval if maxval is not None else VALENCE[el])
        self.dirs.append([])
        self.nbrs.append([])
        return len(self.pos) - 1

    def root(self, el, maxval=None):
        return self._new(self.origin, el, maxval)

    def slots(self, i):
        """Free bond directions at atom i, given the bonds it already has."""
        ds = self.dirs[i]
        rng = self.rng
        k = len(ds)
        if k == 0:
            b = _random_unit(rng)
            return [b] + self._cone(b, rng)
        if k == 1:
            return self._cone(ds[0], rng)
        if k == 2:
            s = _add(ds[0], ds[1])
            if _norm(s) < 1e-6:
                m = _perp(ds[0], rng)
            else:
                m = _unit(_scale(s, -1.0))
            c = _cross(ds[0], ds[1])
            nrm = _unit(c) if _norm(c) > 1e-6 else _perp(m, rng)
            ca, sa = math.cos(math.radians(54.735)), math.sin(math.radians(54.735))
            return [_add(_scale(m, ca), _scale(nrm, sa)), _sub(_scale(m, ca), _scale(nrm, sa))]
        if k == 3:
            s = _add(_add(ds[0], ds[1]), ds[2])
            if _norm(s) < 1e-6:
                return [_unit(_cross(ds[0], ds[1]))]
            return [_unit(_scale(s, -1.0))]
        return []

    @staticmethod
    def _cone(b, rng):
        p = _perp(b, rng)
        q = _cross(b, p)
        phi0 = rng.uniform(0.0, 2.0 * math.pi)
        st = math.sqrt(1.0 - TETRA_COS * TETRA_COS)
        out = []
        for t in range(3):
            phi = phi0 + t * 2.0 * math.pi / 3.0
            out.append(_add(_scale(b, TETRA_COS),
                            _add(_scale(p, st * math.cos(phi)), _scale(q, st * math.sin(phi)))))
        return out

    def _link(self, i, j, length):
        dij = _unit(_sub(self.pos[j], self.pos[i]))
        self.dirs[i].append(dij)
        self.dirs[j].append(_scale(dij, -1.0))
        self.nbrs[i].append(j)
        self.nbrs[j].append(i)
        self.bonds.append((i, j, length))

    def child(self, parent, el, length=None, maxval=None):
        sl = self.slots(parent)
        direction = sl[0]
        if length is None:
            length = bond_length(self.elem[parent], el)
        j = self._new(_add(self.pos[parent], _scale(direction, length)), el, maxval)
        self._link(parent, j, length)
        return j

    def ring(self, anchor, size, elems):
        """Closes a regular ring of ``size`` atoms through ``anchor``.

        Adds size-1 atoms and ``size`` ring bonds (size-1 tree bonds plus one
        closure), all of length RING_BOND.
        """
        rng = self.rng
        s = self.slots(anchor)[0]
        p = _perp(s, rng)
        R = RING_BOND / (2.0 * math.sin(math.pi / size))
        c = _add(self.pos[anchor], _scale(s, R))
        idx = [anchor]
        for t in range(1, size):
            ang = 2.0 * math.pi * t / size
            v = _add(_scale(s, -R * math.cos(ang)), _scale(p, R * math.sin(ang)))
            idx.append(self._new(_add(c, v), elems[t - 1], None))
        for t in range(size):
            self._link(idx[t], idx[(t + 1) % size], RING_BOND)
        return idx

    def hydrogens(self, i, count):
        for _ in range(count):
            self.child(i, "H")

    def to_system(self, name, masses=None) -> System:
        r = np.array(self.pos, dtype=np.float64).reshape(-1, 3)
        pairs = np.array([(a, b) for a, b, _ in self.bonds], dtype=np.int32).reshape(-1, 2)
        # constraint distances come from the reference geometry, so g(r) = 0
        d = np.linalg.norm(r[pairs[:, 0]] - r[pairs[:, 1]], axis=1) if len(pairs) else np.zeros(0)
        if masses is None:
            masses = np.array([MASS[e] for e in self.elem], dtype=np.float64)
        return System(pairs=pairs, d=d, mass=masses, r=r,
                      kind=np.zeros(len(pairs), np.int8), elem=list(self.elem),
                      mol_start=np.zeros(1, np.int64), name=name)


# ----------------------------------------------------------------------------
# united-atom chains

def united_chain(n_atoms: int, seed: int, angles: bool, origin=(0.0, 0.0, 0.0),
                 name="chain") -> System:
    """Linear united-atom chain with bond 0.153 nm and (optionally) 1-3
    distances 0.250 nm.  The bond angle is 2*asin(0.125/0.153) (about
    109.57 degrees) so that both distances hold exactly; dihedrals are
    uniform random.  Masses alternate CH (12.011) / CH2 (14.027)."""
    rng = np.random.default_rng(seed)
    theta = 2.0 * math.asin(0.5 * CHAIN_13 / CHAIN_BOND)
    pos = [origin]
    if n_atoms > 1:
        b = _random_unit(rng)
        pos.append(_add(origin, _scale(b, CHAIN_BOND)))
    prev_dir = None
    for i in range(2, n_atoms):
        b = _unit(_sub(pos[i - 1], pos[i - 2]))     # last bond direction
        if prev_dir is None:
            p = _perp(b, rng)
        else:
            # component of the previous bond perpendicular to b fixes the dihedral frame
            p0 = _sub(prev_dir, _scale(b, _dot(prev_dir, b)))
            p = _unit(p0) if _norm(p0) > 1e-8 else _perp(b, rng)
        q = _cross(b, p)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        ct = math.cos(math.pi - theta)
        st = math.sin(math.pi - theta)
        nd = _add(_scale(b, ct), _add(_scale(p, st * math.cos(phi)), _scale(q, st * math.sin(phi))))
        pos.append(_add(pos[i - 1], _scale(_unit(nd), CHAIN_BOND)))
        prev_dir = b
    r = np.array(pos, dtype=np.float64).reshape(-1, 3)
    pairs = [(i, i + 1) for i in range(n_atoms - 1)]
    kind = [0] * len(pairs)
    d = [CHAIN_BOND] * len(pairs)
    if angles:
        pairs += [(i, i + 2) for i in range(n_atoms - 2)]
        kind += [1] * (n_atoms - 2)
        d += [CHAIN_13] * (n_atoms - 2)
    mass = np.array([MASS["C"] if i % 2 == 0 else MASS["CH2"] for i in range(n_atoms)])
    return System(pairs=np.array(pairs, np.int32).reshape(-1, 2), d=np.array(d, np.float64),
                  mass=mass, r=r, kind=np.array(kind, np.int8),
                  elem=["C" if i % 2 == 0 else "CH2" for i in range(n_atoms)],
                  mol_start=np.zeros(1, np.int64), name=name)


def chain64(seed: int = 0) -> System:
    """64-atom chain: 63 bonds of 0.153 nm and 62 1-3 distances of 0.250 nm."""
    return united_chain(64, seed, angles=True, name="chain64")


def lipid_chain(seed: int, n_atoms: int = 50, origin=(0.0, 0.0, 0.0)) -> System:
    """United-atom lipid-like tail: bonds only."""
    return united_chain(n_atoms, seed, angles=False, origin=origin, name="lipid")


# ----------------------------------------------------------------------------
# protein-like molecule

def _side_chain_len(rng) -> int:
    # 1..10 heavy atoms, skewed short (mean 2.8) so that 300 residues give
    # about 4,700 atoms including hydrogens (15.7 atoms per residue)
    w = np.array([0.38, 0.22, 0.13, 0.08, 0.06, 0.04, 0.03, 0.03, 0.02, 0.01])
    return int(rng.choice(10, p=w / w.sum())) + 1


def _heavy_elem(rng) -> str:
    u = rng.random()
    if u < 0.78:
        return "C"
    if u < 0.88:
        return "N"
    if u < 0.97:
        return "O"
    return "S"


def protein(n_res: int = 300, seed: int = 0, ring_frac: float = 0.10,
            origin=(0.0, 0.0, 0.0)) -> System:
    """Protein-like molecule.

    Backbone N-CA-C(=O) per residue with the peptide bond C-N to the next
    residue; a side chain of 1-10 heavy atoms hangs off CA; ``ring_frac`` of
    the residues carry a 5- or 6-membered ring in the side chain; every heavy
    atom then receives valence-limited hydrogens (at most 3).  All bonds are
    constraints, with lengths by element pair.
    """
    rng = np.random.default_rng(seed)
    mb = _Builder(_Rand(rng.integers(1 << 62)), origin)
    ring_res = set(rng.choice(n_res, size=int(round(ring_frac * n_res)), replace=False).tolist())
    prev_c = None
    heavy = []
    for res in range(n_res):
        if prev_c is None:
            n_at = mb.root("N")
        else:
            n_at = mb.child(prev_c, "N")
        ca = mb.child(n_at, "C")
        c = mb.child(ca, "C", maxval=3)          # carbonyl carbon (sp2)
        o = mb.child(c, "O", maxval=1)           # carbonyl oxygen
        heavy += [n_at, ca, c, o]
        # side chain
        k = _side_chain_len(rng)
        side = [mb.child(ca, "C")]
        heavy.append(side[0])
        if res in ring_res:
            size = 5 if rng.random() < 0.5 else 6
            ring_elems = ["C"] * (size - 1)
            if size == 5 and rng.random() < 0.5:
                ring_elems[1] = "N"
            anchor = side[-1]
            if k >= 2:
                anchor = mb.child(side[-1], "C")
                side.append(anchor)
                heavy.append(anchor)
            idx = mb.ring(anchor, size, ring_elems)
            side += idx[1:]
            heavy += idx[1:]
        else:
            while len(side) < k:
                cand = [a for a in side if mb.free(a) >= 2]
                if not cand:
                    break
                # mostly extend the newest atom: chain-like with some branching
                par = cand[-1] if rng.random() < 0.7 else cand[int(rng.integers(len(cand)))]
                el = _heavy_elem(rng) if len(side) == k - 1 else "C"
                if VALENCE[el] - 1 < 1 and len(side) < k - 1:
                    el = "C"
                j = mb.child(par, el)
                side.append(j)
                heavy.append(j)
        prev_c = c
    for a in heavy:
        nh = min(3, mb.free(a))
        mb.hydrogens(a, max(0, nh))
    sysm = mb.to_system("protein")
    return sysm


# ----------------------------------------------------------------------------
# random recursive trees (many-molecule batches)

def random_tree(n_atoms: int, seed: int, ring_frac: float = 0.05,
                origin=(0.0, 0.0, 0.0)) -> System:
    """Random recursive tree molecule of exactly ``n_atoms`` atoms.

    Each new atom attaches to a uniformly chosen heavy atom with free valence;
    hydrogens only ever appear as leaves; round(ring_frac * n_atoms) 5-/6-ring
    closures are inserted at evenly spaced points of the growth.
    """
    rng = _Rand(seed)
    mb = _Builder(rng, origin)
    mb.root("C")
    open_heavy = [0]            # heavy atoms that still have free valence
    total_free = mb.free(0)
    n_rings = int(round(ring_frac * n_atoms))
    ring_at = sorted(set(int(x) for x in np.linspace(1, max(1, n_atoms - 6), n_rings, endpoint=False))) if n_rings else []
    ring_at.reverse()           # pop() yields the next insertion point

    def close(i):
        nonlocal total_free
        # remove atom i from the open list when it is saturated (swap-pop)
        if mb.free(i) == 0:
            k = open_heavy.index(i)
            open_heavy[k] = open_heavy[-1]
            open_heavy.pop()

    while mb.n < n_atoms:
        rem = n_atoms - mb.n
        if ring_at and mb.n >= ring_at[-1]:
            ring_at.pop()
            if rem >= 5:
                cand = [a for a in open_heavy if mb.free(a) >= 2 and len(mb.dirs[a]) <= 2]
                if cand:
                    size = 5 if (rng.random() < 0.5 or rem < 5 + 1) else 6
                    anchor = cand[rng.integers(len(cand))]
                    idx = mb.ring(anchor, size, ["C"] * (size - 1))
                    total_free += sum(mb.free(a) for a in idx[1:]) - 2
                    open_heavy.extend(idx[1:])
                    close(anchor)
                    continue
        par = open_heavy[rng.integers(len(open_heavy))]
        # keep at least one open slot while atoms remain: force a heavy atom
        want_h = rng.random() < 0.45 and (total_free > 2 or rem == 1)
        if want_h:
            mb.child(par, "H")
            total_free -= 1
        else:
            el = _heavy_elem(rng)
            if VALENCE[el] < 2 or (total_free <= 2 and VALENCE[el] < 3):
                el = "C"
            j = mb.child(par, el)
            open_heavy.append(j)
            total_free += VALENCE[el] - 2
        close(par)
    return mb.to_system("random_tree")


# ----------------------------------------------------------------------------
# angle constraints (h-angles)

def add_h_angles(sysm: System) -> System:
    """Adds H-X-H and then H-X-Y angles as 1-3 distance constraints.

    At each centre X the angles are capped so that X and its neighbours are
    never over-determined: 3*deg(X) - 3 internal degrees of freedom, minus
    the deg(X) bonds, minus one for every heavy-heavy angle Y-X-Y, which is
    left free (otherwise a set of H angles would pin the Y-X-Y angle too and
    a ring whose angles are all pinned is over-constrained, making the
    constraint Jacobian rank deficient).  Distances come from the reference
    geometry.  Angles that are nearly straight (over 150 degrees) are never
    constrained: the 1-3 distance then hardly depends on the angle, the
    constraint is close to a combination of the two bonds, and the Newton
    matrix close to singular.
    """
    s = sysm.n_atoms
    nbrs = [[] for _ in range(s)]
    for k, (a, b) in enumerate(sysm.pairs):
        if sysm.kind[k] == 0:
            nbrs[a].append(b)
            nbrs[b].append(a)
    is_h = np.array([e == "H" for e in sysm.elem], dtype=bool) if sysm.elem else np.zeros(s, bool)
    new_pairs = []
    for x in range(s):
        nb = nbrs[x]
        deg = len(nb)
        if deg < 2:
            continue
        hs = [a for a in nb if is_h[a]]
        ys = [a for a in nb if not is_h[a]]
        budget = 3 * deg - 3 - deg - len(ys) * (len(ys) - 1) // 2
        cand = []
        for i in range(len(hs)):
            for j in range(i + 1, len(hs)):
                cand.append((hs[i], hs[j]))
        for h in hs:
            for y in ys:
                cand.append((h, y))
        def straight(a, b):
            u, v = sysm.r[a] - sysm.r[x], sysm.r[b] - sysm.r[x]
            return np.dot(u, v) < np.cos(np.radians(150.0)) * np.linalg.norm(u) * np.linalg.norm(v)
        cand = [c for c in cand if not straight(*c)]
        for a, b in cand[:max(0, budget)]:
            new_pairs.append((a, b))
    if not new_pairs:
        return sysm
    np_ = np.array(new_pairs, np.int32).reshape(-1, 2)
    dnew = np.linalg.norm(sysm.r[np_[:, 0]] - sysm.r[np_[:, 1]], axis=1)
    return System(pairs=np.concatenate([sysm.pairs, np_]), d=np.concatenate([sysm.d, dnew]),
                  mass=sysm.mass, r=sysm.r, kind=np.concatenate([sysm.kind, np.ones(len(np_), np.int8)]),
                  elem=sysm.elem, mol_start=sysm.mol_start, name=sysm.name + "+hangles")


# ----------------------------------------------------------------------------
# combining molecules

def concat(systems: list, spacing: float = 2.0, name: str = "") -> System:
    """Places molecule centres on a cubic grid ``spacing`` nm apart and
    renumbers atoms.  Molecules may overlap in space (there are no
    interactions between them); the grid keeps coordinates within a box of
    a few tens of nm, like an MD system of the same atom count."""
    nm = len(systems)
    side = max(1, int(math.ceil(nm ** (1.0 / 3.0))))
    pairs, d, mass, r, kind, elem, starts = [], [], [], [], [], [], []
    off = 0
    for i, sm in enumerate(systems):
        gx, gy, gz = i % side, (i // side) % side, i // (side * side)
        shift = np.array([gx, gy, gz], np.float64) * spacing
        centred = sm.r - sm.r.mean(axis=0, keepdims=True) if sm.n_atoms else sm.r
        pairs.append(sm.pairs.astype(np.int64) + off)
        d.append(sm.d)
        mass.append(sm.mass)
        r.append(centred + shift)
        kind.append(sm.kind)
        elem += sm.elem
        starts.append(off)
        off += sm.n_atoms
    return System(pairs=np.concatenate(pairs).astype(np.int32), d=np.concatenate(d),
                  mass=np.concatenate(mass), r=np.concatenate(r), kind=np.concatenate(kind),
                  elem=elem, mol_start=np.array(starts, np.int64), name=name)


# ----------------------------------------------------------------------------
# workloads

def batch_sizes(n_mol: int, seed: int, lo: int = 8, hi: int = 2048) -> np.ndarray:
    """Atom counts drawn log-uniformly from [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_mol))).astype(np.int64)


def random_tree_batch(n_mol: int = 4096, seed: int = 2, lo: int = 8, hi: int = 2048) -> System:
    """Many random-tree molecules of log-uniform size (all bonds constrained)."""
    sizes = batch_sizes(n_mol, seed, lo, hi)
    mols = [random_tree(int(sz), seed * 1_000_003 + i) for i, sz in enumerate(sizes)]
    return concat(mols, spacing=1.5, name=f"random_tree_batch{n_mol}")


def protein_system(seed: int = 1, n_res: int = 300) -> System:
    sm = protein(n_res=n_res, seed=seed)
    sm.name = f"protein{n_res}"
    return sm


def angles_system(seed: int = 3, n_prot: int = 20, n_res: int = 315, n_lipid: int = 1000,
                  lipid_len: int = 50) -> System:
    """Protein-like molecules plus united-atom lipid chains, with bonds and
    H-X-H / H-X-Y angle constraints (lipids have no H so only bonds)."""
    mols = [add_h_angles(protein(n_res=n_res, seed=seed * 7919 + i)) for i in range(n_prot)]
    mols += [lipid_chain(seed * 104729 + j, lipid_len) for j in range(n_lipid)]
    return concat(mols, spacing=1.2, name=f"angles_{n_prot}prot_{n_lipid}lipid")


def _rotations(n: int, rng) -> np.ndarray:
    """n uniformly random rotation matrices (QR of Gaussian matrices)."""
    q, rr = np.linalg.qr(rng.normal(size=(n, 3, 3)))
    q = q * np.sign(np.diagonal(rr, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 2] *= det[:, None]
    return q


def water_box(n_mol: int, seed: int = 0, spacing: float = 0.31) -> System:
    """Rigid waters (three constraints each: O-H, O-H and H-H, the usual
    rigid-water model: O-H 0.09572 nm, H-O-H 104.52 degrees) with random
    orientations, oxygens on a cubic grid ``spacing`` nm apart."""
    rng = np.random.default_rng(seed)
    d_oh, th = 0.09572, math.radians(104.52)
    local = np.array([[0.0, 0.0, 0.0], [d_oh, 0.0, 0.0], [d_oh * math.cos(th), d_oh * math.sin(th), 0.0]])
    local = local - local.mean(axis=0)
    side = max(1, int(math.ceil(n_mol ** (1.0 / 3.0))))
    i = np.arange(n_mol)
    centre = np.stack([i % side, (i // side) % side, i // (side * side)], axis=1) * spacing
    rot = _rotations(n_mol, rng)
    r = (centre[:, None, :] + np.einsum("mij,aj->mai", rot, local)).reshape(-1, 3)
    base = 3 * i
    pairs = np.stack([np.stack([base, base + 1], 1), np.stack([base, base + 2], 1),
                      np.stack([base + 1, base + 2], 1)], axis=1).reshape(-1, 2).astype(np.int32)
    d = np.linalg.norm(r[pairs[:, 0]] - r[pairs[:, 1]], axis=1)
    mass = np.tile([15.999, 1.008, 1.008], n_mol)
    kind = np.tile(np.array([0, 0, 1], np.int8), n_mol)
    return System(pairs=pairs, d=d, mass=mass, r=r, kind=kind, elem=["O", "H", "H"] * n_mol,
                  mol_start=base.astype(np.int64), name=f"water{n_mol}")


def small_molecules(n_each: int, seed: int) -> System:
    """Molecules of one to three constraints on two to four atoms: diatomics,
    bent triatomics (two bonds), rigid waters, four-atom chains and
    three-bond stars, ``n_each`` of each, randomly oriented."""
    rng = np.random.default_rng(seed)
    mols = []
    for j in range(n_each):
        rot = _rotations(4, rng)
        # diatomic C-O
        r = np.array([[0.0, 0.0, 0.0], [0.1128, 0.0, 0.0]]) @ rot[0].T
        mols.append(System(pairs=np.array([[0, 1]], np.int32), d=np.array([0.1128]), mass=np.array([12.011, 15.999]),
                           r=r, kind=np.zeros(1, np.int8), elem=["C", "O"]))
        # bent H-S-H, two bonds only
        th = math.radians(92.1)
        r = np.array([[0.1336, 0.0, 0.0], [0.0, 0.0, 0.0], [0.1336 * math.cos(th), 0.1336 * math.sin(th), 0.0]])
        mols.append(System(pairs=np.array([[0, 1], [1, 2]], np.int32), d=np.array([0.1336, 0.1336]),
                           mass=np.array([1.008, 32.06, 1.008]), r=r @ rot[1].T, kind=np.zeros(2, np.int8),
                           elem=["H", "S", "H"]))
        # rigid water
        w = water_box(1, seed=int(rng.integers(1 << 30)))
        mols.append(w)
        # C-C-C-C chain with random dihedral
        ch = united_chain(4, int(rng.integers(1 << 30)), angles=False)
        mols.append(ch)
        # N with three H (bonds only)
        hs = []
        for k in range(3):
            phi = 2.0 * math.pi * k / 3.0
            hs.append([0.1012 * math.sin(math.radians(68.0)) * math.cos(phi),
                       0.1012 * math.sin(math.radians(68.0)) * math.sin(phi), -0.1012 * math.cos(math.radians(68.0))])
        r = np.concatenate([np.zeros((1, 3)), np.array(hs)]) @ rot[3].T
        pairs = np.array([[0, 1], [0, 2], [0, 3]], np.int32)
        mols.append(System(pairs=pairs, d=np.linalg.norm(r[pairs[:, 0]] - r[pairs[:, 1]], axis=1),
                           mass=np.array([14.007, 1.008, 1.008, 1.008]), r=r, kind=np.zeros(3, np.int8),
                           elem=["N", "H", "H", "H"]))
    return concat(mols, spacing=0.6, name=f"small{n_each}")


def perturb(r: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Unconstrained positions: r + N(0, sigma^2) per coordinate."""
    rng = np.random.default_rng(seed)
    return r + rng.normal(0.0, sigma, size=r.shape)


def soa(x: np.ndarray) -> np.ndarray:
    """[s, 3] -> contiguous [3, s] (structure of arrays)."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)


# ----------------------------------------------------------------------------
# counter-based normal variates (the host side of the device generator)

_PHILOX_M0, _PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
_PHILOX_W0, _PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr: np.ndarray, key) -> np.ndarray:
    """Philox4x32-10 (Salmon et al., SC 2011) on an array of counters
    ``ctr`` [m, 4] (uint32) with one key (k0, k1); returns [m, 4] uint32."""
    c = [np.asarray(ctr[:, i], dtype=np.uint64) for i in range(4)]
    k0, k1 = np.uint64(key[0] & 0xFFFFFFFF), np.uint64(key[1] & 0xFFFFFFFF)
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(_PHILOX_M0) * c[0]
        p1 = np.uint64(_PHILOX_M1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(_PHILOX_W0)) & mask
        k1 = (k1 + np.uint64(_PHILOX_W1)) & mask
    return np.stack(c, axis=1).astype(np.uint32)


def _uniform53(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    x = ((hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)) >> np.uint64(11)
    return (x.astype(np.float64) + 0.5) * 2.0 ** -53


def philox_normals(n_atoms: int, seed: int, step: int) -> np.ndarray:
    """Standard normals z [n_atoms, 3] of atom i at a step: Box-Muller on the
    words of the counters {i, 0, step} (x, y) and {i, 1, step} (z)."""
    i = np.arange(n_atoms, dtype=np.uint64)
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty((n_atoms, 3))
    for half in (0, 1):
        ctr = np.stack([i, np.full_like(i, half), np.full_like(i, step & 0xFFFFFFFF),
                        np.full_like(i, (step >> 32) & 0xFFFFFFFF)], axis=1)
        w = philox4x32_10(ctr, key)
        u1, u2 = _uniform53(w[:, 0], w[:, 1]), _uniform53(w[:, 2], w[:, 3])
        rho = np.sqrt(-2.0 * np.log(u1))
        th = 2.0 * np.pi * u2
        if half == 0:
            out[:, 0], out[:, 1] = rho * np.cos(th), rho * np.sin(th)
        else:
            out[:, 2] = rho * np.cos(th)
    return out


def perturb_philox(r: np.ndarray, sigma: float, seed: int, step: int) -> np.ndarray:
    """r + sigma * philox_normals (AoS [n, 3])."""
    return r + sigma * philox_normals(r.shape[0], seed, step)
