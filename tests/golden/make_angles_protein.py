"""Writes tests/golden/angles_protein0.npz: the dense CPU oracle's solution
of the first protein of the full-size angle-constrained system (20
protein-like molecules with bonds and H-X-H / H-X-Y angle constraints plus
1,000 lipid chains; seed 2, first perturbed input, sigma 0.006 nm).

The protein is solved on its own (molecules are independent blocks of the
Newton matrix, Supplement section 3) by the oracle's dense FP64 Newton
iteration from lambda_0 = 0 (Supplement section 2.3), run until the maximum
relative violation stops decreasing once it is below 1e-13 (Supplement
section 4's stopping rule with the oracle's own rounding as the floor);
the best iterate is stored.  Only ``oracle/`` computes; the inputs come from
the seeded generators.  About two minutes on 8 cores (13 s per dense LU of
the ~10,500 x 10,500 matrix).

    python tests/golden/make_angles_protein.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import newton_dense as O  # noqa: E402
from paper_2503_13075_amd import synth as S  # noqa: E402

OUT = os.path.join(HERE, "angles_protein0.npz")
SEED, SIGMA, INPUT_SEED, MOLECULE = 2, 0.006, 10_000, 0


def main():
    t0 = time.time()
    sm = S.angles_system(seed=SEED)
    ru = S.perturb(sm.r, SIGMA, INPUT_SEED)
    atoms, cons = O.molecules(sm.n_atoms, sm.pairs)[MOLECULE]
    local = np.full(sm.n_atoms, -1, np.int64)
    local[atoms] = np.arange(atoms.size)
    rp, lam, it, st, hist = O.solve_molecule(sm.r[atoms], ru[atoms], local[sm.pairs[cons]], sm.d[cons],
                                             1.0 / sm.mass[atoms], 1e-13, 40, until_stagnation=True)
    viol = float(np.max(O.relative_violation(rp, local[sm.pairs[cons]], sm.d[cons])))
    print(f"molecule {MOLECULE}: {atoms.size} atoms, {cons.size} constraints, status {st}, {it} iterations, "
          f"violation {viol:.2e}, history {['%.1e' % h for h in hist]}, {time.time() - t0:.0f} s", flush=True)
    if st != O.OK:
        raise SystemExit("oracle did not converge")
    np.savez_compressed(OUT, atoms=atoms.astype(np.int32), cons=cons.astype(np.int32), r_new=rp, lam=lam,
                        iters=np.int32(it), history=np.asarray(hist), violation=np.float64(viol),
                        seed=np.int32(SEED), sigma=np.float64(SIGMA), input_seed=np.int32(INPUT_SEED))
    print(f"wrote {OUT} ({os.path.getsize(OUT)} bytes)")


if __name__ == "__main__":
    main()
