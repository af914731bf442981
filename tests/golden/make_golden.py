"""Writes tests/golden/small_system_oracle.json from the FP64 oracle only.

Regression fixture for the 3,000-atom system (30 A cube, seed 1): unique pair count,
total energy, and the forces on a fixed set of atoms. It is produced by the oracle,
never by the GPU library; regenerate only after a change to the oracle that names
the passage of the paper it follows.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1611_04474_amd import workloads as W  # noqa: E402

ATOMS = [0, 1, 2, 100, 777, 1500, 2048, 2999]


def main():
    s = W.small_system()
    r = oracle.forces(s.params(), s.pos, s.types, s.charges, "bruteforce")
    out = {
        "description": "FP64 oracle on the 3,000-atom jittered-lattice system, 30 A cube, seed 1, "
                       "rc 12 A, switch from 10 A, k 332.0636",
        "n_atoms": s.n,
        "n_pairs": int(r.n_pairs),
        "energy": float(r.energy),
        "atoms": ATOMS,
        "forces": [[float(v) for v in r.force[i]] for i in ATOMS],
        "abs_force_sum": float(np.abs(r.force).sum()),
    }
    with open(os.path.join(HERE, "small_system_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
