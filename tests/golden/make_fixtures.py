"""Writes the oracle fixtures in this folder (run from the repository root:
python tests/golden/make_fixtures.py). Calls only the oracle and the seeded
input generator. The paper prints no worked example for the CASCI path
(no energies, no sigma values), so these fixtures pin the oracle against
later changes of its own arithmetic, not against printed numbers."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2405_10197_amd import synth  # noqa: E402


def main():
    out = {}
    # CAS(6e,6o), seed 1: the small configuration of the workload set
    h, eri, _ = synth.integrals(6, 1)
    E, _, s2 = oracle.solve(h, eri, 3, 3, nroots=6)
    Es, _, s2s = oracle.solve(h, eri, 3, 3, nroots=1, spin="singlet")
    out["cas66_seed1"] = {"energies": E.tolist(), "s2": s2.tolist(), "singlet_ground": float(Es[0]),
                          "singlet_ground_s2": float(s2s[0])}
    # CAS(4e,5o) doublet-like (nalpha 3, nbeta 1), seed 7: a row of sigma on a seeded vector
    h, eri, _ = synth.integrals(5, 7)
    na, nb = 3, 1
    x = synth.ci_vector(10, 5, 11)[0]
    s = oracle.sigma(h, eri, na, nb, x)
    out["cas5_31_seed7_sigma"] = {"sigma": s.ravel().tolist()}
    with open(os.path.join(HERE, "oracle_fixtures.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
