"""Write the oracle's result for the 8-atom simple-cubic workload.

Runs the CPU oracle only (no GPU code).  Before writing, the oracle energy is
checked against the brute-force 4-index definition (Eq. Eexx with the LRI
integrals of Eq. Exx-LRI).  Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2412_11081_amd import synth  # noqa: E402
from tests import ref_bruteforce  # noqa: E402


def main():
    oracle.build(force=False)
    st = synth.tiny_cubic().build()
    mats = st.materialize("cpu")
    t0 = time.time()
    r = oracle.evaluate_structure(st, mats=mats, nthreads=int(os.environ.get("THREADS", os.cpu_count())))
    t1 = time.time()
    e_bf = ref_bruteforce.energy_assoc(st, mats)
    assert abs(e_bf - r["E"]) <= 1e-12 * abs(e_bf), (e_bf, r["E"])
    out = {
        "workload": "8-atom simple-cubic cell, a = 5 Bohr, 13 NAO / 40 ABF, r_C = 7, r_V = 14, theta = 0",
        "seed": st.seed,
        "written_by": "tests/golden/make_golden.py (CPU oracle only)",
        "oracle_seconds": t1 - t0,
        "E_bruteforce": e_bf,
        "E": r["E"],
        "F": r["F"].tolist(),
        "sigma": r["sigma"].tolist(),
        "gC": r["gC"].tolist(),
        "gV": r["gV"].tolist(),
        "nC": int(r["gC"].shape[0]),
        "nV": int(r["gV"].shape[0]),
    }
    with open(os.path.join(HERE, "sc8_oracle.json"), "w") as f:
        json.dump(out, f, indent=0)
    print(f"E = {r['E']:.15e}  (brute force {e_bf:.15e}), oracle {t1 - t0:.1f} s")


if __name__ == "__main__":
    main()
