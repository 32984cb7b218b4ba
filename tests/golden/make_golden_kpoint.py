"""Write the oracle's k-point results for two workload cells.

Runs the CPU oracle only (no GPU code): oracle.KProblem on a workload cell
(its own blocks and theta, no step 2) with the complex density matrix per
Born-von Karman offset drawn by synth.kpoint_density.  Cases:

  diamond64_k222  the 64-atom diamond-like cell on a 2 x 2 x 2 mesh (every
                  cell offset is its own negative), theta 1e-4, seed + 6007
  sc8_k331        the 8-atom simple-cubic cell on a 3 x 3 x 1 mesh (offsets
                  and their negatives differ), theta 0, seed + 7

Stores, in tests/golden/<case>_oracle.npz: E, F[N][3], sigma[3][3], gC, gV,
the keep masks of C and V blocks (bit-packed) and of D pairs per offset
(bit-packed), and a fingerprint of the inputs (sums of C, |dC|, V, |dV|, and
of the real and imaginary parts of D(R)).

Usage: python tests/golden/make_golden_kpoint.py [case ...]   (THREADS: default all cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2412_11081_amd import synth  # noqa: E402

# case -> (workload, mesh, seed offset of the density matrix)
CASES = {
    "diamond64_k222": (2, (2, 2, 2), 6007),
    "sc8_k331": (1, (3, 3, 1), 7),
}


def path_of(case):
    return os.path.join(HERE, f"{case}_oracle.npz")


def inputs(case, device="cpu"):
    """The cell, its blocks, the mesh and the k-point density matrix of a case."""
    k, nk, shift = CASES[case]
    st = synth.workload(k).build()
    mats = st.materialize(device)
    Dk = synth.kpoint_density(st.n_tot, nk, st.seed + shift)
    return st, mats, nk, Dk


def fingerprint(mats, Dk):
    out = []
    for kind in ("C", "V"):
        for key, absval in (("val", False), ("dval", True)):
            x = mats[kind][key]
            out.append(float((x.abs() if absval else x).sum()))
    Dk = Dk.detach().cpu().numpy() if hasattr(Dk, "detach") else np.asarray(Dk)
    out += [float(Dk.real.sum()), float(Dk.imag.sum()), float(np.abs(Dk).sum())]
    return np.array(out)


def make(case, threads):
    st, mats, nk, Dk = inputs(case)
    kp = oracle.KProblem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], nk, Dk)
    t0 = time.time()
    r = kp.evaluate(st.theta, nthreads=threads)
    dt = time.time() - t0
    np.savez_compressed(path_of(case), E=r["E"], F=r["F"], sigma=r["sigma"], gC=r["gC"], gV=r["gV"],
                        keepC=np.packbits(r["keepC"] != 0), keepV=np.packbits(r["keepV"] != 0),
                        keepD=np.packbits(r["keepD"].reshape(-1)), nC=kp.nC, nV=kp.nV,
                        theta=st.theta, nk=np.array(nk), fingerprint=fingerprint(mats, Dk), seconds=dt,
                        threads=threads)
    print(f"{case}: E = {r['E']:.15e}, {dt:.0f} s on {threads} threads", flush=True)


def load(case):
    z = np.load(path_of(case), allow_pickle=False)
    out = {k: z[k] for k in z.files}
    out["keepC"] = np.unpackbits(out["keepC"])[: int(out["nC"])]
    out["keepV"] = np.unpackbits(out["keepV"])[: int(out["nV"])]
    return out


if __name__ == "__main__":
    threads = int(os.environ.get("THREADS", os.cpu_count() or 1))
    for case in sys.argv[1:] or list(CASES):
        make(case, threads)
