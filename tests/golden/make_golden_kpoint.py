"""Write the oracle's k-point result for the 64-atom cell on a 2 x 2 x 2 mesh.

Runs the CPU oracle only (no GPU code): oracle.KProblem on the 64-atom
diamond-like cell (its own blocks and theta = 1e-4, no step 2) with the
complex density matrix per Born-von Karman offset drawn by
synth.kpoint_density (seed: the cell's seed + 6007).  Stores, in
tests/golden/diamond64_k222_oracle.npz: E, F[N][3], sigma[3][3], gC, gV,
the keep masks of C and V blocks (bit-packed) and D pairs per offset
(bit-packed), and a fingerprint of the inputs (sums of C, |dC|, V, |dV|,
and of the real and imaginary parts of D(R)).

Usage: python tests/golden/make_golden_kpoint.py   (THREADS: default all cores)
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

CASE = "diamond64_k222"
NK = (2, 2, 2)


def path_of(case=CASE):
    return os.path.join(HERE, f"{case}_oracle.npz")


def inputs(device="cpu"):
    """The cell, its blocks and the k-point density matrix of the case."""
    st = synth.workload(2).build()
    mats = st.materialize(device)
    Dk = synth.kpoint_density(st.n_tot, NK, st.seed + 6007)
    return st, mats, Dk


def fingerprint(mats, Dk):
    out = []
    for kind in ("C", "V"):
        for key, absval in (("val", False), ("dval", True)):
            x = mats[kind][key]
            out.append(float((x.abs() if absval else x).sum()))
    Dk = Dk.detach().cpu().numpy() if hasattr(Dk, "detach") else np.asarray(Dk)
    out += [float(Dk.real.sum()), float(Dk.imag.sum()), float(np.abs(Dk).sum())]
    return np.array(out)


def make(threads):
    st, mats, Dk = inputs()
    kp = oracle.KProblem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], NK, Dk)
    t0 = time.time()
    r = kp.evaluate(st.theta, nthreads=threads)
    dt = time.time() - t0
    np.savez_compressed(path_of(), E=r["E"], F=r["F"], sigma=r["sigma"], gC=r["gC"], gV=r["gV"],
                        keepC=np.packbits(r["keepC"] != 0), keepV=np.packbits(r["keepV"] != 0),
                        keepD=np.packbits(r["keepD"].reshape(-1)), nC=kp.nC, nV=kp.nV,
                        theta=st.theta, nk=np.array(NK), fingerprint=fingerprint(mats, Dk), seconds=dt,
                        threads=threads)
    print(f"{CASE}: E = {r['E']:.15e}, {dt:.0f} s on {threads} threads", flush=True)


def load():
    z = np.load(path_of(), allow_pickle=False)
    out = {k: z[k] for k in z.files}
    out["keepC"] = np.unpackbits(out["keepC"])[: int(out["nC"])]
    out["keepV"] = np.unpackbits(out["keepV"])[: int(out["nV"])]
    return out


if __name__ == "__main__":
    make(int(os.environ.get("THREADS", os.cpu_count() or 1)))
