"""Write the oracle's full results for the 64-, 320- and 1080-atom workloads.

Runs the CPU oracle only (no GPU code).  For each case it stores, in
``tests/golden/<case>_oracle.npz``: E, F[N][3], sigma[3][3], the per-block
gradients gC[nC][3] and gV[nV][3], the keep masks of C and V blocks and D
pairs (bit-packed), the number of V blocks that step 1 alone keeps (so a
test can state how many step 2 removed), the thresholds, the generator seed
and a fingerprint of the generated inputs (sums of the block values and of
D) that the tests compare before trusting the stored values.

Cases (the thresholds are the workloads' own unless stated):
  diamond64      64-atom diamond-like cell, theta 1e-4, theta_cs 1e-7
  diamond64_s2   the same cell with theta_cs = 0.3, where the Cauchy-Schwarz
                 step drops V blocks that step 1 keeps (Sec. Sparsity
                 exploitation, the Cauchy-Schwarz bound)
  abx3_320       320-atom ABX3 cell, theta 1e-4, theta_cs 1e-7
  abx3_1080      1080-atom strained, substituted ABX3 cell, theta 1e-5, theta_cs 1e-8
  diamond64_pt   the 64-atom cell with one threshold per tensor (Table
                 thr_default's five lists): C 1e-4, V 1e-2, D 1e-3, dC 1e-4,
                 dV 1e-3, theta_cs 1e-7; the keep masks are then bit masks
                 (1 value list, 2 derivative list)

Usage: python tests/golden/make_golden_big.py [case ...]   (default: all)
Threads: THREADS (default: all host cores).  The oracle parallelises over V
blocks with private accumulators summed in thread order, so the result does
not depend on the thread count beyond rounding of that final sum.
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

CASES = {
    "diamond64": (2, None),
    "diamond64_s2": (2, 0.3),
    "abx3_320": (3, None),
    "abx3_1080": (4, None),
    "diamond64_pt": (2, None),
}
# per-tensor thresholds (C, V, D, dC, dV) of the cases that use them
PER_TENSOR = {"diamond64_pt": (1e-4, 1e-2, 1e-3, 1e-4, 1e-3)}


def path_of(case):
    return os.path.join(HERE, f"{case}_oracle.npz")


def fingerprint(mats):
    """Sums of the generated inputs (C, |dC|, V, |dV|, D and its trace), taken
    in chunks on whatever device holds them; compared at a relative 1e-10, so
    the summation order does not matter."""
    out = []
    for kind in ("C", "V"):
        for key, absval in (("val", False), ("dval", True)):
            s = 0.0
            for part in mats[kind][key].split(1 << 26):
                s += float((part.abs() if absval else part).sum())
            out.append(s)
    D = mats["D"]
    out += [float(D.sum()), float(D.diagonal().sum())]
    return np.array(out)


def make(case, threads):
    k, theta_cs = CASES[case]
    st = synth.workload(k).build()
    if theta_cs is not None:
        st.theta_cs = theta_cs
    mats = st.materialize("cpu")
    pr = oracle.Problem.from_structure(st, mats)
    t0 = time.time()
    thr = PER_TENSOR.get(case)
    if thr is None:
        keep = pr.screen(st.theta, st.theta_cs)
        s1 = pr.screen(st.theta, 0.0)
        E, gC, gV = pr.contract(keep, nthreads=threads)
    else:
        keep = pr.screen5(thr, st.theta_cs)
        s1 = pr.screen5(thr, 0.0)
        E, gC, gV = pr.contract(keep, nthreads=threads, bits=True)
    F, sig = pr.forces_stress(gC, gV)
    dt = time.time() - t0
    np.savez_compressed(
        path_of(case),
        case=case, workload=k, seed=st.seed, theta=st.theta, theta_cs=st.theta_cs,
        natom=st.natom, nC=pr.nC, nV=pr.nV,
        E=E, F=F, sigma=sig, gC=gC, gV=gV,
        keepC=keep[0] if thr else np.packbits(keep[0]), keepV=keep[1] if thr else np.packbits(keep[1]),
        keepD=np.packbits(keep[2]), kept_v_step1=int((s1[1] != 0).sum()),
        thresholds=np.array(thr if thr else [st.theta] * 5),
        fingerprint=fingerprint(mats),
        oracle_seconds=dt, oracle_threads=threads,
        written_by="tests/golden/make_golden_big.py (CPU oracle only)",
    )
    print(f"{case}: E = {E:.15e}, kept C {int((keep[0] != 0).sum())}/{pr.nC}, kept V {int((keep[1] != 0).sum())}/{pr.nV} "
          f"(step 1 alone {int((s1[1] != 0).sum())}), max|F| {np.abs(F).max():.3e}, oracle {dt:.1f} s on {threads} threads",
          flush=True)


def load(case):
    """The stored result as a dict, masks unpacked to uint8 arrays."""
    z = np.load(path_of(case), allow_pickle=False)
    r = {k: z[k] for k in z.files}
    if str(r["case"]) not in PER_TENSOR:   # bit masks are stored as they are
        r["keepC"] = np.unpackbits(r["keepC"])[: int(r["nC"])]
        r["keepV"] = np.unpackbits(r["keepV"])[: int(r["nV"])]
    n = int(r["natom"])
    r["keepD"] = np.unpackbits(r["keepD"])[: n * n]
    r["E"] = float(r["E"])
    return r


def main():
    oracle.build(force=False)
    threads = int(os.environ.get("THREADS", os.cpu_count() or 1))
    for case in sys.argv[1:] or list(CASES):
        make(case, threads)


if __name__ == "__main__":
    main()
