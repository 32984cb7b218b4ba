"""Shared helpers of the parity tests (HIP path vs CPU oracle)."""
from __future__ import annotations

import functools
import os

import numpy as np

from paper_2412_11081_amd import synth

# Tolerances of the plain FP64 GPU path against the FP64 oracle.
TOL_E_PER_ATOM = 1e-8      # Ha per atom
TOL_F = 1e-5               # Ha/Bohr
TOL_SIGMA = 1e-6           # Ha/Bohr^3
# Both sides compute in FP64 and differ only in summation order, so the
# agreement is also required at this relative level.
REL_FP64 = 1e-9


def golden(case):
    """Stored oracle result of a workload (tests/golden/make_golden_big.py)."""
    from tests.golden import make_golden_big

    return make_golden_big.load(case)


def check_fingerprint(mats, ref):
    """The generated inputs are the ones the stored result was computed from."""
    from tests.golden import make_golden_big

    fp = make_golden_big.fingerprint(mats)
    assert np.allclose(fp, ref["fingerprint"], rtol=1e-10, atol=0), \
        f"inputs differ from the stored ones: {fp} vs {ref['fingerprint']}"


def nthreads():
    return int(os.environ.get("LRX_ORACLE_THREADS", min(16, os.cpu_count() or 1)))


def require_gpu():
    import pytest
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


@functools.lru_cache(maxsize=8)
def workload(k: int):
    st = synth.workload(k).build()
    return st


def block_sizes(st, kind, first, second):
    if kind == "C":
        return st.nabf[first] * st.nao[first] * st.nao[second]
    return st.nabf[first] * st.nabf[second]


def gather_blocks(st, blk, kind, idx):
    """Host copies of a subset of blocks (re-packed) for an oracle sub-problem."""
    import torch

    idx = np.asarray(idx, np.int64)
    first, second = np.asarray(blk["first"])[idx], np.asarray(blk["second"])[idx]
    R, off = np.asarray(blk["R"])[idx], np.asarray(blk["off"])[idx]
    sz = block_sizes(st, kind, first, second).astype(np.int64)
    new_off = np.concatenate([[0], np.cumsum(sz)[:-1]]).astype(np.int64)
    val, dval = blk["val"], blk["dval"]
    vparts, dparts = [], []
    for o, s in zip(off, sz):
        vparts.append(val[o:o + s])
        dparts.append(dval[3 * o:3 * (o + s)])
    v = torch.cat(vparts).cpu().numpy() if vparts else np.zeros(0)
    dv = torch.cat(dparts).cpu().numpy() if dparts else np.zeros(0)
    return dict(first=first, second=second, R=R, off=new_off, val=v, dval=dv)


def subproblem_for_block(st, mats, kind, b):
    """Oracle problem holding every block that can meet block b in a quartet
    and every block whose screening decision those quartets depend on.

    Returns (problem, local index of b)."""
    import oracle

    C, V = mats["C"], mats["V"]
    cf, vf, vs = np.asarray(C["first"]), np.asarray(V["first"]), np.asarray(V["second"])
    if kind == "V":
        A, B = int(vf[b]), int(vs[b])
        vsel = np.nonzero(((vf == A) & (vs == B)) | ((vf == B) & (vs == A)))[0]
        atoms = {A, B}
    else:
        A = int(cf[b])
        vsel = np.nonzero((vf == A) | (vs == A))[0]
        atoms = {A} | set(vf[vsel].tolist()) | set(vs[vsel].tolist())
    csel = np.nonzero(np.isin(cf, sorted(atoms)))[0]
    Cs = gather_blocks(st, C, "C", csel)
    Vs = gather_blocks(st, V, "V", vsel)
    pr = oracle.Problem(st.tau, st.lat, st.nao, st.nabf, Cs, Vs, st.D)
    local = int(np.nonzero((csel if kind == "C" else vsel) == b)[0][0])
    return pr, local


def oracle_block_gradient(st, mats, kind, b, theta, theta_cs):
    pr, loc = subproblem_for_block(st, mats, kind, b)
    keep = pr.screen(theta, theta_cs)
    _, gC, gV = pr.contract(keep, focus=(kind, loc), nthreads=nthreads())
    kept = bool((keep[0] if kind == "C" else keep[1])[loc])
    return (gC if kind == "C" else gV)[loc], kept


def gpu_context(st, mats):
    from paper_2412_11081_amd import lrx

    return lrx.context_for(st, mats)


def assert_close_fp64(name, got, ref, abs_tol):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    err = np.max(np.abs(got - ref)) if got.size else 0.0
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    assert err <= abs_tol, f"{name}: max abs error {err:.3e} > {abs_tol:.1e}"
    assert err <= REL_FP64 * max(scale, 1e-300) + 1e-300 or err <= 1e-14, \
        f"{name}: max abs error {err:.3e} exceeds {REL_FP64:.0e} x scale {scale:.3e}"
