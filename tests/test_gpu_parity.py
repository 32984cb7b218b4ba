"""HIP path (through the C-ABI) against the CPU oracle.

Small cells: every output element (E, F, sigma, per-block gradients, keep
masks) against the oracle run live.  The 8-atom workload: against the stored
oracle result.  The 64-, 320- and 1080-atom workloads: per-block gradients of
sampled blocks against the oracle restricted to the quartets that contain
them, the keep masks of those blocks, and properties that hold at any size.
"""
import json
import os

import numpy as np
import pytest

from paper_2412_11081_amd import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sc8_oracle.json")


def _gpu(st, mats, theta, theta_cs):
    ctx = H.gpu_context(st, mats)
    E, F, S = ctx.evaluate(theta, theta_cs)
    gC, gV = ctx.block_gradients()
    kC, kV, kD = ctx.keep_masks()
    st_ = ctx.stats()
    ctx.close()
    return dict(E=E, F=F, sigma=S, gC=gC, gV=gV, keepC=kC, keepV=kV, keepD=kD, stats=st_)


# (natom, nspecies, n_ao, n_abf, box, rc, rv, theta, seed): tails of every tile
# size, several species, images of the atom itself, screening on and off.
SMALL = [
    (2, 1, 3, 5, 6.0, 4.5, 7.0, 0.0, 31),
    (3, 2, 5, 17, 6.5, 5.0, 8.0, 0.0, 32),
    (3, 2, 13, 33, 7.0, 5.0, 8.0, 1e-4, 33),
    (4, 3, 7, 20, 5.5, 4.5, 7.5, 2e-3, 34),
    (2, 1, 22, 40, 9.0, 5.0, 8.0, 0.0, 35),
    (3, 1, 18, 100, 12.0, 5.0, 7.0, 0.0, 36),
    (2, 2, 16, 64, 3.6, 4.0, 5.0, 0.0, 37),
    (2, 1, 9, 75, 7.5, 5.0, 8.0, 0.0, 38),      # five alpha tiles: the last one reduced a quarter per Z wave
    (2, 2, 11, 90, 8.0, 5.0, 8.0, 1e-4, 39),    # six alpha tiles
]


@pytest.mark.parametrize("case", SMALL, ids=[f"n{c[0]}s{c[1]}ao{c[2]}abf{c[3]}th{c[7]}" for c in SMALL])
def test_small_cells_every_element(oracle_lib, case):
    H.require_gpu()
    natom, nsp, nao, nabf, box, rc, rv, theta, seed = case
    st = synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=rc, rv=rv,
                          seed=seed, theta=theta, theta_cs=1e-3 * theta, jitter=0.5).build()
    print(f"case {case}: nC={len(st.keysC[0])} nV={len(st.keysV[0])}", flush=True)
    mats = st.materialize("cuda")
    g = _gpu(st, mats, st.theta, st.theta_cs)
    r = oracle_lib.Problem.from_structure(st, mats).evaluate(st.theta, st.theta_cs, nthreads=H.nthreads())
    np.testing.assert_array_equal(g["keepC"], r["keepC"])
    np.testing.assert_array_equal(g["keepV"], r["keepV"])
    np.testing.assert_array_equal(g["keepD"], r["keepD"])
    H.assert_close_fp64("E", g["E"], r["E"], H.TOL_E_PER_ATOM * st.natom)
    H.assert_close_fp64("F", g["F"], r["F"], H.TOL_F)
    H.assert_close_fp64("sigma", g["sigma"], r["sigma"], H.TOL_SIGMA)
    H.assert_close_fp64("gC", g["gC"], r["gC"], H.TOL_F)
    H.assert_close_fp64("gV", g["gV"], r["gV"], H.TOL_F)


def test_tiny_cubic_against_stored_oracle():
    """The 8-atom workload (13 NAO / 40 ABF, no screening) in full."""
    H.require_gpu()
    ref = json.load(open(GOLDEN))
    st = H.workload(1)
    mats = st.materialize("cuda")
    g = _gpu(st, mats, 0.0, 0.0)
    assert g["gC"].shape[0] == ref["nC"] and g["gV"].shape[0] == ref["nV"]
    H.assert_close_fp64("E", g["E"], ref["E"], H.TOL_E_PER_ATOM * st.natom)
    H.assert_close_fp64("F", g["F"], ref["F"], H.TOL_F)
    H.assert_close_fp64("sigma", g["sigma"], ref["sigma"], H.TOL_SIGMA)
    H.assert_close_fp64("gC", g["gC"], ref["gC"], H.TOL_F)
    H.assert_close_fp64("gV", g["gV"], ref["gV"], H.TOL_F)


def test_repeat_is_bitwise_identical():
    """No atomics in any reduction: two evaluations agree bit for bit."""
    H.require_gpu()
    st = H.workload(1)
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    a = ctx.evaluate(0.0, 0.0)
    b = ctx.evaluate(0.0, 0.0)
    ctx.close()
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def _sampled(st, mats, nsample, seed):
    g = _gpu(st, mats, st.theta, st.theta_cs)
    rng = np.random.default_rng(seed)
    nC, nV = g["gC"].shape[0], g["gV"].shape[0]
    # properties that hold at any size
    assert np.max(np.abs(g["F"].sum(axis=0))) <= 1e-10 * max(1.0, np.abs(g["F"]).max())
    assert np.max(np.abs(g["sigma"] - g["sigma"].T)) <= 1e-10 * np.abs(g["sigma"]).max()
    # forces and stress are the scatter of the block gradients
    Fh = np.zeros_like(g["F"])
    W = np.zeros((3, 3))
    for kind, gr in (("C", g["gC"]), ("V", g["gV"])):
        blk = mats[kind]
        f, s = np.asarray(blk["first"]), np.asarray(blk["second"])
        np.add.at(Fh, f, gr)
        np.add.at(Fh, s, -gr)
        W += gr.T @ blk["disp"]
    H.assert_close_fp64("F from gradients", g["F"], Fh, H.TOL_F)
    H.assert_close_fp64("sigma from gradients", g["sigma"], -W / st.volume, H.TOL_SIGMA)
    picks = [("C", int(b)) for b in rng.choice(nC, size=min(nsample, nC), replace=False)]
    picks += [("V", int(b)) for b in rng.choice(nV, size=min(nsample, nV), replace=False)]
    for kind, b in picks:
        ref, kept = H.oracle_block_gradient(st, mats, kind, b, st.theta, st.theta_cs)
        got = (g["gC"] if kind == "C" else g["gV"])[b]
        assert bool((g["keepC"] if kind == "C" else g["keepV"])[b]) == kept, (kind, b)
        H.assert_close_fp64(f"g{kind}[{b}]", got, ref, H.TOL_F)
    return g


def test_diamond64_sampled_blocks():
    H.require_gpu()
    st = H.workload(2)
    mats = st.materialize("cuda")
    _sampled(st, mats, 3, 2)


def test_perovskite320_sampled_blocks():
    H.require_gpu()
    st = H.workload(3)
    mats = st.materialize("cuda")
    _sampled(st, mats, 3, 3)


def test_perovskite1080_sampled_blocks():
    """The 1080-atom workload in the configuration the benchmark times."""
    H.require_gpu()
    st = H.workload(4)
    mats = st.materialize("cuda")
    _sampled(st, mats, 2, 4)
