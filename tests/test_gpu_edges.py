"""Edge cases of the HIP path, through the C-ABI, against the CPU oracle:
everything screened away, D blocks screened under live triples, a cell of
one atom (only its own images), the largest block sizes the kernels take
(32 NAOs and 128 ABFs per atom: eight alpha tiles, H slices too large for
the LDS stage), and inputs the library must reject with an error instead of
computing (non-finite values, broken symmetries, block sizes and C partner
counts beyond the kernels)."""
import numpy as np
import pytest

from paper_2412_11081_amd import lrx, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _both(oracle_lib, st, theta, theta_cs):
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    E, F, S = ctx.evaluate(theta, theta_cs)
    gC, gV = ctx.block_gradients()
    keep = ctx.keep_masks()
    ctx.close()
    r = oracle_lib.Problem.from_structure(st, mats).evaluate(theta, theta_cs, nthreads=H.nthreads())
    return (E, F, S, gC, gV, keep), r


def _check(st, got, r):
    E, F, S, gC, gV, keep = got
    np.testing.assert_array_equal(keep[0], r["keepC"])
    np.testing.assert_array_equal(keep[1], r["keepV"])
    np.testing.assert_array_equal(keep[2], r["keepD"])
    H.assert_close_fp64("E", E, r["E"], H.TOL_E_PER_ATOM * st.natom)
    H.assert_close_fp64("F", F, r["F"], H.TOL_F)
    H.assert_close_fp64("sigma", S, r["sigma"], H.TOL_SIGMA)
    H.assert_close_fp64("gC", gC, r["gC"], H.TOL_F)
    H.assert_close_fp64("gV", gV, r["gV"], H.TOL_F)


def test_everything_screened(oracle_lib):
    """A threshold above every block: no block, pair or triple survives; E, F,
    sigma and every gradient are exactly zero, as in the oracle."""
    H.require_gpu()
    st = synth.small_case(natom=3, nspecies=2, n_ao=5, n_abf=17, box=6.5, rc=5.0, rv=8.0, seed=41).build()
    got, r = _both(oracle_lib, st, 1e6, 1e3)
    E, F, S, gC, gV, keep = got
    assert E == 0.0 and not F.any() and not S.any() and not gC.any() and not gV.any()
    assert not keep[0].any() and not keep[1].any() and not keep[2].any()
    _check(st, got, r)


@pytest.mark.parametrize("case", [(4, 2, 3, 9, 6.0, 51, 0.3), (5, 2, 4, 11, 6.5, 52, 0.2)],
                         ids=["n4ao3th0.3", "n5ao4th0.2"])
def test_partially_screened_density_blocks(oracle_lib, case):
    """A threshold that screens some D blocks while C and V blocks survive:
    live triples whose D(A,B) or D(F,B) is screened take that term as zero."""
    H.require_gpu()
    natom, nsp, nao, nabf, box, seed, theta = case
    st = synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=4.5, rv=7.0, seed=seed,
                          theta=theta, theta_cs=0.0).build()
    got, r = _both(oracle_lib, st, theta, 0.0)
    kD = np.asarray(r["keepD"]).reshape(natom, natom)
    cA, cF, _ = st.keysC
    vA, vB, _ = st.keysV
    live_c = {(int(a), int(f)) for a, f, k in zip(cA, cF, r["keepC"]) if k}
    live_v = {(int(a), int(b)) for a, b, k in zip(vA, vB, r["keepV"]) if k}
    touched = sum(1 for a, f in live_c for a2, b in live_v if a2 == a and not (kD[a, b] and kD[f, b]))
    print("live triples with a screened D block:", touched, flush=True)
    assert touched > 0 and r["E"] != 0.0
    _check(st, got, r)


def test_empty_v_list():
    """No V blocks at all (an empty list is valid input): no triple exists,
    so E, F, sigma and every C-block gradient are exactly zero."""
    H.require_gpu()
    import torch

    st, m = _fresh(45)
    V = dict(first=np.zeros(0, np.int32), second=np.zeros(0, np.int32), R=np.zeros((0, 3), np.int32),
              off=np.zeros(0, np.int64), val=torch.zeros(0, dtype=torch.float64, device="cuda"),
              dval=torch.zeros(0, dtype=torch.float64, device="cuda"))
    ctx = lrx.Context(0)
    ctx.set_structure(st.tau, st.lat, st.nao, st.nabf)
    ctx.set_tensors(m["C"], V, m["D"])
    for prec in ("fp64", "bf16x3"):
        E, F, S = ctx.evaluate(0.0, 0.0, precision=prec)
        gC, gV = ctx.block_gradients()
        assert E == 0.0 and not F.any() and not S.any() and not gC.any() and gV.size == 0, prec
    ctx.close()


def test_single_atom_cell(oracle_lib):
    """One atom: every block is an image of the atom itself (force-free by
    symmetry up to rounding, stress from the image displacements)."""
    H.require_gpu()
    st = synth.small_case(natom=1, nspecies=1, n_ao=7, n_abf=23, box=4.0, rc=5.0, rv=7.5, seed=42).build()
    print("blocks", len(st.keysC[0]), len(st.keysV[0]), flush=True)
    got, r = _both(oracle_lib, st, 0.0, 0.0)
    _check(st, got, r)
    assert np.max(np.abs(got[1])) <= 1e-10 * max(1.0, np.abs(got[2]).max())


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_largest_blocks(oracle_lib, prec):
    """32 NAOs and 128 ABFs on every atom: eight alpha tiles, the widest
    column chunks, and H slices that exceed the LDS stage (read from HBM)."""
    H.require_gpu()
    st = synth.small_case(natom=2, nspecies=1, n_ao=32, n_abf=128, box=7.0, rc=4.5, rv=6.0, seed=43).build()
    print("blocks", len(st.keysC[0]), len(st.keysV[0]), flush=True)
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    E, F, S = ctx.evaluate(0.0, 0.0, precision=prec)
    gC, gV = ctx.block_gradients()
    keep = ctx.keep_masks()
    ctx.close()
    r = oracle_lib.Problem.from_structure(st, mats).evaluate(0.0, 0.0, nthreads=H.nthreads())
    if prec == "fp64":
        _check(st, (E, F, S, gC, gV, keep), r)
    else:
        # the BF16x3 bounds of tests/test_gpu_precision.py
        from tests.test_gpu_precision import _check_all

        _check_all("bf16x3", (E, F, S, gC, gV), r)


def _fresh(seed=44):
    st = synth.small_case(natom=2, nspecies=1, n_ao=3, n_abf=5, box=6.0, rc=4.5, rv=7.0, seed=seed).build()
    return st, st.materialize("cuda")


def _expect_rejected(st, C, V, D, words):
    ctx = lrx.Context(0)
    ctx.set_structure(st.tau, st.lat, st.nao, st.nabf)
    with pytest.raises(lrx.LrxError) as e:
        ctx.set_tensors(C, V, D)
    msg = str(e.value)
    print("rejected:", msg, flush=True)
    assert any(w in msg for w in words), msg
    ctx.close()


def test_non_finite_values_are_rejected():
    H.require_gpu()
    st, m = _fresh()
    C = dict(m["C"])
    C["val"] = m["C"]["val"].clone()
    C["val"][3] = float("nan")
    _expect_rejected(st, C, m["V"], m["D"], ["finite", "NaN", "nan"])


def test_non_finite_v_values_are_rejected():
    """V and dV are checked for finiteness in the mirror pass."""
    H.require_gpu()
    st, m = _fresh()
    V = dict(m["V"])
    V["val"] = m["V"]["val"].clone()
    V["val"][-1] = float("nan")
    _expect_rejected(st, m["C"], V, m["D"], ["non-finite V"])
    V = dict(m["V"])
    V["dval"] = m["V"]["dval"].clone()
    V["dval"][2] = float("inf")
    _expect_rejected(st, m["C"], V, m["D"], ["non-finite V"])


def test_v_block_without_mirror_is_rejected():
    """A V block whose (second, first, -R) partner is missing: one block moved
    to a far image breaks the pairing in both directions."""
    H.require_gpu()
    st, m = _fresh()
    V = dict(m["V"])
    R = np.array(V["R"], dtype=np.int32).reshape(-1, 3).copy()
    R[0, 0] += 1000
    V["R"] = R
    _expect_rejected(st, m["C"], V, m["D"], ["mirror"])


def test_asymmetric_density_matrix_is_rejected():
    H.require_gpu()
    st, m = _fresh()
    D = m["D"].clone()
    D[0, 1] += 1e-3
    _expect_rejected(st, m["C"], m["V"], D, ["D", "symmetric"])


def test_broken_v_mirror_is_rejected():
    H.require_gpu()
    st, m = _fresh()
    V = dict(m["V"])
    V["val"] = m["V"]["val"].clone()
    # an off-diagonal element of the first block: its mirror block no longer matches
    V["val"][1] += 1e-3
    _expect_rejected(st, m["C"], V, m["D"], ["mirror", "V"])


def test_block_sizes_beyond_the_kernels_are_rejected():
    H.require_gpu()
    ctx = lrx.Context(0)
    tau = np.zeros((1, 3))
    with pytest.raises(lrx.LrxError):
        ctx.set_structure(tau, np.eye(3) * 5.0, np.array([33], np.int32), np.array([10], np.int32))
    with pytest.raises(lrx.LrxError):
        ctx.set_structure(tau, np.eye(3) * 5.0, np.array([10], np.int32), np.array([129], np.int32))
    ctx.close()


def test_too_many_c_partners_are_rejected():
    """Every C pair takes at least one of the 64 column chunks an atom may
    have, so an atom with more than 64 C partners is refused (the per-slot
    lists of the Hamiltonian rely on that bound)."""
    H.require_gpu()
    # 130 one-NAO atoms in a cell of side 8.5 +- 0.3 Bohr: every pair has an
    # image closer than 8.8 sqrt(3) / 2 < 8 Bohr, so every atom has 130 C
    # partners (130 NAOs, within the depth limit of 508)
    st = synth.small_case(natom=130, n_ao=1, n_abf=1, box=8.5, rc=8.0, rv=8.0, seed=41).build()
    m = st.materialize("cuda")
    _expect_rejected(st, m["C"], m["V"], m["D"], ["64 C-pair column chunks"])
