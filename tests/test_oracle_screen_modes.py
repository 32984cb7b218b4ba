"""Pins of the oracle's paper-literal screening modes (CPU only).

* Per-tensor thresholds (Table thr_default: C, V, D, dC, dV): each term uses
  its own lists, so the screened result equals the unscreened result on
  inputs where exactly the dropped parts are zero (values outside the value
  lists, derivatives outside the derivative lists, D blocks of dropped
  pairs); the energy also equals the brute-force 4-index energy of those
  inputs.
* The item-level Cauchy-Schwarz test (Algorithm 1, Sec. Sparsity
  exploitation): at theta_item = 0 nothing changes; above it, the energy
  moves by at most the sum of the bounds of the skipped items, that sum is
  at most theta_item per skipped item, and it grows with theta_item.
"""
import numpy as np
import pytest

from paper_2412_11081_amd import synth
from tests import ref_bruteforce as bf


def _case(seed=19):
    st = synth.small_case(natom=4, seed=seed, nspecies=2, n_ao=3, n_abf=4, box=7.0, rc=5.5, rv=9.0).build()
    return st, st.materialize("cpu")


def _zeroed(st, mats, kC, kV, kD):
    m2 = {}
    for tag, keep in (("C", kC), ("V", kV)):
        blk = dict(mats[tag])
        val, dval = blk["val"].clone(), blk["dval"].clone()
        for b in range(len(keep)):
            f, s_ = blk["first"][b], blk["second"][b]
            sz = st.nabf[f] * st.nao[f] * st.nao[s_] if tag == "C" else st.nabf[f] * st.nabf[s_]
            o = blk["off"][b]
            if not keep[b] & 1:
                val[o:o + sz] = 0
            if not keep[b] & 2:
                dval[3 * o:3 * (o + sz)] = 0
        blk["val"], blk["dval"] = val, dval
        m2[tag] = blk
    D = st.D.copy()
    N = st.natom
    for X in range(N):
        for Y in range(N):
            if not kD[X * N + Y]:
                D[st.ao_off[X]:st.ao_off[X + 1], st.ao_off[Y]:st.ao_off[Y + 1]] = 0
    return m2, D


@pytest.mark.parametrize("thr", [(3e-3, 2e-2, 1e-1, 5e-3, 3e-2), (1e-3, 0.0, 0.3, 0.0, 5e-2), (0.0, 5e-2, 0.0, 2e-2, 0.0)])
def test_per_tensor_lists_equal_unscreened_with_dropped_parts_zeroed(oracle_lib, thr):
    st, mats = _case()
    pr = oracle_lib.Problem.from_structure(st, mats)
    r = pr.evaluate5(thr, 0.0)
    kC, kV, kD = r["keepC"], r["keepV"], r["keepD"]
    # the thresholds split the lists: some blocks keep only the value or only the derivative
    print("C bits", np.bincount(kC, minlength=4), "V bits", np.bincount(kV, minlength=4), "D kept", kD.sum())
    assert len(set(kC.tolist()) | set(kV.tolist())) >= 3
    m2, D = _zeroed(st, mats, kC, kV, kD)
    r0 = oracle_lib.Problem(st.tau, st.lat, st.nao, st.nabf, m2["C"], m2["V"], D).evaluate(0.0, 0.0)
    assert abs(r0["E"] - r["E"]) <= 1e-12 * abs(r["E"])
    np.testing.assert_allclose(r["F"], r0["F"], rtol=0, atol=1e-12 * np.abs(r0["F"]).max() + 1e-15)
    np.testing.assert_allclose(r["sigma"], r0["sigma"], rtol=0, atol=1e-12 * np.abs(r0["sigma"]).max() + 1e-15)
    assert abs(bf.energy_assoc(st, m2, D=D) - r["E"]) <= 1e-11 * abs(r["E"])


def test_per_tensor_zero_thresholds_are_the_plain_contraction(oracle_lib):
    st, mats = _case(20)
    pr = oracle_lib.Problem.from_structure(st, mats)
    a = pr.evaluate5((0.0,) * 5, 0.0)
    b = pr.evaluate(0.0, 0.0)
    assert a["E"] == b["E"] and np.array_equal(a["F"], b["F"]) and np.array_equal(a["sigma"], b["sigma"])
    assert (a["keepC"] == 3).all() and (a["keepV"] == 3).all()


def test_item_level_cauchy_schwarz_test(oracle_lib):
    st, mats = _case(21)
    pr = oracle_lib.Problem.from_structure(st, mats)
    keep = pr.screen(0.0, 0.0)
    E0, gC0, gV0 = pr.contract(keep)
    E00, _, _ = pr.contract(keep, theta_item=0.0)
    assert E00 == E0 and pr.skipped_bound == 0.0
    prev = 0.0
    skipped_any = False
    for t in (1e-6, 1e-5, 1e-4, 1e-3, 1e-2):
        E, gC, gV = pr.contract(keep, theta_item=t)
        sb = pr.skipped_bound
        print(f"theta_item {t:.0e}: |dE| {abs(E - E0):.3e}, sum of skipped bounds {sb:.3e}")
        assert abs(E - E0) <= sb * (1 + 1e-12) + 1e-15
        assert sb >= prev
        prev = sb
        skipped_any = skipped_any or sb > 0
    assert skipped_any
