"""Preparation of C and dC on the GPU (lrx_prepare_c; Eq. C_VA and the
gradient after Eq. V_inverse) against the oracle (oracle/prepare.py).

Small cells: every element of C and dC, from host and from device inputs
(bit-identical); the prepared C then drives lrx_evaluate, whose E, F and
sigma match the oracle's contraction of the oracle-prepared C.  The 64- and
1080-atom workloads: sampled keys against the oracle's solve of those keys.
Bad inputs (a missing V block, a Coulomb matrix that is not positive
definite) are refused.
"""
import numpy as np
import pytest

from oracle import prepare as prep
from paper_2412_11081_amd import lrx, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

# (natom, nspecies, n_ao, n_abf, box, rc, rv, seed)
CELLS = [
    (3, 2, 3, 5, 7.0, 5.5, 9.0, 51),
    (4, 3, 7, 20, 8.0, 5.0, 8.0, 52),
    (2, 1, 13, 40, 9.0, 5.0, 8.0, 53),
    (3, 2, 22, 33, 9.0, 5.0, 8.0, 54),
    (2, 1, 3, 100, 7.0, 5.0, 8.0, 56),   # four pair keys of n = 200: the LDS triangle near its 201-row limit
    (2, 1, 3, 110, 7.0, 5.0, 8.0, 55),   # four pair keys of n = 220 > 201: M in the device workspace
]
REL = 1e-10


def _cell(c):
    natom, nsp, nao, nabf, box, rc, rv, seed = c
    st = synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=rc, rv=rv, seed=seed).build()
    return st


def _np(x):
    return x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)


@pytest.mark.parametrize("cell", CELLS, ids=[f"n{c[0]}s{c[1]}ao{c[2]}abf{c[3]}" for c in CELLS])
def test_small_cells_every_element(cell):
    H.require_gpu()
    st = _cell(cell)
    mh = st.materialize("cpu")
    Th = synth.three_center(st, "cpu")
    off, val, dval = prep.prepare_c(st.nao, st.nabf, mh["V"], Th)
    print(f"cell {cell}: {len(off)} keys, max|C| {np.abs(val).max():.3e}, max|dC| {np.abs(dval).max():.3e}", flush=True)
    gh, fl = lrx.prepare_c(st.nao, st.nabf, mh["V"], Th)        # host inputs
    md = st.materialize("cuda")
    Td = synth.three_center(st, "cuda")
    gd, _ = lrx.prepare_c(st.nao, st.nabf, md["V"], Td)          # device inputs
    assert fl > 0
    np.testing.assert_array_equal(gh["off"], off)
    for name, got, ref in (("C", gh["val"], val), ("dC", gh["dval"], dval)):
        err = float(np.max(np.abs(got - ref)))
        print(f"  {name}: max abs error {err:.3e} (scale {np.abs(ref).max():.3e})", flush=True)
        assert err <= REL * np.abs(ref).max() + 1e-15, name
    assert np.array_equal(_np(gd["val"]), gh["val"]) and np.array_equal(_np(gd["dval"]), gh["dval"])


def test_prepared_c_drives_the_evaluation(oracle_lib):
    """The prepared C as the input of the forces: E, F, sigma against the
    oracle's contraction of the oracle-prepared C (on-site blocks pass the
    library's symmetry check)."""
    H.require_gpu()
    st = _cell(CELLS[1])
    md = st.materialize("cuda")
    Td = synth.three_center(st, "cuda")
    Cg, _ = lrx.prepare_c(st.nao, st.nabf, md["V"], Td)
    mh = st.materialize("cpu")
    off, val, dval = prep.prepare_c(st.nao, st.nabf, mh["V"], synth.three_center(st, "cpu"))
    Cref = dict(first=mh["C"]["first"], second=mh["C"]["second"], R=mh["C"]["R"], off=off, val=val, dval=dval)
    r = oracle_lib.Problem(st.tau, st.lat, st.nao, st.nabf, Cref, mh["V"], st.D).evaluate(0.0, 0.0)
    ctx = lrx.Context()
    ctx.set_structure(st.tau, st.lat, st.nao, st.nabf)
    ctx.set_tensors(Cg, md["V"], md["D"])
    E, F, S = ctx.evaluate(0.0, 0.0)
    ctx.close()
    print(f"E {E:.12e} oracle {r['E']:.12e}", flush=True)
    H.assert_close_fp64("E", E, r["E"], H.TOL_E_PER_ATOM * st.natom)
    H.assert_close_fp64("F", F, r["F"], H.TOL_F)
    H.assert_close_fp64("sigma", S, r["sigma"], H.TOL_SIGMA)


@pytest.mark.parametrize("k", [2, 4])
def test_workload_sampled_keys(k):
    H.require_gpu()
    st = H.workload(k)
    md = st.materialize("cuda")
    Td = synth.three_center(st, "cuda")
    Cg, fl = lrx.prepare_c(st.nao, st.nabf, md["V"], Td)
    print(f"workload {k}: {len(Cg['off'])} keys, {fl:.3e} FLOP", flush=True)
    vh = {key: _np(v) if key in ("val", "dval") else v for key, v in md["V"].items()}
    th = {key: _np(v) if key in ("val", "dval") else v for key, v in Td.items()}
    vidx = prep._vkeys(vh)
    first = np.asarray(Td["first"])
    rng = np.random.default_rng(9)
    gv, gdv = _np(Cg["val"]), _np(Cg["dval"])
    for b in [0] + [int(i) for i in rng.integers(0, first.shape[0], 12)]:
        A, F = int(first[b]), int(np.asarray(Td["second"])[b])
        mA = st.nabf[A]
        C, dC = prep.solve_pair(st.nao, st.nabf, vh, vidx, th, b)
        n = mA * st.nao[A] * st.nao[F]
        o = int(Cg["off"][b])
        got = gv[o:o + n]
        gotd = gdv[3 * o:3 * (o + n)].reshape(3, -1)
        ref, refd = C[:mA].reshape(-1), dC[:, :mA].reshape(3, -1)
        e1 = float(np.max(np.abs(got - ref))) / float(np.abs(ref).max())
        e2 = float(np.max(np.abs(gotd - refd))) / max(float(np.abs(refd).max()), 1e-300)
        print(f"  key {b} ({A},{F}): relative errors C {e1:.2e} dC {e2:.2e}", flush=True)
        assert e1 <= REL and (e2 <= REL or not refd.any())


def test_rejected_inputs():
    H.require_gpu()
    st = _cell(CELLS[0])
    mh = st.materialize("cpu")
    T = synth.three_center(st, "cpu")
    # a Coulomb matrix that is not positive definite: V scaled so that its
    # off-site blocks dominate the on-site ones
    V = dict(mh["V"])
    vf, vs = np.asarray(V["first"]), np.asarray(V["second"])
    val = _np(V["val"]).copy()
    for i in range(vf.shape[0]):
        if vf[i] != vs[i]:
            n = st.nabf[vf[i]] * st.nabf[vs[i]]
            o = int(V["off"][i])
            val[o:o + n] *= 1e3
    V["val"] = val
    with pytest.raises(lrx.LrxError):
        lrx.prepare_c(st.nao, st.nabf, V, T)
    # a missing V block: drop the on-site block of atom 0
    keep = np.nonzero(~((vf == 0) & (vs == 0) & ~np.asarray(mh["V"]["R"]).any(axis=1)))[0]
    V2 = dict(first=vf[keep], second=vs[keep], R=np.asarray(mh["V"]["R"])[keep], off=np.asarray(mh["V"]["off"])[keep],
              val=_np(mh["V"]["val"]), dval=_np(mh["V"]["dval"]))
    with pytest.raises(lrx.LrxError):
        lrx.prepare_c(st.nao, st.nabf, V2, T)
