"""k-point sampling on the HIP path (lrx_set_kpoint_tensors) against the
oracle's k-point form (oracle.KProblem; Methods, Eq. Eexx with the k-sum
definition of D, and Eq. exx_expand).

The library runs its Gamma-point kernels on the Born-von Karman supercell's
home-cell rows with a block-circulant D, one real pass per part of a complex
D.  Compared element by element with the oracle, which reads every D slot at
its own cell offset with no folding:

  * E, F, sigma and the per-block gradients, real and complex D, several
    meshes (offsets that differ from their negatives need nk > 2), cells whose
    atoms span one to six 16-row ABF tiles, unscreened and screened (joint
    theta; per-tensor thresholds with the D pairs decided per offset on |D|);
  * the keep masks, keepD mapped from supercell atom pairs to (offset, X, Y);
  * host and device inputs bit for bit; nk = (1,1,1) bit for bit equal to the
    Gamma-point entry point; the 64-atom cell on a 2 x 2 x 2 mesh and the
    8-atom cell on a 3 x 3 x 1 mesh against stored oracle results;
  * refused inputs: a D that is not Hermitian, theta_cs > 0, and the entry
    points that do not take k-point contexts.
"""
import numpy as np
import pytest

from paper_2412_11081_amd import lrx, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

CELLS = [  # (natom, nspecies, n_ao, n_abf, box, rc, rv, seed, nk)
    (2, 1, 3, 4, 5.0, 4.0, 6.0, 71, (2, 1, 1)),
    (3, 2, 5, 20, 6.5, 5.0, 7.5, 91, (2, 2, 1)),
    (2, 2, 13, 40, 7.0, 5.0, 8.0, 92, (1, 1, 3)),
    (4, 2, 7, 33, 7.5, 5.0, 8.0, 93, (2, 2, 2)),
    (2, 1, 11, 90, 8.0, 5.0, 8.0, 94, (3, 1, 1)),
    (3, 1, 4, 9, 5.5, 4.5, 6.5, 95, (2, 3, 1)),
]
IDS = [f"n{c[0]}ao{c[2]}abf{c[3]}nk{''.join(map(str, c[8]))}" for c in CELLS]


def _cell(c):
    natom, nsp, nao, nabf, box, rc, rv, seed, nk = c
    st = synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=rc, rv=rv, seed=seed).build()
    return st, nk


def _dk(st, nk, trs):
    Dk = synth.kpoint_density(st.n_tot, nk, st.seed + 5, trs=trs)
    return Dk.real.copy() if trs else Dk


def _gpu(st, mats, nk, Dk, theta=0.0, thresholds=None, precision="fp64", device=True):
    import torch

    ctx = lrx.Context()
    ctx.set_structure(st.tau, st.lat, st.nao, st.nabf)
    D = torch.from_numpy(Dk).to("cuda") if device else Dk
    ctx.set_kpoint_tensors(nk, mats["C"], mats["V"], D)
    E, F, S = ctx.evaluate(theta, 0.0, precision=precision, thresholds=thresholds)
    gC, gV = ctx.block_gradients()
    kC, kV, kD = ctx.keep_masks()
    ctx.close()
    return dict(E=E, F=F, sigma=S, gC=gC, gV=gV, keepC=kC, keepV=kV, keepD=kD)


def _keepd_by_offset(kD, natom, nk):
    """Supercell pairs ((t, X), (u, Y)) -> [offset u - t][X][Y]; every cell t
    must give the same answer."""
    ncell = int(np.prod(nk))
    ns = natom * ncell
    kD = kD.reshape(ns, ns)
    cells = [(r0, r1, r2) for r2 in range(nk[2]) for r1 in range(nk[1]) for r0 in range(nk[0])]
    out = np.full((ncell, natom, natom), 255, np.uint8)
    for ti, t in enumerate(cells):
        for ui, u in enumerate(cells):
            d = [(u[k] - t[k]) % nk[k] for k in range(3)]
            r = d[0] + nk[0] * (d[1] + nk[1] * d[2])
            blk = kD[ti * natom:(ti + 1) * natom, ui * natom:(ui + 1) * natom]
            assert out[r].max() == 255 or np.array_equal(out[r], blk), "keepD differs between cells"
            out[r] = blk
    return out


def _compare(g, r, st, nk, bits=False):
    if bits:
        np.testing.assert_array_equal(g["keepC"], r["keepC"])
        np.testing.assert_array_equal(g["keepV"], r["keepV"])
    else:
        np.testing.assert_array_equal(g["keepC"] != 0, r["keepC"] != 0)
        np.testing.assert_array_equal(g["keepV"] != 0, r["keepV"] != 0)
    np.testing.assert_array_equal(_keepd_by_offset(g["keepD"], st.natom, nk), r["keepD"])
    H.assert_close_fp64("E", g["E"], r["E"], H.TOL_E_PER_ATOM * st.natom)
    H.assert_close_fp64("F", g["F"], r["F"], H.TOL_F)
    H.assert_close_fp64("sigma", g["sigma"], r["sigma"], H.TOL_SIGMA)
    H.assert_close_fp64("gC", g["gC"], r["gC"], H.TOL_F)
    H.assert_close_fp64("gV", g["gV"], r["gV"], H.TOL_F)


@pytest.mark.parametrize("cell", CELLS, ids=IDS)
@pytest.mark.parametrize("trs", [True, False], ids=["real", "complex"])
def test_every_element_unscreened(oracle_lib, cell, trs):
    H.require_gpu()
    st, nk = _cell(cell)
    mats = st.materialize("cuda")
    Dk = _dk(st, nk, trs)
    r = oracle_lib.KProblem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], nk, Dk).evaluate(
        0.0, nthreads=H.nthreads())
    g = _gpu(st, mats, nk, Dk)
    print(f"{cell}: E {g['E']:.15e} oracle {r['E']:.15e}; max|F| {np.abs(r['F']).max():.3e}", flush=True)
    _compare(g, r, st, nk)


def _theta_that_splits(kp, theta0):
    """A joint theta (on a geometric grid below theta0) that drops some D
    pairs and some C or V blocks but not all of them."""
    for th in np.geomspace(theta0, theta0 * 1e-4, 25):
        r = kp.evaluate(th)
        kD = r["keepD"]
        if 0 < kD.sum() < kD.size and (not r["keepC"].all() or not r["keepV"].all()):
            return float(th), r
    return None, None


@pytest.mark.parametrize("cell", CELLS[1:5], ids=IDS[1:5])
def test_every_element_screened(oracle_lib, cell):
    H.require_gpu()
    st, nk = _cell(cell)
    mats = st.materialize("cuda")
    Dk = _dk(st, nk, False)
    kp = oracle_lib.KProblem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], nk, Dk)
    th, r = _theta_that_splits(kp, 0.3)
    assert th is not None, "no theta splits the lists"
    print(f"{cell}: theta {th:.3e}, kept D pairs {int(r['keepD'].sum())}/{r['keepD'].size}, "
          f"C {int(r['keepC'].sum())}/{r['keepC'].size}, V {int(r['keepV'].sum())}/{r['keepV'].size}", flush=True)
    _compare(_gpu(st, mats, nk, Dk, theta=th), r, st, nk)


def test_per_tensor_thresholds(oracle_lib):
    H.require_gpu()
    st, nk = _cell(CELLS[3])
    mats = st.materialize("cuda")
    Dk = _dk(st, nk, False)
    kp = oracle_lib.KProblem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], nk, Dk)
    for s in np.geomspace(1.0, 1e-3, 13):
        thr = tuple(float(x) * s for x in (3e-2, 2e-1, 2e-1, 5e-2, 3e-1))
        r = kp.evaluate(thr=thr)
        split = ((r["keepC"] == 1) | (r["keepC"] == 2)).any() or ((r["keepV"] == 1) | (r["keepV"] == 2)).any()
        if split and 0 < r["keepD"].sum() < r["keepD"].size:
            break
    else:
        pytest.fail("no scaling of the thresholds splits the lists")
    print(f"thresholds {thr}", flush=True)
    _compare(_gpu(st, mats, nk, Dk, thresholds=thr), r, st, nk, bits=True)


@pytest.mark.parametrize("prec,rel_e,rel_f", [("fp32", 1e-7, 1e-5), ("bf16x3", 1e-6, 1e-4)])
def test_reduced_precision_forms(oracle_lib, prec, rel_e, rel_f):
    """The FP32 and BF16x3 forms on the supercell (both passes of a complex D)
    against the FP64 oracle, with the bounds of the Gamma-point forms: |dE| <=
    rel_e |E|, and max|d| <= rel_f times the largest magnitude for F, sigma
    and the block gradients."""
    H.require_gpu()
    st, nk = _cell(CELLS[3])
    mats = st.materialize("cuda")
    Dk = _dk(st, nk, False)
    r = oracle_lib.KProblem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], nk, Dk).evaluate(
        0.0, nthreads=H.nthreads())
    g = _gpu(st, mats, nk, Dk, precision=prec)
    for name, rel in (("E", rel_e), ("F", rel_f), ("sigma", rel_f), ("gC", rel_f), ("gV", rel_f)):
        got, ref = np.asarray(g[name], np.float64), np.asarray(r[name], np.float64)
        err, scale = float(np.max(np.abs(got - ref))), float(np.max(np.abs(ref)))
        print(f"  {prec} {name}: max abs error {err:.3e} (scale {scale:.3e})", flush=True)
        assert err <= rel * scale + 1e-12, name


def test_host_inputs_and_repeat_bitwise():
    H.require_gpu()
    st, nk = _cell(CELLS[3])
    Dk = _dk(st, nk, False)
    gd = _gpu(st, st.materialize("cuda"), nk, Dk)
    gh = _gpu(st, st.materialize("cpu"), nk, Dk, device=False)
    gd2 = _gpu(st, st.materialize("cuda"), nk, Dk)
    for k in ("E", "F", "sigma", "gC", "gV"):
        assert np.array_equal(np.asarray(gd[k]), np.asarray(gh[k])), k
        assert np.array_equal(np.asarray(gd[k]), np.asarray(gd2[k])), k


def test_gamma_mesh_equals_gamma_entry_point():
    """nk = (1,1,1) with the Gamma-point D: the same kernels on the same
    lists, so the same bits as lrx_set_tensors + lrx_evaluate; afterwards the
    context goes back to the Gamma point with lrx_set_tensors."""
    import torch

    H.require_gpu()
    st = synth.small_case(natom=4, nspecies=2, n_ao=7, n_abf=20, box=7.0, rc=5.0, rv=8.0, seed=96).build()
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    ref = ctx.evaluate(1e-3, 0.0)
    ctx.set_kpoint_tensors((1, 1, 1), mats["C"], mats["V"], mats["D"][None].contiguous())
    got = ctx.evaluate(1e-3, 0.0)
    for a, b in zip(got, ref):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    ctx.set_tensors(mats["C"], mats["V"], mats["D"])
    again = ctx.evaluate(1e-3, 0.0)
    for a, b in zip(again, ref):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    ctx.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", ["diamond64_k222", "sc8_k331"])
def test_workload_against_stored_oracle(case):
    """Workload cells with a complex D: the 64-atom cell on a 2 x 2 x 2 mesh
    (theta 1e-4) and the 8-atom cell on a 3 x 3 x 1 mesh (theta 0, offsets
    that differ from their negatives): E, F, sigma and every block gradient
    against the stored oracle results (tests/golden/make_golden_kpoint.py)."""
    import torch

    from tests.golden import make_golden_kpoint as G

    H.require_gpu()
    ref = G.load(case)
    st, mats, nk, Dk = G.inputs(case, "cuda")
    assert np.allclose(G.fingerprint(mats, Dk), ref["fingerprint"], rtol=1e-10, atol=0)
    ctx = lrx.Context()
    ctx.set_structure(st.tau, st.lat, st.nao, st.nabf)
    ctx.set_kpoint_tensors(nk, mats["C"], mats["V"], torch.from_numpy(Dk).to("cuda"))
    E, F, S = ctx.evaluate(float(ref["theta"]), 0.0)
    gC, gV = ctx.block_gradients()
    kC, kV, _ = ctx.keep_masks()
    ctx.close()
    print(f"{case}: E {E:.15e} oracle {float(ref['E']):.15e}; max|F| {np.abs(ref['F']).max():.3e}", flush=True)
    np.testing.assert_array_equal(kC != 0, ref["keepC"] != 0)
    np.testing.assert_array_equal(kV != 0, ref["keepV"] != 0)
    H.assert_close_fp64("E", E, float(ref["E"]), H.TOL_E_PER_ATOM * st.natom)
    H.assert_close_fp64("F", F, ref["F"], H.TOL_F)
    H.assert_close_fp64("sigma", S, ref["sigma"], H.TOL_SIGMA)
    H.assert_close_fp64("gC", gC, ref["gC"], H.TOL_F)
    H.assert_close_fp64("gV", gV, ref["gV"], H.TOL_F)


def test_refused():
    import torch

    H.require_gpu()
    st, nk = _cell(CELLS[1])
    mats = st.materialize("cuda")
    Dk = _dk(st, nk, False)
    bad = Dk.copy()
    bad[1][0, 1] += 0.1   # D(-r) != D(r)^H (offset 1 is its own negative on this mesh)
    ctx = lrx.Context()
    ctx.set_structure(st.tau, st.lat, st.nao, st.nabf)
    with pytest.raises(lrx.LrxError, match="D\\(-R\\)"):
        ctx.set_kpoint_tensors(nk, mats["C"], mats["V"], torch.from_numpy(bad).to("cuda"))
    ctx.set_kpoint_tensors(nk, mats["C"], mats["V"], torch.from_numpy(Dk).to("cuda"))
    with pytest.raises(lrx.LrxError, match="theta_cs"):
        ctx.evaluate(0.0, 1e-3)
    with pytest.raises(lrx.LrxError):
        ctx.evaluate_noalloc(0.0, 0.0)
    with pytest.raises(lrx.LrxError):
        ctx.hamiltonian(0.0, 0.0)
    with pytest.raises(lrx.LrxError):
        lrx.evaluate_batch([ctx], 0.0, 0.0)
    E, F, S = ctx.evaluate(0.0, 0.0)   # still usable
    assert np.isfinite(E) and F.shape == (st.natom, 3)
    ctx.close()
