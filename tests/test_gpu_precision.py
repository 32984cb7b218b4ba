"""FP32 and BF16x3 forms of the HIP path against the FP64 CPU oracle.

Bounds (stated per result; the FP64 path has the tighter ones in helpers):

* FP32: every product in FP32 with FP32 accumulation over at most a few
  thousand terms (unit roundoff 6e-8), gradients reduced in FP64 from the
  FP32 Z and Y.  Bound: max|dF| <= 1e-5 max|F| + 1e-6 Ha/Bohr, the same form
  for the block gradients and sigma, |dE| <= 1e-5 |E| + 1e-8 N.
* BF16x3: the Z and Y products take hi*hi + hi*lo + lo*hi of the bf16 split
  of their FP32 operands (relative product error about 2^-16), H and X are
  FP32.  Bound: max|dF| <= 1e-4 Ha/Bohr (the force target of the refined
  form), max|dsigma| <= 1e-5 Ha/Bohr^3, |dE| <= 1e-4 |E| + 1e-8 N.
The measured errors are printed for every case.
"""
import numpy as np
import pytest

from paper_2412_11081_amd import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

BOUNDS = {
    # (E rel, F rel, F abs, sigma rel, sigma abs)
    "fp32": (1e-5, 1e-5, 1e-6, 1e-5, 1e-7),
    "bf16x3": (1e-4, 0.0, 1e-4, 0.0, 1e-5),
}

CASES = [
    (3, 2, 13, 33, 7.0, 5.0, 8.0, 1e-4, 33),
    (4, 3, 7, 20, 5.5, 4.5, 7.5, 2e-3, 34),
    (3, 1, 18, 100, 12.0, 5.0, 7.0, 0.0, 36),
    (2, 2, 16, 64, 3.6, 4.0, 5.0, 0.0, 37),
    (2, 1, 3, 5, 6.0, 4.5, 7.0, 0.0, 31),       # one alpha tile: reduced a quarter per Z wave
    (2, 1, 9, 75, 7.5, 5.0, 8.0, 0.0, 38),      # five alpha tiles
]


def _check(prec, name, got, ref, rel, abs_tol):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    err = float(np.max(np.abs(got - ref))) if got.size else 0.0
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    bound = rel * scale + abs_tol
    print(f"  {prec} {name}: max abs error {err:.3e} (scale {scale:.3e}, bound {bound:.3e})", flush=True)
    assert err <= bound, f"{prec} {name}: {err:.3e} > {bound:.3e}"


def _run(st, mats, prec):
    ctx = H.gpu_context(st, mats)
    E, F, S = ctx.evaluate(st.theta, st.theta_cs, precision=prec)
    gC, gV = ctx.block_gradients()
    keep = ctx.keep_masks()
    ctx.close()
    return E, F, S, gC, gV, keep


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}s{c[1]}ao{c[2]}abf{c[3]}" for c in CASES])
def test_small_cells_reduced_precision(oracle_lib, case, prec):
    H.require_gpu()
    natom, nsp, nao, nabf, box, rc, rv, theta, seed = case
    st = synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=rc, rv=rv,
                          seed=seed, theta=theta, theta_cs=1e-3 * theta, jitter=0.5).build()
    print(f"case {case} {prec}", flush=True)
    mats = st.materialize("cuda")
    E, F, S, gC, gV, keep = _run(st, mats, prec)
    r = oracle_lib.Problem.from_structure(st, mats).evaluate(st.theta, st.theta_cs, nthreads=H.nthreads())
    # screening stays FP64: decisions are identical in every form
    np.testing.assert_array_equal(keep[0], r["keepC"])
    np.testing.assert_array_equal(keep[1], r["keepV"])
    np.testing.assert_array_equal(keep[2], r["keepD"])
    er, fr, fa, sr, sa = BOUNDS[prec]
    _check(prec, "E", E, r["E"], er, 1e-8 * st.natom)
    _check(prec, "F", F, r["F"], fr, fa)
    _check(prec, "sigma", S, r["sigma"], sr, sa)
    _check(prec, "gC", gC, r["gC"], fr, fa)
    _check(prec, "gV", gV, r["gV"], fr, fa)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_tiny_cubic_reduced_precision(oracle_lib, prec):
    """The 8-atom workload against the stored FP64 oracle result."""
    import json

    from tests.test_gpu_parity import GOLDEN

    H.require_gpu()
    ref = json.load(open(GOLDEN))
    st = H.workload(1)
    mats = st.materialize("cuda")
    E, F, S, gC, gV, _ = _run(st, mats, prec)
    er, fr, fa, sr, sa = BOUNDS[prec]
    _check(prec, "E", E, ref["E"], er, 1e-8 * st.natom)
    _check(prec, "F", F, ref["F"], fr, fa)
    _check(prec, "sigma", S, ref["sigma"], sr, sa)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_perovskite1080_reduced_precision_sampled(oracle_lib, prec):
    """The 1080-atom workload: sampled block gradients against the oracle,
    and the force/virial scatter of the block gradients."""
    H.require_gpu()
    st = H.workload(4)
    mats = st.materialize("cuda")
    E, F, S, gC, gV, keep = _run(st, mats, prec)
    er, fr, fa, sr, sa = BOUNDS[prec]
    assert np.max(np.abs(F.sum(axis=0))) <= 1e-10 * max(1.0, np.abs(F).max())
    rng = np.random.default_rng(40)
    picks = [("C", int(b)) for b in rng.choice(gC.shape[0], size=2, replace=False)]
    picks += [("V", int(b)) for b in rng.choice(gV.shape[0], size=2, replace=False)]
    for kind, b in picks:
        ref, kept = H.oracle_block_gradient(st, mats, kind, b, st.theta, st.theta_cs)
        got = (gC if kind == "C" else gV)[b]
        assert bool((keep[0] if kind == "C" else keep[1])[b]) == kept
        _check(prec, f"g{kind}[{b}]", got, ref, fr, fa)
