"""lrx_evaluate_noalloc (the entry point for callers that cannot allocate
device memory) against lrx_evaluate, through the C-ABI.

Two calls in a row on the fixed scratch, the second on a smaller structure,
so that what the first call leaves in the scratch would show if the second
read it; each result must match lrx_evaluate on the same context to the FP64
parity bar (the same kernels run, so it should match bit for bit).  A
structure whose work buffers exceed the scratch is refused with LRX_EBUDGET.
"""
import numpy as np
import pytest

from paper_2412_11081_amd import lrx, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

LRX_EBUDGET = -5


def _compare(name, got, ref, natom):
    E, F, S = got
    E0, F0, S0 = ref
    print(f"{name}: |dE| {abs(E - E0):.2e} max|dF| {np.max(np.abs(F - F0)):.2e} "
          f"max|dsigma| {np.max(np.abs(S - S0)):.2e}", flush=True)
    H.assert_close_fp64(f"{name} E", E, E0, H.TOL_E_PER_ATOM * natom)
    H.assert_close_fp64(f"{name} F", F, F0, H.TOL_F)
    H.assert_close_fp64(f"{name} sigma", S, S0, H.TOL_SIGMA)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_noalloc_matches_evaluate_twice_second_smaller(prec):
    H.require_gpu()
    big = synth.small_case(natom=4, nspecies=2, n_ao=13, n_abf=33, box=7.5, rc=5.0, rv=8.0, seed=61,
                           theta=1e-4, theta_cs=1e-7).build()
    small = synth.small_case(natom=2, nspecies=1, n_ao=5, n_abf=17, box=6.0, rc=4.5, rv=7.0, seed=62).build()
    ctxs, refs = [], []
    for st in (big, small):
        mats = st.materialize("cuda")
        ctx = H.gpu_context(st, mats)
        s = ctx.stats()
        print(f"{st.name}: natom {st.natom}, work bytes {s['work_bytes']}", flush=True)
        assert s["work_bytes"][lrx.PRECISIONS[prec]] <= lrx.SCRATCH_BYTES
        refs.append(ctx.evaluate(st.theta, st.theta_cs, precision=prec))
        ctxs.append((ctx, mats, st))
    # two calls in a row on the scratch: the larger structure, then the smaller
    for (ctx, _, st), ref in zip(ctxs, refs):
        got = ctx.evaluate_noalloc(st.theta, st.theta_cs, precision=prec)
        _compare(f"{st.name} {prec}", got, ref, st.natom)
        gC, gV = ctx.block_gradients()
        ctx.evaluate(st.theta, st.theta_cs, precision=prec)
        gC0, gV0 = ctx.block_gradients()
        H.assert_close_fp64("gC", gC, gC0, H.TOL_F)
        H.assert_close_fp64("gV", gV, gV0, H.TOL_F)
    # and the larger one again after the smaller one
    ctx, _, st = ctxs[0]
    _compare(f"{st.name} {prec} again", ctx.evaluate_noalloc(st.theta, st.theta_cs, precision=prec), refs[0],
             st.natom)
    for ctx, _, _ in ctxs:
        ctx.close()


def test_noalloc_refuses_structures_beyond_the_scratch():
    H.require_gpu()
    st = H.workload(2)
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    assert ctx.stats()["work_bytes"][0] > lrx.SCRATCH_BYTES
    with pytest.raises(lrx.LrxError) as e:
        ctx.evaluate_noalloc(st.theta, st.theta_cs)
    print("refused:", e.value, flush=True)
    assert e.value.code == LRX_EBUDGET and "scratch" in str(e.value)
    ctx.close()


def test_noalloc_per_tensor_thresholds():
    """Per-tensor lists (the unit roles and liveness bits live in the
    context, the work buffers in the scratch): the same result as
    lrx_evaluate with the same thresholds."""
    H.require_gpu()
    st = synth.small_case(natom=4, nspecies=2, n_ao=13, n_abf=33, box=7.5, rc=5.0, rv=8.0, seed=61).build()
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    thr = (3e-3, 2e-2, 1e-1, 5e-3, 3e-2)
    ref = ctx.evaluate(thresholds=thr)
    kC, kV, _ = ctx.keep_masks()
    print(f"C bits {np.bincount(kC, minlength=4)}, V bits {np.bincount(kV, minlength=4)}", flush=True)
    _compare("per-tensor", ctx.evaluate_noalloc(thresholds=thr), ref, st.natom)
    ctx.close()
