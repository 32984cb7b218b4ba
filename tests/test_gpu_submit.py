"""lrx_submit / lrx_wait through the C-ABI: queued evaluations give the same
results, bit for bit, as lrx_evaluate (first use, captured graph and its
replays), tickets are waited for in any order, each ticket once, and
tickets never waited for are released by lrx_destroy."""
import ctypes

import numpy as np
import pytest

from paper_2412_11081_amd import lrx, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _structure():
    return synth.small_case(natom=3, nspecies=2, n_ao=6, n_abf=21, box=6.5, rc=5.0, rv=8.0, seed=61,
                            theta=1e-4, theta_cs=1e-7).build()


def _same(a, b):
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_submitted_results_equal_evaluate():
    H.require_gpu()
    st = _structure()
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    ref64 = ctx.evaluate(st.theta, st.theta_cs, precision="fp64")
    refb3 = ctx.evaluate(st.theta, st.theta_cs, precision="bf16x3")
    # three fp64 submissions (the plan runs eagerly, is captured, is replayed)
    # and one bf16x3 in between, all outstanding at once
    t = [ctx.submit(st.theta, st.theta_cs, "fp64"), ctx.submit(st.theta, st.theta_cs, "bf16x3"),
         ctx.submit(st.theta, st.theta_cs, "fp64"), ctx.submit(st.theta, st.theta_cs, "fp64")]
    print("tickets", t, flush=True)
    assert len(set(t)) == 4
    for k in (3, 1, 0, 2):
        got = ctx.wait(t[k])
        _same(got, refb3 if k == 1 else ref64)
    # the block gradients describe the latest submitted evaluation (fp64)
    gC, gV = ctx.block_gradients()
    ctx.evaluate(st.theta, st.theta_cs, precision="fp64")
    gC2, gV2 = ctx.block_gradients()
    assert np.array_equal(gC, gC2) and np.array_equal(gV, gV2)
    ctx.close()


def test_ticket_errors_and_release_at_destroy():
    H.require_gpu()
    st = _structure()
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    tk = ctx.submit(st.theta, st.theta_cs, "fp64")
    ctx.wait(tk)
    with pytest.raises(lrx.LrxError):
        ctx.wait(tk)                      # each ticket once
    with pytest.raises(lrx.LrxError):
        ctx.wait(tk + 1000)               # never issued
    # stage timing is for lrx_evaluate only
    o = lrx.Options(st.theta, st.theta_cs, lrx.PRECISIONS["fp64"], 1, 0, 0)
    t = ctypes.c_int64(-7)
    rc = ctx.lib.lrx_submit(ctx.h, ctypes.byref(o), ctypes.byref(t))
    assert rc != 0 and t.value == -7
    # outstanding at destroy: waited for and released there
    ctx.submit(st.theta, st.theta_cs, "fp64")
    ctx.submit(st.theta, st.theta_cs, "bf16x3")
    ctx.close()
