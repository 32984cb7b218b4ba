"""The serving loop on the GPU: each request's result is the same alone and
in the mix (bit for bit: a request's work units and kernels do not depend on
its batch), and within the BF16x3 bounds (relative to each result's
magnitude) of the FP64 result of the same request."""
import numpy as np
import pytest

from paper_2412_11081_amd import lrx, synth
from paper_2412_11081_amd.serve import LrxEngine, Request, Server, poisson_arrivals, replay
from tests import helpers as H

pytestmark = pytest.mark.gpu

REQUESTS = [9, 12, 0, 23, 2, 15, 17, 20]


def test_results_same_alone_and_in_the_mix():
    H.require_gpu()
    structs = [synth.serving_request(i).build() for i in REQUESTS]
    print("natoms", [s.natom for s in structs], flush=True)
    srv = Server(LrxEngine(precision="bf16x3"), hbm_budget=48 << 30, max_batch=4, workers=2)
    reqs = replay(srv, structs, poisson_arrivals(len(structs), rate=200.0, seed=5))
    assert srv.drain(timeout=120)
    srv.close()
    st = srv.stats()
    print("serving stats", st, flush=True)
    assert st["completed"] == len(structs), [r.error for r in reqs]
    for r, s in zip(reqs, structs):
        mats = s.materialize("cuda")
        ctx = lrx.context_for(s, mats)
        alone = ctx.evaluate(s.theta, s.theta_cs, precision="bf16x3")
        ref = ctx.evaluate(s.theta, s.theta_cs, precision="fp64")
        ctx.close()
        E, F, S = r.result
        assert E == alone[0] and np.array_equal(F, alone[1]) and np.array_equal(S, alone[2]), r.rid
        dF, dS, dE = np.max(np.abs(F - ref[1])), np.max(np.abs(S - ref[2])), abs(E - ref[0])
        print(f"request {r.rid} ({s.natom} atoms): |dE| {dE:.2e} max|dF| {dF:.2e} (max|F| "
              f"{np.abs(ref[1]).max():.2e}) max|dsigma| {dS:.2e}", flush=True)
        assert dF <= 1e-4 * np.abs(ref[1]).max() + 1e-12
        assert dS <= 1e-4 * np.abs(ref[2]).max() + 1e-12
        assert dE <= 1e-6 * abs(ref[0])


def test_memory_cache_trim_and_reuse():
    """Contexts come and go: the second pass reuses the library's cached
    device memory; after lrx_pool_trim the next context maps fresh memory and
    still gives the same results."""
    H.require_gpu()
    structs = [synth.serving_request(i).build() for i in REQUESTS[:3]]
    first = []
    for s in structs:
        mats = s.materialize("cuda")
        ctx = lrx.context_for(s, mats)
        first.append(ctx.evaluate(s.theta, s.theta_cs, precision="bf16x3"))
        ctx.close()
    lrx.pool_trim(0, 0)
    for s, ref in zip(structs, first):
        mats = s.materialize("cuda")
        ctx = lrx.context_for(s, mats)
        got = ctx.evaluate(s.theta, s.theta_cs, precision="bf16x3")
        ctx.close()
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    with pytest.raises(lrx.LrxError):
        lrx.pool_trim(999, 0)
