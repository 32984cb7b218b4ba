"""lrx_enumerate_pairs (image pairs within a cutoff, on the device) against
the enumeration oracle, key for key (bit-exact: the same rounded distance
rule on both sides): tiny triclinic cells, a one-atom cell, a cutoff below
every interatomic distance, the four workloads with both cutoffs, serving
requests, and rejected inputs."""
import numpy as np
import pytest

from oracle import pairs as P
from paper_2412_11081_amd import lrx, synth
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _same(tau, lat, rc, capacity=0):
    got = lrx.enumerate_pairs(tau, lat, rc, capacity=capacity)
    ref = P.pairs(tau, lat, rc)
    print(f"natom {len(tau)} rcut {rc:.3f}: {got[0].size} keys (oracle {ref[0].size})", flush=True)
    for x, y in zip(got, ref):
        np.testing.assert_array_equal(x, y)
    return got


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_small_triclinic_cells(seed):
    H.require_gpu()
    rng = np.random.default_rng(seed)
    lat = np.eye(3) * rng.uniform(4, 7) + rng.uniform(-1.2, 1.2, size=(3, 3))
    tau = rng.uniform(0, 1, size=(seed + 1, 3)) @ lat
    _same(tau, lat, rng.uniform(3.0, 11.0))


def test_one_atom_and_short_cutoff():
    H.require_gpu()
    f, s, R = _same(np.zeros((1, 3)), np.eye(3) * 3.0, 7.5)          # only images of itself
    assert (f == 0).all() and (s == 0).all() and f.size > 1
    tau = np.array([[0.0, 0, 0], [2.5, 0, 0], [0, 2.5, 0]])
    f, s, R = _same(tau, np.eye(3) * 10.0, 1.0)                       # only the atoms themselves
    np.testing.assert_array_equal(f, [0, 1, 2])
    np.testing.assert_array_equal(s, [0, 1, 2])
    assert not R.any()


def test_capacity_retry():
    H.require_gpu()
    st = synth.workload(1)
    _same(st.tau, st.lat, st.rv, capacity=5)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_workloads_both_cutoffs(k):
    H.require_gpu()
    st = H.workload(k)
    for rc, keys in ((st.rc, st.keysC), (st.rv, st.keysV)):
        got = _same(st.tau, st.lat, rc)
        # and the generator's keys (its own enumeration) are the same set
        for x, y in zip(got, keys):
            np.testing.assert_array_equal(x, np.asarray(y))


def test_serving_requests():
    H.require_gpu()
    for i in (0, 7, 23):
        st = synth.serving_request(i)
        _same(st.tau, st.lat, st.rv)


def test_rejected_inputs():
    H.require_gpu()
    with pytest.raises(lrx.LrxError):
        lrx.enumerate_pairs(np.array([[np.nan, 0, 0]]), np.eye(3) * 5, 3.0)
    with pytest.raises(lrx.LrxError):
        lrx.enumerate_pairs(np.zeros((2, 3)), np.zeros((3, 3)), 3.0)
    with pytest.raises(lrx.LrxError):
        lrx.enumerate_pairs(np.zeros((2, 3)), np.eye(3) * 0.01, 30.0)   # more than 62 lattice spacings
