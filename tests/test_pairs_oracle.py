"""Pins of the image-pair enumeration oracle (oracle/pairs.py), CPU only:
the vectorised enumeration equals plain loops on tiny cells (also triclinic
ones and cells smaller than the cutoff), the list is closed under the
mirror (second, first, -R), every kept image lies inside and every image
just outside is dropped, and the workload generators' independent
enumeration (sqrt of a matrix-product displacement) finds the same keys."""
import numpy as np
import pytest

from oracle import pairs as P
from paper_2412_11081_amd import synth


def _cells():
    rng = np.random.default_rng(7)
    out = []
    for k in range(4):
        lat = np.eye(3) * rng.uniform(4, 7) + rng.uniform(-1.2, 1.2, size=(3, 3))   # triclinic
        n = 1 + k
        tau = rng.uniform(0, 1, size=(n, 3)) @ lat
        out.append((tau, lat, rng.uniform(3.0, 9.0)))
    return out


@pytest.mark.parametrize("case", range(4))
def test_vectorised_equals_loops(case):
    tau, lat, rc = _cells()[case]
    a = P.pairs(tau, lat, rc)
    b = P.pairs_loops(tau, lat, rc)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert a[0].size > 0


@pytest.mark.parametrize("case", range(4))
def test_mirror_closed_inside_and_sorted(case):
    tau, lat, rc = _cells()[case]
    f, s, R = P.pairs(tau, lat, rc)
    keys = set(zip(f.tolist(), s.tolist(), map(tuple, R.tolist())))
    for a, b, r in keys:
        assert (b, a, tuple(-x for x in r)) in keys
    d = tau[s] - tau[f] + R @ lat
    assert np.all(np.sqrt((d * d).sum(1)) < rc * (1 + 1e-12))
    order = np.lexsort((R[:, 2], R[:, 1], R[:, 0], s, f))
    np.testing.assert_array_equal(order, np.arange(f.size))
    # every image one span further out (and every non-listed image) is outside
    spans = P._spans(lat, rc)
    for a in range(tau.shape[0]):
        for b in range(tau.shape[0]):
            for r in [(spans[0] + 1, 0, 0), (0, -spans[1] - 1, 0), (0, 0, spans[2] + 1)]:
                dd = tau[b] - tau[a] + np.array(r) @ lat
                assert np.sqrt(dd @ dd) >= rc


@pytest.mark.parametrize("k,cut", [(1, "rc"), (1, "rv"), (2, "rc"), (2, "rv")])
def test_workload_generator_agrees(k, cut):
    st = synth.workload(k)
    rc = st.rc if cut == "rc" else st.rv
    a = P.pairs(st.tau, st.lat, rc)
    b = synth.enumerate_pairs(st.tau, st.lat, rc)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
