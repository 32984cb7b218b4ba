"""Pins of the oracle's preparation of C and dC (Eq. C_VA and the gradient
after Eq. V_inverse), CPU only.

* Finite differences: moving one atom moves the displacement of every key it
  belongs to; the central difference of the prepared C along the move equals
  dC times the sign of the key's displacement change (keys frozen).  This
  checks the derivative formula (the -M^-1 dM M^-1 term, its blocks and its
  sign) against the solve itself.
* Swap symmetry: the rows on F of the solution for (A,F,R) are the rows on F
  of the solution for (F,A,-R) with the AO pair swapped, and their
  derivatives change sign (the mirror key's displacement is -r).
* On-site blocks are symmetric in the AO pair, with zero derivative.
"""
import dataclasses

import numpy as np
import pytest

from oracle import prepare as prep
from paper_2412_11081_amd import synth


def _cell(seed=51, tau=None, keys=None):
    st = synth.small_case(natom=3, seed=seed, nspecies=2, n_ao=3, n_abf=5, box=7.0, rc=5.5, rv=9.0)
    if tau is not None:
        st = dataclasses.replace(st, tau=tau)
    st = st.build(keys=keys)
    m = st.materialize("cpu")
    return st, m, synth.three_center(st)


def test_prepared_c_matches_finite_differences():
    st0, m0, T0 = _cell()
    off, val, dval = prep.prepare_c(st0.nao, st0.nabf, m0["V"], T0)
    keys = (st0.keysC, st0.keysV)
    atom, h = 1, 1e-4
    first, second = np.asarray(st0.keysC[0]), np.asarray(st0.keysC[1])
    for x in range(3):
        res = []
        for sgn in (1, -1):
            tau = st0.tau.copy()
            tau[atom, x] += sgn * h
            st, m, T = _cell(tau=tau, keys=keys)
            res.append(prep.prepare_c(st.nao, st.nabf, m["V"], T)[1])
        fd = (res[0] - res[1]) / (2 * h)
        worst = 0.0
        for b in range(first.shape[0]):
            A, F = int(first[b]), int(second[b])
            sign = (1.0 if F == atom else 0.0) - (1.0 if A == atom else 0.0)
            n = st0.nabf[A] * st0.nao[A] * st0.nao[F]
            o = int(off[b])
            an = sign * dval[3 * o + x * n:3 * o + (x + 1) * n]
            err = np.max(np.abs(fd[o:o + n] - an)) / max(np.max(np.abs(an)), 1e-3)
            worst = max(worst, err)
        print(f"direction {x}: worst relative error {worst:.2e}")
        assert worst <= 1e-6


def test_prepared_c_swap_symmetry_and_onsite():
    st, m, T = _cell(52)
    first, second, R = np.asarray(T["first"]), np.asarray(T["second"]), np.asarray(T["R"])
    vidx = prep._vkeys(m["V"])
    key = {(int(first[b]), int(second[b]), *map(int, R[b])): b for b in range(first.shape[0])}
    checked = 0
    for b in range(first.shape[0]):
        A, F = int(first[b]), int(second[b])
        C, dC = prep.solve_pair(st.nao, st.nabf, m["V"], vidx, T, b)
        if A == F and not R[b].any():
            assert np.allclose(C, C.transpose(0, 2, 1), rtol=0, atol=1e-13 * np.abs(C).max())
            assert not dC.any()
            continue
        bm = key[(F, A, *map(int, -R[b]))]
        Cm, dCm = prep.solve_pair(st.nao, st.nabf, m["V"], vidx, T, bm)
        mA, mF = st.nabf[A], st.nabf[F]
        scale = np.abs(C).max()
        np.testing.assert_allclose(C[mA:], Cm[:mF].transpose(0, 2, 1), rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(dC[:, mA:], -dCm[:, :mF].transpose(0, 1, 3, 2), rtol=0,
                                   atol=1e-12 * np.abs(dC).max())
        checked += 1
    assert checked > 0
