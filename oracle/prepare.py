"""CPU oracle of the preparation of C and dC (test infrastructure only).

Only the tests may import this module.  It is numpy only and shares nothing
with the GPU library.

For every C key (A,F,R), Eq. C_VA fixes the LRI coefficients of the pair
(A a, F f) on the ABFs of both atoms:

    [C^A; C^F] = M^-1 [ (P_A|phi_A phi_F); (P_F|phi_A phi_F) ],
    M = [[V(A,A,0), V(A,F,R)], [V(A,F,R)^T, V(F,F,0)]],

and the C block of the key is C^A, the first mA rows.  The on-site key
(A,A,0) uses the ABFs of A alone: C = V(A,A,0)^-1 (P_A|phi_A phi_A).  The
gradient follows the equation after Eq. V_inverse (the derivative of
M^-1 from M M^-1 = I):

    dC = M^-1 ( -[[0, dV], [dV^T, 0]] [C^A; C^F] + d(P|phi phi) ),

with dV the derivative of V(A,F,R) and every derivative taken with respect
to the key's displacement r = tau_F + R.L - tau_A.  On-site blocks do not
change when their atom moves, so their dC is zero.  np.linalg.solve (LAPACK)
is the one library step.
"""
from __future__ import annotations

import numpy as np


def _np(x):
    if hasattr(x, "detach"):
        x = x.detach().cpu().numpy()
    return np.asarray(x)


def _vkeys(V):
    f, s, R = _np(V["first"]), _np(V["second"]), _np(V["R"]).reshape(-1, 3)
    return {(int(f[i]), int(s[i]), int(R[i, 0]), int(R[i, 1]), int(R[i, 2])): i for i in range(f.shape[0])}


def solve_pair(nao, nabf, V, vidx, T, b):
    """The full solution [C^A; C^F] of key b of T (rows of A then F) and its
    derivative [3][rows][nA][nF]; for an on-site key the rows of A only."""
    f, s, R = _np(T["first"]), _np(T["second"]), _np(T["R"]).reshape(-1, 3)
    A, F = int(f[b]), int(s[b])
    Rb = tuple(int(x) for x in R[b])
    mA, mF, nA, nF = int(nabf[A]), int(nabf[F]), int(nao[A]), int(nao[F])
    vval, vdval, voff = _np(V["val"]), _np(V["dval"]), _np(V["off"])
    tval, tdval, toff = _np(T["val"]), _np(T["dval"]), _np(T["off"])
    onsite = A == F and Rb == (0, 0, 0)
    rows = mA if onsite else mA + mF
    k1 = nA * nF
    o = int(toff[b])
    P = tval[o:o + rows * k1].reshape(rows, k1)
    dP = tdval[3 * o:3 * (o + rows * k1)].reshape(3, rows, k1)

    def vblk(key, m1, m2):
        i = vidx[key]
        q = int(voff[i])
        return vval[q:q + m1 * m2].reshape(m1, m2), vdval[3 * q:3 * (q + m1 * m2)].reshape(3, m1, m2)

    VAA, _ = vblk((A, A, 0, 0, 0), mA, mA)
    if onsite:
        C = np.linalg.solve(VAA, P)
        return C.reshape(rows, nA, nF), np.zeros((3, rows, nA, nF))
    VFF, _ = vblk((F, F, 0, 0, 0), mF, mF)
    VAF, dVAF = vblk((A, F) + Rb, mA, mF)
    M = np.block([[VAA, VAF], [VAF.T, VFF]])
    C = np.linalg.solve(M, P)
    dC = np.empty((3, rows, k1))
    for x in range(3):
        Vt = np.block([[np.zeros((mA, mA)), dVAF[x]], [dVAF[x].T, np.zeros((mF, mF))]])
        dC[x] = np.linalg.solve(M, dP[x] - Vt @ C)
    return C.reshape(rows, nA, nF), dC.reshape(3, rows, nA, nF)


def prepare_c(nao, nabf, V, T):
    """C blocks for every key of T, laid out as lrx blocks: (off, val, dval)
    with val [mA][nA][nF] at off and dval [3][mA][nA][nF] at 3 off."""
    nao, nabf = np.asarray(nao), np.asarray(nabf)
    vidx = _vkeys(V)
    f, s = _np(T["first"]), _np(T["second"])
    sizes = np.array([nabf[f[b]] * nao[f[b]] * nao[s[b]] for b in range(f.shape[0])], np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    val = np.empty(int(sizes.sum()))
    dval = np.empty(3 * int(sizes.sum()))
    for b in range(f.shape[0]):
        mA = int(nabf[f[b]])
        C, dC = solve_pair(nao, nabf, V, vidx, T, b)
        n = int(sizes[b])
        o = int(off[b])
        val[o:o + n] = C[:mA].reshape(-1)
        dval[3 * o:3 * (o + n)] = dC[:, :mA].reshape(-1)
    return off, val, dval
