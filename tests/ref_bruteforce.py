"""Brute-force exchange energy from the 4-index definition (test helper).

E = -1/2 sum_{ikjl} (ik|jl) D_kl D_ij  (Methods, Eq. Eexx with N_k = 1), where
the LRI-fitted 4-index integrals are (Eq. Exx-LRI)
    (ik|jl) = sum_{A in {I,K}} sum_{B in {J,L}} C^A_{ik} (P_A|P_B) C^B_{jl}.
The fitted pair density rho_{ik} is expanded on the ABFs of both atoms of the
pair, with the swap symmetry C^A_{ik} = C^A_{ki} (Methods, after the LRI
expansion).  Lattice images are folded into home-cell indices (Gamma point).
Nothing here is shared with the oracle's quartet loop.
"""
import numpy as np


def dense_ri(st, mats, keepC=None, keepV=None):
    """P[A alpha][i][k] fitted-density coefficients and dense V (ABF x ABF)."""
    nao, nabf = st.nao, st.nabf
    ao = np.concatenate([[0], np.cumsum(nao)])
    ab = np.concatenate([[0], np.cumsum(nabf)])
    nt, mt = int(ao[-1]), int(ab[-1])
    P = np.zeros((mt, nt, nt))
    C = mats["C"]
    val = C["val"].cpu().numpy() if hasattr(C["val"], "cpu") else np.asarray(C["val"])
    for b, (X, Y) in enumerate(zip(C["first"], C["second"])):
        if keepC is not None and not keepC[b]:
            continue
        m, nx, ny = nabf[X], nao[X], nao[Y]
        blk = val[C["off"][b]:C["off"][b] + m * nx * ny].reshape(m, nx, ny)
        # ABF on X for the pair (X x, Y y) ...
        P[ab[X]:ab[X] + m, ao[X]:ao[X] + nx, ao[Y]:ao[Y] + ny] += blk
        # ... and for the pair (Y y, X x), by the swap symmetry
        P[ab[X]:ab[X] + m, ao[Y]:ao[Y] + ny, ao[X]:ao[X] + nx] += blk.transpose(0, 2, 1)
    V = mats["V"]
    vval = V["val"].cpu().numpy() if hasattr(V["val"], "cpu") else np.asarray(V["val"])
    Vd = np.zeros((mt, mt))
    for b, (A, B) in enumerate(zip(V["first"], V["second"])):
        if keepV is not None and not keepV[b]:
            continue
        m1, m2 = nabf[A], nabf[B]
        Vd[ab[A]:ab[A] + m1, ab[B]:ab[B] + m2] += vval[V["off"][b]:V["off"][b] + m1 * m2].reshape(m1, m2)
    return P, Vd


def energy_literal(st, mats):
    """Materialise (ik|jl) and contract it with D D (tiny cells only)."""
    P, Vd = dense_ri(st, mats)
    eri = np.einsum("aik,ab,bjl->ikjl", P, Vd, P, optimize=True)
    D = st.D
    return -0.5 * np.einsum("ikjl,kl,ij->", eri, D, D, optimize=True)


def energy_assoc(st, mats, keepC=None, keepV=None, D=None):
    """Same contraction, associated as M_ab = <P_a, D P_b D> (larger cells)."""
    P, Vd = dense_ri(st, mats, keepC, keepV)
    D = st.D if D is None else D
    Q = np.einsum("ij,bjl,lk->bik", D, P, D, optimize=True)
    M = P.reshape(P.shape[0], -1) @ Q.reshape(Q.shape[0], -1).T
    return -0.5 * float(np.sum(Vd * M))


def hamiltonian_literal(st, mats, D=None):
    """H^X_ij = -sum_kl (ik|jl) D_kl (Eq. Exx2) from the same fitted
    4-index integrals, without forming them (small cells)."""
    P, Vd = dense_ri(st, mats)
    D = st.D if D is None else D
    # (PD)[b][j][k] = sum_l P[b][j][l] D[k][l]; W[a][j][k] = sum_b Vd[a][b] (PD)[b][j][k]
    PD = np.einsum("bjl,kl->bjk", P, D, optimize=True)
    W = np.einsum("ab,bjk->ajk", Vd, PD, optimize=True)
    return -np.einsum("aik,ajk->ij", P, W, optimize=True)
