"""Pins of the oracle's k-point form (oracle.KProblem, orc_contract_kp).

The k mesh nk makes a Born-von Karman (BvK) supercell of N_k = prod(nk)
unit cells, and the density matrix depends on the offset of two orbitals'
cells modulo that supercell (Methods, Eq. Eexx and the k-sum definition of
D).  Each pin would fail for a plausible mistake in the oracle's offsets
(which slot reads D at which cell offset), in the complex weight
Re[D_AB D*_FG + D_AG D*_FB] (Eq. exx_expand), or in the per-cell
normalisation:

  * nk = (1,1,1) with a real D is the Gamma-point oracle, bit for bit;
  * the explicit BvK supercell (atoms and keys replicated per cell, D block
    circulant) run through the Gamma-point oracle gives N_k times the
    energy, the k-point forces on every image, and the k-point stress; a
    complex D enters through its real and imaginary parts;
  * the 4-index definition of Eq. Eexx, -1/(2 N_k) sum (IK|JL) D_KL D*_IJ
    over the supercell with the LRI integrals, with a complex D;
  * five-point finite differences of the energy in the atom positions and
    in a homogeneous strain, D(R) held fixed.
"""
import types

import numpy as np
import pytest

from paper_2412_11081_amd import synth
from tests import ref_bruteforce as bf


def _kprob(oracle_lib, st, nk, Dk, mats=None):
    m = mats if mats is not None else st.materialize("cpu")
    return oracle_lib.KProblem(st.tau, st.lat, st.nao, st.nabf, m["C"], m["V"], nk, Dk)


def _cells(nk):
    """Cell offsets in the flat order r0 + nk0 (r1 + nk1 r2)."""
    return [(r0, r1, r2) for r2 in range(nk[2]) for r1 in range(nk[1]) for r0 in range(nk[0])]


def _flat(nk, r):
    r = [int(r[k]) % nk[k] for k in range(3)]
    return r[0] + nk[0] * (r[1] + nk[1] * r[2])


def supercell(st, mats, nk, Dk):
    """The BvK supercell written out: atom (t, i) = index t * N + i at tau_i +
    t.L, lattice rows nk_x L_x, every key (A, F, R) replicated for each cell t
    as ((t, A), (t + R mod nk, F), floor((t + R) / nk)) with the same values,
    and the dense D_sc[(t, i)][(u, j)] = D(u - t)[i][j]."""
    N, nt = st.natom, st.n_tot
    nk = np.asarray(nk)
    cells = np.array(_cells(nk))
    ncell = len(cells)
    tau = np.concatenate([st.tau + c @ st.lat for c in cells])
    lat = st.lat * nk[:, None]
    out = {}
    for tag in ("C", "V"):
        b = mats[tag]
        f, s, R = np.asarray(b["first"]), np.asarray(b["second"]), np.asarray(b["R"]).reshape(-1, 3)
        F, S, RR, OFF = [], [], [], []
        for ti, t in enumerate(cells):
            p = t[None, :] + R
            r = np.mod(p, nk)
            F.append(ti * N + f)
            S.append(np.array([_flat(nk, x) for x in r]) * N + s)
            RR.append((p - r) // nk)
            OFF.append(np.asarray(b["off"]))
        out[tag] = dict(first=np.concatenate(F).astype(np.int32), second=np.concatenate(S).astype(np.int32),
                        R=np.concatenate(RR).astype(np.int32), off=np.concatenate(OFF),
                        val=np.asarray(b["val"]), dval=np.asarray(b["dval"]))
    Dsc = np.zeros((ncell * nt, ncell * nt), Dk.dtype)
    for ti, t in enumerate(cells):
        for ui, u in enumerate(cells):
            Dsc[ti * nt:(ti + 1) * nt, ui * nt:(ui + 1) * nt] = Dk[_flat(nk, u - t)]
    return tau, lat, np.tile(st.nao, ncell), np.tile(st.nabf, ncell), out, Dsc


CASES = [  # (natom, nspecies, n_ao, n_abf, box, rc, rv, seed, nk)
    (2, 1, 3, 4, 5.0, 4.0, 6.0, 71, (2, 1, 1)),
    (3, 2, 2, 3, 5.5, 4.5, 6.5, 72, (1, 2, 2)),
    (2, 2, 3, 4, 4.5, 4.0, 6.0, 73, (3, 1, 1)),
    (2, 1, 2, 3, 4.5, 4.0, 5.5, 81, (2, 3, 1)),   # an offset and its negative differ only where nk > 2
]


def _case(c):
    natom, nsp, nao, nabf, box, rc, rv, seed, nk = c
    st = synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=rc, rv=rv, seed=seed).build()
    return st, nk


def test_gamma_mesh_is_the_gamma_oracle(oracle_lib):
    st = synth.small_case(natom=3, nspecies=2, n_ao=3, n_abf=5, seed=74).build()
    mats = st.materialize("cpu")
    for theta in (0.0, 3e-2):
        ref = oracle_lib.Problem.from_structure(st, mats).evaluate(theta, 0.0)
        got = _kprob(oracle_lib, st, (1, 1, 1), st.D[None], mats).evaluate(theta)
        assert got["E"] == ref["E"]
        assert np.array_equal(got["gC"], ref["gC"]) and np.array_equal(got["gV"], ref["gV"])
        assert np.array_equal(got["keepD"][0], ref["keepD"].reshape(st.natom, st.natom))


@pytest.mark.parametrize("c", CASES, ids=[f"n{c[0]}nk{''.join(map(str, c[8]))}" for c in CASES])
@pytest.mark.parametrize("trs", [True, False], ids=["real", "complex"])
def test_bvk_supercell_through_the_gamma_oracle(oracle_lib, c, trs):
    st, nk = _case(c)
    mats = st.materialize("cpu")
    Dk = synth.kpoint_density(st.n_tot, nk, st.seed + 5, trs=trs)
    if trs:
        Dk = Dk.real.copy()
    got = _kprob(oracle_lib, st, nk, Dk, mats).evaluate(0.0)
    tau, lat, nao, nabf, blk, Dsc = supercell(st, mats, nk, Dk)
    ncell = int(np.prod(nk))
    E = 0.0
    F = np.zeros((ncell * st.natom, 3))
    S = np.zeros((3, 3))
    parts = [Dsc.real] + ([] if trs else [Dsc.imag])
    for part in parts:   # Re[z w*] = Re z Re w + Im z Im w
        r = oracle_lib.Problem(tau, lat, nao, nabf, blk["C"], blk["V"], np.ascontiguousarray(part)).evaluate(0.0, 0.0)
        E += r["E"]
        F += r["F"]
        S += r["sigma"]
    print(f"E_k {got['E']:.15e}  E_sc / N_k {E / ncell:.15e}", flush=True)
    assert abs(got["E"] - E / ncell) <= 1e-12 * abs(E / ncell)
    scale = np.abs(got["F"]).max()
    for t in range(ncell):
        np.testing.assert_allclose(F[t * st.natom:(t + 1) * st.natom], got["F"], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(S, got["sigma"], rtol=0, atol=1e-11 * np.abs(got["sigma"]).max())


@pytest.mark.parametrize("nk", [(2, 1, 1), (1, 2, 2)])
def test_four_index_definition_complex(oracle_lib, nk):
    """Eq. Eexx on the BvK supercell: E = -1/(2 N_k) sum (ik|jl) D_kl D*_ij."""
    st = synth.small_case(natom=2, nspecies=2, n_ao=2, n_abf=3, box=4.5, rc=4.0, rv=6.0, seed=75).build()
    mats = st.materialize("cpu")
    Dk = synth.kpoint_density(st.n_tot, nk, 76)
    assert np.abs(Dk.imag).max() > 0.01
    got = _kprob(oracle_lib, st, nk, Dk, mats).evaluate(0.0)
    tau, lat, nao, nabf, blk, Dsc = supercell(st, mats, nk, Dk)
    sc = types.SimpleNamespace(nao=nao, nabf=nabf)
    P, Vd = bf.dense_ri(sc, blk)
    eri = np.einsum("aik,ab,bjl->ikjl", P, Vd, P, optimize=True)
    E4 = -0.5 / np.prod(nk) * np.einsum("ikjl,kl,ij->", eri, Dsc, Dsc.conj(), optimize=True)
    print(f"E_k {got['E']:.15e}  Eq. Eexx {E4.real:.15e} (imaginary part {E4.imag:.1e})", flush=True)
    assert abs(E4.imag) <= 1e-12 * abs(E4.real)
    assert abs(got["E"] - E4.real) <= 1e-12 * abs(E4.real)
    # the imaginary part of D matters: dropping it changes E
    E_re = _kprob(oracle_lib, st, nk, Dk.real.copy(), mats).evaluate(0.0)["E"]
    assert abs(E_re - got["E"]) > 1e-6 * abs(got["E"])


def _fd5(f, h):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


def _energy_at(oracle_lib, st, nk, Dk, tau, lat):
    s2 = synth.Structure(st.name, tau, lat, st.species, st.species_dims, st.rc, st.rv, 0.0, 0.0, st.seed, st.d_kind)
    s2.build(with_d=False, keys=(st.keysC, st.keysV))
    s2.D = st.D   # unused: the k-point D(R) is passed on its own
    return _kprob(oracle_lib, s2, nk, Dk).evaluate(0.0)["E"]


def test_forces_and_stress_match_finite_differences(oracle_lib):
    st = synth.small_case(natom=2, nspecies=2, n_ao=3, n_abf=4, box=5.0, rc=4.0, rv=6.0, seed=77).build()
    nk = (2, 1, 2)
    Dk = synth.kpoint_density(st.n_tot, nk, 78)
    res = _kprob(oracle_lib, st, nk, Dk).evaluate(0.0)
    h = 1e-3
    for M in range(st.natom):
        for x in range(3):
            def e_of(dx):
                t = st.tau.copy()
                t[M, x] += dx
                return _energy_at(oracle_lib, st, nk, Dk, t, st.lat)
            f_fd = -_fd5(e_of, h)
            assert abs(f_fd - res["F"][M, x]) <= 1e-6, (M, x, f_fd, res["F"][M, x])
    h = 1e-4
    for i, j in ((0, 0), (1, 2), (2, 1)):
        def e_of(e):
            eps = np.zeros((3, 3))
            eps[i, j] = e
            T = np.eye(3) + eps
            return _energy_at(oracle_lib, st, nk, Dk, st.tau @ T.T, st.lat @ T.T)
        s_fd = -_fd5(e_of, h) / st.volume
        assert abs(s_fd - res["sigma"][i, j]) <= 1e-8, (i, j, s_fd, res["sigma"][i, j])
    assert np.abs(res["F"]).max() > 1e-4


def test_screening_per_offset(oracle_lib):
    """theta_D acts on the modulus of each offset's block: a pair dropped at
    one offset stays in at another, and the screened energy equals the
    unscreened one with those D blocks set to zero."""
    st = synth.small_case(natom=3, nspecies=2, n_ao=3, n_abf=4, box=5.5, rc=4.5, rv=6.5, seed=79).build()
    nk = (2, 2, 1)
    Dk = synth.kpoint_density(st.n_tot, nk, 80)
    mats = st.materialize("cpu")
    kp = _kprob(oracle_lib, st, nk, Dk, mats)
    mod = np.abs(Dk)
    ao = np.concatenate([[0], np.cumsum(st.nao)])
    bmax = np.array([[[mod[r, ao[x]:ao[x + 1], ao[y]:ao[y + 1]].max() for y in range(st.natom)]
                      for x in range(st.natom)] for r in range(len(Dk))])
    thD = float(np.median(bmax))
    r = kp.evaluate(thr=(0.0, 0.0, thD, 0.0, 0.0))
    assert 0 < r["keepD"].sum() < r["keepD"].size
    np.testing.assert_array_equal(r["keepD"], (bmax > thD).astype(np.uint8))
    D0 = Dk.copy()
    for rr in range(len(Dk)):
        for x in range(st.natom):
            for y in range(st.natom):
                if not r["keepD"][rr, x, y]:
                    D0[rr, ao[x]:ao[x + 1], ao[y]:ao[y + 1]] = 0
    r0 = _kprob(oracle_lib, st, nk, D0, mats).evaluate(0.0)
    assert abs(r["E"] - r0["E"]) <= 1e-13 * abs(r0["E"])
    np.testing.assert_allclose(r["gC"], r0["gC"], rtol=0, atol=1e-13 * np.abs(r0["gC"]).max())
