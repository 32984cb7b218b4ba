"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test would fail for a plausible mistake in the oracle: a dropped or
mis-paired density-matrix term, a wrong sign or slot, a transposed block, a
wrong image displacement, a wrong volume or stress convention.
"""
import numpy as np
import pytest

from paper_2412_11081_amd import synth
from tests import ref_bruteforce as bf


def _eval(oracle_lib, st, mats=None, theta=None, theta_cs=None):
    return oracle_lib.evaluate_structure(st, theta=theta, theta_cs=theta_cs, mats=mats)


def _energy_at(oracle_lib, st, tau, lat):
    """E with the block lists frozen (keys of the reference geometry)."""
    s2 = synth.Structure(st.name, tau, lat, st.species, st.species_dims, st.rc, st.rv, 0.0, 0.0, st.seed,
                         st.d_kind)
    s2.build(with_d=False, keys=(st.keysC, st.keysV))
    s2.D = st.D
    return _eval(oracle_lib, s2, theta=0.0, theta_cs=0.0)["E"]


# --------------------------------------------------------------------------
# P1: the 4-index textbook energy (Eq. Eexx with Eq. Exx-LRI)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,natom,nspecies", [(5, 2, 1), (6, 3, 2), (7, 4, 1)])
def test_energy_equals_four_index_definition(oracle_lib, seed, natom, nspecies):
    st = synth.small_case(natom=natom, seed=seed, nspecies=nspecies, n_ao=3, n_abf=4).build()
    mats = st.materialize("cpu")
    E = _eval(oracle_lib, st, mats, 0.0, 0.0)["E"]
    E_lit = bf.energy_literal(st, mats)
    E_as = bf.energy_assoc(st, mats)
    assert abs(E - E_lit) <= 1e-12 * abs(E_lit)
    assert abs(E - E_as) <= 1e-12 * abs(E_as)


def test_energy_four_index_self_images(oracle_lib):
    """A cell smaller than the cutoffs: many self-images (A, A, R != 0)."""
    st = synth.small_case(natom=2, seed=9, box=3.2, rc=4.0, rv=6.5, n_ao=2, n_abf=3).build()
    mats = st.materialize("cpu")
    assert any((a == b) and np.any(r != 0) for a, b, r in zip(*st.keysC))
    E = _eval(oracle_lib, st, mats, 0.0, 0.0)["E"]
    assert abs(E - bf.energy_assoc(st, mats)) <= 1e-12 * abs(E)


# --------------------------------------------------------------------------
# P2/P3: five-point finite differences (Results, FD formula), D fixed
# --------------------------------------------------------------------------
def _fd5(f, h):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


def test_forces_match_finite_differences(oracle_lib):
    st = synth.small_case(natom=3, seed=11, nspecies=2, n_ao=3, n_abf=4).build()
    res = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    h = 1e-3
    for M in range(st.natom):
        for x in range(3):
            def e_of(dx):
                t = st.tau.copy()
                t[M, x] += dx
                return _energy_at(oracle_lib, st, t, st.lat)
            f_fd = -_fd5(e_of, h)
            assert abs(f_fd - res["F"][M, x]) <= 1e-6, (M, x, f_fd, res["F"][M, x])


def test_stress_matches_strain_finite_differences(oracle_lib):
    st = synth.small_case(natom=3, seed=12, n_ao=3, n_abf=4, box=5.0).build()
    res = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    h = 1e-4
    omega = st.volume
    for i in range(3):
        for j in range(3):
            def e_of(e):
                eps = np.zeros((3, 3))
                eps[i, j] = e
                T = np.eye(3) + eps
                return _energy_at(oracle_lib, st, st.tau @ T.T, st.lat @ T.T)
            s_fd = -_fd5(e_of, h) / omega
            assert abs(s_fd - res["sigma"][i, j]) <= 1e-8, (i, j, s_fd, res["sigma"][i, j])


# --------------------------------------------------------------------------
# P4: invariants
# --------------------------------------------------------------------------
def test_invariants_sum_force_symmetric_stress(oracle_lib):
    st = synth.small_case(natom=4, seed=13, nspecies=2, n_ao=3, n_abf=5).build()
    r = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    assert np.max(np.abs(r["F"].sum(axis=0))) <= 1e-12 * max(1.0, np.abs(r["F"]).max())
    assert np.max(np.abs(r["sigma"] - r["sigma"].T)) <= 1e-12 * max(1e-30, np.abs(r["sigma"]).max())


def test_translation_and_rotation(oracle_lib):
    st = synth.small_case(natom=3, seed=14, n_ao=3, n_abf=4).build()
    r0 = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    # rigid translation
    e_t = _energy_at(oracle_lib, st, st.tau + np.array([0.37, -1.1, 2.3]), st.lat)
    assert abs(e_t - r0["E"]) <= 1e-12 * abs(r0["E"])
    # rotation: E invariant, F -> Q F, sigma -> Q sigma Q^T
    ang = 0.7
    Q = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1.0]])
    Q = Q @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    s2 = synth.Structure(st.name, st.tau @ Q.T, st.lat @ Q.T, st.species, st.species_dims, st.rc, st.rv,
                         0.0, 0.0, st.seed, st.d_kind)
    s2.build(with_d=False, keys=(st.keysC, st.keysV))
    s2.D = st.D
    r1 = _eval(oracle_lib, s2, theta=0.0, theta_cs=0.0)
    assert abs(r1["E"] - r0["E"]) <= 1e-12 * abs(r0["E"])
    assert np.allclose(r1["F"], r0["F"] @ Q.T, atol=1e-12)
    assert np.allclose(r1["sigma"], Q @ r0["sigma"] @ Q.T, atol=1e-13)


def test_homogeneity(oracle_lib):
    """E is quadratic in C, linear in V, quadratic in D."""
    st = synth.small_case(natom=3, seed=15, n_ao=3, n_abf=4).build()
    mats = st.materialize("cpu")
    pr = oracle_lib.Problem.from_structure(st, mats)
    E0 = pr.evaluate(0.0, 0.0)["E"]
    lam = 1.7
    for tag, power in (("C", 2), ("V", 1)):
        m2 = {k: dict(v) if isinstance(v, dict) else v for k, v in mats.items()}
        m2[tag]["val"] = mats[tag]["val"] * lam
        m2[tag]["dval"] = mats[tag]["dval"] * lam
        E = oracle_lib.Problem(st.tau, st.lat, st.nao, st.nabf, m2["C"], m2["V"], mats["D"]).evaluate(0.0, 0.0)["E"]
        assert abs(E - lam**power * E0) <= 1e-12 * abs(E)
    E = oracle_lib.Problem(st.tau, st.lat, st.nao, st.nabf, mats["C"], mats["V"], mats["D"] * lam).evaluate(0.0, 0.0)["E"]
    assert abs(E - lam**2 * E0) <= 1e-12 * abs(E)


def test_atom_relabelling(oracle_lib):
    st = synth.small_case(natom=4, seed=16, nspecies=2, n_ao=3, n_abf=4).build()
    r0 = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    perm = np.array([2, 0, 3, 1])
    inv = np.argsort(perm)
    s2 = synth.Structure(st.name, st.tau[perm], st.lat, st.species[perm], st.species_dims, st.rc, st.rv,
                         0.0, 0.0, st.seed, st.d_kind)
    s2.build(with_d=False)
    # permute D's atom blocks consistently
    ao = st.ao_off
    idx = np.concatenate([np.arange(ao[a], ao[a + 1]) for a in perm])
    s2.D = st.D[np.ix_(idx, idx)]
    r1 = _eval(oracle_lib, s2, theta=0.0, theta_cs=0.0)
    assert abs(r1["E"] - r0["E"]) <= 1e-12 * abs(r0["E"])
    assert np.allclose(r1["F"], r0["F"][perm], atol=1e-12)
    assert np.allclose(r1["sigma"], r0["sigma"], atol=1e-13)
    del inv


# --------------------------------------------------------------------------
# P5: closed forms
# --------------------------------------------------------------------------
def test_single_atom_closed_form(oracle_lib):
    """One atom in a box larger than every cutoff: only the on-site blocks."""
    st = synth.small_case(natom=1, seed=17, box=30.0, n_ao=3, n_abf=5).build()
    assert len(st.keysC[0]) == 1 and len(st.keysV[0]) == 1
    r = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    m, n = st.nabf[0], st.nao[0]
    mats = st.materialize("cpu")
    C0 = mats["C"]["val"].numpy().reshape(m, n, n)
    V0 = mats["V"]["val"].numpy().reshape(m, m)
    D = st.D
    E = -(np.einsum("xaf,xy,ybg,ab,fg->", C0, V0, C0, D, D) + np.einsum("xaf,xy,ybg,ag,fb->", C0, V0, C0, D, D))
    assert abs(r["E"] - E) <= 1e-12 * abs(E)
    assert np.all(r["F"] == 0.0) and np.all(np.abs(r["sigma"]) == 0.0)


def test_dimer_force_along_bond(oracle_lib):
    """Two atoms in a large box: F_1 = -F_2 parallel to the bond,
    |F| = -dE/dd, and sigma = (1/Omega) F_2 (x) d with d = tau_2 - tau_1: the
    pair blocks (1,2,d) and (2,1,-d) give W = g (x) d - g' (x) d = -F_2 (x) d."""
    st = synth.small_case(natom=2, seed=18, box=40.0, n_ao=3, n_abf=4).build()
    st.tau = np.array([[10.0, 10.0, 10.0], [12.1, 11.3, 9.2]])
    st.build()
    r = _eval(oracle_lib, st, theta=0.0, theta_cs=0.0)
    dvec = st.tau[1] - st.tau[0]
    dhat = dvec / np.linalg.norm(dvec)
    assert np.allclose(r["F"][0], -r["F"][1], atol=1e-14)
    assert np.linalg.norm(np.cross(r["F"][1], dhat)) <= 1e-12 * np.linalg.norm(r["F"][1])

    def e_of(dd):
        t = st.tau.copy()
        t[1] += dd * dhat
        return _energy_at(oracle_lib, st, t, st.lat)

    dEdd = _fd5(e_of, 1e-3)
    assert abs(np.dot(r["F"][1], dhat) + dEdd) <= 1e-7
    sig = np.outer(r["F"][1], dvec) / st.volume
    assert np.allclose(r["sigma"], sig, atol=1e-12 * np.abs(sig).max() + 1e-18)


# --------------------------------------------------------------------------
# Screening
# --------------------------------------------------------------------------
def test_screened_equals_unscreened_with_dropped_blocks_zeroed(oracle_lib):
    """S1/S2 only remove blocks: the screened result equals the unscreened
    result on inputs where exactly the dropped blocks are zero."""
    st = synth.small_case(natom=4, seed=19, nspecies=2, n_ao=3, n_abf=4, box=7.0, rc=5.5, rv=9.0).build()
    mats = st.materialize("cpu")
    pr = oracle_lib.Problem.from_structure(st, mats)
    theta = 2e-3
    r = pr.evaluate(theta, 1e-3 * theta)
    kC, kV, kD = r["keepC"], r["keepV"], r["keepD"]
    assert kC.sum() < len(kC) and kV.sum() < len(kV)
    m2 = {"C": dict(mats["C"]), "V": dict(mats["V"])}
    for tag, keep in (("C", kC), ("V", kV)):
        val = mats[tag]["val"].clone()
        dval = mats[tag]["dval"].clone()
        first, second, off = mats[tag]["first"], mats[tag]["second"], mats[tag]["off"]
        for b in np.nonzero(keep == 0)[0]:
            if tag == "C":
                sz = st.nabf[first[b]] * st.nao[first[b]] * st.nao[second[b]]
            else:
                sz = st.nabf[first[b]] * st.nabf[second[b]]
            val[off[b]:off[b] + sz] = 0
            dval[3 * off[b]:3 * (off[b] + sz)] = 0
        m2[tag]["val"], m2[tag]["dval"] = val, dval
    D = st.D.copy()
    N = st.natom
    for X in range(N):
        for Y in range(N):
            if not kD[X * N + Y]:
                D[st.ao_off[X]:st.ao_off[X + 1], st.ao_off[Y]:st.ao_off[Y + 1]] = 0
    r0 = oracle_lib.Problem(st.tau, st.lat, st.nao, st.nabf, m2["C"], m2["V"], D).evaluate(0.0, 0.0)
    assert abs(r0["E"] - r["E"]) <= 1e-12 * abs(r["E"])
    assert np.allclose(r0["F"], r["F"], atol=1e-13)
    # and the brute-force definition on the zeroed inputs agrees as well
    st2 = st
    assert abs(bf.energy_assoc(st2, m2, D=D) - r["E"]) <= 1e-12 * abs(r["E"])


def test_schwarz_bound_holds(oracle_lib):
    """P6: |E contribution of a V block| <= |V|_F S(A,B) and the same for its
    derivative slot (Cauchy-Schwarz inequality, Sec. Sparsity exploitation)."""
    st = synth.small_case(natom=3, seed=20, nspecies=2, n_ao=3, n_abf=4).build()
    mats = st.materialize("cpu")
    pr = oracle_lib.Problem.from_structure(st, mats)
    keep = pr.screen(0.0, 0.0)
    S = keep[3]
    V = mats["V"]
    vv, dv = V["val"].numpy(), V["dval"].numpy()
    checked = 0
    for b in range(0, pr.nV, max(1, pr.nV // 12)):
        A, B = V["first"][b], V["second"][b]
        sz = st.nabf[A] * st.nabf[B]
        Eb, _, gV = pr.contract(keep, focus=("V", b))
        nV = np.linalg.norm(vv[V["off"][b]:V["off"][b] + sz])
        assert abs(Eb) <= nV * S[A, B] * (1 + 1e-12)
        for x in range(3):
            nd = np.linalg.norm(dv[3 * V["off"][b] + x * sz:3 * V["off"][b] + (x + 1) * sz])
            assert abs(gV[b, x]) <= nd * S[A, B] * (1 + 1e-12)
        checked += 1
    assert checked >= 6


def test_block_screen_decisions(oracle_lib):
    """S1 drops only blocks whose max-abs (with derivatives) is <= theta, and
    every V block shares its fate with its mirror (second, first, -R)."""
    st = synth.small_case(natom=4, seed=21, n_ao=3, n_abf=4, box=7.0, rc=5.5, rv=9.0).build()
    mats = st.materialize("cpu")
    pr = oracle_lib.Problem.from_structure(st, mats)
    theta = 1e-3
    kC, kV, kD, _ = pr.screen(theta, 0.0)
    C = mats["C"]
    for b in range(pr.nC):
        sz = st.nabf[C["first"][b]] * st.nao[C["first"][b]] * st.nao[C["second"][b]]
        mx = max(np.abs(C["val"][C["off"][b]:C["off"][b] + sz]).max().item(),
                 np.abs(C["dval"][3 * C["off"][b]:3 * (C["off"][b] + sz)]).max().item())
        assert bool(kC[b]) == (mx > theta)
    V = mats["V"]
    key = {(int(a), int(c), tuple(r)): i for i, (a, c, r) in enumerate(zip(V["first"], V["second"], V["R"]))}
    for (a, c, r), i in key.items():
        j = key[(c, a, tuple(-np.array(r)))]
        assert kV[i] == kV[j]


def test_schwarz_bound_is_tight_for_positive_scalar_blocks(oracle_lib):
    """P6, equality case: with one NAO and one ABF per atom, positive C and D
    entries and derivatives too small to enter the norms, every term of the
    Cauchy-Schwarz bound S(A,B) is exactly the matching term of the folded
    Z(A,B) = sum_{F,G} C(A,F) C(B,G) [D_AB D_FG + D_AG D_FB] (the triangle
    inequality is an equality for positive terms).  Z is read off the
    oracle's V-block gradients, g_b = -dV_b Z(A,B) for 1 x 1 blocks, so the
    bound's formula is pinned to the contraction itself: a dropped term, a
    wrong index or a missing factor breaks the equality."""
    st = synth.small_case(natom=3, seed=23, nspecies=1, n_ao=1, n_abf=1, box=5.0, rc=4.0, rv=6.0).build()
    mats = st.materialize("cpu")
    C = dict(mats["C"])
    C["val"] = mats["C"]["val"].abs() + 0.05
    C["dval"] = mats["C"]["dval"] * 1e-9
    D = np.abs(st.D)
    pr = oracle_lib.Problem(st.tau, st.lat, st.nao, st.nabf, C, mats["V"], D)
    kC, kV, kD, S = pr.screen(0.0, 0.0)
    _, _, gV = pr.contract((kC, kV, kD))
    V = mats["V"]
    dv = V["dval"].numpy()
    checked = 0
    for b in range(pr.nV):
        o = 3 * int(V["off"][b])
        d3 = dv[o:o + 3]
        x = int(np.argmax(np.abs(d3)))
        if abs(d3[x]) < 1e-6:
            continue   # on-site V block: no derivative to read Z through
        A, B = int(V["first"][b]), int(V["second"][b])
        Z = -gV[b, x] / d3[x]
        assert Z > 0 and abs(S[A, B] - Z) <= 1e-12 * Z, (A, B, S[A, B], Z)
        checked += 1
    assert checked >= 6
