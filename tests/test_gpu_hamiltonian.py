"""The exact-exchange Hamiltonian H^X = dE/dD (Eq. Exx2) of the HIP path
(lrx_hamiltonian) against the oracle.

Small cells: every element of H^X and E = <H^X, D> / 2 against the oracle's
quartet-loop H, with and without screening (joint and per-tensor lists,
dropped D pairs), over several NAO/ABF tile sizes and ragged tails.  The 64-,
320- and 1080-atom cells: sampled D blocks against the oracle's loop over the
quartets that reach them, and E against the stored oracle energy.  At every
size: H^X is symmetric, and it is the derivative of the GPU energy along
random symmetric directions (exact for the quadratic E).
"""
import numpy as np
import pytest

from paper_2412_11081_amd import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

# (natom, nspecies, n_ao, n_abf, box, rc, rv, theta, seed)
CELLS = [
    (2, 1, 3, 5, 6.0, 4.5, 7.0, 0.0, 31),
    (3, 2, 5, 17, 6.5, 5.0, 8.0, 0.0, 32),
    (3, 2, 13, 33, 7.0, 5.0, 8.0, 1e-4, 33),
    (4, 3, 7, 20, 5.5, 4.5, 7.5, 2e-3, 34),
    (2, 1, 22, 40, 9.0, 5.0, 8.0, 0.0, 35),
    (2, 2, 11, 90, 8.0, 5.0, 8.0, 1e-4, 39),
    (2, 2, 16, 64, 3.6, 4.0, 5.0, 0.0, 37),   # atoms see their own images
]
# agreement of two FP64 results that differ in summation order
REL = 1e-10


def _cell(c):
    natom, nsp, nao, nabf, box, rc, rv, theta, seed = c
    return synth.small_case(natom=natom, nspecies=nsp, n_ao=nao, n_abf=nabf, box=box, rc=rc, rv=rv, seed=seed,
                            theta=theta, theta_cs=1e-3 * theta).build()


def _check(name, got, ref):
    err = float(np.max(np.abs(got - ref)))
    scale = float(np.max(np.abs(ref)))
    print(f"  {name}: max abs error {err:.3e} (scale {scale:.3e})", flush=True)
    assert err <= REL * scale + 1e-14, name


@pytest.mark.parametrize("cell", CELLS, ids=[f"n{c[0]}ao{c[2]}abf{c[3]}th{c[7]}" for c in CELLS])
def test_small_cells_every_element(oracle_lib, cell):
    H.require_gpu()
    st = _cell(cell)
    mats = st.materialize("cuda")
    print(f"cell {cell}: n_tot {st.D.shape[0]}", flush=True)
    pr = oracle_lib.Problem.from_structure(st, mats)
    keep = pr.screen(st.theta, st.theta_cs)
    Href = pr.hamiltonian(keep, nthreads=H.nthreads())
    Eref = pr.contract(keep, nthreads=H.nthreads())[0]
    ctx = H.gpu_context(st, mats)
    E, Hx = ctx.hamiltonian(st.theta, st.theta_cs)
    E2 = ctx.evaluate(st.theta, st.theta_cs)[0]
    ctx.close()
    _check("H", Hx, Href)
    assert abs(E - Eref) <= REL * abs(Eref), (E, Eref)
    assert abs(E - E2) <= REL * abs(E2)
    assert np.array_equal(Hx, Hx.T) or float(np.max(np.abs(Hx - Hx.T))) <= 1e-15 * float(np.max(np.abs(Hx)))


@pytest.mark.parametrize("thr", [(1e-3, 0.0, 0.3, 0.0, 5e-2), (3e-3, 2e-2, 1e-1, 5e-3, 3e-2)], ids=["C_D_dV", "all"])
def test_per_tensor_lists(oracle_lib, thr):
    """Per-tensor thresholds: H^X takes the value lists only, and is zero on
    dropped D pairs."""
    H.require_gpu()
    st = synth.small_case(natom=4, seed=19, nspecies=2, n_ao=3, n_abf=4, box=7.0, rc=5.5, rv=9.0).build()
    mats = st.materialize("cuda")
    pr = oracle_lib.Problem.from_structure(st, mats)
    keep = pr.screen5(thr, 0.0)
    print(f"thr {thr}: C bits {np.bincount(keep[0], minlength=4)}, V bits {np.bincount(keep[1], minlength=4)}, "
          f"D kept {int(keep[2].sum())} of {keep[2].size}", flush=True)
    Href = pr.hamiltonian(keep, bits=True)
    ctx = H.gpu_context(st, mats)
    E, Hx = ctx.hamiltonian(0.0, 0.0, thresholds=thr)
    ctx.close()
    _check("H", Hx, Href)
    Eref = pr.contract(keep, bits=True)[0]
    assert abs(E - Eref) <= REL * abs(Eref)


def test_repeat_is_bitwise_identical():
    H.require_gpu()
    st = _cell(CELLS[2])
    mats = st.materialize("cuda")
    ctx = H.gpu_context(st, mats)
    a = ctx.hamiltonian(st.theta, st.theta_cs)
    b = ctx.hamiltonian(st.theta, st.theta_cs)
    ctx.close()
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def _directional(ctx, st, mats, rng, nd=2):
    """<H^X, S> against (E(D + eS) - E(D - eS)) / 2e of the GPU energy,
    unscreened (no decision can flip): exact up to rounding for any e
    because E is quadratic in D."""
    import torch

    _, Hx = ctx.hamiltonian(0.0, 0.0)
    D = mats["D"]
    ao = np.concatenate([[0], np.cumsum(st.nao)])
    for _ in range(nd):
        # a few random symmetric blocks on atom pairs within the Coulomb range
        S = torch.zeros_like(D)
        vf, vs = np.asarray(mats["V"]["first"]), np.asarray(mats["V"]["second"])
        for i in rng.integers(0, len(vf), 6):
            X, Y = int(vf[i]), int(vs[i])
            blk = torch.tensor(rng.standard_normal((st.nao[X], st.nao[Y])), dtype=D.dtype, device=D.device)
            S[ao[X]:ao[X + 1], ao[Y]:ao[Y + 1]] += blk
            S[ao[Y]:ao[Y + 1], ao[X]:ao[X + 1]] += blk.T
        eps = 1e-1
        e = []
        for sgn in (1, -1):
            ctx.set_tensors(mats["C"], mats["V"], (D + sgn * eps * S).contiguous())
            e.append(ctx.evaluate(0.0, 0.0)[0])
        fd = (e[0] - e[1]) / (2 * eps)
        an = float(np.sum(Hx * S.cpu().numpy()))
        print(f"  directional: analytic {an:.12e} finite difference {fd:.12e}", flush=True)
        # E itself carries about 1e-14 |E| of summation rounding
        assert abs(fd - an) <= 1e-9 * abs(an) + 1e-13 * abs(e[0]) / eps
    ctx.set_tensors(mats["C"], mats["V"], D)


@pytest.mark.parametrize("case", ["diamond64", "abx3_320", "abx3_1080"])
def test_workload_sampled_blocks_and_energy(oracle_lib, case):
    """The 64-, 320- and 1080-atom workloads (the last in the configuration
    the benchmark times): E = <H^X, D> / 2 against the stored oracle energy,
    sampled D blocks of H^X against the oracle's loop over the quartets that
    reach them, symmetry, and directional derivatives."""
    import torch

    H.require_gpu()
    ref = H.golden(case)
    st = H.workload(int(ref["workload"]))
    theta, theta_cs = float(ref["theta"]), float(ref["theta_cs"])
    mats = st.materialize("cuda")
    H.check_fingerprint(mats, ref)
    ctx = H.gpu_context(st, mats)
    nt = mats["D"].shape[0]
    out = torch.empty((nt, nt), dtype=torch.float64, device="cuda")
    E, Hd = ctx.hamiltonian(theta, theta_cs, out=out)
    torch.cuda.synchronize()
    print(f"{case}: n_tot {nt}, E {E:.12e} (oracle {float(ref['E']):.12e})", flush=True)
    H.assert_close_fp64("E", E, float(ref["E"]), H.TOL_E_PER_ATOM * st.natom)
    asym = float(torch.max(torch.abs(Hd - Hd.T)))
    assert asym <= 1e-14 * float(torch.max(torch.abs(Hd)))
    Hx = Hd.cpu().numpy()
    pr = oracle_lib.Problem.from_structure(st, mats)
    keep = pr.screen(theta, theta_cs)
    ao = np.concatenate([[0], np.cumsum(st.nao)])
    rng = np.random.default_rng(5)
    # the on-site block of atom 0 and two random pairs within the Coulomb
    # range (a far pair has a zero block)
    vf, vs = np.asarray(mats["V"]["first"]), np.asarray(mats["V"]["second"])
    picks = [(0, 0)] + [(int(vf[i]), int(vs[i])) for i in rng.integers(0, len(vf), 2)]
    for X, Y in picks:
        Hf = pr.hamiltonian(keep, focus=(X, Y), nthreads=H.nthreads())
        blk = (slice(ao[X], ao[X + 1]), slice(ao[Y], ao[Y + 1]))
        print(f" block ({X},{Y}):", flush=True)
        _check("H block", Hx[blk], Hf[blk])
    _directional(ctx, st, mats, rng)
    ctx.close()
