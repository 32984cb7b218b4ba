"""Seeded synthetic inputs with the shapes of the paper's workloads.

This module holds none of the method's arithmetic.  It builds:

* periodic geometries (atom positions ``tau`` in Bohr, lattice rows ``a1..a3``),
* block keys ``(first, second, R)`` of the C and V tensors (all image pairs
  within a cutoff; the ABF of a C block sits on ``first``),
* block values from closed-form radial envelopes times per-species-pair base
  tensors, with analytic derivatives w.r.t. the block's own displacement
  ``r = tau_second + R.L - tau_first``,
* a symmetric Gamma-point density matrix with eigenvalues in [0, 2].

The recipe follows the paper's setting of NAO orbitals and ABFs on atoms
(Methods, Eqs. for the LRI expansion and V) with synthetic values, since the
real basis sets and densities are not available.  Both the CPU oracle and the
GPU library consume what this module produces.

Value layout (shared by both consumers): a block's elements are row-major
(C: ``[m_first][n_first][n_second]``, V: ``[m_first][m_second]``); block ``i``
starts at element ``off[i]`` of ``val`` and its three Cartesian derivatives
start at ``3*off[i]`` of ``dval`` as ``[x][block]``.  Blocks of one species
pair are stored contiguously so one broadcast product fills them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

# (n_ao, n_abf) of the synthetic species used by the workloads.
SPECIES_SI40 = (13, 40)      # 2s2p1d NAOs, small ABF set (tiny cubic cell)
SPECIES_SI75 = (13, 75)      # 2s2p1d NAOs, 75 ABFs (diamond-like cell)
SPECIES_A = (18, 90)         # perovskite A site
SPECIES_B = (13, 75)         # perovskite B site
SPECIES_X = (13, 75)         # perovskite X site
SPECIES_BP = (22, 100)       # substituted B site

TAPER_START = 0.85           # the smooth cutoff acts on the last 15 % of r_c
SEED_BASE = 11081


# ----------------------------------------------------------------------------
# radial envelopes
# ----------------------------------------------------------------------------
def taper(x: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Quintic smootherstep S(x) on [0.85, 1] (C2 at both ends) and dS/dx."""
    x = np.asarray(x, dtype=np.float64)
    t = np.clip((x - TAPER_START) / (1.0 - TAPER_START), 0.0, 1.0)
    s = 1.0 - t**3 * (10.0 - 15.0 * t + 6.0 * t**2)
    ds = -30.0 * t**2 * (1.0 - t) ** 2 / (1.0 - TAPER_START)
    inside = (x > TAPER_START) & (x < 1.0)
    ds = np.where(inside, ds, 0.0)
    s = np.where(x >= 1.0, 0.0, s)
    return s, ds


def env_c(r: np.ndarray, rc: float) -> Tuple[np.ndarray, np.ndarray]:
    """C envelope exp(-0.3 r^2) * S(r/rc) and its radial derivative."""
    g = np.exp(-0.3 * r * r)
    s, ds = taper(r / rc)
    return g * s, -0.6 * r * g * s + g * ds / rc


def env_v(r: np.ndarray, rv: float) -> Tuple[np.ndarray, np.ndarray]:
    """V envelope S(r/rv) / (1 + r^2) and its radial derivative."""
    q = 1.0 / (1.0 + r * r)
    s, ds = taper(r / rv)
    return q * s, -2.0 * r * q * q * s + q * ds / rv


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def enumerate_pairs(tau: np.ndarray, lat: np.ndarray, rcut: float):
    """All (first, second, R) with |tau_second + R.L - tau_first| < rcut.

    Returned sorted by (first, second, R lexicographic).  The list is closed
    under the mirror (second, first, -R).
    """
    tau = np.asarray(tau, np.float64)
    lat = np.asarray(lat, np.float64)
    n = tau.shape[0]
    vol = abs(np.linalg.det(lat))
    heights = [vol / np.linalg.norm(np.cross(lat[(i + 1) % 3], lat[(i + 2) % 3])) for i in range(3)]
    span = [int(math.ceil(rcut / h)) + 1 for h in heights]
    rr = np.array(np.meshgrid(*[np.arange(-s, s + 1) for s in span], indexing="ij")).reshape(3, -1).T
    rr = rr[np.lexsort((rr[:, 2], rr[:, 1], rr[:, 0]))]
    shifts = rr.astype(np.float64) @ lat                      # [nR, 3]
    out_f, out_s, out_r = [], [], []
    for a in range(n):
        d = tau[:, None, :] + shifts[None, :, :] - tau[a][None, None, :]   # [n, nR, 3]
        dist = np.sqrt(np.einsum("ijk,ijk->ij", d, d))
        sec, ridx = np.nonzero(dist < rcut)
        order = np.lexsort((ridx, sec))
        sec, ridx = sec[order], ridx[order]
        out_f.append(np.full(sec.shape, a, np.int32))
        out_s.append(sec.astype(np.int32))
        out_r.append(rr[ridx].astype(np.int32))
    return np.concatenate(out_f), np.concatenate(out_s), np.concatenate(out_r).reshape(-1, 3)


def displacement(tau, lat, first, second, R):
    """r = (tau_second - tau_first) + R.L, associated so that the mirror block
    (second, first, -R) gets exactly -r (IEEE negation is exact)."""
    return (tau[second] - tau[first]) + R.astype(np.float64) @ lat


# ----------------------------------------------------------------------------
# structure
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Structure:
    name: str
    tau: np.ndarray            # [N, 3] Bohr
    lat: np.ndarray            # [3, 3] rows a1..a3, Bohr
    species: np.ndarray        # [N] int
    species_dims: List[Tuple[int, int]]   # per species (n_ao, n_abf)
    rc: float                  # C (orbital) cutoff, Bohr
    rv: float                  # V (Coulomb range) cutoff, Bohr
    theta: float               # block screening threshold
    theta_cs: float            # Schwarz threshold
    seed: int
    d_kind: str = "haar"       # "haar" (Q diag(U[0,2]) Q^T), "goe" (I + S/rho) or "gersh" (drawn on the device)

    # filled by build()
    nao: np.ndarray = None
    nabf: np.ndarray = None
    ao_off: np.ndarray = None
    base_c: Dict = None        # (s, s2) -> [m_s, n_s, n_s2]; ("on", s) -> symmetric on-site
    base_v: Dict = None        # (s, s2) -> [m_s, m_s2]
    D: np.ndarray = None       # [n_tot, n_tot]
    keysC: Tuple = None        # (first, second, R)
    keysV: Tuple = None

    @property
    def natom(self) -> int:
        return int(self.tau.shape[0])

    @property
    def n_tot(self) -> int:
        return int(self.nao.sum())

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.lat)))

    # ------------------------------------------------------------------
    def build(self, with_d: bool = True, keys=None):
        """Draw the species tensors and D from the seed, enumerate block keys.

        ``keys`` = (keysC, keysV) freezes the block lists (finite-difference
        use); otherwise they are enumerated from the cutoffs.
        """
        rng = np.random.default_rng(self.seed + 7919)
        dims = self.species_dims
        self.nao = np.array([dims[s][0] for s in self.species], np.int32)
        self.nabf = np.array([dims[s][1] for s in self.species], np.int32)
        self.ao_off = np.concatenate([[0], np.cumsum(self.nao)]).astype(np.int64)
        used = sorted(set(int(s) for s in self.species))
        self.base_c, self.base_v = {}, {}
        for s in used:
            n, m = dims[s]
            t = rng.normal(0.0, 0.1, size=(m, n, n))
            self.base_c[("on", s)] = 0.5 * (t + t.transpose(0, 2, 1))
        for s in used:
            for s2 in used:
                n, m = dims[s]
                n2 = dims[s2][0]
                self.base_c[(s, s2)] = rng.normal(0.0, 0.1, size=(m, n, n2))
        for s in used:
            m = dims[s][1]
            g = rng.normal(0.0, 1.0, size=(m, m))
            b = g @ g.T / m + np.eye(m)
            self.base_v[(s, s)] = 0.5 * (b + b.T)
        for i, s in enumerate(used):
            for s2 in used[i + 1:]:
                m, m2 = dims[s][1], dims[s2][1]
                b = 0.5 * rng.normal(0.0, 1.0, size=(m, m2)) / math.sqrt(max(m, m2))
                k = min(m, m2)
                b[np.arange(k), np.arange(k)] += 1.0
                self.base_v[(s, s2)] = b
                self.base_v[(s2, s)] = np.ascontiguousarray(b.T)
        if keys is None:
            self.keysC = enumerate_pairs(self.tau, self.lat, self.rc)
            self.keysV = enumerate_pairs(self.tau, self.lat, self.rv)
        else:
            self.keysC, self.keysV = keys
        if with_d and self.d_kind != "gersh":
            self.D = make_density(self.n_tot, self.d_kind, rng)
        return self

    # ------------------------------------------------------------------
    def _layout(self, kind: str):
        """Group blocks by value template; return offsets and group list.

        Groups are laid out in the order of str(template key), the blocks of
        a group in key order."""
        first, second, R = self.keysC if kind == "C" else self.keysV
        first, second = np.asarray(first), np.asarray(second)
        sp = np.asarray(self.species, np.int64)
        sa, sb = sp[first], sp[second]
        if kind == "C":
            onsite = (first == second) & np.all(np.asarray(R) == 0, axis=1)
        else:
            onsite = np.zeros(first.shape[0], bool)
        code = np.where(onsite, -1 - sa, sa * 4096 + sb)
        uniq, inv = np.unique(code, return_inverse=True)
        keys = [("on", int(-1 - c)) if c < 0 else (int(c // 4096), int(c % 4096)) for c in uniq]
        off = np.zeros(first.shape[0], np.int64)
        glist = []
        cur = 0
        for g in sorted(range(len(keys)), key=lambda g: str(keys[g])):
            k = keys[g]
            idx = np.nonzero(inv == g)[0].astype(np.int64)
            base = self.base_c[k] if kind == "C" else self.base_v[k]
            size = base.size
            off[idx] = cur + np.arange(idx.size, dtype=np.int64) * size
            glist.append((k, idx, cur, size))
            cur += idx.size * size
        return off, glist, cur

    def radial(self, kind: str):
        """Per-block scalar f(|r|) and derivative factors f'(|r|) r_x/|r|."""
        first, second, R = self.keysC if kind == "C" else self.keysV
        d = displacement(self.tau, self.lat, first, second, R)
        r = np.sqrt(np.einsum("ij,ij->i", d, d))
        f, fp = env_c(r, self.rc) if kind == "C" else env_v(r, self.rv)
        with np.errstate(invalid="ignore", divide="ignore"):
            unit = np.where(r[:, None] > 0, d / np.where(r > 0, r, 1.0)[:, None], 0.0)
        return f, fp[:, None] * unit, d

    def materialize(self, device: str = "cpu"):
        """Block arrays as torch float64 tensors on ``device`` (+ host keys).

        Each element is one IEEE product base*f, identical on CPU and GPU.
        """
        import torch

        out = {}
        on_gpu = torch.device(device).type == "cuda"

        def up(a):
            # small host arrays go to the device through pinned memory,
            # asynchronously on the current stream: a copy from pageable memory
            # would block the calling thread behind other work on the device
            t = torch.from_numpy(np.ascontiguousarray(a))
            return t.pin_memory().to(device, non_blocking=True) if on_gpu else t.to(device)

        for kind in ("C", "V"):
            off, glist, total = self._layout(kind)
            f, fpx, disp = self.radial(kind)
            val = torch.empty(total, dtype=torch.float64, device=device)
            dval = torch.empty(3 * total, dtype=torch.float64, device=device)
            for key, idx, start, size in glist:
                base = self.base_c[key] if kind == "C" else self.base_v[key]
                b = up(np.ascontiguousarray(base).reshape(-1))
                fi = up(f[idx])
                fpi = up(fpx[idx])
                nb = idx.size
                # written in place: no temporaries the size of the blocks
                torch.mul(fi[:, None], b[None, :], out=val[start:start + nb * size].view(nb, size))
                torch.mul(fpi[:, :, None], b[None, None, :],
                          out=dval[3 * start:3 * (start + nb * size)].view(nb, 3, size))
            first, second, R = self.keysC if kind == "C" else self.keysV
            out[kind] = dict(first=first, second=second, R=R, off=off, val=val, dval=dval, disp=disp)
        if self.d_kind == "gersh" and self.D is None:
            out["D"] = gersh_density(self.n_tot, self.seed + 104729, device)
        else:
            out["D"] = up(self.D)
        return out


# ----------------------------------------------------------------------------
# three-centre integrals (P|phi phi) for the preparation of C
# ----------------------------------------------------------------------------
def three_center(st: Structure, device: str = "cpu", seed_shift: int = 104723):
    """Synthetic (P|phi_A phi_F) for every C key (A,F,R): the ABFs of A then
    those of F against the AO pair (A a, F f), [mA + mF][nA][nF], or
    [mA][nA][nA] for the on-site key (A,A,0), with d/dr as [3][block] (r the
    key's displacement).  Base tensors per species pair times the C envelope;
    the rows on F of (A,F,R) are the rows on F of (F,A,-R) with the AO pair
    swapped, as for real integrals, and on-site blocks are symmetric in the
    AO pair.  Returns a dict like the C and V blocks of materialize()."""
    import torch

    rng = np.random.default_rng(st.seed + seed_shift)
    dims = st.species_dims
    used = sorted(set(int(x) for x in st.species))
    u = {}
    for s_ in used:
        n, m = dims[s_]
        t = rng.normal(0.0, 0.1, size=(m, n, n))
        u[("on", s_)] = 0.5 * (t + t.transpose(0, 2, 1))
    for s_ in used:
        for s2 in used:
            n, m = dims[s_]
            u[(s_, s2)] = rng.normal(0.0, 0.1, size=(m, n, dims[s2][0]))
    first, second, R = st.keysC
    first, second, R = np.asarray(first), np.asarray(second), np.asarray(R)
    d = displacement(st.tau, st.lat, first, second, R)
    r = np.sqrt(np.einsum("ij,ij->i", d, d))
    f, fp = env_c(r, st.rc)
    with np.errstate(invalid="ignore", divide="ignore"):
        unit = np.where(r[:, None] > 0, d / np.where(r > 0, r, 1.0)[:, None], 0.0)
    sp = np.asarray(st.species)
    nb = first.shape[0]
    rows = np.zeros(nb, np.int64)
    sizes = np.zeros(nb, np.int64)
    onsite = (first == second) & np.all(R == 0, axis=1)
    for b in range(nb):
        A, F = int(first[b]), int(second[b])
        rows[b] = st.nabf[A] if onsite[b] else st.nabf[A] + st.nabf[F]
        sizes[b] = rows[b] * st.nao[A] * st.nao[F]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    total = int(sizes.sum())
    val = np.empty(total)
    dval = np.empty(3 * total)
    for b in range(nb):
        A, F = int(first[b]), int(second[b])
        sA, sF = int(sp[A]), int(sp[F])
        if onsite[b]:
            base = u[("on", sA)]
        else:
            base = np.concatenate([u[(sA, sF)], u[(sF, sA)].transpose(0, 2, 1)], axis=0)
        flat = base.reshape(-1)
        o, n = int(off[b]), int(sizes[b])
        val[o:o + n] = f[b] * flat
        for x in range(3):
            dval[3 * o + x * n:3 * o + (x + 1) * n] = (fp[b] * unit[b, x]) * flat
    return dict(first=first, second=second, R=R, off=off, rows=rows, onsite=onsite,
                val=torch.from_numpy(val).to(device), dval=torch.from_numpy(dval).to(device))


# ----------------------------------------------------------------------------
# density matrices
# ----------------------------------------------------------------------------
def make_density(n: int, kind: str, rng: np.random.Generator) -> np.ndarray:
    """Symmetric n x n matrix with eigenvalues in [0, 2].

    ``haar``: Q diag(U[0,2]) Q^T, Q Haar-distributed (sign-fixed QR).
    ``goe``:  I + S / rho, S a GOE matrix, rho = 1.001 * spectral radius.
    """
    if kind == "haar":
        g = rng.normal(size=(n, n))
        q, r = np.linalg.qr(g)
        q = q * np.sign(np.diag(r))[None, :]
        lam = rng.uniform(0.0, 2.0, size=n)
        d = (q * lam[None, :]) @ q.T
    elif kind == "goe":
        g = rng.normal(size=(n, n))
        s = (g + g.T) / math.sqrt(2.0)
        del g
        from scipy.sparse.linalg import eigsh

        lam = eigsh(s, k=1, which="LM", return_eigenvectors=False, tol=1e-6)
        rho = 1.001 * float(abs(lam[0]))
        s /= rho
        s[np.diag_indices(n)] += 1.0
        d = s
    else:
        raise ValueError(kind)
    d = 0.5 * (d + d.T)
    return np.ascontiguousarray(d)


def gersh_density(n: int, seed: int, device: str = "cpu"):
    """Symmetric n x n torch matrix with eigenvalues in (0, 2), drawn on ``device``:
    I + S / rho with S = (G + G^T)/sqrt(2), G Gaussian from a seeded torch
    generator, and rho = 1.001 * max_i sum_j |S_ij| (Gershgorin: every
    eigenvalue of S lies in [-rho, rho]).  Cheap for the serving stream."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    G = torch.randn(n, n, generator=g, device=device, dtype=torch.float64)
    S = (G + G.T) * (1.0 / math.sqrt(2.0))
    del G
    rho = 1.001 * S.abs().sum(dim=1).max()   # stays on the device: no wait for the stream
    S /= rho
    S.diagonal().add_(1.0)
    return S.contiguous()


def kpoint_density(n: int, nk, seed: int, trs: bool = False) -> np.ndarray:
    """Density matrix per Born-von Karman cell offset, drawn through the k-sum
    definition of D (Methods): on the Gamma-centred mesh k_m = m / nk, a
    Hermitian D(k_m) with eigenvalues in (0, 2) (I + S/rho, S = (G + G^H)/sqrt 2
    from complex Gaussian G, rho = 1.001 * max_i sum_j |S_ij|, so Gershgorin
    bounds the spectrum), then
        D(r)[i][j] = (1/N_k) sum_m exp(-2 pi i k_m . r) D(k_m)[i][j],
    returned as a complex array [N_k][n][n] with r = r0 + nk0 (r1 + nk1 r2).
    D(-r) = D(r)^H for every draw.  trs=True draws D(k_-m) = conj(D(k_m))
    (time-reversal symmetry; real D(k) where k_m = k_-m), which makes every
    D(r) real; otherwise the D(k_m) are independent and D(r) is complex."""
    nk = tuple(int(x) for x in nk)
    rng = np.random.default_rng(seed)
    Dk = np.zeros(nk + (n, n), np.complex128)
    done = np.zeros(nk, bool)
    for m in np.ndindex(*nk):
        if done[m]:
            continue
        mm = tuple((-mi) % ni for mi, ni in zip(m, nk))
        self_conj = mm == m
        if trs and self_conj:
            g = rng.normal(size=(n, n))
        else:
            g = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
        S = (g + g.conj().T) / math.sqrt(2.0)
        S /= 1.001 * float(np.abs(S).sum(axis=1).max())
        S[np.diag_indices(n)] += 1.0
        Dk[m] = S
        done[m] = True
        if trs and not self_conj:
            Dk[mm] = S.conj()
            done[mm] = True
    # sum_m exp(-2 pi i m.r / nk) over the three mesh axes is numpy's forward FFT
    Dr = np.fft.fftn(Dk, axes=(0, 1, 2)) / float(np.prod(nk))
    # [r0][r1][r2] -> flat index r0 + nk0 (r1 + nk1 r2)
    Dr = np.ascontiguousarray(Dr.transpose(2, 1, 0, 3, 4)).reshape(-1, n, n)
    if trs:
        assert np.abs(Dr.imag).max() <= 1e-12 * max(1.0, np.abs(Dr.real).max())
    return Dr


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def _cubic_sites(ncell: int, a: float, basis: np.ndarray) -> np.ndarray:
    g = np.array(np.meshgrid(*[np.arange(ncell)] * 3, indexing="ij")).reshape(3, -1).T
    pts = (g[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return pts * a


def tiny_cubic(seed: int = SEED_BASE + 1) -> Structure:
    """8 atoms on a 2x2x2 simple-cubic lattice (a = 5 Bohr), one 13/40 species.

    Orbital cutoff 7 Bohr, Coulomb range 14 Bohr, no screening.
    """
    rng = np.random.default_rng(seed)
    tau = _cubic_sites(2, 5.0, np.zeros((1, 3))) + rng.uniform(-0.2, 0.2, size=(8, 3))
    return Structure("sc8", tau, np.eye(3) * 10.0, np.zeros(8, np.int32), [SPECIES_SI40],
                     rc=7.0, rv=14.0, theta=0.0, theta_cs=0.0, seed=seed, d_kind="haar")


def diamond64(seed: int = SEED_BASE + 2) -> Structure:
    """64-atom diamond-like cell: 8-atom conventional cell a = 10.26 Bohr, 2x2x2."""
    rng = np.random.default_rng(seed)
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])
    tau = _cubic_sites(2, 10.26, basis) + rng.uniform(-0.1, 0.1, size=(64, 3))
    return Structure("diamond64", tau, np.eye(3) * 20.52, np.zeros(64, np.int32), [SPECIES_SI75],
                     rc=8.0, rv=20.0, theta=1e-4, theta_cs=1e-7, seed=seed, d_kind="haar")


def _perovskite(ncell: int, seed: int, strain: float, n_sub: int, theta: float, name: str) -> Structure:
    """ABX3 cubic cells (a = 11.6 Bohr): A at 0, B at centre, X at face centres.

    Each X is displaced 0.3 Bohr along a seeded direction perpendicular to its
    B-X-B axis; optional symmetric strain of the lattice (fractional
    coordinates kept) and substitution of ``n_sub`` B sites by species 3.
    """
    rng = np.random.default_rng(seed)
    a = 11.6
    basis = np.array([[0, 0, 0], [.5, .5, .5], [.5, .5, 0], [.5, 0, .5], [0, .5, .5]])
    spec_cell = np.array([0, 1, 2, 2, 2], np.int32)
    axis_cell = np.array([-1, -1, 2, 1, 0])            # B-X-B axis of each X site
    frac = _cubic_sites(ncell, 1.0, basis) / ncell
    species = np.tile(spec_cell, ncell**3)
    axes = np.tile(axis_cell, ncell**3)
    lat = np.eye(3) * (a * ncell)
    tau = frac @ lat
    for i in np.nonzero(species == 2)[0]:
        v = rng.normal(size=3)
        v[axes[i]] = 0.0
        tau[i] += 0.3 * v / np.linalg.norm(v)
    dims = [SPECIES_A, SPECIES_B, SPECIES_X]
    if strain > 0:
        e = rng.uniform(-1.0, 1.0, size=(3, 3))
        e = 0.5 * (e + e.T)
        e *= strain / np.max(np.abs(e))
        frac_now = tau @ np.linalg.inv(lat)
        lat = lat @ (np.eye(3) + e).T
        tau = frac_now @ lat
    if n_sub > 0:
        bsites = np.nonzero(species == 1)[0]
        pick = rng.choice(bsites, size=n_sub, replace=False)
        species = species.copy()
        species[pick] = 3
        dims = dims + [SPECIES_BP]
    return Structure(name, tau, lat, species, dims, rc=8.0, rv=20.0, theta=theta,
                     theta_cs=1e-3 * theta, seed=seed, d_kind="goe")


def perovskite320(seed: int = SEED_BASE + 3) -> Structure:
    return _perovskite(4, seed, 0.0, 0, 1e-4, "abx3_320")


def perovskite1080(seed: int = SEED_BASE + 4) -> Structure:
    return _perovskite(6, seed, 0.01, int(round(0.02 * 216)), 1e-5, "abx3_1080")


def serving_request(i: int, rng_seed: Optional[int] = None) -> Structure:
    """One request of the serving stream: 20..500 atoms, ABX3-like species mix.

    Cubic or orthorhombic cell (aspect ratios in [0.8, 1.25]) at perovskite
    density 5 / 11.6^3, atoms on a jittered grid, species A:B:X = 1:1:3.
    """
    seed = SEED_BASE * 1000 + i if rng_seed is None else rng_seed
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 501))
    vol = n * 11.6**3 / 5.0
    asp = np.ones(3) if rng.uniform() < 0.5 else rng.uniform(0.8, 1.25, size=3)
    side = asp * (vol / np.prod(asp)) ** (1.0 / 3.0)
    grid = np.maximum(1, np.round(side / np.mean(side) * n ** (1.0 / 3.0))).astype(int)
    while np.prod(grid) < n:
        grid[np.argmin(grid / side)] += 1
    pts = np.array(np.meshgrid(*[np.arange(g) for g in grid], indexing="ij")).reshape(3, -1).T
    pts = pts[rng.permutation(pts.shape[0])[:n]]
    frac = (pts + 0.5 + rng.uniform(-0.2, 0.2, size=pts.shape)) / grid
    lat = np.diag(side)
    species = rng.permutation(np.array([0] * (n // 5) + [1] * (n // 5) + [2] * (n - 2 * (n // 5)), np.int32))
    return Structure(f"req{i}", frac @ lat, lat, species, [SPECIES_A, SPECIES_B, SPECIES_X],
                     rc=8.0, rv=20.0, theta=1e-4, theta_cs=1e-7, seed=seed, d_kind="gersh")


def workload(k: int) -> Structure:
    """The four fixed workloads: 1 = 8-atom cubic, 2 = 64-atom diamond,
    3 = 320-atom perovskite, 4 = 1080-atom strained/substituted perovskite."""
    return {1: tiny_cubic, 2: diamond64, 3: perovskite320, 4: perovskite1080}[k]()


def small_case(natom: int = 3, n_ao: int = 3, n_abf: int = 5, box: float = 6.0, rc: float = 4.5,
               rv: float = 7.0, seed: int = 5, theta: float = 0.0, theta_cs: float = 0.0,
               nspecies: int = 1) -> Structure:
    """Tiny random periodic cell for pins (finite differences, brute force):
    a lattice within 0.3 Bohr of a cube of side ``box`` and atoms at uniform
    random fractional positions."""
    rng = np.random.default_rng(seed)
    lat = np.eye(3) * box + rng.uniform(-0.3, 0.3, size=(3, 3))
    frac = rng.uniform(0, 1, size=(natom, 3))
    tau = frac @ lat
    dims = [(n_ao + k, n_abf + 2 * k) for k in range(nspecies)]
    species = (np.arange(natom) % nspecies).astype(np.int32)
    return Structure(f"small{natom}", tau, lat, species, dims, rc=rc, rv=rv, theta=theta,
                     theta_cs=theta_cs, seed=seed, d_kind="haar")
