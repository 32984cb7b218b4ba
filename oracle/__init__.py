"""CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``lrx_oracle.c`` (plain FP64
C, built with gcc by :func:`build`) through ctypes and shares nothing with the
GPU library.  See ``lrx_oracle.c`` for what is computed and which passages of
the paper each part follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lrx_oracle.c")
_LIB = os.path.join(_HERE, "liblrx_oracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class OrcInput(ctypes.Structure):
    _fields_ = [
        ("natom", ctypes.c_int32), ("tau", _f64p), ("lat", _f64p), ("nao", _i32p), ("nabf", _i32p),
        ("nC", ctypes.c_int64), ("C_first", _i32p), ("C_second", _i32p), ("C_R", _i32p), ("C_off", _i64p),
        ("C_val", _f64p), ("C_dval", _f64p),
        ("nV", ctypes.c_int64), ("V_first", _i32p), ("V_second", _i32p), ("V_R", _i32p), ("V_off", _i64p),
        ("V_val", _f64p), ("V_dval", _f64p),
        ("D", _f64p),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP enabled; one thread unless asked)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_screen.argtypes = [ctypes.POINTER(OrcInput), ctypes.c_double, ctypes.c_double, _u8p, _u8p, _u8p, _f64p]
        lib.orc_screen.restype = ctypes.c_int
        lib.orc_contract.argtypes = [ctypes.POINTER(OrcInput), _u8p, _u8p, _u8p, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_int64, ctypes.c_int, _f64p, _f64p, _f64p]
        lib.orc_contract.restype = ctypes.c_int
        lib.orc_contract2.argtypes = [ctypes.POINTER(OrcInput), _u8p, _u8p, _u8p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _f64p, _f64p,
                                      _f64p, _f64p]
        lib.orc_contract2.restype = ctypes.c_int
        lib.orc_screen5.argtypes = [ctypes.POINTER(OrcInput), _f64p, ctypes.c_double, _u8p, _u8p, _u8p, _f64p]
        lib.orc_screen5.restype = ctypes.c_int
        lib.orc_hamiltonian.argtypes = [ctypes.POINTER(OrcInput), _u8p, _u8p, _u8p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, _f64p]
        lib.orc_hamiltonian.restype = ctypes.c_int
        lib.orc_forces_stress.argtypes = [ctypes.POINTER(OrcInput), _f64p, _f64p, _f64p, _f64p]
        lib.orc_has_openmp.restype = ctypes.c_int
        lib.orc_screen_d_kp.argtypes = [ctypes.POINTER(OrcInput), _i32p, _f64p, _f64p, ctypes.c_double, _u8p]
        lib.orc_screen_d_kp.restype = None
        lib.orc_contract_kp.argtypes = [ctypes.POINTER(OrcInput), _i32p, _f64p, _f64p, _u8p, _u8p, _u8p,
                                        ctypes.c_int, _f64p, _f64p, _f64p]
        lib.orc_contract_kp.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


class Problem:
    """Host copies of one structure's inputs, in the oracle's C struct."""

    def __init__(self, tau, lat, nao, nabf, C, V, D):
        self.keep = []   # keep numpy arrays alive

        def arr(x, dt):
            if hasattr(x, "detach"):
                x = x.detach().cpu().numpy()
            a = np.ascontiguousarray(np.asarray(x), dtype=dt)
            self.keep.append(a)
            return a

        self.tau = arr(tau, np.float64)
        self.lat = arr(lat, np.float64)
        self.nao = arr(nao, np.int32)
        self.nabf = arr(nabf, np.int32)
        self.natom = int(self.nao.shape[0])
        s = OrcInput()
        s.natom = self.natom
        s.tau, s.lat = _p(self.tau, _f64p), _p(self.lat, _f64p)
        s.nao, s.nabf = _p(self.nao, _i32p), _p(self.nabf, _i32p)
        for tag, blk in (("C", C), ("V", V)):
            first = arr(blk["first"], np.int32)
            setattr(s, f"n{tag}", int(first.shape[0]))
            setattr(s, f"{tag}_first", _p(first, _i32p))
            setattr(s, f"{tag}_second", _p(arr(blk["second"], np.int32), _i32p))
            setattr(s, f"{tag}_R", _p(arr(blk["R"], np.int32), _i32p))
            setattr(s, f"{tag}_off", _p(arr(blk["off"], np.int64), _i64p))
            setattr(s, f"{tag}_val", _p(arr(blk["val"], np.float64), _f64p))
            setattr(s, f"{tag}_dval", _p(arr(blk["dval"], np.float64), _f64p))
        self.Dm = arr(D, np.float64)
        s.D = _p(self.Dm, _f64p)
        self.s = s
        self.nC, self.nV = int(s.nC), int(s.nV)

    @classmethod
    def from_structure(cls, st, mats=None):
        m = mats if mats is not None else st.materialize("cpu")
        return cls(st.tau, st.lat, st.nao, st.nabf, m["C"], m["V"], m["D"])

    # ------------------------------------------------------------------
    def screen(self, theta, theta_cs):
        lib = _load()
        kC = np.zeros(self.nC, np.uint8)
        kV = np.zeros(self.nV, np.uint8)
        kD = np.zeros(self.natom * self.natom, np.uint8)
        S = np.zeros(self.natom * self.natom, np.float64)
        rc = lib.orc_screen(ctypes.byref(self.s), theta, theta_cs, _p(kC, _u8p), _p(kV, _u8p), _p(kD, _u8p), _p(S, _f64p))
        if rc != 0:
            raise ValueError("V block without mirror (second, first, -R)")
        return kC, kV, kD, S.reshape(self.natom, self.natom)

    def screen5(self, thr, theta_cs):
        """Per-tensor screening, thr = (theta_C, theta_V, theta_D, theta_dC,
        theta_dV): bit masks (bit 0 value kept, bit 1 derivative kept) for C
        and V blocks, 0/1 for D pairs, and S(A,B)."""
        lib = _load()
        t = np.ascontiguousarray(thr, np.float64)
        assert t.shape == (5,)
        kC = np.zeros(self.nC, np.uint8)
        kV = np.zeros(self.nV, np.uint8)
        kD = np.zeros(self.natom * self.natom, np.uint8)
        S = np.zeros(self.natom * self.natom, np.float64)
        rc = lib.orc_screen5(ctypes.byref(self.s), _p(t, _f64p), theta_cs, _p(kC, _u8p), _p(kV, _u8p), _p(kD, _u8p),
                             _p(S, _f64p))
        if rc != 0:
            raise ValueError("V block without mirror (second, first, -R)")
        return kC, kV, kD, S.reshape(self.natom, self.natom)

    def contract(self, keep, v_begin=0, v_end=None, focus=None, nthreads=1, bits=False, theta_item=0.0):
        """E and block gradients from the quartets of V blocks [v_begin, v_end).

        keep = (keepC, keepV, keepD): 0/1 masks from screen() (a kept block in
        both lists), or with bits=True the bit masks of screen5().
        theta_item > 0 adds the item-level Cauchy-Schwarz test; the sum of the
        bounds of the skipped energy items is then in self.skipped_bound."""
        lib = _load()
        kC, kV, kD = keep[:3]
        if not bits:
            kC = np.where(np.asarray(kC) != 0, 3, 0).astype(np.uint8)
            kV = np.where(np.asarray(kV) != 0, 3, 0).astype(np.uint8)
        kC = np.ascontiguousarray(kC, np.uint8)
        kV = np.ascontiguousarray(kV, np.uint8)
        kD = np.ascontiguousarray(kD, np.uint8)
        E = np.zeros(1)
        sk = np.zeros(1)
        gC = np.zeros((self.nC, 3))
        gV = np.zeros((self.nV, 3))
        fk, fi = (0, 0) if focus is None else ({"C": 1, "V": 2}[focus[0]], int(focus[1]))
        lib.orc_contract2(ctypes.byref(self.s), _p(kC, _u8p), _p(kV, _u8p), _p(kD, _u8p), int(v_begin),
                          int(self.nV if v_end is None else v_end), fk, fi, int(nthreads), float(theta_item),
                          _p(E, _f64p), _p(gC, _f64p), _p(gV, _f64p), _p(sk, _f64p))
        self.skipped_bound = float(sk[0])
        return float(E[0]), gC, gV

    def hamiltonian(self, keep, nthreads=1, bits=False, focus=None):
        """H^X = dE/dD (Eq. Exx2), dense [n_tot][n_tot], from the quartets'
        energy items; keep as for contract().  focus = (X, Y): only the
        quartets that reach the D block of atoms (X, Y), whose H block is
        then complete (the rest of the matrix is not)."""
        lib = _load()
        kC, kV, kD = keep[:3]
        if not bits:
            kC = np.where(np.asarray(kC) != 0, 3, 0).astype(np.uint8)
            kV = np.where(np.asarray(kV) != 0, 3, 0).astype(np.uint8)
        kC = np.ascontiguousarray(kC, np.uint8)
        kV = np.ascontiguousarray(kV, np.uint8)
        kD = np.ascontiguousarray(kD, np.uint8)
        nt = int(self.nao.sum())
        H = np.zeros((nt, nt))
        fx, fy = (-1, -1) if focus is None else (int(focus[0]), int(focus[1]))
        lib.orc_hamiltonian(ctypes.byref(self.s), _p(kC, _u8p), _p(kV, _u8p), _p(kD, _u8p), fx, fy, int(nthreads),
                            _p(H, _f64p))
        return H

    def forces_stress(self, gC, gV):
        lib = _load()
        F = np.zeros((self.natom, 3))
        sig = np.zeros((3, 3))
        gC = np.ascontiguousarray(gC, np.float64)
        gV = np.ascontiguousarray(gV, np.float64)
        lib.orc_forces_stress(ctypes.byref(self.s), _p(gC, _f64p), _p(gV, _f64p), _p(F, _f64p), _p(sig, _f64p))
        return F, sig

    def evaluate(self, theta, theta_cs, nthreads=1):
        """E_X, F^{X1}[natom][3], sigma^{X1}[3][3] (Ha, Ha/Bohr, Ha/Bohr^3)."""
        keep = self.screen(theta, theta_cs)
        E, gC, gV = self.contract(keep, nthreads=nthreads)
        F, sig = self.forces_stress(gC, gV)
        return dict(E=E, F=F, sigma=sig, gC=gC, gV=gV, keepC=keep[0], keepV=keep[1], keepD=keep[2])


    def evaluate5(self, thr, theta_cs, theta_item=0.0, nthreads=1):
        """E, F, sigma with per-tensor thresholds (screen5) and, for
        theta_item > 0, the item-level Cauchy-Schwarz test."""
        keep = self.screen5(thr, theta_cs)
        E, gC, gV = self.contract(keep, nthreads=nthreads, bits=True, theta_item=theta_item)
        F, sig = self.forces_stress(gC, gV)
        return dict(E=E, F=F, sigma=sig, gC=gC, gV=gV, keepC=keep[0], keepV=keep[1], keepD=keep[2],
                    skipped_bound=self.skipped_bound)


class KProblem(Problem):
    """A unit cell with k-point sampling on an nk[0] x nk[1] x nk[2] mesh:
    the density matrix per cell offset of the Born-von Karman supercell,
    Dk[r][n_tot][n_tot] complex (or real), r = r0 + nk0 (r1 + nk1 r2)
    (lrx_oracle.c, orc_contract_kp)."""

    def __init__(self, tau, lat, nao, nabf, C, V, nk, Dk):
        Dk = Dk.detach().cpu().numpy() if hasattr(Dk, "detach") else np.asarray(Dk)
        self.nk = np.ascontiguousarray(nk, np.int32)
        nr = int(np.prod(self.nk))
        nt = int(np.asarray(nao).sum())
        assert Dk.shape == (nr, nt, nt), Dk.shape
        self.Dre = np.ascontiguousarray(Dk.real, np.float64)
        self.Dim = np.ascontiguousarray(Dk.imag, np.float64) if np.iscomplexobj(Dk) else None
        super().__init__(tau, lat, nao, nabf, C, V, self.Dre[0])

    def screen_d(self, theta_D):
        lib = _load()
        nr = int(np.prod(self.nk))
        kD = np.zeros(nr * self.natom * self.natom, np.uint8)
        lib.orc_screen_d_kp(ctypes.byref(self.s), _p(self.nk, _i32p), _p(self.Dre, _f64p),
                            None if self.Dim is None else _p(self.Dim, _f64p), float(theta_D), _p(kD, _u8p))
        return kD

    def evaluate(self, theta=0.0, thr=None, nthreads=1):
        """E, F, sigma per unit cell: joint screening with theta (C, V, D),
        or per-tensor thresholds thr = (C, V, D, dC, dV); no step 2.
        keepD is [n_cells][natom][natom]."""
        if thr is None:
            kC, kV, _, _ = self.screen(theta, 0.0)
            kC = np.where(kC != 0, 3, 0).astype(np.uint8)
            kV = np.where(kV != 0, 3, 0).astype(np.uint8)
            kD = self.screen_d(theta)
        else:
            kC, kV, _, _ = self.screen5(thr, 0.0)
            kD = self.screen_d(thr[2])
        kC = np.ascontiguousarray(kC, np.uint8)
        kV = np.ascontiguousarray(kV, np.uint8)
        lib = _load()
        E = np.zeros(1)
        gC = np.zeros((self.nC, 3))
        gV = np.zeros((self.nV, 3))
        lib.orc_contract_kp(ctypes.byref(self.s), _p(self.nk, _i32p), _p(self.Dre, _f64p),
                            None if self.Dim is None else _p(self.Dim, _f64p), _p(kC, _u8p), _p(kV, _u8p),
                            _p(kD, _u8p), int(nthreads), _p(E, _f64p), _p(gC, _f64p), _p(gV, _f64p))
        F, sig = self.forces_stress(gC, gV)
        return dict(E=float(E[0]), F=F, sigma=sig, gC=gC, gV=gV, keepC=kC, keepV=kV,
                    keepD=kD.reshape(-1, self.natom, self.natom))


def evaluate_structure(st, theta=None, theta_cs=None, nthreads=1, mats=None):
    pr = Problem.from_structure(st, mats)
    th = st.theta if theta is None else theta
    tcs = st.theta_cs if theta_cs is None else theta_cs
    return pr.evaluate(th, tcs, nthreads=nthreads)


def has_openmp() -> bool:
    return bool(_load().orc_has_openmp())


def timed_sample(pr: Problem, theta, theta_cs, v_count: int, nthreads=1):
    """Time the quartet loop over the first ``v_count`` kept-or-not V blocks.

    Returns (seconds, fraction of all kept V blocks covered).
    """
    keep = pr.screen(theta, theta_cs)
    kV = keep[1]
    t0 = time.perf_counter()
    pr.contract(keep, 0, v_count, nthreads=nthreads)
    dt = time.perf_counter() - t0
    frac = float(kV[:v_count].sum()) / max(1.0, float(kV.sum()))
    return dt, frac
