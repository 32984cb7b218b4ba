"""ctypes binding of the HIP library (C-ABI in ``include/lrx.h``).

Argument marshalling only: every step of an evaluation runs in the library's
kernels.  Block values may be torch CUDA tensors (passed as device pointers,
borrowed by the library) or host arrays (copied).  The library is loaded from
this package's directory; if it is missing the binding raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrx.so")

FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}
NSTAGES = 9

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_f32p = ctypes.POINTER(ctypes.c_float)
_u8p = ctypes.POINTER(ctypes.c_uint8)


class LrxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lrx error {code}: {msg}")
        self.code = code


BATCH_EAGER = 1
BATCH_NO_TUNE = 2
MAX_ALPHA_TILES = 8
SCRATCH_BYTES = 128 << 20     # LRX_SCRATCH_BYTES of include/lrx.h


class Options(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("theta_cs", ctypes.c_double),
                ("precision", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("theta_tensor", ctypes.c_double * 5)]


SCREEN_PER_TENSOR = 4


def _options(theta, theta_cs, precision, timing=0, flags=0, thresholds=None):
    """lrx_options; thresholds = (C, V, D, dC, dV) selects per-tensor screening."""
    o = Options(float(theta), float(theta_cs), PRECISIONS.get(precision, precision), int(bool(timing)), int(flags), 0)
    if thresholds is not None:
        t = [float(x) for x in thresholds]
        assert len(t) == 5
        o.flags |= SCREEN_PER_TENSOR
        for k in range(5):
            o.theta_tensor[k] = t[k]
    return o


class Blocks(ctypes.Structure):
    _fields_ = [("nblk", ctypes.c_int64), ("first", _i32p), ("second", _i32p), ("R", _i32p),
                ("off", _i64p), ("val", ctypes.c_void_p), ("dval", ctypes.c_void_p), ("nval", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("kept_c_blocks", ctypes.c_int64), ("kept_v_blocks", ctypes.c_int64),
                ("alive_c_pairs", ctypes.c_int64), ("alive_v_pairs", ctypes.c_int64),
                ("alive_triples", ctypes.c_int64), ("h_slots", ctypes.c_int64),
                ("flop_alg", ctypes.c_double), ("flop_triple", ctypes.c_double),
                ("flop_triple_group", ctypes.c_double * 9),
                ("bytes_alg", ctypes.c_double), ("device_bytes", ctypes.c_double),
                ("work_bytes", ctypes.c_double * 3), ("work_held", ctypes.c_int32 * 3),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        for k in ("flop_triple_group", "work_bytes", "work_held"):
            out[k] = list(out[k])
        return out


_lib = None

EXPORTS = ["lrx_create", "lrx_set_structure", "lrx_set_tensors", "lrx_evaluate", "lrx_block_gradients",
           "lrx_keep_masks", "lrx_get_stats", "lrx_stage_times", "lrx_stage_name", "lrx_evaluate_batch",
           "lrx_batch_tuning", "lrx_last_error", "lrx_destroy", "lrx_pool_trim", "lrx_group_times",
           "lrx_submit", "lrx_wait", "lrx_evaluate_noalloc", "lrx_enumerate_pairs", "lrx_hamiltonian",
           "lrx_hamiltonian_info", "lrx_prepare_c", "lrx_set_kpoint_tensors"]


def load(path: Optional[str] = None):
    """Load ``liblrx.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2412_11081_amd.build`")
    lib = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    lib.lrx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp]
    lib.lrx_set_structure.argtypes = [vp, ctypes.c_int32, _f64p, _f64p, _i32p, _i32p]
    lib.lrx_set_tensors.argtypes = [vp, ctypes.POINTER(Blocks), ctypes.POINTER(Blocks), vp, ctypes.c_int32]
    lib.lrx_set_kpoint_tensors.argtypes = [vp, _i32p, ctypes.POINTER(Blocks), ctypes.POINTER(Blocks), vp, vp,
                                           ctypes.c_int32]
    lib.lrx_evaluate.argtypes = [vp, ctypes.POINTER(Options), _f64p, _f64p, _f64p]
    lib.lrx_block_gradients.argtypes = [vp, _f64p, _f64p]
    lib.lrx_keep_masks.argtypes = [vp, _u8p, _u8p, _u8p]
    lib.lrx_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.lrx_stage_times.argtypes = [vp, _f32p, ctypes.c_int32]
    lib.lrx_stage_name.argtypes = [ctypes.c_int32]
    lib.lrx_stage_name.restype = ctypes.c_char_p
    lib.lrx_evaluate_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(Options), _f64p, _f64p, _f64p]
    lib.lrx_batch_tuning.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
    lib.lrx_last_error.argtypes = [vp]
    lib.lrx_last_error.restype = ctypes.c_char_p
    lib.lrx_destroy.argtypes = [vp]
    lib.lrx_destroy.restype = None
    lib.lrx_pool_trim.argtypes = [ctypes.c_int32, ctypes.c_uint64]
    lib.lrx_group_times.argtypes = [vp, _f32p, ctypes.c_int32]
    lib.lrx_submit.argtypes = [vp, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_int64)]
    lib.lrx_wait.argtypes = [vp, ctypes.c_int64, _f64p, _f64p, _f64p]
    lib.lrx_evaluate_noalloc.argtypes = [vp, ctypes.POINTER(Options), _f64p, _f64p, _f64p]
    lib.lrx_enumerate_pairs.argtypes = [ctypes.c_int32, ctypes.c_int32, _f64p, _f64p, ctypes.c_double, ctypes.c_int64,
                                        _i32p, _i32p, _i32p, ctypes.POINTER(ctypes.c_int64)]
    lib.lrx_hamiltonian.argtypes = [vp, ctypes.POINTER(Options), _f64p, vp, ctypes.c_int32]
    lib.lrx_hamiltonian_info.argtypes = [vp, _f32p, _f64p]
    lib.lrx_prepare_c.argtypes = [ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, ctypes.POINTER(Blocks),
                                  ctypes.POINTER(Blocks), ctypes.c_int32, vp, vp, ctypes.POINTER(ctypes.c_double)]
    for f in ("lrx_prepare_c", "lrx_hamiltonian", "lrx_hamiltonian_info", "lrx_evaluate_noalloc", "lrx_enumerate_pairs", "lrx_create", "lrx_set_structure", "lrx_set_tensors", "lrx_evaluate", "lrx_block_gradients",
              "lrx_keep_masks", "lrx_get_stats", "lrx_stage_times", "lrx_evaluate_batch", "lrx_batch_tuning",
              "lrx_pool_trim", "lrx_group_times", "lrx_submit", "lrx_wait"):
        getattr(lib, f).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _np(a, dt):
    return np.ascontiguousarray(np.asarray(a), dtype=dt)


def _ptr(a, t):
    return a.ctypes.data_as(t)


class Context:
    """One structure on one device.  Mirrors the lrx_* calls one to one."""

    def __init__(self, device: int = 0, stream=None):
        self.lib = load()
        self.h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
        self._check(self.lib.lrx_create(ctypes.byref(self.h), int(device), s), init=True)
        self._keep = []
        self.natom = 0
        self.nC = self.nV = 0
        self.ncell = 1   # cells of the k-point supercell (1: the Gamma point)

    def _check(self, rc, init=False):
        if rc != 0:
            msg = "" if init else self.lib.lrx_last_error(self.h).decode()
            raise LrxError(rc, msg)

    def set_structure(self, tau, lat, nao, nabf):
        self._tau, self._lat = _np(tau, np.float64), _np(lat, np.float64)
        self._nao, self._nabf = _np(nao, np.int32), _np(nabf, np.int32)
        self.natom = int(self._nao.shape[0])
        self.ncell = 1
        self._check(self.lib.lrx_set_structure(self.h, self.natom, _ptr(self._tau, _f64p), _ptr(self._lat, _f64p),
                                               _ptr(self._nao, _i32p), _ptr(self._nabf, _i32p)))

    def _blocks(self, blk: Dict, keep):
        first, second = _np(blk["first"], np.int32), _np(blk["second"], np.int32)
        R, off = _np(blk["R"], np.int32).reshape(-1), _np(blk["off"], np.int64)
        val, dval = blk["val"], blk["dval"]
        keep += [first, second, R, off]
        b = Blocks()
        b.nblk = int(first.shape[0])
        b.first, b.second, b.R, b.off = _ptr(first, _i32p), _ptr(second, _i32p), _ptr(R, _i32p), _ptr(off, _i64p)
        if hasattr(val, "data_ptr"):
            b.val, b.dval, b.nval = val.data_ptr(), dval.data_ptr(), int(val.numel())
            on_dev = val.is_cuda
            keep += [val, dval]
        else:
            v, dv = _np(val, np.float64), _np(dval, np.float64)
            keep += [v, dv]
            b.val, b.dval, b.nval = v.ctypes.data, dv.ctypes.data, int(v.size)
            on_dev = False
        return b, on_dev

    def set_tensors(self, C: Dict, V: Dict, D):
        keep = []
        bc, dc = self._blocks(C, keep)
        bv, dv = self._blocks(V, keep)
        if hasattr(D, "data_ptr"):
            dptr, dd = D.data_ptr(), D.is_cuda
            keep.append(D)
        else:
            Dm = _np(D, np.float64)
            keep.append(Dm)
            dptr, dd = Dm.ctypes.data, False
        if not (dc == dv == dd):
            raise ValueError("C, V and D must all be on the device or all on the host")
        if dc:
            # the library reads the tensors on its own stream: finish the work
            # that produced them on the caller's streams first
            import torch

            torch.cuda.current_stream().synchronize()
        self._check(self.lib.lrx_set_tensors(self.h, ctypes.byref(bc), ctypes.byref(bv), ctypes.c_void_p(dptr), int(dc)))
        self._keep = keep
        self.nC, self.nV = int(bc.nblk), int(bv.nblk)
        self.ncell = 1

    def set_kpoint_tensors(self, nk, C: Dict, V: Dict, Dk):
        """lrx_set_kpoint_tensors: Dk [n_cells][n_tot][n_tot], complex or real
        (numpy, or a torch tensor on the context's device), per offset
        r = r0 + nk0 (r1 + nk1 r2) of the Born-von Karman supercell."""
        keep = []
        bc, dc = self._blocks(C, keep)
        bv, dv = self._blocks(V, keep)
        nkv = np.ascontiguousarray(nk, np.int32)
        assert nkv.shape == (3,)
        keep.append(nkv)
        if hasattr(Dk, "data_ptr"):
            import torch

            dd = Dk.is_cuda
            re = Dk.real.contiguous() if Dk.is_complex() else Dk.to(torch.float64).contiguous()
            im = Dk.imag.contiguous() if Dk.is_complex() else None
            keep += [re] + ([im] if im is not None else [])
            pre, pim = re.data_ptr(), (im.data_ptr() if im is not None else None)
        else:
            Dn = np.asarray(Dk)
            re = np.ascontiguousarray(Dn.real, np.float64)
            im = np.ascontiguousarray(Dn.imag, np.float64) if np.iscomplexobj(Dn) else None
            keep += [re] + ([im] if im is not None else [])
            pre, pim, dd = re.ctypes.data, (im.ctypes.data if im is not None else None), False
        if not (dc == dv == dd):
            raise ValueError("C, V and D must all be on the device or all on the host")
        if dc:
            import torch

            torch.cuda.current_stream().synchronize()
        self._check(self.lib.lrx_set_kpoint_tensors(self.h, _ptr(nkv, _i32p), ctypes.byref(bc), ctypes.byref(bv),
                                                    ctypes.c_void_p(pre), ctypes.c_void_p(pim), int(dc)))
        self._keep = keep
        self.nC, self.nV = int(bc.nblk), int(bv.nblk)
        self.ncell = int(np.prod(nkv))

    def evaluate(self, theta=0.0, theta_cs=0.0, precision="fp64", timing=False, thresholds=None):
        """lrx_evaluate; thresholds = (C, V, D, dC, dV) for per-tensor screening."""
        o = _options(theta, theta_cs, precision, timing, thresholds=thresholds)
        E = ctypes.c_double()
        F = np.zeros((self.natom, 3))
        S = np.zeros((3, 3))
        self._check(self.lib.lrx_evaluate(self.h, ctypes.byref(o), ctypes.byref(E), _ptr(F, _f64p), _ptr(S, _f64p)))
        return E.value, F, S

    def evaluate_noalloc(self, theta=0.0, theta_cs=0.0, precision="fp64", thresholds=None):
        """lrx_evaluate_noalloc: the evaluation with the library's fixed device
        scratch for its work buffers (no device allocation)."""
        o = _options(theta, theta_cs, precision, thresholds=thresholds)
        E = ctypes.c_double()
        F = np.zeros((self.natom, 3))
        S = np.zeros((3, 3))
        self._check(self.lib.lrx_evaluate_noalloc(self.h, ctypes.byref(o), ctypes.byref(E), _ptr(F, _f64p),
                                                  _ptr(S, _f64p)))
        return E.value, F, S

    def hamiltonian(self, theta=0.0, theta_cs=0.0, thresholds=None, out=None, timing=False):
        """lrx_hamiltonian: (E, H^X).  out: a contiguous float64 torch tensor
        [n_tot][n_tot] on the context's device to write H^X into (returned
        as is); otherwise H^X comes back as a numpy array."""
        o = _options(theta, theta_cs, "fp64", timing, thresholds=thresholds)
        E = ctypes.c_double()
        if out is not None:
            if not (out.is_cuda and out.is_contiguous() and str(out.dtype) == "torch.float64"):
                raise ValueError("out: a contiguous float64 device tensor")
            import torch

            torch.cuda.current_stream().synchronize()
            self._check(self.lib.lrx_hamiltonian(self.h, ctypes.byref(o), ctypes.byref(E),
                                                 ctypes.c_void_p(out.data_ptr()), 1))
            return E.value, out
        nt = int(np.sum(self._nao))
        H = np.zeros((nt, nt))
        self._check(self.lib.lrx_hamiltonian(self.h, ctypes.byref(o), ctypes.byref(E),
                                             ctypes.c_void_p(H.ctypes.data), 0))
        return E.value, H

    def hamiltonian_info(self, timing=True):
        """lrx_hamiltonian_info: ({stage: ms} or None, {flop kind: count})."""
        ms = (ctypes.c_float * 5)()
        fl = (ctypes.c_double * 4)()
        self._check(self.lib.lrx_hamiltonian_info(self.h, ms if timing else None, fl))
        names = ("screen", "hbuild", "slot", "g3", "final")
        return ({n: float(ms[i]) for i, n in enumerate(names)} if timing else None,
                {"total": fl[0], "slot": fl[1], "g3": fl[2], "hbuild": fl[3]})

    def submit(self, theta=0.0, theta_cs=0.0, precision="fp64", thresholds=None):
        """lrx_submit: queue an evaluation on the context's stream; returns its ticket."""
        o = _options(theta, theta_cs, precision, thresholds=thresholds)
        t = ctypes.c_int64()
        self._check(self.lib.lrx_submit(self.h, ctypes.byref(o), ctypes.byref(t)))
        return t.value

    def wait(self, ticket):
        """lrx_wait: (E, F, sigma) of a submitted evaluation."""
        E = ctypes.c_double()
        F = np.zeros((self.natom, 3))
        S = np.zeros((3, 3))
        self._check(self.lib.lrx_wait(self.h, int(ticket), ctypes.byref(E), _ptr(F, _f64p), _ptr(S, _f64p)))
        return E.value, F, S

    def block_gradients(self):
        gC, gV = np.zeros((self.nC, 3)), np.zeros((self.nV, 3))
        self._check(self.lib.lrx_block_gradients(self.h, _ptr(gC, _f64p), _ptr(gV, _f64p)))
        return gC, gV

    def keep_masks(self):
        kC, kV = np.zeros(self.nC, np.uint8), np.zeros(self.nV, np.uint8)
        ns = self.natom * self.ncell   # supercell atoms with k-point sampling
        kD = np.zeros(ns * ns, np.uint8)
        self._check(self.lib.lrx_keep_masks(self.h, _ptr(kC, _u8p), _ptr(kV, _u8p), _ptr(kD, _u8p)))
        return kC, kV, kD

    def stats(self):
        s = Stats()
        self._check(self.lib.lrx_get_stats(self.h, ctypes.byref(s)))
        return s.as_dict()

    def stage_times(self):
        ms = (ctypes.c_float * NSTAGES)()
        rc = self.lib.lrx_stage_times(self.h, ms, NSTAGES)
        if rc < 0:
            self._check(rc)
        return {self.lib.lrx_stage_name(i).decode(): float(ms[i]) for i in range(NSTAGES)}

    def group_times(self):
        """lrx_group_times: {MT: ms} of the triple launches of the last timed evaluation."""
        ms = (ctypes.c_float * (MAX_ALPHA_TILES + 1))()
        rc = self.lib.lrx_group_times(self.h, ms, MAX_ALPHA_TILES + 1)
        if rc < 0:
            self._check(rc)
        return {mt: float(ms[mt]) for mt in range(MAX_ALPHA_TILES + 1) if ms[mt] > 0}

    def close(self):
        if self.h:
            self.lib.lrx_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def context_for(structure, mats, device: int = 0, stream=None) -> Context:
    """Context holding one synthetic structure (``synth.Structure``) and its
    materialised blocks (``Structure.materialize``)."""
    ctx = Context(device, stream)
    ctx.set_structure(structure.tau, structure.lat, structure.nao, structure.nabf)
    ctx.set_tensors(mats["C"], mats["V"], mats["D"])
    return ctx


def evaluate_batch(contexts, theta=0.0, theta_cs=0.0, precision="fp64", eager=False, tune=True, thresholds=None):
    """lrx_evaluate_batch over ``contexts`` (distinct, one device): returns
    lists of E, F [natom][3] and sigma [3][3], one entry per context."""
    if not contexts:
        return [], [], []
    lib = contexts[0].lib
    n = len(contexts)
    handles = (ctypes.c_void_p * n)(*[c.h.value for c in contexts])
    flags = (BATCH_EAGER if eager else 0) | (0 if tune else BATCH_NO_TUNE)
    o = _options(theta, theta_cs, precision, flags=flags, thresholds=thresholds)
    E = np.zeros(n)
    nat = [c.natom for c in contexts]
    F = np.zeros((sum(nat), 3))
    S = np.zeros((n, 3, 3))
    contexts[0]._check(lib.lrx_evaluate_batch(handles, n, ctypes.byref(o), _ptr(E, _f64p), _ptr(F, _f64p),
                                              _ptr(S, _f64p)))
    out_f, k = [], 0
    for a in nat:
        out_f.append(F[k:k + a].copy())
        k += a
    return list(E), out_f, [S[i].copy() for i in range(n)]


def batch_tuning(context):
    """Launch shapes of the last plan built with ``context`` first:
    {MT: (mode, ms_mode0, ms_mode1)}; the times are 0 for groups that plan did
    not time (shapes already chosen earlier in the process)."""
    mode = (ctypes.c_int32 * (MAX_ALPHA_TILES + 1))()
    ms = (ctypes.c_float * (2 * (MAX_ALPHA_TILES + 1)))()
    context.lib.lrx_batch_tuning(context.h, mode, ms)
    return {mt: (int(mode[mt]), float(ms[2 * mt]), float(ms[2 * mt + 1])) for mt in range(1, MAX_ALPHA_TILES + 1)}


def prepare_c(nao, nabf, V, T, device: int = 0):
    """lrx_prepare_c (Eq. C_VA and the gradient of C): the C blocks of the keys
    of T from V and the three-centre integrals T, in key order.  Returns
    (blocks, flop): blocks as for lrx_set_tensors (keys of T, offsets, val,
    dval) on the device when T's values are device tensors, else numpy."""
    lib = load()
    keep = []
    bv, v_dev = Context._blocks(None, V, keep)
    bt, t_dev = Context._blocks(None, T, keep)
    if v_dev != t_dev:
        raise ValueError("V and T must both be on the device or both on the host")
    nao_, nabf_ = _np(nao, np.int32), _np(nabf, np.int32)
    first, second = _np(T["first"], np.int32), _np(T["second"], np.int32)
    sizes = nabf_[first].astype(np.int64) * nao_[first] * nao_[second]
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    total = int(sizes.sum())
    if t_dev:
        import torch

        dev = T["val"].device
        torch.cuda.current_stream().synchronize()
        cv = torch.empty(max(total, 1), dtype=torch.float64, device=dev)
        cd = torch.empty(max(3 * total, 1), dtype=torch.float64, device=dev)
        pv, pd = ctypes.c_void_p(cv.data_ptr()), ctypes.c_void_p(cd.data_ptr())
    else:
        cv, cd = np.empty(max(total, 1)), np.empty(max(3 * total, 1))
        pv, pd = ctypes.c_void_p(cv.ctypes.data), ctypes.c_void_p(cd.ctypes.data)
    fl = ctypes.c_double()
    rc = lib.lrx_prepare_c(int(device), int(nao_.shape[0]), _ptr(nao_, _i32p), _ptr(nabf_, _i32p), ctypes.byref(bv),
                           ctypes.byref(bt), int(t_dev), pv, pd, ctypes.byref(fl))
    if rc != 0:
        raise LrxError(rc, "lrx_prepare_c failed (bad arguments, a missing V block, or a Coulomb matrix of a "
                           "pair that is not positive definite)")
    return dict(first=T["first"], second=T["second"], R=T["R"], off=off, val=cv[:total], dval=cd[:3 * total]), fl.value


def enumerate_pairs(tau, lat, rcut, device: int = 0, capacity: int = 0):
    """lrx_enumerate_pairs: keys (first, second, R[n][3]) of every image pair
    within rcut, sorted by (first, second, R).  Calls the library again with
    the exact size when the first buffer (``capacity``, default an estimate
    from the cell's density) is too small."""
    lib = load()
    tau = _np(tau, np.float64)
    lat = _np(lat, np.float64)
    n = int(tau.shape[0])
    if capacity <= 0:
        vol = abs(float(np.linalg.det(lat)))
        dens = n / vol if vol > 0 and np.isfinite(vol) else 0.0   # the library rejects a singular lattice
        capacity = int(min(n * (1 + 1.5 * 4.19 * rcut ** 3 * dens), 1 << 30)) + 64
    for _ in range(2):
        f = np.zeros(capacity, np.int32)
        s = np.zeros(capacity, np.int32)
        R = np.zeros((capacity, 3), np.int32)
        cnt = ctypes.c_int64()
        rc = lib.lrx_enumerate_pairs(int(device), n, _ptr(tau, _f64p), _ptr(lat, _f64p), float(rcut), int(capacity),
                                     _ptr(f, _i32p), _ptr(s, _i32p), _ptr(R, _i32p), ctypes.byref(cnt))
        if rc == 0:
            k = int(cnt.value)
            return f[:k].copy(), s[:k].copy(), R[:k].copy()
        if rc != -5:
            raise LrxError(rc, "lrx_enumerate_pairs failed (bad arguments or device error)")
        capacity = int(cnt.value)
    raise LrxError(-5, "lrx_enumerate_pairs: capacity")


def pool_trim(device: int = 0, keep_bytes: int = 0):
    """lrx_pool_trim: hand the device pool's unused memory back to the driver."""
    rc = load().lrx_pool_trim(int(device), int(keep_bytes))
    if rc != 0:
        raise LrxError(rc, f"lrx_pool_trim(device={device}) failed")
