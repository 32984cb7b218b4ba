"""Image-pair enumeration oracle (test infrastructure only).

Methods of the paper: every basis function carries a combined index of an
atom and a lattice vector, and each two-centre block (C within the orbital
cutoff, V within the Coulomb range) is a function of the displacement
r = tau[second] + R.L - tau[first] of its two atoms.  The pairs are every
(first, second, R) whose image lies inside the cutoff sphere of ``first``.

The decision is written out with each operation rounded on its own, in this
order (numpy element-wise operations, no fused multiply-add):

    shift = (R_0 * a1 + R_1 * a2) + R_2 * a3
    r     = (tau[second] - tau[first]) + shift
    d2    = (r_x * r_x + r_y * r_y) + r_z * r_z        kept iff d2 < rcut * rcut

over R_i in [-span_i, span_i], span_i = ceil(rcut / h_i) + 1 with h_i the
spacing of the lattice planes spanned by the other two vectors.  Output
sorted by (first, second, R_0, R_1, R_2).  ``pairs_loops`` is the same rule as
plain Python loops for tiny cells.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def _spans(lat, rcut):
    lat = np.asarray(lat, np.float64)
    vol = abs(float(np.linalg.det(lat)))
    out = []
    for i in range(3):
        c = np.cross(lat[(i + 1) % 3], lat[(i + 2) % 3])
        h = vol / float(np.sqrt(np.dot(c, c)))
        out.append(int(math.ceil(rcut / h) + 1))
    return out


def _images(spans):
    return [r for r in itertools.product(*[range(-s, s + 1) for s in spans])]   # lexicographic


def pairs(tau, lat, rcut):
    """Keys (first [n], second [n], R [n][3]) as int32 arrays."""
    tau = np.asarray(tau, np.float64)
    lat = np.asarray(lat, np.float64)
    n = tau.shape[0]
    imgs = np.array(_images(_spans(lat, rcut)), np.float64)               # [nR, 3]
    shift = (imgs[:, 0:1] * lat[0][None, :] + imgs[:, 1:2] * lat[1][None, :]) + imgs[:, 2:3] * lat[2][None, :]
    rc2 = rcut * rcut
    F, S, R = [], [], []
    for f in range(n):
        rel = tau - tau[f][None, :]                                        # [n, 3]: tau[second] - tau[first]
        r = rel[:, None, :] + shift[None, :, :]                            # [n, nR, 3]
        d2 = (r[..., 0] * r[..., 0] + r[..., 1] * r[..., 1]) + r[..., 2] * r[..., 2]
        s_idx, r_idx = np.nonzero(d2 < rc2)                                # second-major, then R order
        F.append(np.full(s_idx.shape, f, np.int32))
        S.append(s_idx.astype(np.int32))
        R.append(imgs[r_idx].astype(np.int32).reshape(-1, 3))
    return np.concatenate(F), np.concatenate(S), np.concatenate(R).reshape(-1, 3)


def pairs_loops(tau, lat, rcut):
    """The same keys from plain Python loops (tiny cells only)."""
    tau = [list(map(float, t)) for t in np.asarray(tau, np.float64)]
    lat = [list(map(float, a)) for a in np.asarray(lat, np.float64)]
    rc2 = rcut * rcut
    out = []
    imgs = _images(_spans(lat, rcut))
    for f in range(len(tau)):
        for s in range(len(tau)):
            for R in imgs:
                r = []
                for x in range(3):
                    sh = (R[0] * lat[0][x] + R[1] * lat[1][x]) + R[2] * lat[2][x]
                    r.append((tau[s][x] - tau[f][x]) + sh)
                d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]
                if d2 < rc2:
                    out.append((f, s, R))
    F = np.array([o[0] for o in out], np.int32)
    S = np.array([o[1] for o in out], np.int32)
    R = np.array([o[2] for o in out], np.int32).reshape(-1, 3)
    return F, S, R
