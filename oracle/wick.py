"""Python entry to the O-W oracle (``wick.c``): plain Wick enumeration, direct O(V^2) sum.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import operators as ops

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wick.c")
_LIB = os.path.join(_HERE, "liboracle_wick.so")
_lib = None

_FL = {"u": 0, "d": 1, "s": 2}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc and OpenMP (FP64 throughout)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        f = lib.oracle_wick
        P = ctypes.c_void_p
        f.argtypes = [ctypes.c_int] * 3 + [P, P, P, P, P, P, P, P, ctypes.c_int, P, P]
        f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _term_arrays(ch):
    nterm = np.zeros(4, dtype=np.int32)
    w = np.zeros((4, 3), dtype=np.float64)
    fl = np.zeros((4, 3, 3), dtype=np.int32)
    for b, terms in enumerate(ops.channel_terms(ch)):
        nterm[b] = len(terms)
        for t, (wt, f) in enumerate(terms):
            w[b, t] = wt
            fl[b, t] = [_FL[q] for q in f]
    return nterm, w, fl


def correlate(S_l, S_s, ch, r_list, lower=False, offsets=None):
    """C_ch(r) for one time slice at the given relative coordinates.

    S_l, S_s: complex128 arrays [Lz][Ly][Lx][12][12].
    ch:       channel tuple (B1, B2, B3, B4), names as in ``operators.BARYONS``.
    r_list:   int array [n][3] of (rx, ry, rz).
    offsets:  per baryon B1..B4 the first of its two spin components (0 upper,
              2 lower); default all 2 if ``lower`` else all 0.
    Returns complex128 [n][16], spin index a + 2*(b + 2*(a' + 2*b')), each spin
    relative to its baryon's offset.
    """
    lib = _load()
    S_l = np.ascontiguousarray(S_l, dtype=np.complex128)
    S_s = np.ascontiguousarray(S_s, dtype=np.complex128)
    Lz, Ly, Lx = S_l.shape[:3]
    assert S_l.shape == (Lz, Ly, Lx, 12, 12) and S_s.shape == S_l.shape
    r = np.ascontiguousarray(np.asarray(r_list, dtype=np.int32).reshape(-1, 3))
    M1 = np.ascontiguousarray([ops.spin_structure(b)[0] for b in ch], dtype=np.complex128)
    M2 = np.ascontiguousarray([ops.spin_structure(b)[1] for b in ch], dtype=np.complex128)
    nterm, w, fl = _term_arrays(ch)
    if offsets is None:
        offsets = (2 if lower else 0,) * 4
    glo = np.ascontiguousarray(offsets, dtype=np.int32)
    assert glo.shape == (4,) and all(g in (0, 2) for g in glo)
    out = np.zeros((r.shape[0], 16), dtype=np.complex128)
    rc = lib.oracle_wick(Lx, Ly, Lz, S_l.ctypes.data, S_s.ctypes.data, M1.ctypes.data, M2.ctypes.data,
                         nterm.ctypes.data, w.ctypes.data, fl.ctypes.data, glo.ctypes.data,
                         r.shape[0], r.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle_wick failed with code %d" % rc)
    return out


def correlate_full(S_l, S_s, ch, r_list):
    """All 256 spin components: [n][256], index alpha + 4*(beta + 4*(alpha' + 4*beta'))
    with every spin over 0..3, assembled from the 16 choices of upper or lower pair
    per baryon (each a call of ``correlate`` with those offsets)."""
    r = np.asarray(r_list, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((r.shape[0], 256), dtype=np.complex128)
    for h in range(16):
        off = tuple(2 * ((h >> i) & 1) for i in range(4))
        part = correlate(S_l, S_s, ch, r, offsets=off)
        for s in range(16):
            sp = [off[i] + ((s >> i) & 1) for i in range(4)]
            out[:, sp[0] + 4 * (sp[1] + 4 * (sp[2] + 4 * sp[3]))] = part[:, s]
    return out


def all_r(Lx, Ly, Lz):
    """Every relative coordinate, x fastest (the order of the output field)."""
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.int32)
