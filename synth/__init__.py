"""Seeded synthetic quark propagators (shared input generator).

This module only draws random numbers; it holds none of the correlator's
arithmetic.  Both the GPU path (through its tests and the benchmark) and the
CPU oracle consume the arrays it returns.

The paper's inputs are wall-source propagators on a CP-PACS/JLQCD N_f=2+1
gauge configuration (Sec. 6), which are not available; these stand-ins have the
same per-site shape: for each flavour f in {light (u=d), strange}, each time
slice t and each site x, a 12x12 complex matrix S_f(x,t)[i][j] with
i = 3*mu + c (sink spin-colour) and j = 3*mu' + c' (source spin-colour).

Every slice is drawn from its own counter-keyed stream
``SeedSequence([seed, flavour, t])`` (Philox4x32-10 bit generator), so a slice
can be regenerated on its own, in any order.

Layout of the arrays: ``[T][z][y][x][12][12]`` complex, C order (x fastest
among the sites).
"""
from __future__ import annotations

import numpy as np

LIGHT, STRANGE = 0, 1
MASSES = (0.5, 0.7)          # decay rates per time slice: light, strange
BASE_SEED = 1510009030


def _rng(seed: int, flavour: int, t: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence([seed, flavour, t, stream])))


def complex_gaussian(rng: np.random.Generator, shape, dtype=np.complex128) -> np.ndarray:
    """Real and imaginary parts independent N(0,1)."""
    rd = np.float64 if dtype == np.complex128 else np.float32
    out = np.empty(shape, dtype=dtype)
    out.real = rng.standard_normal(shape, dtype=rd)
    out.imag = rng.standard_normal(shape, dtype=rd)
    return out


def slice_gaussian(L, t, flavour, seed=BASE_SEED, dtype=np.complex128, masses=MASSES):
    """One time slice: entries N(0,1) complex times exp(-m_f t)."""
    Lx, Ly, Lz = (L, L, L) if np.isscalar(L) else L
    z = complex_gaussian(_rng(seed, flavour, t), (Lz, Ly, Lx, 12, 12), dtype)
    z *= np.exp(-masses[flavour] * t)
    return z


def slice_correlated(L, t, flavour, seed=BASE_SEED, noise=1e-3, dtype=np.complex128, masses=MASSES):
    """One time slice: exp(-m_f t) * (Z_f(x) + noise * eta_f(x, t)).

    Z_f is a t-independent complex Gaussian field and eta_f fresh complex
    Gaussian noise per slice, so that neighbouring slices are strongly
    correlated the way slices of a real propagator are.
    """
    Lx, Ly, Lz = (L, L, L) if np.isscalar(L) else L
    shape = (Lz, Ly, Lx, 12, 12)
    base = complex_gaussian(_rng(seed, flavour, 0, 1), shape, np.complex128)
    eta = complex_gaussian(_rng(seed, flavour, t, 2), shape, np.complex128)
    out = (base + noise * eta) * np.exp(-masses[flavour] * t)
    return out.astype(dtype, copy=False)


def propagators(L, T, seed=BASE_SEED, kind="gaussian", t_list=None, dtype=np.complex128, su3=False):
    """Light and strange propagators for the time slices ``t_list`` (default 0..T-1).

    Returns ``(S_light, S_strange)``, each ``[n_t][Lz][Ly][Lx][12][12]``.
    With ``su3=True`` the strange propagator is the light one (S_s := S_l),
    the flavour-SU(3) limit.
    """
    if t_list is None:
        t_list = range(T)
    t_list = list(t_list)
    f = slice_gaussian if kind == "gaussian" else slice_correlated
    Sl = np.stack([f(L, t, LIGHT, seed=seed, dtype=dtype) for t in t_list])
    if su3:
        Ss = Sl.copy()
    else:
        Ss = np.stack([f(L, t, STRANGE, seed=seed, dtype=dtype) for t in t_list])
    return Sl, Ss


def smooth_diagonal(L, seed=BASE_SEED):
    """Site-dependent scalar fields phi_f(x) (complex Gaussian), one per flavour.

    Used to build propagators proportional to the identity in spin-colour
    space, S_f(x) = phi_f(x) * 1_12, for the cross-correlation closed form.
    """
    Lx, Ly, Lz = (L, L, L) if np.isscalar(L) else L
    phl = complex_gaussian(_rng(seed, LIGHT, 0, 7), (Lz, Ly, Lx))
    phs = complex_gaussian(_rng(seed, STRANGE, 0, 7), (Lz, Ly, Lx))
    return phl, phs
