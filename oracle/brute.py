"""O-0: literal brute-force evaluation on tiny lattices.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Evaluates the four-point function exactly as it is written in Sec. 3,
Eq. (LN.pLLp.ududsu): a sum over every nonzero entry of the four baryon tensors
(sink and source, Sec. 2 fields) of the product of tensor values and of the
Wick contraction of the twelve quark fields, the latter taken as the
determinant of the 6x6 propagator matrix P_ij = [f_i == f'_j] S_{f_i}(x_i)[xi_i][xi'_j]
(Sec. 3, Eq. (Qexchdiag)).  The determinant is computed by LAPACK (LU), not by
enumerating permutations, so that it checks the sign bookkeeping of ``wick.c``.
Cost: 24^4 determinants per (X, r, spin, term tuple); only for V of a few sites.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import operators as ops

_FL = {"u": 0, "d": 1, "s": 2}


def tensor_entries(g, name="p"):
    """Nonzero entries of eps(c_a c_b c_c) Gamma_1(mu_a, mu_b) Gamma_2(g, mu_c) of field `name`
    (octet fields: Gamma_1 = C gamma_5, Gamma_2 = 1)."""
    eps = ops.levi_civita()
    M1, M2 = ops.spin_structure(name)
    idx, val = [], []
    for ca, cb, cc in itertools.product(range(3), repeat=3):
        if eps[ca, cb, cc] == 0:
            continue
        for ma, mb, mc in itertools.product(range(4), repeat=3):
            if M1[ma, mb] == 0 or M2[g, mc] == 0:
                continue
            idx.append((3 * ma + ca, 3 * mb + cb, 3 * mc + cc))
            val.append(eps[ca, cb, cc] * M1[ma, mb] * M2[g, mc])
    return np.array(idx), np.array(val)


def correlate(S_l, S_s, ch, r_list, spins=None, lower=False, offsets=None):
    """C_ch(r) by brute force for one time slice.

    spins: iterable of spin indices a + 2*(b + 2*(a' + 2*b')) (default: all 16).
    lower: take the lower two Dirac components of every spinor index (component
           2 + a for a, Sec. 6) instead of the upper two.
    offsets: per baryon B1..B4 the first Dirac component of its pair (0 or 2),
           overriding ``lower``.
    Returns complex128 [n_r][16] (entries not requested are left 0).
    """
    Lz, Ly, Lx = S_l.shape[:3]
    V = Lx * Ly * Lz
    Sl = S_l.reshape(V, 12, 12)
    Ss = S_s.reshape(V, 12, 12)
    props = [Sl, Sl, Ss]          # u, d, s (u = d numerically, distinct as fields)
    if spins is None:
        spins = range(16)
    if offsets is None:
        offsets = (2 if lower else 0,) * 4
    ent = [[tensor_entries(g + offsets[i], b) for g in range(2)] for i, b in enumerate(ch)]
    terms = ops.channel_terms(ch)
    out = np.zeros((len(r_list), 16), dtype=np.complex128)
    for ir, (rx, ry, rz) in enumerate(r_list):
        for X in range(V):
            x, y, z = X % Lx, (X // Lx) % Ly, X // (Lx * Ly)
            x1 = ((x + rx) % Lx) + Lx * (((y + ry) % Ly) + Ly * ((z + rz) % Lz))
            sites = [x1] * 3 + [X] * 3
            for sp in spins:
                a, b, a3, b4 = sp & 1, (sp >> 1) & 1, (sp >> 2) & 1, (sp >> 3) & 1
                total = 0.0 + 0.0j
                for (w1, f1), (w2, f2), (w3, f3), (w4, f4) in itertools.product(*terms):
                    fsnk = [_FL[q] for q in f1 + f2]
                    fsrc = [_FL[q] for q in f3 + f4]
                    (i1, v1), (i2, v2), (i3, v3), (i4, v4) = ent[0][a], ent[1][b], ent[2][a3], ent[3][b4]
                    # all index combinations: grid over the four entry lists
                    g1, g2, g3, g4 = np.meshgrid(np.arange(len(v1)), np.arange(len(v2)), np.arange(len(v3)),
                                                 np.arange(len(v4)), indexing="ij")
                    g1, g2, g3, g4 = g1.ravel(), g2.ravel(), g3.ravel(), g4.ravel()
                    xi = np.concatenate([i1[g1], i2[g2]], axis=1)      # [N, 6] sink indices
                    xp = np.concatenate([i3[g3], i4[g4]], axis=1)      # [N, 6] source indices
                    coef = v1[g1] * v2[g2] * v3[g3] * v4[g4]
                    P = np.zeros((len(coef), 6, 6), dtype=np.complex128)
                    for i in range(6):
                        for j in range(6):
                            if fsnk[i] != fsrc[j]:
                                continue
                            P[:, i, j] = props[fsnk[i]][sites[i]][xi[:, i], xp[:, j]]
                    total += w1 * w2 * w3 * w4 * np.sum(coef * np.linalg.det(P))
                out[ir, sp] += total
    return out
