"""O-U: unified-style evaluation of the same correlator (FFT over X).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The cross-check of Sec. 6 compares the block algorithm with the unified
contraction algorithm, whose idea is to fold every Wick permutation and every
source-tensor entry into one weight tensor over the open source indices before
any spatial sum.  Here:

  1. per sink term and site, G(x; g; e_a, e_b, e_c) = sum_xi T(xi; g) prod S  (as in wick.c);
  2. W_{a'b'}(A, B) = sum_{terms 3,4} w3 w4 sum_sigma sgn(sigma) sum_{source entries}
     T3 T4, with A = (e'_{sigma(1)}, e'_{sigma(2)}, e'_{sigma(3)}) and
     B = (e'_{sigma(4)}, e'_{sigma(5)}, e'_{sigma(6)});                        (Sec. 3, Eq. (Qexchdiag))
  3. sum_X G1(X+r)[A] G2(X)[B] = (1/V) sum_q G1~(q)[A] G2~(-q)[B] e^{iqr}      (Sec. 3, Eq. (LN.pLLp.FFT))
     with numpy's FFT as the library step;
  4. C(r) = sum_{A,B} W(A,B) x [that correlation].
No effective blocks, no diagram classification.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import operators as ops
from .brute import tensor_entries

_FL = {"u": 0, "d": 1, "s": 2}


def _sign(p):
    p = list(p)
    s = 1
    for i in range(len(p)):
        while p[i] != i:
            j = p[i]
            p[i], p[j] = p[j], p[i]
            s = -s
    return s


def sink_G(S_l, S_s, flav, lower=False):
    """G(x; g; A) for one sink term: [V][2][1728] complex."""
    V = S_l.shape[0] * S_l.shape[1] * S_l.shape[2]
    props = {"u": S_l.reshape(V, 12, 12), "d": S_l.reshape(V, 12, 12), "s": S_s.reshape(V, 12, 12)}
    Sa, Sb, Sc = (props[f] for f in flav)
    G = np.zeros((V, 2, 12, 12, 12), dtype=np.complex128)
    g0 = 2 if lower else 0
    for g in range(2):
        idx, val = tensor_entries(g0 + g)
        for (ia, ib, ic), v in zip(idx, val):
            G[:, g] += v * np.einsum("xi,xj,xk->xijk", Sa[:, ia], Sb[:, ib], Sc[:, ic])
    return G.reshape(V, 2, 1728)


def source_weights(ch, t1f, t2f, lower=False):
    """W[(a', b')] as sparse 1728x1728 matrices for given sink-term flavours.

    Sums over the source terms of B3 and B4 and over sigma.
    """
    g0 = 2 if lower else 0
    ents = [tensor_entries(g0 + g) for g in range(2)]
    fs = [_FL[q] for q in t1f + t2f]
    W = {}
    for a3, a4 in itertools.product(range(2), repeat=2):
        rows, cols, vals = [], [], []
        (i3, v3), (i4, v4) = ents[a3], ents[a4]
        for (w3, f3), (w4, f4) in itertools.product(ops.BARYONS[ch[2]], ops.BARYONS[ch[3]]):
            fsrc = [_FL[q] for q in f3 + f4]
            for p in itertools.permutations(range(6)):
                if any(fs[i] != fsrc[p[i]] for i in range(6)):
                    continue
                sg = _sign(p)
                e = np.concatenate([np.repeat(i3, len(v4), axis=0), np.tile(i4, (len(v3), 1))], axis=1)
                c = np.repeat(v3, len(v4)) * np.tile(v4, len(v3)) * (w3 * w4 * sg)
                A = 144 * e[:, p[0]] + 12 * e[:, p[1]] + e[:, p[2]]
                B = 144 * e[:, p[3]] + 12 * e[:, p[4]] + e[:, p[5]]
                rows.append(A); cols.append(B); vals.append(c)
        if rows:
            W[(a3, a4)] = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                        shape=(1728, 1728))
        else:
            W[(a3, a4)] = sp.csr_matrix((1728, 1728), dtype=np.complex128)
    return W


def correlate(S_l, S_s, ch, lower=False):
    """C_ch(r) for every r of one time slice: complex128 [Lz][Ly][Lx][16]."""
    Lz, Ly, Lx = S_l.shape[:3]
    V = Lx * Ly * Lz
    out = np.zeros((16, V), dtype=np.complex128)
    for (w1, f1), (w2, f2) in itertools.product(ops.BARYONS[ch[0]], ops.BARYONS[ch[1]]):
        G1 = sink_G(S_l, S_s, f1, lower).reshape(Lz, Ly, Lx, 2, 1728)
        G2 = sink_G(S_l, S_s, f2, lower).reshape(Lz, Ly, Lx, 2, 1728)
        F1 = np.fft.fftn(G1, axes=(0, 1, 2)).reshape(V, 2, 1728)            # sum_x f(x) e^{-iqx}
        F2m = (V * np.fft.ifftn(G2, axes=(0, 1, 2))).reshape(V, 2, 1728)    # sum_x g(x) e^{+iqx}
        W = source_weights(ch, f1, f2, lower)
        for (a3, a4), Wm in W.items():
            if Wm.nnz == 0:
                continue
            for b in range(2):
                H = (Wm @ F2m[:, b, :].T).T                     # [V][1728]: sum_B W(A,B) G2~(-q)[B]
                for a in range(2):
                    ct = np.sum(F1[:, a, :] * H, axis=1)       # C~(q)
                    cr = np.fft.ifftn(ct.reshape(Lz, Ly, Lx)).reshape(V)   # (1/V) sum_q e^{iqr}
                    out[a + 2 * (b + 2 * (a3 + 2 * a4))] += w1 * w2 * cr
    return out.T.reshape(Lz, Ly, Lx, 16)
