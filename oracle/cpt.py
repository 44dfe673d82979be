"""Forward/backward (CPT) average of the correlator (Sec. 6), FP64.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper takes the upper two components of every spinor index forward in time
(the baryon pair) and the lower two backward in time (the antibaryon pair,
related to the first by charge conjugation, parity and time reversal), maps both
to spin indices 0, 1 and averages the two, which doubles the statistics.

Readings of the paper taken here:
  * time slices: forward t0 + tau, backward t0 - tau, both taken mod Lt;
  * both parts are normalised by exp(E tau), tau >= 0 being the distance from t0;
  * lower component 2 + s is re-indexed to s, with no spin flip;
  * R(r, tau) = 1/2 (C_up(r; t0 + tau) + sign * C_low(r; t0 - tau)); sign = +1 by
    default (a factor common to each baryon's backward part enters the pair
    squared), the caller may choose -1.
"""
from __future__ import annotations

import numpy as np

from . import wick


def cpt_average(S_l, S_s, ch, t0, tau, sign=1.0, energy=0.0):
    """R_ch(r, tau) for every relative coordinate r.

    S_l, S_s: complex128 [Lt][Lz][Ly][Lx][12][12], every time slice of the lattice.
    ch:       channel tuple (B1, B2, B3, B4).
    Returns complex128 [V][16], spin index a + 2*(b + 2*(a' + 2*b')).
    """
    Lt, Lz, Ly, Lx = S_l.shape[:4]
    r = wick.all_r(Lx, Ly, Lz)
    tf, tb = (t0 + tau) % Lt, (t0 - tau) % Lt
    forward = wick.correlate(S_l[tf], S_s[tf], ch, r)
    backward = wick.correlate(S_l[tb], S_s[tb], ch, r, lower=True)
    return 0.5 * np.exp(energy * tau) * (forward + sign * backward)
