"""Pins of the oracle for all 256 spin components of C(r) (alpha, beta, alpha', beta'
each over the four Dirac components), i.e. with the spin pair of every baryon
chosen on its own: the upper two (0, 1) or the lower two (2, 3) components of the
index of the baryon tensor T(xi_a xi_b xi_c; g) = eps Gamma_1 Gamma_2(g, .) of
Sec. 2, Eq. (FieldOperator_B), the lower pair being what Sec. 6 uses for the
backward propagating states.  Pinned against:

* brute force (literal 6x6 determinants by LU over every nonzero tensor entry)
  with the same per-baryon offsets; the offset tuples are asymmetric, so that an
  offset applied to the wrong baryon, or a shared offset, fails;
* the upper and lower oracles: the all-upper and all-lower blocks of the
  256-component assembly are those fields;
* the index formula alpha + 4 (beta + 4 (alpha' + 4 beta')) at hand-placed entries.
"""
import numpy as np
import pytest

import synth
from oracle import brute, operators as ops, wick


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("ch,offsets,spins", [
    (ops.CHANNELS[2], (0, 2, 0, 0), [0, 9]),      # p Lambda > Sigma+ n: beta lower
    (ops.CHANNELS[1], (2, 0, 0, 2), [3, 12]),     # p Lambda > p Lambda: alpha and beta' lower
    (ops.CHANNELS[51], (0, 0, 2, 0), [5, 10]),    # Xi- Xi0 > Xi- Xi0: alpha' lower
    (("D++(1)", "O-(2)", "D++(1)", "O-(2)"), (2, 0, 2, 0), [1, 14]),   # decuplet, complex Gamma_1
])
def test_mixed_offsets_equal_brute_force(ch, offsets, spins):
    Sl, Ss = synth.propagators((1, 1, 1), 1, seed=41)
    r = [(0, 0, 0)]
    ob = brute.correlate(Sl[0], Ss[0], ch, r, spins=spins, offsets=offsets)
    ow = wick.correlate(Sl[0], Ss[0], ch, r, offsets=offsets)
    assert np.abs(ow[:, spins]).max() > 0
    assert rel(ob[:, spins], ow[:, spins]) < 1e-12
    # the same spins with the offsets of another baryon differ
    other = offsets[1:] + offsets[:1]
    ox = wick.correlate(Sl[0], Ss[0], ch, r, offsets=other)
    assert rel(ox[:, spins], ow[:, spins]) > 1e-6


def test_mixed_offsets_equal_brute_force_two_sites():
    """Two sites and a nonzero r (the sink baryons at different points)."""
    Sl, Ss = synth.propagators((2, 1, 1), 1, seed=43)
    ch = ops.CHANNELS[2]
    r = [(1, 0, 0)]
    off = (2, 0, 0, 2)
    ob = brute.correlate(Sl[0], Ss[0], ch, r, spins=[6], offsets=off)
    ow = wick.correlate(Sl[0], Ss[0], ch, r, offsets=off)
    assert rel(ob[:, [6]], ow[:, [6]]) < 1e-12


def test_full_assembly_blocks_and_index():
    lat = (2, 2, 1)
    Sl, Ss = synth.propagators(lat, 1, seed=47)
    ch = ops.CHANNELS[1]
    r = wick.all_r(*lat)
    full = wick.correlate_full(Sl[0], Ss[0], ch, r)
    up = wick.correlate(Sl[0], Ss[0], ch, r)
    lo = wick.correlate(Sl[0], Ss[0], ch, r, lower=True)
    idx = np.arange(16)
    a, b, ap, bp = idx & 1, (idx >> 1) & 1, (idx >> 2) & 1, (idx >> 3) & 1
    assert np.array_equal(full[:, a + 4 * b + 16 * ap + 64 * bp], up)
    assert np.array_equal(full[:, (a + 2) + 4 * (b + 2) + 16 * (ap + 2) + 64 * (bp + 2)], lo)
    # alpha = 3, beta = 0, alpha' = 2, beta' = 1: offsets (2, 0, 2, 0), spin 1 + 8
    mixed = wick.correlate(Sl[0], Ss[0], ch, r, offsets=(2, 0, 2, 0))
    assert np.array_equal(full[:, 3 + 4 * 0 + 16 * 2 + 64 * 1], mixed[:, 1 + 8])
    assert np.abs(full).max() > 0 and np.count_nonzero(np.abs(full).max(axis=0)) > 16
