"""Wick contraction of a string of quark fields by explicit pairing.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For free quark fields the vacuum expectation value of a product of Grassmann
fields is the sum over complete pairings of each quark with an antiquark of
the same flavour, each pairing weighted by the product of propagators and by
the sign of the permutation that brings every paired couple next to each other
(quark on the left).  This module carries that rule out literally, by repeated
contraction of the leftmost field, with no reference to determinants; the
tests compare it with the determinant rule used by the oracle and with the
expansions printed in Sec. 3, Eq. (Qexchdiag) and Appendix A,
Eq. (Qexchdiag_SpnnSp).
"""
from __future__ import annotations


def expand(fields):
    """Wick expansion of a field string.

    fields: list of (kind, flavour, label) with kind 'q' or 'qbar'.
    Returns {frozenset of (q_label, qbar_label): sign}.
    """
    out = {}
    _rec(list(fields), 1, [], out)
    return out


def _rec(rest, sign, pairs, out):
    if not rest:
        key = frozenset(pairs)
        out[key] = out.get(key, 0) + sign
        return
    kind0, fl0, lab0 = rest[0]
    for j in range(1, len(rest)):
        kind, fl, lab = rest[j]
        if fl != fl0 or kind == kind0:
            continue
        # moving field j next to field 0 crosses j-1 Grassmann fields
        s = -1 if (j - 1) % 2 else 1
        if kind0 == "q":
            pair = (lab0, lab)
        else:
            # <qbar q> = -<q qbar>
            pair = (lab, lab0)
            s = -s
        _rec(rest[1:j] + rest[j + 1:], sign * s, pairs + [pair], out)
