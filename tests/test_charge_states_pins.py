"""Other charge states than the 52 listed channels (Sec. 4 notes the extension):
pins of the Wick oracle on them through exact isospin relations (S_u = S_d),
and the channel-id ABI on the CPU.

Isospin with the operator phases of Sec. 2: T_- p = -n (eps (d C g5 d) vanishes),
so (p, -n) is a doublet; u <-> d maps p -> -n, n -> -p, S+ <-> S- (up to signs
that cancel in pairs), X0 <-> X-.  Hence, elementwise in r and spins:
  C[pp > pp] = C[nn > nn],
  C[pp > pp] = 1/2 (C[pn > pn] + C[pn > np] + C[np > pn] + C[np > np])   (I = 1),
  C[S+S+ > S+S+] = C[S-S- > S-S-],  C[X0X0 > X0X0] = C[X-X- > X-X-],
  C[S+p > S+p] = C[S-n > S-n].
"""
import numpy as np
import pytest

import synth
from oracle import wick


@pytest.fixture(scope="module")
def field():
    L = 2
    Sl, Ss = synth.propagators(L, 1, seed=71)
    return Sl[0], Ss[0], wick.all_r(L, L, L)


def C(field, ch):
    Sl, Ss, r = field
    return wick.correlate(Sl, Ss, ch, r)


def close(a, b):
    return np.abs(a - b).max() <= 1e-12 * max(np.abs(a).max(), np.abs(b).max())


def test_nn_equals_pp(field):
    pp = C(field, ("p", "p", "p", "p"))
    assert np.abs(pp).max() > 0
    assert close(pp, C(field, ("n", "n", "n", "n")))


def test_isospin_one_nucleon_pair(field):
    pp = C(field, ("p", "p", "p", "p"))
    i1 = 0.5 * (C(field, ("p", "n", "p", "n")) + C(field, ("p", "n", "n", "p")) +
                C(field, ("n", "p", "p", "n")) + C(field, ("n", "p", "n", "p")))
    assert close(pp, i1)
    # and the I = 0 combination is something else
    i0 = 0.5 * (C(field, ("p", "n", "p", "n")) - C(field, ("p", "n", "n", "p")) -
                C(field, ("n", "p", "p", "n")) + C(field, ("n", "p", "n", "p")))
    assert not close(pp, i0)


@pytest.mark.parametrize("a,b", [(("S+", "S+", "S+", "S+"), ("S-", "S-", "S-", "S-")),
                                 (("X0", "X0", "X0", "X0"), ("X-", "X-", "X-", "X-")),
                                 (("S+", "p", "S+", "p"), ("S-", "n", "S-", "n"))])
def test_u_d_exchange(field, a, b):
    ca = C(field, a)
    assert np.abs(ca).max() > 0
    assert close(ca, C(field, b))


def test_channel_ids_and_names():
    import paper_1510_00903_amd as bbc
    names = bbc.baryon_names()
    assert names[:8] == ["p", "n", "S+", "S-", "X0", "X-", "L", "S0"]
    # listed channels keep their index
    assert bbc.channel_id("p", "n", "p", "n") == 0
    assert bbc.channel_id("X-", "X0", "X-", "X0") == 51
    assert bbc.channel_id("L", "L", "S0", "L") == 52
    # other charge states get 56 + ((b1 * 8 + b2) * 8 + b3) * 8 + b4
    c = bbc.channel_id("p", "p", "p", "p")
    assert c == 56 and bbc.channel_name(c) == "p p > p p"
    c = bbc.channel_id("S+", "p", "S+", "p")
    assert c == 56 + ((2 * 8 + 0) * 8 + 2) * 8 + 0
    assert bbc.channel_content(c) == (5, 1)
    with pytest.raises(bbc.BBCError):
        bbc.channel_id("p", "p", "p", "n")           # quark content differs
    with pytest.raises(bbc.BBCError):
        bbc.plan_stats([56 + 1])                      # p p > p n: not a channel
    st = bbc.plan_stats([bbc.channel_id("p", "p", "p", "p")])
    assert st["iterations"] > 0


def test_general_field_ids():
    import paper_1510_00903_amd as bbc
    names = bbc.baryon_names()
    fams = ("D++", "D-", "O-", "D+", "D0", "S*+", "S*0", "S*-", "X*0", "X*-")
    assert names[8:] == ["p2", "n2"] + ["%s(%d)" % (f, l) for f in fams for l in (1, 2, 3)]
    # quadruples with a general field: 4152 + ((b1 * 40 + b2) * 40 + b3) * 40 + b4
    c = bbc.channel_id("O-(3)", "O-(3)", "O-(3)", "O-(3)")
    assert c == 4152 + ((18 * 40 + 18) * 40 + 18) * 40 + 18
    assert bbc.channel_name(c) == "O-(3) O-(3) > O-(3) O-(3)"
    assert bbc.channel_content(c) == (0, 6)
    c = bbc.channel_id("p2", "n", "p", "n2")
    assert c == 4152 + ((8 * 40 + 1) * 40 + 0) * 40 + 9
    assert bbc.channel_content(c) == (6, 0)
    c = bbc.channel_id("S*0(2)", "p", "S*0(2)", "p")
    assert c == 4152 + ((29 * 40 + 0) * 40 + 29) * 40 + 0 and bbc.channel_content(c) == (5, 1)
    assert bbc.channel_id("p", "n", "p", "n") == 0             # octet ids unchanged
    with pytest.raises(bbc.BBCError):
        bbc.channel_id("O-(1)", "p", "O-(1)", "n")            # quark content differs
    with pytest.raises(bbc.BBCError):
        bbc.channel_name(4152)                                 # octet quadruple in the general range
    st = bbc.plan_stats([bbc.channel_id("O-(1)", "O-(2)", "O-(1)", "O-(2)")])
    assert st["iterations"] > 0
