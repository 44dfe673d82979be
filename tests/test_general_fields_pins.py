"""Pins of the oracle for general interpolating fields B = eps((q1 Gamma_1 q2) Gamma_2 q3)
(Sec. 2, Eq. (FieldOperator_B)): the decuplet fields with {C gamma_l, 1} (Sec. 4
footnote) and the nucleon field with {C, gamma_5}, against facts that do not come
from the Wick oracle:

* Clifford-algebra facts the fields rest on: C gamma_mu^T C^-1 = -gamma_mu, hence
  C gamma_l symmetric (a diquark of identical flavours survives the colour
  antisymmetry) and C, C gamma_5 antisymmetric;
* brute force: literal 6x6 determinants over every nonzero tensor entry, with
  complex Gamma entries (C gamma_1, C gamma_3 are imaginary or complex);
* exact flavour relations: with S_u = S_d the Delta++ and Delta- correlators agree,
  and with S_s = S_l (flavour SU(3) limit) the Omega- correlators equal the Delta++
  ones;
* the octet field through the general path: {C gamma_5, 1} is the listed proton.
"""
import numpy as np
import pytest

import synth
from oracle import brute, operators as ops, wick


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_clifford_facts():
    g1, g2, g3, g4, g5 = ops.dirac_gammas()
    C = ops.charge_conjugation()
    Ci = np.linalg.inv(C)
    for g in (g1, g2, g3, g4):
        assert np.allclose(C @ g.T @ Ci, -g)
    for l, g in enumerate((g1, g2, g3), start=1):
        M = C @ g
        assert np.allclose(M.T, M)
        G1, G2 = ops.spin_structure("O-(%d)" % l)
        assert np.allclose(G1, M) and np.allclose(G2, np.eye(4))
    assert np.allclose(C.T, -C)
    assert np.allclose((C @ g5).T, -(C @ g5))
    G1, G2 = ops.spin_structure("p2")
    assert np.allclose(G1, C) and np.allclose(G2, g5)
    # every Gamma used is monomial in the Dirac representation (one nonzero per row)
    for name in ["p", "p2", "D++(1)", "D++(2)", "D++(3)"]:
        for M in ops.spin_structure(name):
            assert all(np.count_nonzero(np.abs(row) > 0) == 1 for row in M)


@pytest.mark.parametrize("ch,spins", [
    (("O-(3)", "O-(3)", "O-(3)", "O-(3)"), [0, 9]),
    (("D++(1)", "O-(2)", "D++(1)", "O-(2)"), [3, 12]),
    (("p2", "n", "p", "n2"), [5, 10]),
])
def test_general_fields_equal_brute_force(ch, spins):
    Sl, Ss = synth.propagators((1, 1, 1), 1, seed=23)
    r = [(0, 0, 0)]
    ob = brute.correlate(Sl[0], Ss[0], ch, r, spins=spins)
    ow = wick.correlate(Sl[0], Ss[0], ch, r)
    assert np.abs(ow[:, spins]).max() > 0
    assert rel(ob[:, spins], ow[:, spins]) < 1e-12


def test_general_fields_lower_equal_brute_force():
    Sl, Ss = synth.propagators((1, 1, 1), 1, seed=29)
    ch = ("D++(3)", "p2", "D++(3)", "p2")
    spins = [6, 9]
    ob = brute.correlate(Sl[0], Ss[0], ch, [(0, 0, 0)], spins=spins, lower=True)
    ow = wick.correlate(Sl[0], Ss[0], ch, [(0, 0, 0)], lower=True)
    assert rel(ob[:, spins], ow[:, spins]) < 1e-12


@pytest.mark.parametrize("l1,l2", [(1, 1), (3, 2)])
def test_decuplet_flavour_relations(l1, l2):
    lat = (2, 2, 1)
    r = wick.all_r(*lat)
    Sl, Ss = synth.propagators(lat, 1, seed=31)
    dpp = ("D++(%d)" % l1, "D++(%d)" % l2, "D++(%d)" % l1, "D++(%d)" % l2)
    dm = tuple(n.replace("D++", "D-") for n in dpp)
    om = tuple(n.replace("D++", "O-") for n in dpp)
    a = wick.correlate(Sl[0], Ss[0], dpp, r)
    assert np.abs(a).max() > 0
    assert rel(wick.correlate(Sl[0], Ss[0], dm, r), a) < 1e-12
    # S_s = S_l: Omega- is Delta++ with relabelled flavour
    assert rel(wick.correlate(Sl[0], Sl[0], om, r), a) < 1e-12
    assert rel(wick.correlate(Sl[0], Ss[0], om, r), a) > 1e-3


def test_octet_through_general_path():
    """{C gamma_5, 1} through the general tensor code is the proton of Sec. 2 (same field
    object), so the listed channel is unchanged; and p2 differs from p."""
    lat = (2, 1, 1)
    r = wick.all_r(*lat)
    Sl, Ss = synth.propagators(lat, 1, seed=37)
    a = wick.correlate(Sl[0], Ss[0], ("p", "n", "p", "n"), r)
    b = wick.correlate(Sl[0], Ss[0], ("p2", "n2", "p2", "n2"), r)
    assert rel(b, a) > 1e-3
    ob = brute.correlate(Sl[0], Ss[0], ("p", "n", "p", "n"), r, spins=[0, 15])
    assert rel(ob[:, [0, 15]], a[:, [0, 15]]) < 1e-12


@pytest.mark.parametrize("ch,spins", [
    (("D+(1)", "D+(2)", "D+(1)", "D+(2)"), [0, 15]),
    (("S*0(3)", "p", "S*0(3)", "p"), [5]),
])
def test_mixed_decuplet_equals_brute_force(ch, spins):
    Sl, Ss = synth.propagators((1, 1, 1), 1, seed=41)
    ob = brute.correlate(Sl[0], Ss[0], ch, [(0, 0, 0)], spins=spins)
    ow = wick.correlate(Sl[0], Ss[0], ch, [(0, 0, 0)])
    assert np.abs(ow[:, spins]).max() > 0
    assert rel(ob[:, spins], ow[:, spins]) < 1e-12


def test_decuplet_isospin_three():
    """S_u = S_d: the I = 3, I3 = 2 state (D++ D+ + D+ D++)/sqrt2 has the correlator of the
    I3 = 3 state D++ D++, elementwise (D+ = T_- D++ / sqrt3 fixes its normalisation and phase)."""
    lat = (2, 2, 1)
    r = wick.all_r(*lat)
    Sl, Ss = synth.propagators(lat, 1, seed=43)
    a, b = "D++(1)", "D+(1)"
    top = wick.correlate(Sl[0], Ss[0], (a, a, a, a), r)
    pair = 0.5 * sum(wick.correlate(Sl[0], Ss[0], snk + src, r)
                     for snk in ((a, b), (b, a)) for src in ((a, b), (b, a)))
    assert np.abs(top).max() > 0
    assert rel(pair, top) < 1e-12
    # D+ D+ mixes I = 3, 2, 1, 0: its correlator is a different quantity
    assert rel(wick.correlate(Sl[0], Ss[0], (b, b, b, b), r), top) > 1e-3


@pytest.mark.parametrize("x,y,su3", [("S*+(2)", "S*-(2)", False), ("X*0(1)", "X*-(1)", False),
                                     ("S*+(2)", "D+(2)", True), ("X*0(3)", "D0(3)", True)])
def test_mixed_decuplet_flavour_relations(x, y, su3):
    """u <-> d (S_u = S_d): S*+ <-> S*-, X*0 <-> X*-; with S_s = S_l the s quarks relabel:
    S*+ (u s u) <-> D+ (u d u), X*0 (s u s) <-> D0 (d u d)."""
    lat = (2, 2, 1)
    r = wick.all_r(*lat)
    Sl, Ss = synth.propagators(lat, 1, seed=47)
    if su3:
        Ss = Sl.copy()
    cx = wick.correlate(Sl[0], Ss[0], (x, x, x, x), r)
    cy = wick.correlate(Sl[0], Ss[0], (y, y, y, y), r)
    assert np.abs(cx).max() > 0
    assert rel(cy, cx) < 1e-12
