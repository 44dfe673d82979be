"""Pins of the CPU oracle against facts outside the oracle itself (no GPU).

Each check is chosen so that a plausible slip in the oracle -- a wrong Wick sign,
a dropped or mis-weighted Lambda/Sigma0 term, a wrong operator phase, a
transposed propagator, r taken as X-r instead of X+r -- fails at least one test.
"""
import itertools
import os

import numpy as np
import pytest

import synth
from oracle import brute, grassmann, operators as ops, unified, wick

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SPIN_SWAP = [((s >> 1) & 1) + 2 * (s & 1) + 4 * ((s >> 3) & 1) + 8 * ((s >> 2) & 1) for s in range(16)]
SINK_SWAP = [((s >> 1) & 1) + 2 * (s & 1) + 4 * ((s >> 2) & 3) for s in range(16)]
SRC_SWAP = [(s & 3) + 4 * ((s >> 3) & 1) + 8 * ((s >> 2) & 1) for s in range(16)]


def minus_r_index(L):
    r = wick.all_r(L, L, L)
    m = (-r) % L
    return m[:, 0] + L * (m[:, 1] + L * m[:, 2])


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(a).max(), np.abs(b).max())


# ---------------------------------------------------------------- gamma algebra
def test_dirac_representation_and_cg5():
    """Clifford algebra of the Dirac-representation gammas; C gamma_5 real antisymmetric."""
    g = ops.dirac_gammas()
    for i in range(4):
        for j in range(4):
            ac = g[i] @ g[j] + g[j] @ g[i]
            assert np.allclose(ac, 2 * np.eye(4) * (i == j))
    M = ops.cg5()
    assert np.allclose(M.imag, 0)
    assert np.allclose(M, -M.T)
    assert np.allclose(M @ M.T, np.eye(4))        # orthogonal: each row has one +-1
    assert np.count_nonzero(np.round(M.real)) == 4


# ---------------------------------------------------------------- Wick sign convention
def _read_wick_fixture(name):
    fields, lines = None, []
    for ln in open(os.path.join(GOLDEN, name)):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        if ln.startswith("string:"):
            fields = []
            for tok in ln.split()[1:]:
                kind, fl, lab = tok.split(":")
                fields.append((kind, fl, int(lab)))
            continue
        sgn = 1 if ln[0] == "+" else -1
        pairs = frozenset(tuple(int(v) for v in p.split(":")) for p in ln[1:].split())
        lines.append((pairs, sgn))
    return fields, dict(lines)


@pytest.mark.parametrize("fixture", ["wick_pLambda.txt", "wick_SigmaN.txt"])
def test_grassmann_expansion_matches_paper(fixture):
    """Explicit Grassmann pairing reproduces the printed Wick expansion, term by term."""
    fields, want = _read_wick_fixture(fixture)
    got = {k: v for k, v in grassmann.expand(fields).items() if v != 0}
    assert got == want


@pytest.mark.parametrize("fixture", ["wick_pLambda.txt", "wick_SigmaN.txt"])
def test_determinant_rule_matches_grassmann(fixture):
    """Mirrored order: <q1..q6 qbar6'..qbar1'> = det[<q_i qbar_j'>], the rule used in wick.c."""
    fields, _ = _read_wick_fixture(fixture)
    qs = [f for f in fields if f[0] == "q"]
    qb = [f for f in fields if f[0] == "qbar"][::-1]      # undo the mirror: position j <-> j'
    assert [f[2] for f in qb] == [f[2] for f in qs]
    det_rule = {}
    for p in itertools.permutations(range(6)):
        if any(qs[i][1] != qb[p[i]][1] for i in range(6)):
            continue
        sgn = np.linalg.det(np.eye(6)[list(p)])
        det_rule[frozenset((qs[i][2], qb[p[i]][2]) for i in range(6))] = int(round(sgn))
    assert det_rule == grassmann.expand(fields)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("ch", [ops.CHANNELS[0], ops.CHANNELS[5], ops.CHANNELS[51]])
def test_wick_oracle_equals_brute_force(ch):
    """O-W (sigma enumeration) equals literal LAPACK determinants summed over all tensor entries."""
    Sl, Ss = synth.propagators((2, 1, 1), 1, seed=11)
    r = [(0, 0, 0), (1, 0, 0)]
    spins = [0, 6, 9, 15]
    ob = brute.correlate(Sl[0], Ss[0], ch, r, spins=spins)
    ow = wick.correlate(Sl[0], Ss[0], ch, r)
    assert rel(ob[:, spins], ow[:, spins]) < 1e-12


def test_wick_oracle_equals_brute_force_lambda():
    """Same for a channel with three Lambda sink and source terms (p Lambda -> p Lambda)."""
    Sl, Ss = synth.propagators((1, 1, 1), 1, seed=12)
    ob = brute.correlate(Sl[0], Ss[0], ops.CHANNELS[1], [(0, 0, 0)], spins=[3, 12])
    ow = wick.correlate(Sl[0], Ss[0], ops.CHANNELS[1], [(0, 0, 0)])
    assert rel(ob[:, [3, 12]], ow[:, [3, 12]]) < 1e-12


# ---------------------------------------------------------------- exact zeros
@pytest.mark.parametrize("ch", ops.ZERO_CHANNELS)
def test_omitted_channels_vanish(ch):
    """The four off-diagonal channels left out in Sec. 4 vanish identically when S_u = S_d."""
    Sl, Ss = synth.propagators(2, 1, seed=13)
    ref = wick.correlate(Sl[0], Ss[0], ("L", "L", "L", "L"), wick.all_r(2, 2, 2))
    z = wick.correlate(Sl[0], Ss[0], ch, wick.all_r(2, 2, 2))
    assert np.abs(z).max() < 1e-12 * np.abs(ref).max()


def test_identical_sink_baryons_antisymmetry():
    """Sec. 6 footnote: identical sink baryons give C(r)_{ab..} = -C(-r)_{ba..}, zero at r = -r."""
    L = 4
    Sl, Ss = synth.propagators(L, 1, seed=14)
    mi = minus_r_index(L)
    for ch in [("L", "L", "p", "X-"), ("S0", "S0", "S+", "S-")]:
        c = wick.correlate(Sl[0], Ss[0], ch, wick.all_r(L, L, L))
        assert rel(c, -c[mi][:, SINK_SWAP]) < 1e-12
        fixed = [i for i in range(L ** 3) if mi[i] == i]
        assert len(fixed) == 8
        for s in range(16):
            if (s & 1) == ((s >> 1) & 1):
                assert np.abs(c[fixed, s]).max() < 1e-12 * np.abs(c).max()


def test_identical_source_baryons_antisymmetry():
    """Sec. 6 footnote: identical source baryons (one wall source) give C_{..a'b'} = -C_{..b'a'}."""
    Sl, Ss = synth.propagators(2, 1, seed=15)
    for ch in [("p", "X-", "L", "L"), ("S0", "L", "S0", "S0")]:
        if ch in ops.CHANNELS:
            c = wick.correlate(Sl[0], Ss[0], ch, wick.all_r(2, 2, 2))
            assert rel(c, -c[:, SRC_SWAP]) < 1e-12


# ---------------------------------------------------------------- isospin / SU(3)
ISOSPIN = [  # (channel a, channel b, sign): C_a = sign * C_b when S_u = S_d
    (("p", "X-", "p", "X-"), ("n", "X0", "n", "X0"), +1),
    (("p", "X-", "n", "X0"), ("n", "X0", "p", "X-"), +1),
    (("L", "L", "p", "X-"), ("L", "L", "n", "X0"), -1),
    (("p", "X-", "L", "L"), ("n", "X0", "L", "L"), -1),
    (("S0", "S0", "p", "X-"), ("S0", "S0", "n", "X0"), -1),
    (("S0", "L", "p", "X-"), ("S0", "L", "n", "X0"), +1),
]


@pytest.mark.parametrize("a,b,s", ISOSPIN)
def test_isospin_relations(a, b, s):
    """u <-> d maps p<->n, Xi- -> -Xi0, Lambda -> -Lambda, Sigma0 -> Sigma0 (operator phases of Sec. 2)."""
    Sl, Ss = synth.propagators(2, 1, seed=16)
    r = wick.all_r(2, 2, 2)
    assert rel(wick.correlate(Sl[0], Ss[0], a, r), s * wick.correlate(Sl[0], Ss[0], b, r)) < 1e-12


def test_su3_limit_relations():
    """With S_s = S_l, u <-> s maps Sigma+ n onto Sigma- Xi0 (r -> -r, baryons swapped)."""
    L = 3
    Sl, Ss = synth.propagators(L, 1, seed=17, su3=True)
    r = wick.all_r(L, L, L)
    mi = minus_r_index(L)
    a = wick.correlate(Sl[0], Ss[0], ("S+", "n", "S+", "n"), r)
    b = wick.correlate(Sl[0], Ss[0], ("S-", "X0", "S-", "X0"), r)
    assert rel(a, b[mi][:, SPIN_SWAP]) < 1e-12
    c = wick.correlate(Sl[0], Ss[0], ("p", "X-", "p", "X-"), r)
    assert rel(c, c[mi][:, SPIN_SWAP]) < 1e-12


# ---------------------------------------------------------------- algebraic structure
def test_homogeneity_in_each_propagator():
    """C(a S_l, b S_s) = a^{n_l} b^{n_s} C(S_l, S_s) (six propagators per term)."""
    Sl, Ss = synth.propagators(2, 1, seed=18)
    r = wick.all_r(2, 2, 2)
    for ch in [ops.CHANNELS[1], ops.CHANNELS[10], ops.CHANNELS[42]]:
        nl, ns = ops.quark_content(ch)
        a, b = 1.3 - 0.4j, 0.7 + 0.2j
        c0 = wick.correlate(Sl[0], Ss[0], ch, r)
        c1 = wick.correlate(a * Sl[0], b * Ss[0], ch, r)
        assert rel(c1, a ** nl * b ** ns * c0) < 1e-12


def test_linear_in_strange_for_s_minus_1():
    """S = -1 channels hold one strange quark: C is linear in S_s."""
    Sl, S1 = synth.propagators(2, 1, seed=19)
    _, S2 = synth.propagators(2, 1, seed=20)
    r = wick.all_r(2, 2, 2)
    ch = ops.CHANNELS[3]
    c12 = wick.correlate(Sl[0], S1[0] + S2[0], ch, r)
    assert rel(c12, wick.correlate(Sl[0], S1[0], ch, r) + wick.correlate(Sl[0], S2[0], ch, r)) < 1e-12


def test_translation_invariance():
    """Shifting both propagator fields by a lattice vector leaves C(r) unchanged."""
    L = 3
    Sl, Ss = synth.propagators(L, 1, seed=21)
    r = wick.all_r(L, L, L)
    ch = ops.CHANNELS[2]
    sh = lambda a: np.roll(a, shift=(1, 2, 1), axis=(0, 1, 2))
    assert rel(wick.correlate(Sl[0], Ss[0], ch, r), wick.correlate(sh(Sl[0]), sh(Ss[0]), ch, r)) < 1e-12


def test_diagonal_propagator_closed_form():
    """S_f(x) = phi_f(x) 1: C(r) = K * sum_X Phi1(X+r) Phi2(X) with K = C on one site with S = 1.

    Pins the X+r convention (an X-r slip gives the reflected correlation) and the
    periodic wrap; the correlation is evaluated with numpy, the constant K by brute force.
    """
    L = 3
    phl, phs = synth.smooth_diagonal(L, seed=22)
    eye = np.eye(12, dtype=complex)
    Sl = phl[..., None, None] * eye
    Ss = phs[..., None, None] * eye
    for ch in [ops.CHANNELS[1], ops.CHANNELS[46]]:
        f1 = [q for _, f in ops.BARYONS[ch[0]][:1] for q in f]
        f2 = [q for _, f in ops.BARYONS[ch[1]][:1] for q in f]
        ph = {"u": phl, "d": phl, "s": phs}
        P1 = np.prod([ph[q] for q in f1], axis=0)
        P2 = np.prod([ph[q] for q in f2], axis=0)
        corr = np.zeros((L, L, L), dtype=complex)
        for rz, ry, rx in itertools.product(range(L), repeat=3):
            corr[rz, ry, rx] = np.sum(np.roll(P1, shift=(-rz, -ry, -rx), axis=(0, 1, 2)) * P2)
        one = np.ones((1, 1, 1), dtype=complex)[..., None, None] * eye
        K = brute.correlate(one, one, ch, [(0, 0, 0)])[0]
        got = wick.correlate(Sl, Ss, ch, wick.all_r(L, L, L))
        want = corr.reshape(-1)[:, None] * K[None, :]
        assert np.abs(K).max() > 1.0
        assert rel(got, want) < 1e-12


def test_propagator_not_transposed():
    """A transposed propagator (source and sink spin-colour swapped) changes C."""
    Sl, Ss = synth.propagators((2, 1, 1), 1, seed=23)
    r = [(0, 0, 0), (1, 0, 0)]
    ch = ops.CHANNELS[0]
    c = wick.correlate(Sl[0], Ss[0], ch, r)
    ob = brute.correlate(Sl[0], Ss[0], ch, r, spins=[0, 9])
    assert rel(c[:, [0, 9]], ob[:, [0, 9]]) < 1e-12
    ct = wick.correlate(np.swapaxes(Sl[0], -1, -2), np.swapaxes(Ss[0], -1, -2), ch, r)
    assert rel(c, ct) > 1e-3


# ---------------------------------------------------------------- second oracle
@pytest.mark.parametrize("ci", [1, 10, 20, 51])
def test_unified_equals_wick(ci):
    """O-U (folded weights + FFT) equals O-W (direct O(V^2) sum) on every r of a 3^3 lattice."""
    Sl, Ss = synth.propagators(3, 1, seed=24)
    ch = ops.CHANNELS[ci]
    ou = unified.correlate(Sl[0], Ss[0], ch).reshape(-1, 16)
    ow = wick.correlate(Sl[0], Ss[0], ch, wick.all_r(3, 3, 3))
    assert rel(ou, ow) < 1e-12
