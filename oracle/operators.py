"""Oracle operator table: gamma matrices, baryon interpolating fields, channels.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use the oracle.

Every baryon term is the literal field of the paper:
    B_gamma(x) = w * eps(c_a, c_b, c_c) (C gamma_5)(mu_a, mu_b) delta(gamma, mu_c)
                   q_{f_a}(a) q_{f_b}(b) q_{f_c}(c)
with the quark fields in the Grassmann order (a, b, c) as printed:
  * p, n and C = gamma_4 gamma_2: Sec. 2, Eq. (FieldOperator_N);
  * Sigma^{+-}, Sigma^0, Lambda, Xi^{0,-}: Sec. 2, Eq. (FieldOperator_SLXi);
  * X_u, X_d, X_s: Sec. 2, Eq. (FieldOperator_xxx);
  * Dirac representation: Sec. 6 (benchmark section).
Each term is stored as (weight, (f_a, f_b, f_c)) in that field order, so for
example X_d = eps (s C gamma_5 u) d is (1, ('s', 'u', 'd')).
"""
from __future__ import annotations

import math

import numpy as np


def dirac_gammas():
    """Euclidean gamma matrices in the Dirac representation.

    gamma_4 = diag(1, 1, -1, -1) and gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]
    (the convention of lattice codes such as Bridge++ named in Sec. 6);
    gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4.
    """
    sig = [np.array([[0, 1], [1, 0]], dtype=complex),
           np.array([[0, -1j], [1j, 0]], dtype=complex),
           np.array([[1, 0], [0, -1]], dtype=complex)]
    z = np.zeros((2, 2), dtype=complex)
    gk = [np.block([[z, -1j * s], [1j * s, z]]) for s in sig]
    g4 = np.diag([1, 1, -1, -1]).astype(complex)
    g5 = gk[0] @ gk[1] @ gk[2] @ g4
    return gk[0], gk[1], gk[2], g4, g5


def cg5():
    """The diquark spin matrix C gamma_5 with C = gamma_4 gamma_2 (Sec. 2)."""
    g1, g2, g3, g4, g5 = dirac_gammas()
    return (g4 @ g2) @ g5


def charge_conjugation():
    """C = gamma_4 gamma_2 (Sec. 2)."""
    g1, g2, g3, g4, g5 = dirac_gammas()
    return g4 @ g2


def levi_civita():
    e = np.zeros((3, 3, 3))
    for (a, b, c), s in (((0, 1, 2), 1), ((1, 2, 0), 1), ((2, 0, 1), 1),
                         ((0, 2, 1), -1), ((2, 1, 0), -1), ((1, 0, 2), -1)):
        e[a, b, c] = s
    return e


_X = {"Xu": ("d", "s", "u"), "Xd": ("s", "u", "d"), "Xs": ("u", "d", "s")}
_R6, _R2 = 1.0 / math.sqrt(6.0), 1.0 / math.sqrt(2.0)

# Sec. 2, Eqs. (FieldOperator_N), (FieldOperator_SLXi), (FieldOperator_xxx).
BARYONS = {
    "p":   [(+1.0, ("u", "d", "u"))],
    "n":   [(-1.0, ("u", "d", "d"))],
    "S+":  [(-1.0, ("u", "s", "u"))],
    "S-":  [(-1.0, ("d", "s", "d"))],
    "X0":  [(+1.0, ("u", "s", "s"))],
    "X-":  [(-1.0, ("d", "s", "s"))],
    "Xu":  [(1.0, _X["Xu"])],
    "Xd":  [(1.0, _X["Xd"])],
    "Xs":  [(1.0, _X["Xs"])],
    "S0":  [(+_R2, _X["Xu"]), (-_R2, _X["Xd"])],
    "L":   [(+_R6, _X["Xu"]), (+_R6, _X["Xd"]), (-2.0 * _R6, _X["Xs"])],
}

# General fields of Sec. 2, Eq. (FieldOperator_B): B = eps ((q1 Gamma_1 q2) Gamma_2 q3).
#  * "p2", "n2": the nucleon with {Gamma_1, Gamma_2} = {C, gamma_5} (same flavour terms as p, n);
#  * decuplet fields with {C gamma_l, 1} (Sec. 4 footnote), l = 1, 2, 3 in the name:
#    Delta++ (uuu), Delta- (ddd), Omega- (sss), one term each; the members of
#    mixed flavour as the symmetric flavour combinations (a reading: the paper gives
#    no flavour wavefunctions), each term the literal Grassmann string eps (q1 G q2) q3:
#      Delta+  = (2 (u G d) u + (u G u) d) / sqrt3      Delta0 = (2 (d G u) d + (d G d) u) / sqrt3
#      Sigma*+ = (2 (u G s) u + (u G u) s) / sqrt3      Sigma*- = (2 (d G s) d + (d G d) s) / sqrt3
#      Sigma*0 = sqrt(2/3) ((u G d) s + (d G s) u + (s G u) d)
#      Xi*0    = (2 (s G u) s + (s G s) u) / sqrt3      Xi*-   = (2 (s G d) s + (s G s) d) / sqrt3
#    (Delta+ is T_- Delta++ / sqrt3 with T_- replacing one u by d.)
_R3, _R23 = 1.0 / math.sqrt(3.0), math.sqrt(2.0 / 3.0)
DECUPLET = {
    "D++": [(1.0, ("u", "u", "u"))],
    "D-": [(1.0, ("d", "d", "d"))],
    "O-": [(1.0, ("s", "s", "s"))],
    "D+": [(2 * _R3, ("u", "d", "u")), (_R3, ("u", "u", "d"))],
    "D0": [(2 * _R3, ("d", "u", "d")), (_R3, ("d", "d", "u"))],
    "S*+": [(2 * _R3, ("u", "s", "u")), (_R3, ("u", "u", "s"))],
    "S*0": [(_R23, ("u", "d", "s")), (_R23, ("d", "s", "u")), (_R23, ("s", "u", "d"))],
    "S*-": [(2 * _R3, ("d", "s", "d")), (_R3, ("d", "d", "s"))],
    "X*0": [(2 * _R3, ("s", "u", "s")), (_R3, ("s", "s", "u"))],
    "X*-": [(2 * _R3, ("s", "d", "s")), (_R3, ("s", "s", "d"))],
}
BARYONS["p2"] = BARYONS["p"]
BARYONS["n2"] = BARYONS["n"]
for _name, _terms in DECUPLET.items():
    for _l in (1, 2, 3):
        BARYONS["%s(%d)" % (_name, _l)] = _terms


def spin_structure(name):
    """(Gamma_1, Gamma_2) of a field, 4x4 complex (Dirac representation)."""
    g = dirac_gammas()
    if name in ("p2", "n2"):
        return charge_conjugation(), g[4]
    for d in DECUPLET:
        if name.startswith(d + "("):
            ell = int(name[len(d) + 1])
            return charge_conjugation() @ g[ell - 1], np.eye(4, dtype=complex)
    if name not in BARYONS:
        raise KeyError(name)
    return cg5(), np.eye(4, dtype=complex)


# The 52 channels in the order printed in Sec. 4, Eqs. (GeneralBB_NN)-(GeneralBB_XX):
# (B1, B2, B3, B4) = sink pair B1(X+r) B2(X), source pair with B3 <-> alpha', B4 <-> beta'.
_NL = [("p", "L"), ("S+", "n"), ("S0", "p")]
_LL_SINK = [("L", "L"), ("p", "X-"), ("n", "X0"), ("S+", "S-"), ("S0", "S0"), ("S0", "L")]
_LL_SRC = [("L", "L"), ("p", "X-"), ("n", "X0"), ("S+", "S-"), ("S0", "S0"), ("S0", "L")]
_OMITTED = {(("L", "L"), ("S0", "L")), (("S0", "S0"), ("S0", "L")),
            (("S0", "L"), ("L", "L")), (("S0", "L"), ("S0", "S0"))}
_XL = [("X-", "L"), ("S-", "X0"), ("S0", "X-")]


def _channels():
    ch = [("p", "n", "p", "n")]
    ch += [a + b for a in _NL for b in _NL]
    ch += [a + b for a in _LL_SINK for b in _LL_SRC if (a, b) not in _OMITTED]
    ch += [a + b for a in _XL for b in _XL]
    ch.append(("X-", "X0", "X-", "X0"))
    return ch


CHANNELS = _channels()
assert len(CHANNELS) == 52

# The four off-diagonal channels left out of the list because they vanish in the
# isospin limit (Sec. 4, after Eq. (GeneralBB_XX)).
ZERO_CHANNELS = [("L", "L", "S0", "L"), ("S0", "S0", "S0", "L"),
                 ("S0", "L", "L", "L"), ("S0", "L", "S0", "S0")]


def channel_terms(ch):
    """The four term lists (sink B1, sink B2, source B3, source B4) of a channel."""
    return [BARYONS[b] for b in ch]


def quark_content(ch):
    """(n_light, n_strange) quark propagators in every term of the channel."""
    f = BARYONS[ch[0]][0][1] + BARYONS[ch[1]][0][1]
    ns = sum(1 for q in f if q == "s")
    return 6 - ns, ns
