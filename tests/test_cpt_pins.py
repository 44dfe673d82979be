"""Pins of the lower spinor components and of the forward/backward (CPT) average
(oracle/cpt.py, Sec. 6) against facts that do not come from the oracle:

* brute force (literal 6x6 determinants over every tensor entry) with the lower
  components;
* in the Dirac representation gamma_5 = [[0, 1], [1, 0]] (2x2 blocks) swaps the
  upper and lower components and leaves the diquark matrix invariant
  (gamma_5^T C gamma_5 gamma_5 = C gamma_5), so with S' = gamma_5 S gamma_5 at every
  site the lower-component correlator of S' is the upper-component correlator of
  S, exactly (sink and source indices alike);
* the correlator is a product of six propagators, so scaling a slice by lambda
  scales it by lambda^6, which fixes the direction of the exp(E tau) normalisation
  on both sides of t0.
"""
import numpy as np
import pytest

import synth
from oracle import brute, cpt, operators as ops, wick

G5 = np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]]).astype(complex)
G5SC = np.kron(G5, np.eye(3))           # on spin-colour index 3 * mu + c


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def conj5(S):
    """gamma_5 S gamma_5 at every site (and slice)."""
    return np.einsum("ij,...jk,kl->...il", G5SC, S, G5SC)


def test_gamma5_premises():
    M = ops.cg5()
    assert np.allclose(G5.T @ M @ G5, M)
    assert np.abs(M).max() > 0
    v = np.arange(4.0)
    assert np.array_equal(G5 @ v, [2.0, 3.0, 0.0, 1.0])
    # general fields: C gamma_l picks up a sign per tensor, C and Gamma_2 = gamma_5 do not
    for name in ("O-(1)", "O-(2)", "O-(3)"):
        G1, G2 = ops.spin_structure(name)
        assert np.allclose(G5.T @ G1 @ G5, -G1) and np.allclose(G2, np.eye(4))
    G1, G2 = ops.spin_structure("p2")
    assert np.allclose(G5.T @ G1 @ G5, G1) and np.allclose(G5 @ G2 @ G5, G2)


@pytest.mark.parametrize("ch", [ops.CHANNELS[0], ops.CHANNELS[51]])
def test_lower_components_equal_brute_force(ch):
    Sl, Ss = synth.propagators((2, 1, 1), 1, seed=13)
    r = [(0, 0, 0), (1, 0, 0)]
    spins = [0, 6, 9, 15]
    ob = brute.correlate(Sl[0], Ss[0], ch, r, spins=spins, lower=True)
    ow = wick.correlate(Sl[0], Ss[0], ch, r, lower=True)
    assert rel(ob[:, spins], ow[:, spins]) < 1e-12
    up = wick.correlate(Sl[0], Ss[0], ch, r)
    assert rel(ow, up) > 1e-3                  # the lower components are another quantity


@pytest.mark.parametrize("ch", [ops.CHANNELS[0], ops.CHANNELS[10], ops.CHANNELS[33], ops.CHANNELS[51],
                                ("O-(1)", "O-(2)", "O-(1)", "O-(2)"), ("p2", "n", "p", "n2"),
                                ("S*0(3)", "D+(1)", "S*0(3)", "D+(1)")])
def test_gamma5_maps_upper_to_lower(ch):
    """Also for the general fields: gamma_5^T (C gamma_l) gamma_5 = -C gamma_l gives one sign per
    tensor (four in all), C is invariant, and Gamma_2 = gamma_5 commutes with gamma_5."""
    Sl, Ss = synth.propagators((2, 2, 1), 1, seed=17)
    r = wick.all_r(2, 2, 1)
    up = wick.correlate(Sl[0], Ss[0], ch, r)
    lo5 = wick.correlate(conj5(Sl[0]), conj5(Ss[0]), ch, r, lower=True)
    assert rel(lo5, up) < 1e-12
    lo = wick.correlate(Sl[0], Ss[0], ch, r, lower=True)
    up5 = wick.correlate(conj5(Sl[0]), conj5(Ss[0]), ch, r)
    assert rel(up5, lo) < 1e-12


def cpt_symmetric(lat, Lt, t0, alpha, seed):
    """Slices with S(t0 + tau) = e^{-alpha tau} A_tau, S(t0 - tau) = e^{-alpha tau} g5 A_tau g5,
    S(t0) = A_0 + g5 A_0 g5 (Lt odd, so the two sides never share a slice)."""
    n = Lt // 2 + 1
    Al, As = synth.propagators(lat, n, seed=seed)
    Sl = np.empty((Lt,) + Al.shape[1:], dtype=complex)
    Ss = np.empty_like(Sl)
    Sl[t0], Ss[t0] = Al[0] + conj5(Al[0]), As[0] + conj5(As[0])
    for tau in range(1, n):
        f = np.exp(-alpha * tau)
        Sl[(t0 + tau) % Lt], Ss[(t0 + tau) % Lt] = f * Al[tau], f * As[tau]
        Sl[(t0 - tau) % Lt], Ss[(t0 - tau) % Lt] = f * conj5(Al[tau]), f * conj5(As[tau])
    return Sl, Ss, Al, As


@pytest.mark.parametrize("ci", [1, 10])
def test_cpt_average_of_symmetric_inputs(ci):
    ch = ops.CHANNELS[ci]
    lat, Lt, t0, alpha = (2, 2, 2), 5, 1, 0.3
    Sl, Ss, Al, As = cpt_symmetric(lat, Lt, t0, alpha, seed=19)
    r = wick.all_r(*lat)
    for tau in range(3):                       # tau = 2 wraps: t0 - 2 = -1 -> slice 4
        want = wick.correlate(Sl[t0] if tau == 0 else Al[tau], Ss[t0] if tau == 0 else As[tau], ch, r)
        got = cpt.cpt_average(Sl, Ss, ch, t0, tau, sign=1.0, energy=6 * alpha)
        assert rel(got, want) < 1e-12, tau
        odd = cpt.cpt_average(Sl, Ss, ch, t0, tau, sign=-1.0, energy=6 * alpha)
        assert np.abs(odd).max() < 1e-12 * np.abs(want).max(), tau
    # the two halves are not interchangeable: forward slices read with lower components differ
    wrong = 0.5 * (wick.correlate(Sl[t0 + 1], Ss[t0 + 1], ch, r) +
                   wick.correlate(Sl[t0 + 1], Ss[t0 + 1], ch, r, lower=True)) * np.exp(6 * alpha)
    assert rel(wrong, wick.correlate(Al[1], As[1], ch, r)) > 1e-3
