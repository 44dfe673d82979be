"""Pins of the post-processing oracle (oracle/postproc.py) against facts that do
not come from it: spin algebra of two spin-1/2 particles, the group structure
of the cube's rotations, eigenfunctions of the lattice Laplacian, and the
antisymmetry of identical-baryon sources (Sec. 6) through the Wick oracle."""
import itertools

import numpy as np
import pytest

from oracle import operators as ops
from oracle import postproc as pp
from oracle import wick

# Pauli matrices (textbook); basis |0> = up, |1> = down
SX = np.array([[0, 1], [1, 0]], dtype=complex)
SY = np.array([[0, -1j], [1j, 0]])
SZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2)


def total_spin():
    S = [0.5 * (np.kron(s, I2) + np.kron(I2, s)) for s in (SX, SY, SZ)]
    S2 = sum(s @ s for s in S)
    Splus = S[0] + 1j * S[1]
    return S2, S[2], Splus


def cg_vector(J, M):
    P = pp.clebsch_gordan(J, M)
    return np.array([P[a][b] for a in range(2) for b in range(2)], dtype=complex)  # kron order: a outer


@pytest.mark.parametrize("J,M", [(0, 0), (1, 1), (1, 0), (1, -1)])
def test_clebsch_gordan_are_spin_eigenstates(J, M):
    S2, Sz, _ = total_spin()
    v = cg_vector(J, M)
    assert np.allclose(np.linalg.norm(v), 1.0)
    assert np.allclose(S2 @ v, J * (J + 1) * v)
    assert np.allclose(Sz @ v, M * v)


def test_clebsch_gordan_phases_condon_shortley():
    # S_+ |1,M> = sqrt(2 - M(M+1)) |1,M+1> fixes the relative signs of the triplet;
    # the singlet is orthogonal to the triplet and has + on |up,down>.
    _, _, Sp = total_spin()
    for M in (-1, 0):
        assert np.allclose(Sp @ cg_vector(1, M), np.sqrt(2 - M * (M + 1)) * cg_vector(1, M + 1))
    assert np.allclose(Sp @ cg_vector(0, 0), 0)
    assert cg_vector(0, 0)[1] > 0                   # |up, down> component
    vs = [cg_vector(*jm) for jm in [(0, 0), (1, 1), (1, 0), (1, -1)]]
    G = np.array([[np.vdot(a, b) for b in vs] for a in vs])
    assert np.allclose(G, np.eye(4))


def test_cubic_rotations_form_the_group_O():
    Rs = pp.cubic_rotations()
    keys = {R.tobytes() for R in Rs}
    assert len(Rs) == 24 and len(keys) == 24
    for A in Rs:
        assert round(np.linalg.det(A)) == 1
        assert np.array_equal(A @ A.T, np.eye(3, dtype=int))
        for B in Rs:
            assert (A @ B).tobytes() in keys
    c4z = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])
    c3 = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]])
    assert c4z.tobytes() in keys and c3.tobytes() in keys
    # element orders of O: 1 identity, 9 of order 2 (3 C2 about axes + 6 about edges), 8 of order 3, 6 of order 4
    def order(R):
        P, k = R.copy(), 1
        while not np.array_equal(P, np.eye(3, dtype=int)):
            P, k = P @ R, k + 1
        return k
    counts = {}
    for R in Rs:
        counts[order(R)] = counts.get(order(R), 0) + 1
    assert counts == {1: 1, 2: 9, 3: 8, 4: 6}


def coords(L):
    z, y, x = np.indices((L, L, L))
    return x, y, z


@pytest.mark.parametrize("L", [4, 5, 6])
def test_cubic_projection_properties(L):
    rng = np.random.default_rng(3)
    F = rng.standard_normal((2, L, L, L, 3)) + 1j * rng.standard_normal((2, L, L, L, 3))
    P = pp.cubic_project(F, L)
    assert np.allclose(pp.cubic_project(P, L), P)                  # idempotent
    Q = F - P
    assert abs(np.vdot(P, Q)) < 1e-9 * np.vdot(F, F).real          # P and 1-P orthogonal
    x, y, z = coords(L)
    dx, dy, dz = [np.minimum(c, L - c) for c in (x, y, z)]
    g = np.exp(-0.3 * (dx ** 2 + dy ** 2 + dz ** 2))[..., None]    # rotation invariant (min image)
    assert np.allclose(pp.cubic_project(g, L), g)
    s = np.sin(2 * np.pi * x / L)[..., None]                       # l = 1: no A1 part
    assert np.allclose(pp.cubic_project(s, L), 0)
    c = np.cos(2 * np.pi * x / L)[..., None]
    want = (np.cos(2 * np.pi * x / L) + np.cos(2 * np.pi * y / L) + np.cos(2 * np.pi * z / L))[..., None] / 3
    assert np.allclose(pp.cubic_project(c, L), want)


def test_potential_closed_form():
    # R = cos(2 pi n.r / L) exp(-E t) is an eigenfunction of the six-point Laplacian with
    # eigenvalue sum_d 2 (cos(2 pi n_d / L) - 1); the symmetric difference gives -sinh(E) R.
    L, E, inv2mu = 6, 0.37, 0.81
    n = (1, 2, 0)
    x, y, z = coords(L)
    phase = 2 * np.pi * (n[0] * x + n[1] * y + n[2] * z) / L
    lam = sum(2 * (np.cos(2 * np.pi * k / L) - 1) for k in n)
    R = [np.cos(phase + 0.3) * np.exp(-E * t) + 0j for t in (3, 4, 5)]
    V = pp.central_potential(R[0], R[1], R[2], inv2mu)
    assert np.allclose(V, lam * inv2mu + np.sinh(E))


def test_spin_projection_of_identical_source_baryons():
    # Identical source baryons (Lambda Lambda) make C antisymmetric in (a', b') (Sec. 6):
    # every source triplet projection vanishes, the singlet does not.
    L = 2
    rng_seed = 5
    import synth
    Sl, Ss = synth.propagators(L, 1, seed=rng_seed)
    ch = 10                                           # Lambda Lambda -> Lambda Lambda
    C = wick.correlate(Sl[0], Ss[0], ops.CHANNELS[ch], wick.all_r(L, L, L))   # [r][16]
    for (J, M) in [(1, 1), (1, 0), (1, -1), (0, 0)]:
        P = pp.clebsch_gordan(J, M)
        W = np.zeros((4, 16), dtype=complex)          # keep sink (a, b), project the source
        for a, b, ap, bp in itertools.product(range(2), repeat=4):
            W[a + 2 * b, pp.spin_index(a, b, ap, bp)] = P[ap][bp]
        out = pp.spin_project(C, W)
        if J == 1:
            assert np.abs(out).max() < 1e-12 * np.abs(C).max()
        else:
            assert np.abs(out).max() > 0.1 * np.abs(C).max()
