"""Rotation covariance of the correlators (a pin of the general fields of Sec. 2,
Eq. (FieldOperator_B), that does not come from the Wick oracle's arithmetic).

A rotation R by 90 degrees about z acts on a quark propagator as
S'(x) = Lam S(R^-1 x) Lam^-1, with the spinor rotation Lam defined by
Lam^-1 gamma_i Lam = R_ij gamma_j (textbook Clifford algebra; block diagonal in the
Dirac representation, so upper components stay upper).  Every baryon tensor
T(xi; gamma) then transforms linearly -- the octet fields as spinors, the decuplet
fields {C gamma_l, 1} as vector-spinors (the index l rotates with R) -- and the
correlator built from S' is the same linear map applied to the correlator of S at
R^-1 r.  The maps are read off the tensors (least squares, residual checked) and
must equal the textbook forms; the correlators come from the Wick oracle.  A wrong
gamma matrix, a mislabelled l or a wrong site map breaks one of the checks."""
import itertools

import numpy as np
import pytest

import synth
from oracle import operators as ops, wick

R = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])


def spinor_rotation():
    g1, g2, g3, g4, g5 = ops.dirac_gammas()
    lam = np.cos(np.pi / 4) * np.eye(4) - np.sin(np.pi / 4) * (g1 @ g2)
    li = np.linalg.inv(lam)
    for i, g in enumerate((g1, g2, g3)):
        assert np.allclose(li @ g @ lam, sum(R[i, j] * (g1, g2, g3)[j] for j in range(3)))
    assert np.allclose(lam[:2, 2:], 0) and np.allclose(lam[2:, :2], 0)
    return lam


def dense_tensor(name):
    """T[gamma, xi_a, xi_b, xi_c] = eps(c_a c_b c_c) Gamma_1(mu_a, mu_b) Gamma_2(gamma, mu_c)."""
    M1, M2 = ops.spin_structure(name)
    eps = ops.levi_civita()
    T = np.zeros((4, 12, 12, 12), dtype=complex)
    for ca, cb, cc in itertools.product(range(3), repeat=3):
        if eps[ca, cb, cc] == 0:
            continue
        for ma, mb, mc in itertools.product(range(4), repeat=3):
            T[:, 3 * ma + ca, 3 * mb + cb, 3 * mc + cc] += eps[ca, cb, cc] * M1[ma, mb] * M2[:, mc]
    return T


def family_maps(family, lam):
    """Linear maps of a field family (index k = member * 4 + gamma) at the sink and the source.
    They must be the textbook ones: from Lam^T C = C Lam^-1 and Lam^-1 gamma_i Lam = R_ij gamma_j,
    a spinor field maps with Lam at the sink and Lam^-T at the source, a vector-spinor
    field (C gamma_l) with R (x) Lam and R^T (x) Lam^-T -- which fixes the labels l = 1, 2, 3
    to the x, y, z axes."""
    L = np.kron(lam, np.eye(3))
    Li = np.linalg.inv(L)
    T = np.concatenate([dense_tensor(n) for n in family]).reshape(4 * len(family), -1)
    Tk = T.reshape(-1, 12, 12, 12)
    sink = np.einsum("kabc,ax,by,cz->kxyz", Tk, L, L, L).reshape(T.shape[0], -1)
    src = np.einsum("kabc,xa,yb,zc->kxyz", Tk, Li, Li, Li).reshape(T.shape[0], -1)
    P = np.linalg.pinv(T)
    A, B = sink @ P, src @ P
    assert np.abs(A @ T - sink).max() < 1e-10 and np.abs(B @ T - src).max() < 1e-10
    Rf = R if len(family) == 3 else np.eye(1)
    assert np.abs(A - np.kron(Rf, lam)).max() < 1e-12
    assert np.abs(B - np.kron(Rf.T, np.linalg.inv(lam).T)).max() < 1e-12
    for M in (A, B):               # upper spin components do not mix with lower ones
        for k, j in itertools.product(range(M.shape[0]), repeat=2):
            if (k % 4 < 2) != (j % 4 < 2):
                assert abs(M[k, j]) < 1e-12
    return A, B


def rotate_props(S, lam):
    """S'(x) = Lam S(R^-1 x) Lam^-1 on [z][y][x][12][12]; R^-1 (x, y, z) = (y, -x, z)."""
    L = np.kron(lam, np.eye(3))
    Li = np.linalg.inv(L)
    Lz, Ly, Lx = S.shape[:3]
    assert Lx == Ly
    out = np.empty_like(S)
    for z, y, x in itertools.product(range(Lz), range(Ly), range(Lx)):
        out[z, y, x] = L @ S[z, (-x) % Ly, y] @ Li
    return out


FAMILIES = {"O": ["O-(1)", "O-(2)", "O-(3)"], "D": ["D++(1)", "D++(2)", "D++(3)"], "p": ["p"], "n": ["n"],
            "p2": ["p2"], "L": ["L"]}


@pytest.mark.parametrize("fams,members", [
    (("O", "p", "O", "p"), (0, 0, 1, 0)),          # O-(1) p > O-(2) p
    (("O", "O", "O", "O"), (2, 2, 2, 2)),          # O-(3) O-(3) > O-(3) O-(3)
    (("D", "O", "D", "O"), (1, 0, 0, 2)),          # D++(2) O-(1) > D++(1) O-(3)
    (("p2", "n", "p", "n"), (0, 0, 0, 0)),
    (("p", "L", "p", "L"), (0, 0, 0, 0)),
])
def test_rotation_covariance(fams, members):
    lam = spinor_rotation()
    maps = [family_maps(FAMILIES[f], lam) for f in fams]
    lat = (3, 3, 2)
    Sl, Ss = synth.propagators(lat, 1, seed=151)
    Sl, Ss = Sl[0], Ss[0]
    r = wick.all_r(*lat)
    target = tuple(FAMILIES[f][m] for f, m in zip(fams, members))
    got = wick.correlate(rotate_props(Sl, lam), rotate_props(Ss, lam), target, r)
    # R^-1 r for every r, as an index into the all-r list (x fastest)
    Lx, Ly, Lz = lat
    rinv = [((ry % Lx) + Lx * (((-rx) % Ly) + Ly * rz)) for rx, ry, rz in r]
    want = np.zeros_like(got)
    rows = [maps[i][0] if i < 2 else maps[i][1] for i in range(4)]
    ups = [[(m, d) for m in range(len(FAMILIES[f])) for d in range(2)] for f in fams]
    cache = {}
    for a, b, ap, bp in itertools.product(range(2), repeat=4):
        s_out = a + 2 * (b + 2 * (ap + 2 * bp))
        k = [members[0] * 4 + a, members[1] * 4 + b, members[2] * 4 + ap, members[3] * 4 + bp]
        for (m1, d1), (m2, d2), (m3, d3), (m4, d4) in itertools.product(*ups):
            c = (rows[0][k[0], m1 * 4 + d1] * rows[1][k[1], m2 * 4 + d2] *
                 rows[2][k[2], m3 * 4 + d3] * rows[3][k[3], m4 * 4 + d4])
            if abs(c) < 1e-14:
                continue
            key = (m1, m2, m3, m4)
            if key not in cache:
                ch = tuple(FAMILIES[f][m] for f, m in zip(fams, key))
                cache[key] = wick.correlate(Sl, Ss, ch, r)
            s_in = d1 + 2 * (d2 + 2 * (d3 + 2 * d4))
            want[:, s_out] += c * cache[key][rinv, s_in]
    assert np.abs(got).max() > 0
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()
