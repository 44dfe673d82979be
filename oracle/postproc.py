"""Post-processing of C(r, t) as the paper describes it (Sec. 2): spin projection
to total spin (J, M), projection of the spatial dependence onto the A1+
representation of the cubic group, and the leading-order central potential of
the HAL QCD method.  Plain definitions, FP64, numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Conventions (readings of the paper taken here):
  * Spinor components: Dirac representation, upper (or lower) two components
    of each baryon index; component 0 is spin up and 1 spin down along z
    (Sigma_z = diag(sigma_z, sigma_z) in this representation).
  * Spin index of a correlator value: s = a + 2 (b + 2 (a' + 2 b')) for sink
    spins a (B1), b (B2) and source spins a' (B3), b' (B4).
  * P^(J,M)_{a b}: Clebsch-Gordan coefficients of two spin-1/2 particles,
    |J M> = sum_{ab} P^(J,M)_{ab} |a>|b>  (Sec. 2, source operator J^(J,M)).
  * The cubic-group projection acts on the relative coordinate r only
    (the orbital part), averaging over the 24 proper rotations O; Q = 1 - P.
  * The potential uses the six-point periodic lattice Laplacian and the
    symmetric time difference (R(t+1) - R(t-1)) / 2; V = (lap R / (2 mu) -
    d_t R) / R, elementwise (Sec. 2, leading order of the velocity expansion).
"""
from __future__ import annotations

import itertools

import numpy as np

SQ2 = np.sqrt(0.5)

# (J, M) -> 2x2 table P[a][b] (component 0 = up, 1 = down)
_CG = {
    (0, 0): np.array([[0.0, SQ2], [-SQ2, 0.0]]),
    (1, 1): np.array([[1.0, 0.0], [0.0, 0.0]]),
    (1, 0): np.array([[0.0, SQ2], [SQ2, 0.0]]),
    (1, -1): np.array([[0.0, 0.0], [0.0, 1.0]]),
}


def clebsch_gordan(J, M):
    """P^(J,M)_{ab} for two spin-1/2 baryons (a, b in {0 = up, 1 = down})."""
    return _CG[(J, M)].copy()


def spin_index(a, b, ap, bp):
    return a + 2 * (b + 2 * (ap + 2 * bp))


def spin_weights(sink, source):
    """Weight vector w[s] (16) of the combination sum_{ab a'b'} sink[a][b]^* source[a'][b'] C_s.

    sink / source are 2x2 tables (None keeps that pair unprojected is not
    expressible as one vector; use spin_weight_matrix for that)."""
    w = np.zeros(16, dtype=np.complex128)
    for a, b, ap, bp in itertools.product(range(2), repeat=4):
        w[spin_index(a, b, ap, bp)] = np.conj(sink[a][b]) * source[ap][bp]
    return w


def spin_project(C, W):
    """out[..., m] = sum_s W[m, s] C[..., s]  (C has 16 spin values last)."""
    return np.einsum("ms,...s->...m", np.asarray(W), C)


def cubic_rotations():
    """The 24 proper rotations of the cube: signed 3x3 permutation matrices with det +1."""
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            if round(np.linalg.det(R)) == 1:
                mats.append(R)
    return mats


def cubic_project(F, L):
    """A1+ projection of the spatial argument: (1/24) sum_{R in O} F(R r).

    F: array [..., L, L, L, n] indexed [z][y][x][component] (x fastest in r);
    r is taken mod L on the periodic lattice."""
    F = np.asarray(F)
    out = np.zeros_like(F, dtype=np.complex128)
    idx = np.indices((L, L, L))            # idx[0] = z, idx[1] = y, idx[2] = x
    r = np.stack([idx[2], idx[1], idx[0]])  # (x, y, z)
    for R in cubic_rotations():
        rr = np.tensordot(R, r, axes=1) % L  # rotated (x, y, z)
        out += F[..., rr[2], rr[1], rr[0], :]
    return out / 24.0


def laplacian(F, L):
    """Six-point periodic lattice Laplacian over the three axes of F[..., z, y, x]."""
    out = -6.0 * F
    for ax in (-1, -2, -3):
        out = out + np.roll(F, 1, axis=ax) + np.roll(F, -1, axis=ax)
    return out


def central_potential(R_prev, R_now, R_next, inv_2mu):
    """V(r, t) = (lap R(r,t) * inv_2mu - (R(r,t+1) - R(r,t-1)) / 2) / R(r,t).

    R_*: complex arrays [z][y][x] at t-1, t, t+1 (cubic lattice)."""
    L = R_now.shape[-1]
    return (laplacian(R_now, L) * inv_2mu - 0.5 * (R_next - R_prev)) / R_now
