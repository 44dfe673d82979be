"""Post-processing kernels (spin projection, cubic-group A1+ projection, central
potential) on the GPU through the C ABI, against the oracle (oracle/postproc.py)
on the same seeded inputs."""
import itertools

import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle import postproc as pp
from oracle import wick

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1510_00903_amd as mod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = mod.Context(0)
    yield c
    c.close()


def rand_field(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def cg_weight_sets():
    """Weight matrices used in the tests: full (J, M) projection at sink and source;
    source projection keeping the sink pair; and a random 7 x 16 matrix (ragged n_out)."""
    sets = []
    for J, M in [(0, 0), (1, 1), (1, 0), (1, -1)]:
        P = pp.clebsch_gordan(J, M)
        sets.append(pp.spin_weights(P, P)[None, :])
        W = np.zeros((4, 16), dtype=complex)
        for a, b, ap, bp in itertools.product(range(2), repeat=4):
            W[a + 2 * b, pp.spin_index(a, b, ap, bp)] = P[ap][bp]
        sets.append(W)
    sets.append(rand_field((7, 16), 11))
    return sets


def tol(dtype):
    return 1e-13 if dtype == torch.complex128 else 2e-6


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("lat", [(4, 4, 4), (5, 3, 2)])
def test_spin_project_matches_oracle(ctx, dtype, lat):
    Lx, Ly, Lz = lat
    C = rand_field((3, 2, Lz, Ly, Lx, 16), 21)
    dC = torch.from_numpy(C).to("cuda:0", dtype)
    Cin = dC.cpu().numpy().astype(np.complex128)            # the values the kernel sees
    for W in cg_weight_sets():
        got = ctx.spin_project(dC, W).cpu().numpy().astype(np.complex128)
        ref = pp.spin_project(Cin, W)
        assert np.abs(got - ref).max() <= tol(dtype) * np.abs(ref).max()


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
@pytest.mark.parametrize("L,ncomp", [(4, 16), (5, 3), (6, 1), (8, 4), (17, 2), (21, 1)])
def test_cubic_project_matches_oracle(ctx, dtype, L, ncomp):
    # L^3 values of one component up to 64 KB go through LDS, larger ones are
    # gathered from global memory (17^3 FP64, 21^3 both forms)
    F = rand_field((2, L, L, L, ncomp), 31 + L)
    dF = torch.from_numpy(F).to("cuda:0", dtype)
    Fin = dF.cpu().numpy().astype(np.complex128)
    ref = pp.cubic_project(Fin, L)
    got = ctx.cubic_project(dF).cpu().numpy().astype(np.complex128)
    assert np.abs(got - ref).max() <= tol(dtype) * np.abs(ref).max()
    gotq = ctx.cubic_project(dF, complement=True).cpu().numpy().astype(np.complex128)
    assert np.abs(gotq - (Fin - ref)).max() <= tol(dtype) * np.abs(Fin).max()


@pytest.mark.parametrize("lat", [(4, 4, 4), (6, 5, 3)])
def test_central_potential_matches_oracle(ctx, lat):
    Lx, Ly, Lz = lat
    n_f, n_t = 3, 6
    R = rand_field((n_f, n_t, Lz, Ly, Lx), 41) + 3.0      # keep |R| away from 0
    dR = torch.from_numpy(R).to("cuda:0")
    got = ctx.central_potential(dR, 0.73).cpu().numpy()
    assert got.shape == (n_f, n_t - 2, Lz, Ly, Lx)
    for f in range(n_f):
        for t in range(1, n_t - 1):
            ref = pp.central_potential(R[f, t - 1], R[f, t], R[f, t + 1], 0.73)
            assert np.abs(got[f, t - 1] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_correlate_then_project_identical_source(ctx):
    """End to end on the GPU: Lambda Lambda -> Lambda Lambda on 3^3, source projected to
    (J, M) by the kernel, against the oracle's projection of the Wick oracle's C; the
    triplet projections vanish (identical source baryons)."""
    L = 3
    Sl, Ss = synth.propagators(L, 1, seed=61)
    ch = 10
    dev = torch.device("cuda:0")
    C = ctx.correlate(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), [0], [ch])
    Cref = wick.correlate(Sl[0], Ss[0], ops.CHANNELS[ch], wick.all_r(L, L, L)).reshape(L, L, L, 16)
    for J, M in [(0, 0), (1, 0)]:
        P = pp.clebsch_gordan(J, M)
        W = np.zeros((4, 16), dtype=complex)
        for a, b, ap, bp in itertools.product(range(2), repeat=4):
            W[a + 2 * b, pp.spin_index(a, b, ap, bp)] = P[ap][bp]
        got = ctx.spin_project(C, W).cpu().numpy()[0, 0]
        ref = pp.spin_project(Cref, W)
        scale = np.abs(Cref).max()
        assert np.abs(got - ref).max() <= 1e-12 * scale
        if J == 1:
            assert np.abs(got).max() <= 1e-12 * scale


def test_postproc_argument_errors(ctx):
    import paper_1510_00903_amd as mod
    dC = torch.zeros((1, 4, 4, 4, 16), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(mod.BBCError):
        ctx.spin_project(dC, np.zeros((17, 16)))                    # n_out > 16
    with pytest.raises(mod.BBCError):
        ctx.cubic_project(torch.zeros((1, 4, 4, 2, 3), dtype=torch.complex128, device="cuda:0"))  # not cubic
    with pytest.raises(mod.BBCError):
        ctx.central_potential(torch.zeros((2, 4, 4, 4), dtype=torch.complex128, device="cuda:0"), 1.0)
    with pytest.raises(mod.BBCError):
        ctx.spin_project(dC.cpu(), np.zeros((1, 16)))              # host tensor
