"""Forward/backward (CPT) average (Sec. 6) on the GPU through the C ABI: against
the oracle (oracle/cpt.py) element by element on small lattices, and at larger
sizes through the exact property of CPT-symmetric inputs (S(t0 - tau) =
gamma_5 S(t0 + tau) gamma_5 makes the backward part equal the forward one)."""
import numpy as np
import pytest

import synth
from oracle import cpt, operators as ops

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G5 = np.block([[np.zeros((2, 2)), np.eye(2)], [np.eye(2), np.zeros((2, 2))]])
G5SC = np.kron(G5, np.eye(3))


@pytest.fixture(scope="module")
def bbc():
    import paper_1510_00903_amd as mod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mod.load()
    return mod


@pytest.fixture(scope="module")
def ctx(bbc):
    c = bbc.Context(0)
    yield c
    c.close()


def run(ctx, Sl, Ss, t0, taus, chans, **kw):
    dev = torch.device("cuda:0")
    out = ctx.correlate_cpt(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), t0, taus, chans, **kw)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return out[0].cpu().numpy().astype(np.complex128) * out[1].cpu().numpy()[:, :, None, None, None, None]
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype,tol", [(np.complex128, 1e-12), (np.complex64, 1e-5)])
@pytest.mark.parametrize("lat,t0,sign", [((3, 2, 2), 1, 1), ((2, 3, 4), 4, -1)])
def test_cpt_matches_oracle(ctx, dtype, tol, lat, t0, sign):
    Lt = 5
    Sl, Ss = synth.propagators(lat, Lt, seed=131, dtype=dtype)
    chans = [0, 1, 10, 51, 56]
    energy = [0.1, -0.2, 0.3, 0.0, 0.25]
    taus = [0, 1, 2, 4]                      # t0 - tau wraps; tau = 4 reads the far slices
    got = run(ctx, Sl, Ss, t0, taus, chans, sign=sign, energy=energy)
    Lx, Ly, Lz = lat
    assert got.shape == (len(taus), len(chans), Lz, Ly, Lx, 16)
    S64l, S64s = Sl.astype(np.complex128), Ss.astype(np.complex128)
    for n, tau in enumerate(taus):
        for m, c in enumerate(chans):
            name = ctx_name(c)
            ref = cpt.cpt_average(S64l, S64s, name, t0, tau, sign=sign, energy=energy[m])
            err = np.abs(got[n, m].reshape(-1, 16) - ref).max() / np.abs(ref).max()
            assert err <= tol, (tau, c, err)


@pytest.mark.parametrize("dtype,tol", [(np.complex128, 1e-12), (np.complex64, 1e-5)])
@pytest.mark.parametrize("lat,sign", [((1, 1, 1), 1), ((2, 1, 3), -1)])
def test_cpt_single_time_slice(ctx, bbc, dtype, tol, lat, sign):
    """Lt = 1 (degenerate): tau = 0 is the only distance and both halves read slice 0;
    on lattices with unit extents, octet and general-field channels."""
    Sl, Ss = synth.propagators(lat, 1, seed=137, dtype=dtype)
    chans = [0, 10, 51, bbc.channel_id("O-(3)", "O-(3)", "O-(3)", "O-(3)")]
    print("case: Lt=1 lattice", lat, np.dtype(dtype).name, flush=True)
    got = run(ctx, Sl, Ss, 0, [0], chans, sign=sign, energy=[0.1, -0.2, 0.3, 0.0])
    S64l, S64s = Sl.astype(np.complex128), Ss.astype(np.complex128)
    for m, c in enumerate(chans):
        ref = cpt.cpt_average(S64l, S64s, ctx_name(c), 0, 0, sign=sign, energy=0.0)
        err = np.abs(got[0, m].reshape(-1, 16) - ref).max() / np.abs(ref).max()
        assert err <= tol, (c, err)


def test_cpt_empty_tau_list(ctx):
    """No distances: a valid empty request."""
    dev = torch.device("cuda:0")
    S = torch.zeros((3, 2, 2, 2, 12, 12), dtype=torch.complex128, device=dev)
    out = ctx.correlate_cpt(S, S, 1, [], [0, 51])
    assert tuple(out.shape) == (0, 2, 2, 2, 2, 16)
    S32 = S.to(torch.complex64)
    out, scale = ctx.correlate_cpt(S32, S32, 1, [], [10])
    assert tuple(out.shape) == (0, 1, 2, 2, 2, 16) and tuple(scale.shape) == (0, 1)


def ctx_name(c):
    import paper_1510_00903_amd as mod
    a, b = mod.channel_name(c).split(">")
    return tuple(a.split() + b.split())


def conj5(S):
    return np.einsum("ij,...jk,kl->...il", G5SC, S, G5SC)


@pytest.mark.parametrize("lat,dtype,tol", [((8, 8, 8), np.complex128, 1e-12), ((16, 16, 16), np.complex64, 1e-5)])
def test_cpt_symmetric_inputs(ctx, lat, dtype, tol):
    """S(t0 + tau) = A_tau, S(t0 - tau) = g5 A_tau g5, S(t0) = A_0 + g5 A_0 g5: the average
    with sign +1 is the upper-component correlator of A_tau, with sign -1 it vanishes."""
    Lt, t0 = 5, 3
    A_l, A_s = synth.propagators(lat, 3, seed=137, dtype=dtype)
    Sl = np.empty((Lt,) + A_l.shape[1:], dtype=dtype)
    Ss = np.empty_like(Sl)
    Sl[t0], Ss[t0] = A_l[0] + conj5(A_l[0]), A_s[0] + conj5(A_s[0])
    for tau in (1, 2):
        Sl[(t0 + tau) % Lt], Ss[(t0 + tau) % Lt] = A_l[tau], A_s[tau]
        Sl[(t0 - tau) % Lt], Ss[(t0 - tau) % Lt] = conj5(A_l[tau]), conj5(A_s[tau])
    chans = [1, 10, 33]
    taus = [0, 1, 2]
    even = run(ctx, Sl, Ss, t0, taus, chans, sign=1)
    odd = run(ctx, Sl, Ss, t0, taus, chans, sign=-1)
    dev = torch.device("cuda:0")
    B_l = np.stack([Sl[t0], A_l[1], A_l[2]])
    B_s = np.stack([Ss[t0], A_s[1], A_s[2]])
    fwd = ctx.correlate(torch.from_numpy(B_l).to(dev), torch.from_numpy(B_s).to(dev), [0, 1, 2], chans)
    torch.cuda.synchronize()
    if isinstance(fwd, tuple):
        fwd = fwd[0].cpu().numpy().astype(np.complex128) * fwd[1].cpu().numpy()[:, :, None, None, None, None]
    else:
        fwd = fwd.cpu().numpy()
    for n in range(3):
        for m in range(len(chans)):
            scale = np.abs(fwd[n, m]).max()
            assert np.abs(even[n, m] - fwd[n, m]).max() <= tol * scale, (n, m)
            assert np.abs(odd[n, m]).max() <= tol * scale, (n, m)


def test_cpt_argument_errors(ctx, bbc):
    dev = torch.device("cuda:0")
    S = torch.zeros((3, 2, 2, 2, 12, 12), dtype=torch.complex128, device=dev)
    with pytest.raises(bbc.BBCError):
        ctx.correlate_cpt(S, S, 0, [0], [0], sign=0)
    with pytest.raises(bbc.BBCError):
        ctx.correlate_cpt(S, S, 0, [3], [0])                 # tau >= Lt
    with pytest.raises(bbc.BBCError):
        ctx.correlate_cpt(S, S, 3, [0], [0])                 # t0 >= Lt
    with pytest.raises(bbc.BBCError):
        ctx.correlate_cpt(S.cpu(), S.cpu(), 0, [0], [0])     # host tensors
    with pytest.raises(bbc.BBCError):
        ctx.correlate_cpt(S, S, 0, [0], [57])                # not a channel
