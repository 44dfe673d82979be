"""Degenerate inputs on the GPU: lattices with extents of 1 (a single site, lines
along one axis; Sec. 3's transforms then act on one or two axes only, and the
momentum groups are mostly padding), an empty slice list and an empty channel
list.  Correlators are compared with the oracle element by element."""
import numpy as np
import pytest

import synth
from oracle import wick

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GENERAL = [("O-(3)", "O-(3)", "O-(3)", "O-(3)"), ("p2", "n", "p", "n2"), ("D+(1)", "S*0(3)", "D+(2)", "S*0(3)")]


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


def _names(bbc, c):
    a, b = bbc.channel_name(c).split(">")
    return tuple(a.split() + b.split())


@pytest.mark.parametrize("dtype,tol", [(np.complex128, 1e-12), (np.complex64, 1e-5)])
@pytest.mark.parametrize("lat", [(1, 1, 1), (2, 1, 1), (1, 3, 1), (1, 1, 4)])
def test_degenerate_lattices_match_oracle(bbc, ctx, lat, dtype, tol):
    """Every listed channel and some general fields on lattices with unit extents."""
    Sl, Ss = synth.propagators(lat, 2, seed=171, dtype=dtype)
    chans = list(range(56)) + [bbc.channel_id(*q) for q in GENERAL]
    print("case: lattice", lat, np.dtype(dtype).name, flush=True)
    dev = torch.device("cuda:0")
    res = ctx.correlate(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), [0, 1], chans)
    torch.cuda.synchronize()
    if isinstance(res, tuple):
        got = res[0].cpu().numpy().astype(np.complex128) * res[1].cpu().numpy()[:, :, None, None, None, None]
    else:
        got = res.cpu().numpy()
    S64l, S64s = Sl.astype(np.complex128), Ss.astype(np.complex128)
    r = wick.all_r(*lat)
    for t in range(2):
        scale = 0.0
        for m, c in enumerate(chans):
            ref = wick.correlate(S64l[t], S64s[t], _names(bbc, c), r)
            g = got[t, m].reshape(-1, 16)
            if 52 <= c < 56:                       # isospin-zero channels vanish
                assert np.abs(ref).max() < 1e-12 * scale
                assert np.abs(g).max() < tol * scale, (lat, t, c)
                continue
            scale = max(scale, np.abs(ref).max())
            err = np.abs(g - ref).max() / np.abs(ref).max()
            assert err <= tol, (lat, t, bbc.channel_name(c), err)


def test_empty_slice_list(bbc, ctx):
    """No slices: nothing to compute, an empty result and no error."""
    dev = torch.device("cuda:0")
    S = torch.empty((0, 2, 2, 2, 12, 12), dtype=torch.complex128, device=dev)
    out = ctx.correlate(S, S.clone(), [], [0, 51])
    assert tuple(out.shape) == (0, 2, 2, 2, 2, 16)
    S32 = S.to(torch.complex64)
    out, scale = ctx.correlate(S32, S32.clone(), [], [10])
    assert tuple(out.shape) == (0, 1, 2, 2, 2, 16) and tuple(scale.shape) == (0, 1)


def test_empty_channel_list_rejected(bbc, ctx):
    Sl, Ss = synth.propagators((2, 2, 2), 1, seed=173)
    dev = torch.device("cuda:0")
    with pytest.raises(bbc.BBCError):
        ctx.correlate(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), [0], [])

