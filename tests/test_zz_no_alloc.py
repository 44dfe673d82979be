"""The allocation-free entry point (bbc_correlate_noalloc) through the C ABI: its
output equals bbc_correlate's bit for bit (same kernels, same reduction order) on
two calls in a row, the second with a smaller request, in both precisions; the
device's free memory does not change across a call (the library allocates
nothing); a request beyond the 192 MiB scratch is refused before any launch."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bbc():
    import paper_1510_00903_amd as mod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mod.load()
    return mod


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_noalloc_equals_correlate_two_calls(bbc, dtype):
    fp32 = dtype == np.complex64
    ref_ctx = bbc.Context(0)
    ctx = bbc.Context(0)
    cases = [((6, 6, 6), [0, 1], list(range(52)), [0.1 * k for k in range(52)]),      # large request
             ((4, 2, 3), [3], [1, 10, 51, 5, 30], None)]                              # then a smaller one
    for n, (lat, t_list, chans, energy) in enumerate(cases):
        Lx, Ly, Lz = lat
        Sl, Ss = synth.propagators(lat, max(t_list) + 1, seed=401 + n, t_list=t_list, dtype=dtype)
        dl, ds = _dev(Sl), _dev(Ss)
        print("case: noalloc", lat, "channels", len(chans), "fp32" if fp32 else "fp64", flush=True)
        want = ref_ctx.correlate(dl, ds, t_list, chans, t0=1, energy=energy)
        torch.cuda.synchronize()
        out = torch.full((len(t_list), len(chans), Lz, Ly, Lx, 16), float("nan"), dtype=dl.dtype, device="cuda:0")
        scale = torch.full((len(t_list), len(chans)), float("nan"), dtype=torch.float64,
                           device="cuda:0") if fp32 else None
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(0)[0]
        got = ctx.correlate_noalloc(dl, ds, t_list, chans, out, scale, t0=1, energy=energy)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(0)[0]
        assert free1 == free0, (free0, free1)
        if fp32:
            assert torch.equal(got[0], want[0]) and torch.equal(got[1], want[1])
        else:
            assert torch.equal(got, want)
    ctx.close()
    ref_ctx.close()


def test_noalloc_rejects_oversized_request(bbc):
    ctx = bbc.Context(0)
    lat = (8, 8, 8)
    chans = list(range(52))
    Sl, Ss = synth.propagators(lat, 1, seed=405)
    dl, ds = _dev(Sl), _dev(Ss)
    out = torch.empty((1, 52, 8, 8, 8, 16), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(bbc.BBCError) as e:
        ctx.correlate_noalloc(dl, ds, [0], chans, out)
    assert e.value.status == bbc.ENOMEM
    assert "192 MiB" in str(e.value)
    with pytest.raises(bbc.BBCError):               # host memory is refused
        ctx.correlate_noalloc(torch.from_numpy(Sl), torch.from_numpy(Ss), [0], chans, out.cpu())
    ctx.close()
