"""Graph mode: a correlate call captured into a HIP graph and replayed gives the
eager result bit for bit, on every replay, with eager work and synchronisations
between the replays and with the input buffers changed in place."""
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


@pytest.mark.parametrize("lat,dtype,chans", [((6, 6, 6), np.complex128, list(range(52))),
                                             ((4, 2, 3), np.complex64, [1, 10, 33, 51])])
def test_graph_replays_equal_eager(bbc, lat, dtype, chans):
    dev = torch.device("cuda:0")
    Sl, Ss = synth.propagators(lat, 3, seed=121, dtype=dtype)
    dl, ds = torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)
    fp32 = dtype == np.complex64
    eager, graph = bbc.Context(0), bbc.Context(0)
    graph.graph_mode(True)
    Lx, Ly, Lz = lat
    out = torch.empty((3, len(chans), Lz, Ly, Lx, 16), dtype=dl.dtype, device=dev)
    scale = torch.empty((3, len(chans)), dtype=torch.float64, device=dev) if fp32 else None
    t_list = [0, 1, 2]

    def run_eager():
        r = eager.correlate(dl, ds, t_list, chans, t0=0, energy=[0.3] * len(chans))
        torch.cuda.synchronize()
        return r if fp32 else (r, None)

    def run_graph():
        graph.correlate(dl, ds, t_list, chans, t0=0, energy=[0.3] * len(chans), out=out, scale=scale)
        torch.cuda.synchronize()

    ref, ref_s = run_eager()
    for rep in range(3):
        out.zero_()                                  # eager work between replays
        if scale is not None:
            scale.fill_(-1.0)
        x = torch.randn(256, 256, device=dev)
        (x @ x).sum().item()
        torch.cuda.synchronize()
        run_graph()
        assert torch.equal(out, ref), rep
        if fp32:
            assert torch.equal(scale, ref_s), rep
    # inputs changed in place: the replay reads the buffers' current contents
    dl.mul_(1.5)
    ds.mul_(0.5)
    ref2, ref2_s = run_eager()
    run_graph()
    assert torch.equal(out, ref2)
    if fp32:
        assert torch.equal(scale, ref2_s)
    # other time labels: a new capture, same agreement
    t_list = [2, 0, 1]
    ref3, ref3_s = run_eager()
    run_graph()
    assert torch.equal(out, ref3)
    graph.graph_mode(False)
    eager.close()
    graph.close()


@pytest.mark.skip(reason="graph-timed autotuning is not built: the first run of a build that captured each "
                         "candidate's round ended in a host segmentation fault inside bbc_autotune (FP64 case), "
                         "with no cause found in the code; the autotuner times ordinary launches")
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_autotune_in_graph_mode(bbc, dtype):
    """In graph mode the autotuner would time each candidate as replays of one captured
    graph; it returns a valid choice and keeps it for the shape, and graph replays with
    that choice still give the eager bits (8^3, three slices, channels 1 and 51)."""
    lat, chans = (8, 8, 8), [1, 51]
    print("case: autotune in graph mode", np.dtype(dtype).name, lat, flush=True)
    dev = torch.device("cuda:0")
    Sl, Ss = synth.propagators(lat, 3, seed=123, dtype=dtype)
    dl, ds = torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)
    prec = bbc.F32 if dtype == np.complex64 else bbc.F64
    eager = bbc.Context(0)
    ref = eager.correlate(dl, ds, [0, 1, 2], chans)
    torch.cuda.synchronize()
    ref = tuple(x.clone() for x in ref) if isinstance(ref, tuple) else (ref.clone(),)
    eager.close()
    ctx = bbc.Context(0)
    ctx.graph_mode(True)
    best, ms = ctx.autotune(dl[0].contiguous(), ds[0].contiguous(), chans, reps=2)
    assert ms > 0
    assert 0 <= best["pairs"] < (9 if prec == bbc.F64 else 6) and 0 <= best["blocks"] < 3
    assert 0 <= best["slices"] < 4 and 0 <= best["combine"] < 3 and best["planes"] == 0
    assert ctx.tuning(lat, chans, precision=prec) == (best, True)
    for rep in range(3):                             # capture, then replays with eager work between
        got = ctx.correlate(dl, ds, [0, 1, 2], chans)
        torch.cuda.synchronize()
        got = got if isinstance(got, tuple) else (got,)
        for a, b in zip(got, ref):
            assert torch.equal(a, b), (rep, best)
        x = torch.randn(128, 128, device=dev)
        (x @ x).sum().item()
    ctx.graph_mode(False)
    ctx.close()
