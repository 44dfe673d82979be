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
