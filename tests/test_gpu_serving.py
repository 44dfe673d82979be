"""Serving (continuous batching) on the GPU: results in the mix equal results alone,
admission by HBM footprint, cancellation, timeouts."""
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


def _props(lat, T, seed, dtype):
    Sl, Ss = synth.propagators(lat, T, seed=seed, dtype=dtype)
    dev = torch.device("cuda:0")
    return torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mix_equals_alone(bbc, prec):
    """Jobs of different lattices, channel subsets and slices, submitted together to a
    3-slot server, give bit-identical results to the same jobs run alone."""
    dtype = np.complex128 if prec == "f64" else np.complex64
    tdt = torch.complex128 if prec == "f64" else torch.complex64
    ctx = bbc.Context(0)
    sets = {(4, 4, 4): _props((4, 4, 4), 6, 301, dtype), (6, 6, 6): _props((6, 6, 6), 5, 302, dtype),
            (4, 2, 3): _props((4, 2, 3), 4, 303, dtype)}
    rng = np.random.default_rng(304)
    jobs = []
    for i in range(12):
        lat = list(sets)[i % 3]
        T = sets[lat][0].shape[0]
        n_t = int(rng.integers(1, T + 1))
        sl = sorted(rng.choice(T, size=n_t, replace=False).tolist())
        n_ch = int(rng.integers(1, 20))
        ch = rng.choice(56, size=n_ch, replace=False).tolist()
        jobs.append((lat, sl, ch))
    # alone: direct correlate
    alone = []
    for lat, sl, ch in jobs:
        Sl, Ss = sets[lat]
        r = ctx.correlate(Sl[sl], Ss[sl], sl, ch, t0=1, energy=[0.1 * k for k in range(len(ch))])
        torch.cuda.synchronize()
        alone.append(tuple(x.cpu() for x in r) if isinstance(r, tuple) else r.cpu())
    # mix: server
    ctx.server_start(3)
    handles = {lat: ctx.prop_upload(*sets[lat]) for lat in sets}
    outs, ids = [], []
    for lat, sl, ch in jobs:
        Lx, Ly, Lz = lat
        out = torch.zeros((len(sl), len(ch), Lz, Ly, Lx, 16), dtype=tdt, device="cuda:0")
        scale = torch.zeros((len(sl), len(ch)), dtype=torch.float64, device="cuda:0") if prec == "f32" else None
        ids.append(ctx.submit(handles[lat], sl, sl, ch, out, scale, t0=1,
                              energy=[0.1 * k for k in range(len(ch))]))
        outs.append((out, scale))
    for j in ids:
        ctx.wait(j, 60000)
        assert ctx.poll(j) == "done"
        q, r, tot = ctx.job_times(j)
        assert 0 <= q <= tot and 0 <= r <= tot
    torch.cuda.synchronize()
    for (out, scale), ref in zip(outs, alone):
        if prec == "f64":
            assert torch.equal(out.cpu(), ref)
        else:
            assert torch.equal(out.cpu(), ref[0]) and torch.equal(scale.cpu(), ref[1])
    for h in handles.values():
        ctx.prop_release(h)
    ctx.server_stop()
    ctx.close()


def test_cancel_timeout_and_budget(bbc):
    ctx = bbc.Context(0)
    Sl, Ss = _props((16, 16, 16), 8, 305, np.complex128)
    ctx.server_start(1)
    h = ctx.prop_upload(Sl, Ss)
    big = torch.empty((8, 52, 16, 16, 16, 16), dtype=torch.complex128, device="cuda:0")
    j1 = ctx.submit(h, list(range(8)), list(range(8)), list(range(52)), big)
    j2 = ctx.submit(h, [0], [0], [1], torch.empty((1, 1, 16, 16, 16, 16), dtype=torch.complex128, device="cuda:0"))
    with pytest.raises(bbc.BBCError) as e:
        ctx.wait(j1, 0)
    assert e.value.status == bbc.ETIMEOUT
    ctx.cancel(j2)                      # still queued behind j1 on the single slot
    with pytest.raises(bbc.BBCError) as e:
        ctx.wait(j2, 60000)
    assert e.value.status == bbc.ECANCELLED
    ctx.wait(j1, 120000)
    assert ctx.poll(j1) == "done"
    ctx.job_forget(j1)
    with pytest.raises(bbc.BBCError):
        ctx.poll(j1)
    ctx.prop_release(h)
    with pytest.raises(bbc.BBCError):    # released handle
        ctx.submit(h, [0], [0], [1], big)
    ctx.server_stop()
    ctx.close()
    # a budget too small for the job's workspace is refused at submission
    small = bbc.Context(0, hbm_budget_bytes=64 << 20)
    small.server_start(1)
    h2 = small.prop_upload(Sl[:1], Ss[:1])
    with pytest.raises(bbc.BBCError) as e:
        small.submit(h2, [0], [0], list(range(52)), big)
    assert e.value.status == bbc.ENOMEM
    small.server_stop()
    small.close()
