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


@pytest.mark.parametrize("graphs", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mix_equals_alone(bbc, prec, graphs):
    """Jobs of different lattices, channel subsets and slices, submitted together to a
    3-slot server, give bit-identical results to the same jobs run alone.  With graph
    mode on, the slots replay one captured slice per request shape (the slice's
    pointers written to the slot's argument record first); the jobs then run twice,
    so the second round replays graphs captured in the first."""
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
    if graphs:
        ctx.graph_mode(True)
    ctx.server_start(3)
    handles = {lat: ctx.prop_upload(*sets[lat]) for lat in sets}
    outs, ids = [], []
    for lat, sl, ch in jobs * (2 if graphs else 1):
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
    for (out, scale), ref in zip(outs, alone * (2 if graphs else 1)):
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
        small.submit(h2, [0], [0], list(range(52)), big[:1].contiguous())
    assert e.value.status == bbc.ENOMEM
    small.server_stop()
    small.close()


def _job_bytes(bbc, lat, chans, prec):
    """Device bytes the server commits to a job: its workspace plus its energies."""
    return bbc.footprint(lat, chans, prec) + 8 * len(chans) + 256


def test_finite_budget_admission(bbc):
    """Admission by HBM footprint with a finite budget.  Two small jobs leave idle
    workspaces in both slots; a large job that fits the budget only once an idle
    workspace is released must still run (and equal the direct result bit for bit).
    A job that cannot fit beside its own propagator set is refused at submission; one
    that cannot fit beside another resident set while nothing runs fails with
    BBC_ENOMEM instead of waiting for ever, and runs once that set is released."""
    lat = (4, 4, 4)
    Lx, Ly, Lz = lat
    Sl, Ss = _props(lat, 2, 306, np.complex128)
    props = 2 * Sl.numel() * 16
    small_ch, large_ch = [30], list(range(52))
    f_small = _job_bytes(bbc, lat, small_ch, bbc.F64)
    f_large = _job_bytes(bbc, lat, large_ch, bbc.F64)
    assert f_large >= 1.5 * f_small
    budget = props + f_large + f_small // 2
    dev = torch.device("cuda:0")

    def out_for(chans, n_t=2):
        return torch.zeros((n_t, len(chans), Lz, Ly, Lx, 16), dtype=torch.complex128, device=dev)

    ref = bbc.Context(0)
    want = ref.correlate(Sl, Ss, [0, 1], large_ch)
    torch.cuda.synchronize()
    ref.close()

    ctx = bbc.Context(0, hbm_budget_bytes=budget)
    ctx.server_start(2)
    h = ctx.prop_upload(Sl, Ss)
    print("case: two small jobs, then a large one", flush=True)
    j1 = ctx.submit(h, [0, 1], [0, 1], small_ch, out_for(small_ch))
    j2 = ctx.submit(h, [0, 1], [0, 1], small_ch, out_for(small_ch))
    ctx.wait(j1, 60000)
    ctx.wait(j2, 60000)
    big = out_for(large_ch)
    j3 = ctx.submit(h, [0, 1], [0, 1], large_ch, big)
    ctx.wait(j3, 60000)
    assert ctx.poll(j3) == "done"
    torch.cuda.synchronize()
    assert torch.equal(big, want)
    ctx.server_stop()
    ctx.close()

    # cannot fit beside its own propagator set: refused by submit
    tight = bbc.Context(0, hbm_budget_bytes=props + f_small + (f_large - f_small) // 2)
    tight.server_start(1)
    h = tight.prop_upload(Sl, Ss)
    with pytest.raises(bbc.BBCError) as e:
        tight.submit(h, [0, 1], [0, 1], large_ch, out_for(large_ch))
    assert e.value.status == bbc.ENOMEM
    tight.server_stop()
    tight.close()

    # cannot fit beside another resident set while no job runs: fails, then runs
    ctx = bbc.Context(0, hbm_budget_bytes=budget)
    ctx.server_start(2)
    h = ctx.prop_upload(Sl, Ss)
    S2l, S2s = _props((6, 6, 6), 4, 307, np.complex128)
    assert 2 * S2l.numel() * 16 > f_small // 2
    h2 = ctx.prop_upload(S2l, S2s)
    print("case: large job beside a second resident set", flush=True)
    j4 = ctx.submit(h, [0, 1], [0, 1], large_ch, out_for(large_ch))
    with pytest.raises(bbc.BBCError) as e:
        ctx.wait(j4, 60000)
    assert e.value.status == bbc.ENOMEM
    ctx.prop_release(h2)
    big = out_for(large_ch)
    j5 = ctx.submit(h, [0, 1], [0, 1], large_ch, big)
    ctx.wait(j5, 60000)
    torch.cuda.synchronize()
    assert torch.equal(big, want)
    ctx.server_stop()
    ctx.close()


def test_bypass_admits_small_job_behind_blocked_head(bbc):
    """With the head job waiting for memory held by a running job, a later small job
    that fits a free slot starts first (without the bypass it would queue behind the
    head job); every result equals the direct one bit for bit."""
    lat = (6, 6, 6)
    Lx, Ly, Lz = lat
    T = 8
    Sl, Ss = _props(lat, T, 308, np.complex128)
    props = 2 * Sl.numel() * 16
    small_ch, large_ch = [30], list(range(52))
    f_small = _job_bytes(bbc, lat, small_ch, bbc.F64)
    f_large = _job_bytes(bbc, lat, large_ch, bbc.F64)
    # room for one large job and a small one, not for two large ones
    budget = props + f_large + f_small + f_small // 2
    assert 2 * f_large > budget - props
    dev = torch.device("cuda:0")
    tl = list(range(T))
    ref = bbc.Context(0)
    want_l = ref.correlate(Sl, Ss, tl, large_ch)
    want_s = ref.correlate(Sl, Ss, tl, small_ch)
    torch.cuda.synchronize()
    ref.close()
    ctx = bbc.Context(0, hbm_budget_bytes=budget)
    ctx.server_start(3)
    h = ctx.prop_upload(Sl, Ss)

    def out_for(chans):
        return torch.zeros((T, len(chans), Lz, Ly, Lx, 16), dtype=torch.complex128, device=dev)

    # warm-up: both plans built and cached before the timed submissions
    for chans in (large_ch, small_ch):
        ctx.wait(ctx.submit(h, [0], [0], chans, out_for(chans)[:1].contiguous()), 60000)
    print("case: large, large, small on a budget for one large job", flush=True)
    outs = [out_for(c) for c in (large_ch, large_ch, small_ch)]
    ids = [ctx.submit(h, tl, tl, c, o) for c, o in zip((large_ch, large_ch, small_ch), outs)]
    for j in ids:
        ctx.wait(j, 120000)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], want_l) and torch.equal(outs[1], want_l) and torch.equal(outs[2], want_s)
    q = [ctx.job_times(j)[0] for j in ids]
    assert q[2] < q[1], q
    ctx.server_stop()
    ctx.close()


def test_buffer_checks(bbc):
    """Wrong output buffers are rejected before anything reaches the library."""
    Sl, Ss = _props((2, 2, 2), 1, 309, np.complex128)
    ctx = bbc.Context(0)
    dev = torch.device("cuda:0")
    good = torch.empty((1, 2, 2, 2, 2, 16), dtype=torch.complex128, device=dev)
    bad = [torch.empty((1, 2, 2, 2, 2, 8), dtype=torch.complex128, device=dev),       # shape
           torch.empty((1, 2, 2, 2, 2, 16), dtype=torch.complex64, device=dev),        # dtype
           torch.empty((1, 2, 2, 2, 16, 2), dtype=torch.complex128, device=dev).transpose(-1, -2)]  # strides
    for b in bad:
        with pytest.raises(bbc.BBCError):
            ctx.correlate(Sl, Ss, [0], [0, 1], out=b)
    ctx.correlate(Sl, Ss, [0], [0, 1], out=good)
    with pytest.raises(bbc.BBCError):
        ctx.prop_upload(Sl.real.contiguous(), Ss.real.contiguous())
    ctx.server_start(1)
    h = ctx.prop_upload(Sl, Ss)
    for b in bad:
        with pytest.raises(bbc.BBCError):
            ctx.submit(h, [0], [0], [0, 1], b)
    ctx.prop_release(h)
    ctx.server_stop()
    ctx.close()
