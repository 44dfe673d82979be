"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerance (FP64 form): normwise per (channel, time slice),
    max_{r,spin} |C_gpu - C_oracle| <= 1e-12 * max_{r,spin} |C_oracle|,
the reading taken here of the near-double-precision agreement the paper reports
(Sec. 6); relative errors near zeros are not meaningful.
"""
import os

import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle import unified, wick

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL64 = 1e-12
ALL = list(range(56))


def _name_to_tuple(name):
    a, b = name.split(">")
    return tuple(a.split() + b.split())


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


def gpu_correlate(ctx, Sl, Ss, t_list, channels, **kw):
    dev = torch.device("cuda:0")
    tl = torch.from_numpy(np.ascontiguousarray(Sl)).to(dev)
    ts = torch.from_numpy(np.ascontiguousarray(Ss)).to(dev)
    out = ctx.correlate(tl, ts, t_list, channels, **kw)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


def normwise(a, ref):
    return np.abs(a - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("lat", [(3, 3, 3), (4, 4, 4), (4, 2, 3)])
def test_all_channels_full_field_small(bbc, ctx, lat):
    """Every channel (52 + the 4 isospin-zero ones), every r, two time slices, ragged tiles."""
    Lx, Ly, Lz = lat
    Sl, Ss = synth.propagators(lat, 2, seed=101)
    print("case: lattice", lat, flush=True)
    out = gpu_correlate(ctx, Sl, Ss, [0, 1], ALL)
    r = wick.all_r(Lx, Ly, Lz)
    for t in range(2):
        scale = None
        for c in ALL:
            ch = _name_to_tuple(bbc.channel_name(c))
            ref = wick.correlate(Sl[t], Ss[t], ch, r)
            got = out[t, c].reshape(-1, 16)
            if c < 52:
                assert normwise(got, ref) < TOL64, (lat, t, c)
                scale = max(scale or 0, np.abs(ref).max())
            else:
                assert np.abs(got).max() < TOL64 * scale, (lat, t, c)
                assert np.abs(ref).max() < TOL64 * scale


OTHER_CHARGE_STATES = [("p", "p", "p", "p"), ("n", "n", "n", "n"), ("p", "n", "n", "p"), ("n", "p", "p", "n"),
                       ("n", "p", "n", "p"), ("S+", "p", "S+", "p"), ("S-", "n", "S-", "n"),
                       ("S+", "S+", "S+", "S+"), ("X0", "X0", "X0", "X0"), ("X-", "X0", "X0", "X-"),
                       ("L", "n", "S0", "n"), ("S-", "p", "L", "n")]


@pytest.mark.parametrize("lat", [(3, 3, 3), (4, 2, 3)])
def test_other_charge_states_full_field(bbc, ctx, lat):
    """Channels beyond the listed 52 (extended ids), every r, FP64, against the oracle."""
    Lx, Ly, Lz = lat
    Sl, Ss = synth.propagators(lat, 1, seed=111)
    chans = [bbc.channel_id(*q) for q in OTHER_CHARGE_STATES]
    assert min(chans) >= 56
    print("case: lattice", lat, "channels", chans, flush=True)
    out = gpu_correlate(ctx, Sl, Ss, [0], chans)
    r = wick.all_r(Lx, Ly, Lz)
    for m, q in enumerate(OTHER_CHARGE_STATES):
        ref = wick.correlate(Sl[0], Ss[0], q, r)
        assert normwise(out[0, m].reshape(-1, 16), ref) < TOL64, (lat, q)


def test_other_charge_states_isospin_on_gpu_8cubed(bbc, ctx):
    """At 8^3 the GPU results obey C[pp>pp] = C[nn>nn] = 1/2 sum of the four pn/np
    channels (I = 1), exactly up to rounding; no oracle involved."""
    L = 8
    Sl, Ss = synth.propagators(L, 1, seed=112)
    qs = [("p", "p", "p", "p"), ("n", "n", "n", "n"), ("p", "n", "p", "n"), ("p", "n", "n", "p"),
          ("n", "p", "p", "n"), ("n", "p", "n", "p")]
    out = gpu_correlate(ctx, Sl, Ss, [0], [bbc.channel_id(*q) for q in qs])[0]
    pp, nn = out[0], out[1]
    i1 = 0.5 * (out[2] + out[3] + out[4] + out[5])
    assert normwise(nn, pp) < TOL64
    assert normwise(i1, pp) < TOL64


@pytest.mark.parametrize("lat", [(32, 32, 2), (24, 24, 3), (96, 96, 2), (24, 24, 32), (32, 32, 24)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_plane_fft_extents(bbc, ctx, lat, prec):
    """Lattices whose x and y extents (24, 32; 96 in FP32) take the plane FFT pass,
    forward and inverse, with the z pass writing into the momentum groups: sampled r
    points of two channels against the oracle."""
    Lx, Ly, Lz = lat
    dtype = np.complex128 if prec == "f64" else np.complex64
    Sl, Ss = synth.propagators(lat, 1, seed=113, dtype=dtype)
    chans = [0, 5]
    print("case: lattice", lat, prec, flush=True)
    res = gpu_correlate(ctx, Sl, Ss, [0], chans)
    out = res[0] * res[1][:, :, None, None, None, None] if prec == "f32" else res
    rng = np.random.default_rng(114)
    r = np.concatenate([np.array([[0, 0, 0], [Lx - 1, Ly - 1, Lz - 1], [Lx // 2, 1, 0]]),
                        np.stack([rng.integers(0, Lx, 13), rng.integers(0, Ly, 13), rng.integers(0, Lz, 13)], 1)])
    r = r.astype(np.int32)
    Sl64, Ss64 = Sl.astype(np.complex128), Ss.astype(np.complex128)
    for m, c in enumerate(chans):
        ref = wick.correlate(Sl64[0], Ss64[0], ops.CHANNELS[c], r)
        got = np.stack([out[0, m, rz, ry, rx] for rx, ry, rz in r])
        assert normwise(got, ref) < (TOL64 if prec == "f64" else 1e-5), (lat, prec, c)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_z96_sampled_points(bbc, ctx, prec):
    """A 96-point z axis after a plane pass (24 x 24 x 96): in FP32 the z pass writes
    into the momentum groups, in FP64 it takes the two-factor LDS form and the copy;
    sampled r points of two channels against the oracle."""
    lat = (24, 24, 96)
    Lx, Ly, Lz = lat
    dtype = np.complex128 if prec == "f64" else np.complex64
    Sl, Ss = synth.propagators(lat, 1, seed=117, dtype=dtype)
    chans = [0, 5]
    print("case: lattice", lat, prec, flush=True)
    res = gpu_correlate(ctx, Sl, Ss, [0], chans)
    out = res[0] * res[1][:, :, None, None, None, None] if prec == "f32" else res
    r = np.array([[0, 0, 0], [3, 20, 95], [12, 12, 48], [7, 1, 33]], dtype=np.int32)
    Sl64, Ss64 = Sl.astype(np.complex128), Ss.astype(np.complex128)
    for m, c in enumerate(chans):
        ref = wick.correlate(Sl64[0], Ss64[0], ops.CHANNELS[c], r)
        got = np.stack([out[0, m, rz, ry, rx] for rx, ry, rz in r])
        assert normwise(got, ref) < (TOL64 if prec == "f64" else 1e-5), (prec, c)


@pytest.mark.parametrize("lat", [(48, 2, 2), (2, 48, 2), (2, 2, 48), (96, 1, 2), (1, 64, 1)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_long_line_fft_extents(bbc, ctx, lat, prec):
    """Extents 48, 64 and 96 on each axis (forward and inverse): the two-factor LDS
    FFT (6 x 8, 8 x 8, 12 x 8) in FP64 and one line per thread in registers in FP32;
    full field of two channels against the oracle."""
    Lx, Ly, Lz = lat
    dtype = np.complex128 if prec == "f64" else np.complex64
    Sl, Ss = synth.propagators(lat, 1, seed=115, dtype=dtype)
    chans = [0, 5]
    print("case: lattice", lat, prec, flush=True)
    res = gpu_correlate(ctx, Sl, Ss, [0], chans)
    out = res[0] * res[1][:, :, None, None, None, None] if prec == "f32" else res
    r = wick.all_r(Lx, Ly, Lz)
    Sl64, Ss64 = Sl.astype(np.complex128), Ss.astype(np.complex128)
    for m, c in enumerate(chans):
        ref = wick.correlate(Sl64[0], Ss64[0], ops.CHANNELS[c], r)
        assert normwise(out[0, m].reshape(-1, 16), ref) < (TOL64 if prec == "f64" else 1e-5), (lat, prec, c)


def test_p_lambda_8cubed_all_t(bbc, ctx):
    """The 8^3 x 8 p-Lambda workload: every r at two slices (O-U), sampled r at every slice (O-W)."""
    L, T = 8, 8
    Sl, Ss = synth.propagators(L, T, seed=102)
    out = gpu_correlate(ctx, Sl, Ss, list(range(T)), [1])
    ch = ops.CHANNELS[1]
    for t in (0, 5):
        ref = unified.correlate(Sl[t], Ss[t], ch).reshape(-1, 16)
        assert normwise(out[t, 0].reshape(-1, 16), ref) < TOL64, t
    rs = np.array([[0, 0, 0], [4, 4, 4], [1, 2, 3], [7, 0, 5], [3, 6, 1]])
    idx = rs[:, 0] + L * (rs[:, 1] + L * rs[:, 2])
    for t in range(T):
        ref = wick.correlate(Sl[t], Ss[t], ch, rs)
        assert normwise(out[t, 0].reshape(-1, 16)[idx], ref) < TOL64, t


def test_energy_normalisation_and_time_labels(bbc, ctx):
    """exp(E (t - t0)) of Sec. 2 Eq. (2): output scales per channel and per slice."""
    Sl, Ss = synth.propagators(2, 2, seed=103)
    a = gpu_correlate(ctx, Sl, Ss, [3, 4], [1, 5])
    b = gpu_correlate(ctx, Sl, Ss, [3, 4], [1, 5], t0=1, energy=[1.2, -0.3])
    for n, t in enumerate([3, 4]):
        assert normwise(b[n, 0], a[n, 0] * np.exp(1.2 * (t - 1))) < 1e-14
        assert normwise(b[n, 1], a[n, 1] * np.exp(-0.3 * (t - 1))) < 1e-14


def test_lower_components(bbc, ctx):
    """Spin selection LOWER (components 2, 3, Sec. 6) against the oracle."""
    Sl, Ss = synth.propagators(3, 1, seed=104)
    out = gpu_correlate(ctx, Sl, Ss, [0], [1, 10, 46], spin=1)
    r = wick.all_r(3, 3, 3)
    for m, c in enumerate([1, 10, 46]):
        ref = wick.correlate(Sl[0], Ss[0], ops.CHANNELS[c], r, lower=True)
        assert normwise(out[0, m].reshape(-1, 16), ref) < TOL64


def test_repeated_and_reordered_channels(bbc, ctx):
    """Channel lists are taken in the caller's order, repeats allowed."""
    Sl, Ss = synth.propagators(2, 1, seed=105)
    a = gpu_correlate(ctx, Sl, Ss, [0], [51, 3, 3, 0])
    b = gpu_correlate(ctx, Sl, Ss, [0], [0, 3, 51])
    assert np.array_equal(a[0, 0], b[0, 2])
    assert np.array_equal(a[0, 1], a[0, 2])
    assert np.array_equal(a[0, 3], b[0, 0])


def test_errors_are_reported(bbc, ctx):
    Sl, Ss = synth.propagators(2, 1, seed=106)
    dev = torch.device("cuda:0")
    tl, ts = torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)
    with pytest.raises(bbc.BBCError):
        ctx.correlate(tl, ts, [0], [57])            # p p > p n: quark content differs
    with pytest.raises(bbc.BBCError):
        ctx.correlate(tl.cpu(), ts, [0], [0])
    bad = torch.zeros((1, 5, 5, 5, 12, 12), dtype=torch.complex128, device=dev)
    with pytest.raises(bbc.BBCError):
        ctx.correlate(bad, bad, [0], [0])


# ---------------------------------------------------------------- full size (16^3)
@pytest.fixture(scope="module")
def big(bbc, ctx):
    """All 52 channels on a 16^3 lattice, slices t = 0 and 7 (SU(3)-broken inputs)."""
    L = 16
    Sl, Ss = synth.propagators(L, 8, seed=107, t_list=[0, 7])
    out = gpu_correlate(ctx, Sl, Ss, [0, 7], list(range(56)))
    return L, Sl, Ss, out


SAMPLED = [1, 5, 10, 16, 30, 41, 46, 51]


@pytest.mark.parametrize("c", SAMPLED)
def test_16cubed_sampled_points(big, c):
    """Sampled r (including 0 and L/2 points) of representative channels at full size."""
    L, Sl, Ss, out = big
    rs = np.array([[0, 0, 0], [8, 8, 8], [3, 11, 6]])
    idx = rs[:, 0] + L * (rs[:, 1] + L * rs[:, 2])
    t = 1
    print("case: 16^3 channel", c, flush=True)
    ref = wick.correlate(Sl[t], Ss[t], ops.CHANNELS[c], rs)
    assert normwise(out[t, c].reshape(-1, 16)[idx], ref) < TOL64


def test_16cubed_invariants(big, bbc):
    """Properties that hold at any size, over all channels: the isospin-zero channels
    vanish, identical sink baryons are antisymmetric, and the isospin relations hold."""
    L, Sl, Ss, out = big
    for t in range(2):
        scale = np.abs(out[t, :52]).max()
        assert np.abs(out[t, 52:]).max() < TOL64 * scale
        C = out[t].reshape(56, -1, 16)
        r = wick.all_r(L, L, L)
        m = (-r) % L
        mi = m[:, 0] + L * (m[:, 1] + L * m[:, 2])
        sink_swap = [((s >> 1) & 1) + 2 * (s & 1) + 4 * ((s >> 2) & 3) for s in range(16)]
        names = {bbc.channel_name(c): c for c in range(56)}
        for c in range(52):
            ch = _name_to_tuple(bbc.channel_name(c))
            if ch[0] == ch[1]:
                assert normwise(C[c], -C[c][mi][:, sink_swap]) < TOL64, c
        iso = [("p X- > p X-", "n X0 > n X0", 1), ("p X- > n X0", "n X0 > p X-", 1),
               ("L L > p X-", "L L > n X0", -1), ("p X- > L L", "n X0 > L L", -1),
               ("S0 S0 > p X-", "S0 S0 > n X0", -1), ("S0 L > p X-", "S0 L > n X0", 1)]
        for a, b, s in iso:
            assert normwise(C[names[a]], s * C[names[b]]) < TOL64, (a, b)


# ---------------------------------------------------------------- FP32 form
TOL32 = 1e-5


def _fp32_inputs(lat, t_list, seed):
    """Correlated slices (t-independent field + 1e-3 noise, exp(-m t) decay), rounded to FP32."""
    Sl = np.stack([synth.slice_correlated(lat, t, synth.LIGHT, seed=seed, dtype=np.complex64) for t in t_list])
    Ss = np.stack([synth.slice_correlated(lat, t, synth.STRANGE, seed=seed, dtype=np.complex64) for t in t_list])
    return Sl, Ss


def test_fp32_all_channels_small_with_deep_slice(bbc, ctx):
    """FP32 form against the FP64 oracle (on the same FP32-rounded inputs), every channel,
    including t = 63 where unscaled six-propagator products would underflow FP32."""
    lat = (3, 3, 3)
    t_list = [0, 63]
    Sl, Ss = _fp32_inputs(lat, t_list, seed=201)
    out, scale = gpu_correlate(ctx, Sl, Ss, t_list, ALL)
    assert out.dtype == np.complex64 and scale.dtype == np.float64
    r = wick.all_r(*lat)
    for n in range(2):
        ref_scale = None
        for c in ALL:
            ch = _name_to_tuple(bbc.channel_name(c))
            ref = wick.correlate(Sl[n].astype(np.complex128), Ss[n].astype(np.complex128), ch, r)
            got = out[n, c].reshape(-1, 16).astype(np.complex128) * scale[n, c]
            if c < 52:
                assert np.isfinite(got).all()
                assert normwise(got, ref) < TOL32, (t_list[n], c, normwise(got, ref))
                ref_scale = max(ref_scale or 0, np.abs(ref).max())
            else:
                assert np.abs(got).max() < TOL32 * ref_scale


def test_fp32_vs_fp64_16cubed_all_channels(bbc, ctx):
    """FP32 form against the FP64 form on a 16^3 lattice, every r, all 52 channels;
    the per-channel normwise error table is written to the directory named by
    BBC_REPORT_DIR, if set."""
    lat = (16, 16, 16)
    t_list = [5, 40]
    Sl, Ss = _fp32_inputs(lat, t_list, seed=202)
    chans = list(range(52))
    out32, scale = gpu_correlate(ctx, Sl, Ss, t_list, chans)
    out64 = gpu_correlate(ctx, Sl.astype(np.complex128), Ss.astype(np.complex128), t_list, chans)
    errs = np.zeros((len(t_list), 52))
    for n in range(len(t_list)):
        for c in chans:
            got = out32[n, c].astype(np.complex128) * scale[n, c]
            errs[n, c] = normwise(got, out64[n, c])
    out_dir = os.environ.get("BBC_REPORT_DIR")
    if out_dir and os.path.isdir(out_dir):
        with open(os.path.join(out_dir, "fp32_errors_16c.txt"), "w") as f:
            f.write("# channel  normwise error of the FP32 form vs the FP64 form, 16^3, t=%s\n" % t_list)
            for c in chans:
                f.write("%2d %-16s %s\n" % (c, bbc.channel_name(c), " ".join("%.3e" % e for e in errs[:, c])))
    assert errs.max() < TOL32, errs.max()


def test_fp32_vs_fp64_32cubed_all_channels(bbc, ctx):
    """The 32^3 x 64 configuration's inputs (t-independent field + 1e-3 noise per
    slice, exp(-m t) decay) at t = 0, 31, 63 (the deepest slice): FP32 form against
    the FP64 form over every r, all 52 channels; the per-channel error table is
    written to the directory named by BBC_REPORT_DIR, if set."""
    L = 32
    t_list = [0, 31, 63]
    Sl, Ss = synth.propagators(L, 64, seed=synth.BASE_SEED + 2, kind="correlated", t_list=t_list,
                               dtype=np.complex64)
    chans = list(range(52))
    errs = np.zeros((len(t_list), 52))
    for n, t in enumerate(t_list):                      # one slice at a time (device memory)
        out32, scale = gpu_correlate(ctx, Sl[n:n + 1], Ss[n:n + 1], [t], chans)
        out64 = gpu_correlate(ctx, Sl[n:n + 1].astype(np.complex128), Ss[n:n + 1].astype(np.complex128), [t], chans)
        for c in chans:
            errs[n, c] = normwise(out32[0, c].astype(np.complex128) * scale[0, c], out64[0, c])
        del out32, out64
    out_dir = os.environ.get("BBC_REPORT_DIR")
    if out_dir and os.path.isdir(out_dir):
        with open(os.path.join(out_dir, "fp32_errors_32c64.txt"), "w") as f:
            f.write("# channel  normwise error of the FP32 form vs the FP64 form, 32^3, t=%s\n" % t_list)
            for c in chans:
                f.write("%2d %-16s %s\n" % (c, bbc.channel_name(c), " ".join("%.3e" % e for e in errs[:, c])))
    assert errs.max() < TOL32, errs.max()


def test_16cubed_su3_limit_relations(bbc, ctx):
    """SU(3)-limit run (S_s := S_l) at 16^3: u <-> s maps Sigma+ n onto Sigma- Xi0 and
    p Xi- onto itself, with r -> -r and both baryon pairs swapped."""
    L = 16
    Sl, Ss = synth.propagators(L, 8, seed=108, t_list=[3], su3=True)
    names = {bbc.channel_name(c): c for c in range(52)}
    chans = [names["S+ n > S+ n"], names["S- X0 > S- X0"], names["p X- > p X-"]]
    out = gpu_correlate(ctx, Sl, Ss, [3], chans)[0].reshape(3, -1, 16)
    r = wick.all_r(L, L, L)
    m = (-r) % L
    mi = m[:, 0] + L * (m[:, 1] + L * m[:, 2])
    swap = [((s >> 1) & 1) + 2 * (s & 1) + 4 * ((s >> 3) & 1) + 8 * ((s >> 2) & 1) for s in range(16)]
    assert normwise(out[0], out[1][mi][:, swap]) < TOL64
    assert normwise(out[2], out[2][mi][:, swap]) < TOL64


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_host_streamed_path_equals_device_path(bbc, ctx, dtype):
    """Propagators and output in (pinned) host memory: slices are staged through the device
    with overlapped copies; the result is bit-identical to the all-device path."""
    lat = (4, 4, 4)
    Sl, Ss = synth.propagators(lat, 5, seed=109, dtype=dtype)
    chans = [0, 10, 30, 51]
    dev = torch.device("cuda:0")
    ref = ctx.correlate(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), list(range(5)), chans)
    hl = torch.from_numpy(Sl).pin_memory()
    hs = torch.from_numpy(Ss).pin_memory()
    got = ctx.correlate(hl, hs, list(range(5)), chans)
    torch.cuda.synchronize()
    if isinstance(ref, tuple):
        assert not got[0].is_cuda
        assert torch.equal(got[0], ref[0].cpu()) and torch.equal(got[1].cpu(), ref[1].cpu())
    else:
        assert not got.is_cuda
        assert torch.equal(got, ref.cpu())
    # pageable host memory (no pinning) works too
    got2 = ctx.correlate(torch.from_numpy(Sl), torch.from_numpy(Ss), list(range(5)), chans,
                         out=torch.empty_like(got[0] if isinstance(got, tuple) else got))
    torch.cuda.synchronize()
    a = got2[0] if isinstance(got2, tuple) else got2
    b = got[0] if isinstance(got, tuple) else got
    assert torch.equal(a, b)


def test_96cubed_fp32_relations_full_field(bbc, ctx):
    """The largest lattice (96^3, FP32 form, one slice, device-resident): exact
    relations over every r, which fail if any momentum is missing from a launch:
    the isospin-zero channel vanishes, C[LL>pX-] = -C[LL>nX0], and identical sink
    baryons give C(r)_{ab..} = -C(-r)_{ba..} for LL>LL."""
    L = 96
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(131)
    shape = (1, L, L, L, 12, 12)
    Sl = torch.randn(shape, dtype=torch.complex64, device=dev, generator=g)
    Ss = torch.randn(shape, dtype=torch.complex64, device=dev, generator=g) * 0.5
    chans = [10, 11, 12, 52]
    out, scale = ctx.correlate(Sl, Ss, [0], chans)
    torch.cuda.synchronize()
    C = out[0].to(torch.complex128) * scale[0].view(-1, 1, 1, 1, 1)
    del out, Sl, Ss
    ref = C[0].abs().max().item()
    assert ref > 0
    assert C[3].abs().max().item() <= 1e-5 * ref                               # zero channel
    assert (C[1] + C[2]).abs().max().item() <= 1e-5 * C[1].abs().max().item()  # isospin pair
    # C(r)_{a b a' b'} = -C(-r)_{b a a' b'}: -r = (L - r) mod L per axis, swap a <-> b
    LL = C[0]
    neg = torch.roll(torch.flip(LL, dims=(0, 1, 2)), shifts=(1, 1, 1), dims=(0, 1, 2))
    idx = torch.tensor([((s >> 1) & 1) + 2 * (s & 1) + 4 * (s >> 2) for s in range(16)], device=dev)
    swapped = neg[..., idx]
    assert (LL + swapped).abs().max().item() <= 1e-5 * ref

