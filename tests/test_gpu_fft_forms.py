"""Every forward and inverse FFT form the library can choose, against the FP64 oracle.

The 3-D transforms of Sec. 3 Eq. (LN.pLLp.FFT) take different kernels by
lattice shape and precision: the fused one-pass form for cubic lattices with
L in {4, 6, 8, 12, 16} (both precisions), the plane pass with the z pass
written into the momentum groups (24- and 32-point planes, z in
{2, 3, 4, 6, 8, 12, 16, 24, 32}; 96-point planes in FP32), the one-pass form of
cubic 32^3 lattices in FP32, and per-axis line
transforms otherwise (inverse transforms always).  This file reaches the forms
the other parity tests do not: the fused form in FP32 for every L and in FP64
for L = 6 and 12, 6- and 12-point lines, and the z pass for z in
{4, 6, 8, 12, 16}.  Tolerances as everywhere: normwise per channel,
1e-12 (FP64) and 1e-5 (FP32), both forms checked against the oracle on the
same inputs (FP32-rounded values, taken exactly in FP64).
"""
import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle import unified, wick

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


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


def _inputs(lat, t_list, seed):
    """Correlated slices (t-independent field + 1e-3 noise, exp(-m t) decay) rounded to
    FP32; returned as complex64 and as the same values in complex128."""
    Sl = np.stack([synth.slice_correlated(lat, t, synth.LIGHT, seed=seed, dtype=np.complex64) for t in t_list])
    Ss = np.stack([synth.slice_correlated(lat, t, synth.STRANGE, seed=seed, dtype=np.complex64) for t in t_list])
    return (Sl, Ss), (Sl.astype(np.complex128), Ss.astype(np.complex128))


def _run(ctx, Sl, Ss, t_list, chans):
    """Correlator through the C ABI; FP32 results multiplied by their FP64 scale."""
    dev = torch.device("cuda:0")
    out = ctx.correlate(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), t_list, chans)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return out[0].cpu().numpy().astype(np.complex128) * out[1].cpu().numpy()[:, :, None, None, None, None]
    return out.cpu().numpy()


def _both(ctx, lat, t_list, chans, seed):
    (s32l, s32s), (s64l, s64s) = _inputs(lat, t_list, seed)
    print("case: lattice", lat, "t", t_list, "channels", chans, flush=True)
    return {"f32": _run(ctx, s32l, s32s, t_list, chans), "f64": _run(ctx, s64l, s64s, t_list, chans)}, s64l, s64s


def normwise(a, ref):
    return np.abs(a - ref).max() / np.abs(ref).max()


def _tuple(bbc, c):
    a, b = bbc.channel_name(c).split(">")
    return tuple(a.split() + b.split())


def _special_and_random(lat, n_random, seed):
    """The points of {0, L/2}^3 (where the identical-baryon relations force zeros) and
    a few seeded random points."""
    Lx, Ly, Lz = lat
    pts = {(x, y, z) for x in {0, Lx // 2} for y in {0, Ly // 2} for z in {0, Lz // 2}}
    rng = np.random.default_rng(seed)
    for _ in range(n_random):
        pts.add((int(rng.integers(Lx)), int(rng.integers(Ly)), int(rng.integers(Lz))))
    return np.array(sorted(pts), dtype=np.int32)


def _at(field, r):
    return np.stack([field[rz, ry, rx] for rx, ry, rz in r])


def test_fused_fp32_4cubed_full_field(bbc, ctx):
    """Fused one-pass FFT in FP32 at 4^3 (and 4-point inverse lines): seven octet channels,
    an isospin-zero one and two decuplet channels, every r, at t = 0 and t = 63."""
    lat = (4, 4, 4)
    t_list = [0, 63]
    gen = [bbc.channel_id("O-(3)", "O-(3)", "O-(3)", "O-(3)"), bbc.channel_id("D++(1)", "D++(2)", "D++(2)", "D++(1)")]
    chans = [0, 1, 5, 16, 30, 46, 51, 52] + gen
    (s32l, s32s), (s64l, s64s) = _inputs(lat, t_list, seed=301)
    print("case: lattice", lat, "fp32 fused", flush=True)
    got = _run(ctx, s32l, s32s, t_list, chans)
    r = wick.all_r(*lat)
    for n in range(len(t_list)):
        big = 0.0
        for m, c in enumerate(chans):
            ref = wick.correlate(s64l[n], s64s[n], _tuple(bbc, c), r)
            g = got[n, m].reshape(-1, 16)
            if c == 52:
                continue
            big = max(big, np.abs(ref).max())
            assert normwise(g, ref) < TOL["f32"], (t_list[n], c, normwise(g, ref))
        z = chans.index(52)
        assert np.abs(got[n, z]).max() < TOL["f32"] * big


def test_fused_6cubed_full_field_both_forms(bbc, ctx):
    """Fused FFT at 6^3 (radix 2 x 3) and 6-point inverse lines, FP32 and FP64, every r of
    four channels at the deep slice t = 63, against the unified oracle."""
    lat = (6, 6, 6)
    chans = [1, 5, 30, 51]
    res, s64l, s64s = _both(ctx, lat, [63], chans, seed=302)
    for m, c in enumerate(chans):
        ref = unified.correlate(s64l[0], s64s[0], ops.CHANNELS[c]).reshape(-1, 16)
        for prec in ("f64", "f32"):
            e = normwise(res[prec][0, m].reshape(-1, 16), ref)
            assert e < TOL[prec], (prec, c, e)


@pytest.mark.parametrize("L,precs,chans", [(8, ("f32",), [1, 5, 16, 51]), (12, ("f64", "f32"), [5, 16, 51]),
                                           (16, ("f32",), [5, 30])])
def test_fused_cubic_sampled_points(bbc, ctx, L, precs, chans):
    """Fused FFT at 8^3, 12^3 (radix 4 x 3) and 16^3 in the forms no other oracle test
    covers: r at the eight points of {0, L/2}^3 and one more."""
    lat = (L, L, L)
    res, s64l, s64s = _both(ctx, lat, [7], chans, seed=303 + L)
    r = _special_and_random(lat, 1, seed=L)
    for m, c in enumerate(chans):
        ref = wick.correlate(s64l[0], s64s[0], ops.CHANNELS[c], r)
        for prec in precs:
            e = normwise(_at(res[prec][0, m], r), ref)
            assert e < TOL[prec], (L, prec, c, e)


@pytest.mark.parametrize("lat", [(12, 2, 2), (2, 12, 3), (6, 1, 4)])
def test_ragged_6_and_12_point_lines_full_field(bbc, ctx, lat):
    """6- and 12-point line transforms on non-cubic lattices (per-axis passes and the
    grouped copy), both forms, every r of seven channels."""
    chans = [0, 1, 5, 16, 30, 46, 51]
    res, s64l, s64s = _both(ctx, lat, [2], chans, seed=310)
    r = wick.all_r(*lat)
    for m, c in enumerate(chans):
        ref = wick.correlate(s64l[0], s64s[0], ops.CHANNELS[c], r)
        for prec in ("f64", "f32"):
            e = normwise(res[prec][0, m].reshape(-1, 16), ref)
            assert e < TOL[prec], (lat, prec, c, e)


@pytest.mark.parametrize("lat", [(24, 24, 4), (32, 32, 6), (24, 24, 8), (32, 32, 12), (24, 24, 16)])
def test_plane_pass_z_grouped_lengths(bbc, ctx, lat):
    """Plane pass followed by the z pass into the momentum groups for z lengths 4, 6, 8,
    12 and 16 (and the matching inverse lines), both forms, sampled r of two channels."""
    chans = [5, 30]
    res, s64l, s64s = _both(ctx, lat, [3], chans, seed=320)
    Lx, Ly, Lz = lat
    r = np.array([[0, 0, 0], [Lx // 2, Ly // 2, Lz // 2], [5, 17, Lz - 1], [Lx - 1, 3, 1]], dtype=np.int32)
    for m, c in enumerate(chans):
        ref = wick.correlate(s64l[0], s64s[0], ops.CHANNELS[c], r)
        for prec in ("f64", "f32"):
            e = normwise(_at(res[prec][0, m], r), ref)
            assert e < TOL[prec], (lat, prec, c, e)


@pytest.mark.parametrize("L,chans", [(24, [0, 5, 30, 51]), (32, [1, 30])])
def test_onepass_cubic_fp32_sampled_points(bbc, ctx, L, chans):
    """Cubic 24^3 and 32^3 lattices in both forms against the oracle at r in {0, L/2}^3
    and two more points: at 32^3 the FP32 form takes the one-pass forward FFT (z lines
    in registers, x and y planes in LDS in two mirror-closed batches, written into the
    run-ordered groups), the others the plane pass and then the z pass."""
    lat = (L, L, L)
    res, s64l, s64s = _both(ctx, lat, [5], chans, seed=330 + L)
    r = _special_and_random(lat, 2, seed=L + 1)
    for m, c in enumerate(chans):
        ref = wick.correlate(s64l[0], s64s[0], ops.CHANNELS[c], r)
        for prec in ("f64", "f32"):
            e = normwise(_at(res[prec][0, m], r), ref)
            assert e < TOL[prec], (L, prec, c, e)
