"""Kernel variants and the autotuner (bbc_tuning_*, bbc_autotune) through the C ABI.

Every variant of the block kernel (Sec. 3 blocks), of the forward FFT's plane
pass and of the open-index contraction on the matrix cores (Sec. 3 Eq.
(LN.pLLp.FFT)) forms the same values in the same order, so the results must be
the same bits for every choice; the autotuner must return a valid choice, keep
it for the request shape, and write and read it back through the tuning file.
Lattices: 8^3 (fused one-pass FFT) and 24 x 24 x 4 (plane pass, then the z
pass that writes whole x-row runs of momentum groups), both precisions, the
52 channels, five time slices (so that 2, 4 or 8 slices run at once on the
library's streams, round robin, give the bits of one at a time).  The 24 x 24 x 4 results are also checked against the oracle at
sampled points, since its momentum groups come in x-row runs.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import operators as ops
from oracle import wick

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CHANNELS = list(range(52))
N_PAIRS = {"f64": 9, "f32": 6}


@pytest.fixture(scope="module")
def bbc():
    import paper_1510_00903_amd as mod
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mod.load()
    return mod


def _inputs(lat, prec, seed, n_t=1):
    dt = np.complex64 if prec == "f32" else np.complex128
    Sl = np.stack([synth.slice_correlated(lat, t, synth.LIGHT, seed=seed, dtype=dt) for t in range(n_t)])
    Ss = np.stack([synth.slice_correlated(lat, t, synth.STRANGE, seed=seed, dtype=dt) for t in range(n_t)])
    dev = torch.device("cuda:0")
    return torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)


def _run(ctx, dl, ds):
    out = ctx.correlate(dl, ds, list(range(dl.shape[0])), CHANNELS)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return out[0].clone(), out[1].clone()
    return out.clone(), None


def _variants(prec, lat):
    """Each dimension on its own from the plain choice."""
    planes = 2 if lat[0] in (24, 32) and lat[0] == lat[1] else 1
    base = {"pairs": 0, "blocks": 0, "planes": 0, "slices": 0, "combine": 0}
    out = [dict(base, pairs=p) for p in range(N_PAIRS[prec])]
    out += [dict(base, blocks=b) for b in range(1, 3)]
    out += [dict(base, planes=pl) for pl in range(1, planes)]
    out += [dict(base, slices=s) for s in range(1, 4)]
    out += [dict(base, combine=c) for c in (1, 2)]
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("lat", [(8, 8, 8), (24, 24, 4)])
def test_every_variant_gives_the_same_bits(bbc, prec, lat):
    print("case: variants", prec, lat, flush=True)
    ctx = bbc.Context(0)
    P = bbc.F64 if prec == "f64" else bbc.F32
    # five slices: with 2, 4 or 8 run at once the streams take them round robin
    dl, ds = _inputs(lat, prec, seed=1510009050, n_t=5)
    ctx.set_tuning(lat, CHANNELS, {"pairs": 0, "blocks": 0, "planes": 0, "slices": 0}, precision=P)
    ref, ref_s = _run(ctx, dl, ds)
    for v in _variants(prec, lat):
        ctx.set_tuning(lat, CHANNELS, v, precision=P)
        got, got_s = _run(ctx, dl, ds)
        assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), v
        if ref_s is not None:
            assert torch.equal(got_s, ref_s), v
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_run_ordered_groups_against_oracle(bbc, prec):
    """24 x 24 x 4: sampled r of four channels against the direct-Wick oracle (FP64 values
    of the FP32-rounded inputs), normwise 1e-12 (FP64) / 1e-5 (FP32)."""
    lat = (24, 24, 4)
    print("case: run-ordered oracle", prec, lat, flush=True)
    Sl = synth.slice_correlated(lat, 0, synth.LIGHT, seed=1510009051, dtype=np.complex64)
    Ss = synth.slice_correlated(lat, 0, synth.STRANGE, seed=1510009051, dtype=np.complex64)
    dt = np.complex64 if prec == "f32" else np.complex128
    dev = torch.device("cuda:0")
    ctx = bbc.Context(0)
    chans = [0, 1, 10, 51]
    out = ctx.correlate(torch.from_numpy(Sl.astype(dt)[None]).to(dev), torch.from_numpy(Ss.astype(dt)[None]).to(dev),
                        [0], chans)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        C = out[0].cpu().numpy().astype(np.complex128) * out[1].cpu().numpy()[:, :, None, None, None, None]
    else:
        C = out.cpu().numpy()
    ctx.close()
    rng = np.random.default_rng(7)
    pts = [(0, 0, 0), (12, 12, 2), (1, 23, 3), (5, 7, 1)] + [tuple(int(v) for v in rng.integers(0, lat, 3))
                                                               for _ in range(2)]
    Sl64, Ss64 = Sl.astype(np.complex128), Ss.astype(np.complex128)
    tol = 1e-12 if prec == "f64" else 1e-5
    r = np.array(pts, dtype=np.int32)
    for j, c in enumerate(chans):
        ref = wick.correlate(Sl64, Ss64, ops.CHANNELS[c], r)
        got = np.stack([C[0, j, rz, ry, rx] for rx, ry, rz in pts])
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (c, np.abs(got - ref).max())


def test_autotune_stores_and_round_trips(bbc, tmp_path):
    lat = (8, 8, 8)
    print("case: autotune", lat, flush=True)
    path = str(tmp_path / "tuning.json")
    os.environ["BBC_TUNING_CACHE"] = path
    try:
        ctx = bbc.Context(0)
        dl, ds = _inputs(lat, "f64", seed=1510009052)
        t0, tuned0 = ctx.tuning(lat, CHANNELS)
        assert not tuned0
        best, ms = ctx.autotune(dl[0].contiguous(), ds[0].contiguous(), CHANNELS, reps=2)
        assert 0 <= best["pairs"] < 9 and 0 <= best["blocks"] < 3 and best["planes"] == 0
        assert 0 <= best["slices"] < 4 and 0 <= best["combine"] < 3
        assert ms > 0
        t1, tuned1 = ctx.tuning(lat, CHANNELS)
        assert tuned1 and t1 == best
        # the autotuner rewrote the cache file; a new context loads it
        rec = json.load(open(path))
        assert rec["bbc_tuning"] == 1 and len(rec["entries"]) == 1
        e = rec["entries"][0]
        assert e["lattice"] == [8, 8, 8] and e["precision"] == 0 and e["pairs"] == best["pairs"]
        ctx.close()
        ctx2 = bbc.Context(0)
        t2, tuned2 = ctx2.tuning(lat, CHANNELS)
        assert tuned2 and t2 == best
        # another channel list is another shape
        _, tuned3 = ctx2.tuning(lat, CHANNELS[:4])
        assert not tuned3
        # explicit save / load, and reset to the built-in choice
        p2 = str(tmp_path / "copy.json")
        ctx2.save_tuning(p2)
        ctx2.set_tuning(lat, CHANNELS, None)
        assert not ctx2.tuning(lat, CHANNELS)[1]
        ctx2.load_tuning(p2)
        assert ctx2.tuning(lat, CHANNELS) == (best, True)
        ctx2.close()
    finally:
        del os.environ["BBC_TUNING_CACHE"]


def test_tuning_errors(bbc, tmp_path):
    ctx = bbc.Context(0)
    with pytest.raises(bbc.BBCError):
        ctx.set_tuning((8, 8, 8), CHANNELS, {"pairs": 9, "blocks": 0, "planes": 0})
    with pytest.raises(bbc.BBCError):
        ctx.set_tuning((8, 8, 8), CHANNELS, {"pairs": 6, "blocks": 0, "planes": 0}, precision=bbc.F32)
    with pytest.raises(bbc.BBCError):
        ctx.set_tuning((8, 8, 8), CHANNELS, {"pairs": 0, "blocks": 0, "planes": 0, "slices": 4})
    bad = tmp_path / "bad.json"
    bad.write_text('{"something": 2}')
    with pytest.raises(bbc.BBCError):
        ctx.load_tuning(str(bad))
    with pytest.raises(bbc.BBCError):
        ctx.load_tuning(str(tmp_path / "missing.json"))
    ctx.close()


def test_builtin_choices(bbc):
    """The built-in choice per shape (no tuning entry): row tiles for the contraction,
    4 x 4 block workgroups up to 512 sites, slices at once by lattice size (8 up to
    2,048 sites, 2 up to 4,096, else 1), and in FP32 the LDS-staged channel sums."""
    ctx = bbc.Context(0)
    cases = [((8, 8, 8), bbc.F64, {"pairs": 8, "blocks": 1, "planes": 0, "slices": 3, "combine": 0}),
             ((12, 12, 12), bbc.F64, {"pairs": 8, "blocks": 0, "planes": 0, "slices": 3, "combine": 0}),
             ((16, 16, 16), bbc.F64, {"pairs": 8, "blocks": 0, "planes": 0, "slices": 1, "combine": 0}),
             ((32, 32, 32), bbc.F64, {"pairs": 8, "blocks": 0, "planes": 0, "slices": 0, "combine": 0}),
             ((8, 8, 8), bbc.F32, {"pairs": 5, "blocks": 1, "planes": 1, "slices": 3, "combine": 2}),
             ((16, 16, 16), bbc.F32, {"pairs": 5, "blocks": 2, "planes": 1, "slices": 1, "combine": 2}),
             ((32, 32, 32), bbc.F32, {"pairs": 5, "blocks": 2, "planes": 1, "slices": 0, "combine": 2})]
    for lat, prec, want in cases:
        got, tuned = ctx.tuning(lat, CHANNELS, precision=prec)
        assert not tuned and got == want, (lat, prec, got)
    ctx.close()
