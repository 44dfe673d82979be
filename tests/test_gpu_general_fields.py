"""General interpolating fields on the GPU (Sec. 2, Eq. (FieldOperator_B)): decuplet
fields {C gamma_l, 1} and the nucleon {C, gamma_5}, alone and mixed with octet
fields, against the oracle element by element; exact flavour relations at a
larger size."""
import numpy as np
import pytest

import synth
from oracle import wick

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

QUADS = [
    ("O-(3)", "O-(3)", "O-(3)", "O-(3)"),
    ("O-(1)", "O-(2)", "O-(1)", "O-(2)"),
    ("O-(2)", "O-(2)", "O-(3)", "O-(3)"),
    ("D++(1)", "D++(2)", "D++(2)", "D++(1)"),
    ("D++(1)", "O-(2)", "D++(1)", "O-(2)"),
    ("D-(3)", "D-(3)", "D-(1)", "D-(1)"),
    ("p2", "n", "p", "n2"),
    ("p2", "n2", "p2", "n2"),
    ("D++(3)", "p2", "D++(3)", "p2"),
    ("O-(1)", "X0", "O-(2)", "X0"),
    ("n2", "D-(1)", "n", "D-(1)"),
    ("D+(1)", "D+(2)", "D+(1)", "D+(2)"),
    ("S*0(3)", "p", "S*0(3)", "p"),
    ("D0(1)", "X*0(2)", "D0(1)", "X*0(2)"),
    ("X*-(2)", "L", "X*-(2)", "L"),
    ("D++(1)", "D+(1)", "D+(1)", "D++(1)"),
]


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


def run(ctx, Sl, Ss, chans, spin=0):
    dev = torch.device("cuda:0")
    out = ctx.correlate(torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev), list(range(Sl.shape[0])),
                        chans, spin=spin)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return out[0].cpu().numpy().astype(np.complex128) * out[1].cpu().numpy()[:, :, None, None, None, None]
    return out.cpu().numpy()


@pytest.mark.parametrize("dtype,tol", [(np.complex128, 1e-12), (np.complex64, 1e-5)])
@pytest.mark.parametrize("lat,spin", [((3, 3, 3), 0), ((4, 2, 3), 0), ((3, 2, 2), 1)])
def test_general_fields_match_oracle(bbc, ctx, dtype, tol, lat, spin):
    Sl, Ss = synth.propagators(lat, 1, seed=141, dtype=dtype)
    # octet channels in the same request: one plan holding every spin structure
    chans = [bbc.channel_id(*q) for q in QUADS] + [0, 10, 51]
    got = run(ctx, Sl, Ss, chans, spin=spin)
    S64l, S64s = Sl.astype(np.complex128), Ss.astype(np.complex128)
    r = wick.all_r(*lat)
    for m, c in enumerate(chans):
        a, b = bbc.channel_name(c).split(">")
        ref = wick.correlate(S64l[0], S64s[0], tuple(a.split() + b.split()), r, lower=spin == 1)
        err = np.abs(got[0, m].reshape(-1, 16) - ref).max() / np.abs(ref).max()
        assert err <= tol, (bbc.channel_name(c), err)


@pytest.mark.parametrize("dtype,tol", [(np.complex128, 1e-12), (np.complex64, 1e-5)])
def test_decuplet_flavour_relations_8cubed(bbc, ctx, dtype, tol):
    """S_u = S_d: Delta++ and Delta- agree; S_s = S_l: Omega- equals Delta++ (same kernels,
    different flavour tables)."""
    lat = (8, 8, 8)
    Sl, Ss = synth.propagators(lat, 1, seed=143, dtype=dtype)
    qs = [("D++(1)", "D++(2)", "D++(1)", "D++(2)"), ("D-(1)", "D-(2)", "D-(1)", "D-(2)"),
          ("O-(1)", "O-(2)", "O-(1)", "O-(2)")]
    chans = [bbc.channel_id(*q) for q in qs]
    a = run(ctx, Sl, Ss, chans)
    b = run(ctx, Sl, Sl.copy(), chans)                 # flavour SU(3) limit
    scale = np.abs(a[0, 0]).max()
    assert scale > 0
    assert np.abs(a[0, 1] - a[0, 0]).max() <= tol * scale
    assert np.abs(b[0, 2] - b[0, 0]).max() <= tol * np.abs(b[0, 0]).max()
    assert np.abs(a[0, 2] - a[0, 0]).max() > 1e-3 * scale


def test_rotation_covariance_on_gpu(bbc, ctx):
    """The GPU's correlators of 90-degree-rotated propagators are the rotated GPU
    correlators (maps from the Clifford algebra, see test_rotation_pins), at 6^3 x 4."""
    import itertools
    import test_rotation_pins as rp
    lam = rp.spinor_rotation()
    fams, members = ("O", "p", "O", "p"), (0, 0, 1, 0)
    maps = [rp.family_maps(rp.FAMILIES[f], lam) for f in fams]
    lat = (6, 6, 4)
    Sl, Ss = synth.propagators(lat, 1, seed=157)
    Slr, Ssr = rp.rotate_props(Sl[0], lam)[None], rp.rotate_props(Ss[0], lam)[None]
    keys = list(itertools.product(*[range(len(rp.FAMILIES[f])) for f in fams]))
    names = {k: tuple(rp.FAMILIES[f][m] for f, m in zip(fams, k)) for k in keys}
    chans = [bbc.channel_id(*names[k]) for k in keys]
    base = run(ctx, Sl, Ss, chans)[0]
    target = bbc.channel_id(*names[members])
    got = run(ctx, Slr, Ssr, [target])[0, 0].reshape(-1, 16)
    Lx, Ly, Lz = lat
    r = wick.all_r(*lat)
    rinv = [((ry % Lx) + Lx * (((-rx) % Ly) + Ly * rz)) for rx, ry, rz in r]
    rows = [maps[i][0] if i < 2 else maps[i][1] for i in range(4)]
    want = np.zeros_like(got)
    for a, b, ap, bp in itertools.product(range(2), repeat=4):
        s_out = a + 2 * (b + 2 * (ap + 2 * bp))
        k = [members[0] * 4 + a, members[1] * 4 + b, members[2] * 4 + ap, members[3] * 4 + bp]
        for j, key in enumerate(keys):
            field = base[j].reshape(-1, 16)
            for d1, d2, d3, d4 in itertools.product(range(2), repeat=4):
                c = (rows[0][k[0], key[0] * 4 + d1] * rows[1][k[1], key[1] * 4 + d2] *
                     rows[2][k[2], key[2] * 4 + d3] * rows[3][k[3], key[3] * 4 + d4])
                if abs(c) > 1e-14:
                    want[:, s_out] += c * field[rinv, d1 + 2 * (d2 + 2 * (d3 + 2 * d4))]
    assert np.abs(got).max() > 0
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_general_fields_served_and_graphed(bbc, dtype):
    """General-field channels (decuplet, {C, gamma_5} nucleon, mixed with octet fields)
    through the serving loop and through graph mode give bit-identical results to the
    direct calls."""
    fp32 = dtype == np.complex64
    tdt = torch.complex64 if fp32 else torch.complex128
    dev = torch.device("cuda:0")
    lat, T = (4, 4, 2), 3
    Sl, Ss = synth.propagators(lat, T, seed=161, dtype=dtype)
    dl, ds = torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)
    jobs = [([0, 2], [bbc.channel_id(*QUADS[0]), bbc.channel_id(*QUADS[4])]),
            ([1], [bbc.channel_id(*QUADS[6]), 10, bbc.channel_id(*QUADS[8])]),
            ([2, 1, 0], [bbc.channel_id(*QUADS[9])])]
    direct = bbc.Context(0)
    alone = []
    for sl, ch in jobs:
        r = direct.correlate(dl[sl], ds[sl], sl, ch)
        torch.cuda.synchronize()
        alone.append(tuple(x.cpu() for x in r) if fp32 else (r.cpu(), None))
    direct.close()
    Lx, Ly, Lz = lat
    # serving loop, all jobs in flight together
    srv = bbc.Context(0)
    srv.server_start(2)
    h = srv.prop_upload(dl, ds)
    outs, ids = [], []
    for sl, ch in jobs:
        out = torch.zeros((len(sl), len(ch), Lz, Ly, Lx, 16), dtype=tdt, device=dev)
        scale = torch.zeros((len(sl), len(ch)), dtype=torch.float64, device=dev) if fp32 else None
        ids.append(srv.submit(h, sl, sl, ch, out, scale))
        outs.append((out, scale))
    for j in ids:
        srv.wait(j, 60000)
    torch.cuda.synchronize()
    for (out, scale), (ref, ref_s) in zip(outs, alone):
        assert torch.equal(out.cpu(), ref)
        if fp32:
            assert torch.equal(scale.cpu(), ref_s)
    srv.prop_release(h)
    srv.server_stop()
    srv.close()
    # graph mode: captured once, replayed twice
    gctx = bbc.Context(0)
    gctx.graph_mode(True)
    for sl, ch in jobs:
        out = torch.empty((len(sl), len(ch), Lz, Ly, Lx, 16), dtype=tdt, device=dev)
        scale = torch.empty((len(sl), len(ch)), dtype=torch.float64, device=dev) if fp32 else None
        ref, ref_s = alone[jobs.index((sl, ch))]
        jl, js = dl[sl].contiguous(), ds[sl].contiguous()      # fixed inputs: the second call replays
        for _ in range(2):
            out.zero_()
            gctx.correlate(jl, js, sl, ch, out=out, scale=scale)
            torch.cuda.synchronize()
            assert torch.equal(out.cpu(), ref)
            if fp32:
                assert torch.equal(scale.cpu(), ref_s)
    gctx.graph_mode(False)
    gctx.close()
