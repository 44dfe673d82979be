#!/usr/bin/env python3
"""Benchmark of the effective-block correlator on one MI355X.

One step = the whole hot path over one job: all 52 channels, all 32 time slices
of a 16^3 x 32 lattice in the FP64 form (block construction, forward FFT,
transpose, open-index contraction, inverse FFT, normalisation) -- the workload
of the paper's timing table (Sec. 5, Table 5: 16^3 x 32, 52 channels), with
seeded synthetic propagators in place of the CP-PACS/JLQCD configuration.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line: throughput in site-channels/s (one output point
C_ch(r, t) with its 16 spin components), per-stage device times from HIP
events recorded on the library's stream, the roofline figures of the
dominant kernel, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6        # dense matrix (and vector) FP64
PEAK_FP32_TFLOPS = 157.3       # dense matrix FP32

PAPER_SITE_CH_PER_S = 6815744 / 19.0   # best BG/Q layout of Table 5 (32 nodes), context only


def stage_model(stage, L, nc, n_ch, csize):
    """Algorithmic HBM bytes of one time slice of each stage: every
    array read and written once.  nc = intermediate components per sink spin."""
    V = L ** 3
    field = 2 * nc * V * csize                      # all block intermediates, both sink spins
    out_field = n_ch * 16 * V * csize
    return {
        "blocks": V * 2 * 144 * csize + field,      # two propagator slices in, intermediates out
        "fft_forward": 2 * field,
        "transpose": 2 * field,
        "contract": field,                          # intermediates in (pair products written besides)
        "fft_inverse": 2 * out_field,
        "finalize": 2 * out_field,
    }.get(stage)


def traffic_for(kernel, csize_tag, L):
    """HBM bytes per dispatch from the committed rocprofv3 counter summary for this
    kernel, form and lattice, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_%dc.json" % (kernel, csize_tag, L))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_1510_00903_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("kernels_sha256") != sha:
        return None
    return rec.get("bytes_per_dispatch")


def cpu_model():
    """Model name of the host CPU (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(Sl, Ss, t_idx, budget_s=20.0):
    """The FP64 oracle (direct Wick, O(V^2)) on a bounded sample of the same job:
    time slice t_idx, one r point per channel, channels 0, 4, 8, ..., 48 and then
    further r points, until about budget_s of CPU time has been spent."""
    import numpy as np
    from oracle import operators as ops
    from oracle import wick
    wick.build(force=False)
    r_points = [(3, 11, 6), (8, 8, 8), (1, 0, 13), (15, 7, 2), (0, 0, 0), (5, 9, 12)]
    done = []
    t0 = time.perf_counter()
    for rp in r_points:
        r = np.array([rp], dtype=np.int32)
        for c in range(0, 52, 4):
            wick.correlate(Sl[t_idx], Ss[t_idx], ops.CHANNELS[c], r)
            done.append((c, rp))
            if time.perf_counter() - t0 > budget_s:
                break
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": len(done) / el, "unit": "site-channels/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "direct-Wick O(V^2) oracle on the 16^3 slice t=%d: %d (channel, r) points "
                      "(channels 0,4,...,48 at r in %s, in that order) in %.1f s"
                      % (t_idx, len(done), [list(p) for p in r_points[:1 + (len(done) - 1) // 13]], el)}


SERVE_LARGE = ((16, 32), (24, 48), (32, 64))
SERVE_SMALL = ((8, 8), (12, 12), (16, 16))


def serve_sweep(bbc, torch, np, n_jobs=64, budget_gb=96, lattices=SERVE_LARGE, max_t=16, presets=0,
                runs=((0.5, 4, False), (0.8, 4, False), (0.8, 4, True), (1.2, 4, False), (1.2, 4, True),
                      (1.2, 1, False))):
    """Continuous-batching serving on a Poisson stream of mixed jobs (FP32 form),
    under a finite HBM budget (resident propagator sets plus slot workspaces).

    Jobs: lattice (L, T) uniform over `lattices` (default 16^3x32, 24^3x48,
    32^3x64), channel subset of size U[4,52] drawn without replacement (or, with
    presets > 0, one of that many such subsets drawn first: recurring analysis
    requests), n_t U[4,max_t] distinct slices (at most T), one of 4 resident
    propagator sets per lattice (seeded PCG64, seed 1510009034).
    The service rate mu is measured by running all jobs one after another on a
    single slot, which also gives every job's result alone (kept on the device).
    Each run (load, slots, graphs) then replays the stream with Poisson arrivals
    at load x mu on the given number of slots, with the slots replaying captured
    slices (graph mode) or launching every kernel, and reports p50/p99 latency
    (submit to completion) and throughput; every job's result in the mix is
    compared bit for bit with its result alone.
    """
    dev = torch.device("cuda:0")
    lattices = list(lattices)
    rng = np.random.Generator(np.random.PCG64(1510009034))
    budget = int(budget_gb) << 30
    ctx = bbc.Context(0, hbm_budget_bytes=budget)
    ctx.server_start(1)
    # propagator sets: seeded Gaussian entries x exp(-m t), generated on the device (FP32)
    props = {}
    for li, (L, T) in enumerate(lattices):
        decay_l = torch.exp(-0.5 * torch.arange(T, dtype=torch.float32, device=dev)).view(T, 1, 1, 1, 1, 1)
        decay_s = torch.exp(-0.7 * torch.arange(T, dtype=torch.float32, device=dev)).view(T, 1, 1, 1, 1, 1)
        for k in range(4):
            g = torch.Generator(device=dev)
            g.manual_seed(1510009034 + 16 * li + k)
            shape = (T, L, L, L, 12, 12)
            Sl = torch.randn(shape, dtype=torch.complex64, device=dev, generator=g) * decay_l
            Ss = torch.randn(shape, dtype=torch.complex64, device=dev, generator=g) * decay_s
            props[(li, k)] = ctx.prop_upload(Sl, Ss)
            del Sl, Ss
    torch.cuda.empty_cache()
    jobs = []
    preset = [sorted(rng.choice(52, size=int(rng.integers(4, 53)), replace=False).tolist()) for _ in range(presets)]
    for _ in range(n_jobs):
        li = int(rng.integers(0, 3))
        L, T = lattices[li]
        if presets:
            ch = preset[int(rng.integers(0, presets))]
        else:
            n_ch = int(rng.integers(4, 53))
            ch = sorted(rng.choice(52, size=n_ch, replace=False).tolist())
        n_t = int(rng.integers(4, min(max_t, T) + 1))
        sl = sorted(rng.choice(T, size=n_t, replace=False).tolist())
        jobs.append({"li": li, "L": L, "prop": props[(li, int(rng.integers(0, 4)))], "ch": ch, "sl": sl,
                     "sites": L ** 3 * n_t * len(ch)})

    def run_job(j):
        L = j["L"]
        out = torch.empty((len(j["sl"]), len(j["ch"]), L, L, L, 16), dtype=torch.complex64, device=dev)
        scale = torch.empty((len(j["sl"]), len(j["ch"])), dtype=torch.float64, device=dev)
        jid = ctx.submit(j["prop"], j["sl"], j["sl"], j["ch"], out, scale)
        return jid, out, scale

    # single stream: service rate and results alone
    jid, _, _ = run_job(jobs[0])     # warm-up: plans and workspaces
    ctx.wait(jid)
    alone, service = [], []
    t0 = time.perf_counter()
    for j in jobs:
        jid, out, scale = run_job(j)
        ctx.wait(jid)
        service.append(ctx.job_times(jid)[1])
        alone.append((out, scale))
        ctx.job_forget(jid)
    single_s = time.perf_counter() - t0
    ctx.server_stop()
    # the same single stream with the slot replaying captured slices (each job's
    # first slice captures its shape's graph; later slices replay it)
    ctx.graph_mode(True)
    ctx.server_start(1)
    service_g, same_g = [], 0
    t0 = time.perf_counter()
    for j, (aout, ascale) in zip(jobs, alone):
        jid, out, scale = run_job(j)
        ctx.wait(jid)
        service_g.append(ctx.job_times(jid)[1])
        same_g += bool(torch.equal(out, aout)) and bool(torch.equal(scale, ascale))
        ctx.job_forget(jid)
        del out, scale
    single_g = time.perf_counter() - t0
    ctx.server_stop()
    ctx.graph_mode(False)
    mu = n_jobs / single_s
    sites = sum(j["sites"] for j in jobs)
    results = []
    for load, n_slots, graphs in runs:
        lam = load * mu
        gaps = rng.exponential(1.0 / lam, size=n_jobs)
        arrivals = np.cumsum(gaps) - gaps[0]
        ctx.graph_mode(graphs)
        ctx.server_start(n_slots)
        print("serve: load %.1f on %d slots (%.1f jobs/s)%s" % (load, n_slots, lam, ", graphs" if graphs else ""),
              file=sys.stderr, flush=True)
        inflight = []
        start = time.perf_counter()
        for j, at in zip(jobs, arrivals):
            now = time.perf_counter() - start
            if at > now:
                time.sleep(at - now)
            inflight.append(run_job(j))
        lat, same = [], 0
        for (jid, out, scale), (aout, ascale) in zip(inflight, alone):
            ctx.wait(jid)
            lat.append(ctx.job_times(jid)[2])
            ctx.job_forget(jid)
            same += bool(torch.equal(out, aout)) and bool(torch.equal(scale, ascale))
        makespan = time.perf_counter() - start
        ctx.server_stop()
        del inflight
        lat = np.array(lat)
        ctx.graph_mode(False)
        results.append({"load": load, "slots": n_slots, "slot_graphs": graphs,
                        "arrival_rate_jobs_per_s": round(lam, 3),
                        "site_channels_per_s": round(sites / makespan, 1), "makespan_s": round(makespan, 3),
                        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 2),
                                       "p99": round(float(np.percentile(lat, 99)), 2),
                                       "mean": round(float(lat.mean()), 2), "max": round(float(lat.max()), 2)},
                        "results_identical_alone_vs_mix": "%d/%d" % (same, n_jobs)})
    del alone
    ctx.close()
    torch.cuda.empty_cache()
    return {
        "metric": "serving: job latency p50/p99 and throughput (site-channels/s)",
        "unit": "site-channels/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f32",
        "data": "synthetic (seeded on the device)", "hbm_budget_bytes": budget,
        "single_stream": {"jobs_per_s": round(mu, 3), "site_channels_per_s": round(sites / single_s, 1),
                          "mean_service_ms": round(float(np.mean(service)), 2)},
        "single_stream_slot_graphs": {"jobs_per_s": round(n_jobs / single_g, 3),
                                      "site_channels_per_s": round(sites / single_g, 1),
                                      "mean_service_ms": round(float(np.mean(service_g)), 2),
                                      "results_identical_to_eager": "%d/%d" % (same_g, n_jobs)},
        "runs": results, "jobs": n_jobs,
        "config": {"workload": "%d-job Poisson mix: lattices %s, %s, 4-%d slices, 4 resident "
                               "propagator sets per lattice, FP32 form"
                               % (n_jobs, "/".join("%d^3x%d" % lt for lt in lattices),
                                  "one of %d channel subsets of 4-52 channels" % presets if presets
                                  else "4-52 channels", max_t)},
    }


def stream96(bbc, torch, np, n_slices):
    """96^3 lattice, 52 channels, FP32 form, time slices streamed from host memory.

    Slices (about 1 GB per flavour) are drawn on the host (seeded torch generator,
    Gaussian entries x exp(-m t)) into pinned memory; bbc_correlate copies each
    slice in and its 5.9 GB output back through device staging buffers on two
    copy streams, overlapped with the kernels of the neighbouring slices.  One
    warm-up slice, then n_slices timed slices (t = 0 .. n_slices-1).
    """
    L, n_ch = 96, 52
    V = L ** 3
    chans = list(range(n_ch))
    g = torch.Generator()
    g.manual_seed(1510009035)
    T = n_slices
    shape = (T, L, L, L, 12, 12)
    print("bench: drawing %d host slices of %d^3" % (T, L), file=sys.stderr, flush=True)
    Sl = torch.empty(shape, dtype=torch.complex64, pin_memory=True)
    Ss = torch.empty(shape, dtype=torch.complex64, pin_memory=True)
    for t in range(T):
        Sl[t] = torch.randn(shape[1:], dtype=torch.complex64, generator=g) * float(np.exp(-0.5 * t))
        Ss[t] = torch.randn(shape[1:], dtype=torch.complex64, generator=g) * float(np.exp(-0.7 * t))
    out = torch.empty((T, n_ch, L, L, L, 16), dtype=torch.complex64, pin_memory=True)
    scale = torch.empty((T, n_ch), dtype=torch.float64, device="cuda:0")
    ctx = bbc.Context(0)
    print("bench: warm-up slice", file=sys.stderr, flush=True)
    ctx.correlate(Sl[:1], Ss[:1], [0], chans, out=out[:1], scale=scale[:1])
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    ctx.correlate(Sl, Ss, list(range(T)), chans, out=out, scale=scale)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.close()
    # exact relations on the last slice (host copy of the output): the isospin pair
    # C[L L > p X-] = -C[L L > n X0] on two z planes, and for identical sink baryons
    # C(r)_{a b a' b'} = -C(-r)_{b a a' b'} (L L > L L) over every r
    sc = scale[-1].cpu()
    a = out[-1, 11, [0, 48]].to(torch.complex128) * float(sc[11])
    b = out[-1, 12, [0, 48]].to(torch.complex128) * float(sc[12])
    iso = float((a + b).abs().max() / a.abs().max())
    C = out[-1, 10].to(torch.complex128)
    neg = torch.roll(torch.flip(C, dims=(0, 1, 2)), shifts=(1, 1, 1), dims=(0, 1, 2))
    idx = torch.tensor([((s >> 1) & 1) + 2 * (s & 1) + 4 * (s >> 2) for s in range(16)])
    anti = float((C + neg[..., idx]).abs().max() / C.abs().max())
    del a, b, C, neg
    ok = iso <= 1e-5 and anti <= 1e-5
    site_ch = V * T * n_ch
    stages = {k: {"ms_total": round(v[0], 2), "ms_per_slice": round(v[0] / max(1, T), 2)} for k, v in prof.items()}
    return {"metric": "correlator site-channels/sec (C_ch(r,t))", "value": round(site_ch / el, 1),
            "unit": "site-channels/s", "n_gpus": 1, "steps": T, "warmup": 1,
            "ms_per_slice": round(1000 * el / T, 2), "higher_is_better": True, "dtype": "f32",
            "data": "synthetic (seeded on the host, streamed from pinned memory)",
            "relations_hold": ok,
            "relations": {"isospin_LL_pXm_plus_LL_nX0": iso, "identical_sink_antisymmetry_LL": anti,
                          "tolerance": 1e-5, "slice": T - 1},
            "config": {"workload": "96^3 lattice, all 52 channels, FP32 form, slices streamed host->device, "
                                   "outputs streamed back", "lattice": [L, L, L], "slices": T,
                       "input_GB_per_slice": round(2 * V * 144 * 8 / 1e9, 3),
                       "output_GB_per_slice": round(n_ch * V * 16 * 8 / 1e9, 3)},
            "stages": stages}


def postproc(bbc, torch, np, steps):
    """Post-processing of the 16^3 x 32, 52-channel FP64 output (Sec. 2): spin
    projection (J = 0 at sink and source; source J = 1, M = 0 keeping the sink
    pair), A1+ projection over the cubic group of the 4-component field, and the
    central potential of every channel's J = 0 field.  Inputs: a seeded random field
    of the correlator's shape (the kernels' cost does not depend on the values).
    Each kernel is timed over `steps` calls with HIP events on the current stream;
    rates are algorithmic bytes (every array read and written once) per second."""
    L, T, n_ch = 16, 32, 52
    V = L ** 3
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(1510009036)
    C = torch.randn((T, n_ch, L, L, L, 16), dtype=torch.complex128, device=dev, generator=g)
    sq = np.sqrt(0.5)
    P00 = np.array([[0, sq], [-sq, 0]])
    P10 = np.array([[0, sq], [sq, 0]])
    def sidx(a, b, ap, bp):
        return a + 2 * (b + 2 * (ap + 2 * bp))
    W0 = np.zeros((1, 16), dtype=complex)
    W1 = np.zeros((4, 16), dtype=complex)
    for a in range(2):
        for b in range(2):
            for ap in range(2):
                for bp in range(2):
                    W0[0, sidx(a, b, ap, bp)] = P00[a][b] * P00[ap][bp]
                    W1[a + 2 * b, sidx(a, b, ap, bp)] = P10[ap][bp]
    ctx = bbc.Context(0)
    out0 = torch.empty((T, n_ch, L, L, L, 1), dtype=C.dtype, device=dev)
    out1 = torch.empty((T, n_ch, L, L, L, 4), dtype=C.dtype, device=dev)
    outc = torch.empty_like(out1)
    ctx.spin_project(C, W0, out=out0)
    R = out0[..., 0].permute(1, 0, 2, 3, 4).contiguous()          # [channel][t][z][y][x]
    Vp = torch.empty((n_ch, T - 2, L, L, L), dtype=C.dtype, device=dev)
    cs = 16
    jobs = {
        "spin_project_J0": (lambda: ctx.spin_project(C, W0, out=out0), T * n_ch * V * (16 + 1) * cs),
        "spin_project_src_J1M0": (lambda: ctx.spin_project(C, W1, out=out1), T * n_ch * V * (16 + 4) * cs),
        "cubic_project_A1": (lambda: ctx.cubic_project(out1, out=outc), 2 * T * n_ch * V * 4 * cs),
        "central_potential": (lambda: ctx.central_potential(R, 0.5, out=Vp),
                              n_ch * (T + T - 2) * V * cs),
    }
    res = {}
    for name, (fn, nbytes) in jobs.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "alg_GB": round(nbytes / 1e9, 3), "GB_s": round(gbs, 1),
                     "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)}
    ok = bool(torch.isfinite(Vp).all().item())
    ctx.close()
    total_ms = sum(v["ms"] for v in res.values())
    return {"metric": "post-processing of C(r,t): site-channels/sec", "value": round(T * n_ch * V / (total_ms * 1e-3), 1),
            "unit": "site-channels/s", "n_gpus": 1, "steps": steps, "higher_is_better": True, "dtype": "f64",
            "data": "synthetic (seeded random field of the correlator's shape)", "outputs_finite": ok,
            "config": {"workload": "16^3x32, 52 channels: spin projection J=0 and source J=1 M=0, A1+ cubic "
                                   "projection, central potential per channel", "lattice": [L, L, L], "T": T,
                       "channels": n_ch},
            "kernels": res}


def next_rows(bbc, torch, np, synth, steps):
    """The paths beyond the 52-channel correlator, on the 16^3 x 32 FP64 propagators
    of the default job:
      * CPT average (Sec. 6): bbc_correlate_cpt over tau = 0..15 with t0 = 0 (two
        correlator slices per tau: upper at t0 + tau, lower at t0 - tau mod 32), 52 channels;
      * general fields (Sec. 2, Eq. (FieldOperator_B)): 31 channels -- Omega- Omega- and
        Delta++ Delta++ for every (l1, l2) pair (source = sink), four {C, gamma_5} nucleon
        channels, Omega- p, Delta+ Delta+ and Sigma*0 p for l = 1, 2, 3 -- over all 32 slices.
    Wall time over `steps` calls after one warm-up call, per-stage HIP-event times
    from one more profiled call."""
    L, T = 16, 32
    V = L ** 3
    dev = torch.device("cuda:0")
    Sl, Ss = synth.propagators(L, T, seed=synth.BASE_SEED + 1)
    d_l, d_s = torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)
    ctx = bbc.Context(0)
    out = {}

    def timed(fn, n_units):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0) / steps
        ctx.profile(True)
        ctx.profile_read()
        fn()
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        stages = {k: round(v[0], 3) for k, v in prof.items() if v[1] > 0}
        return {"ms_per_step": round(ms, 3), "value": round(n_units / (ms * 1e-3), 1), "stages_ms": stages}

    taus = list(range(16))
    chans = list(range(52))
    R = torch.empty((len(taus), len(chans), L, L, L, 16), dtype=torch.complex128, device=dev)
    r = timed(lambda: ctx.correlate_cpt(d_l, d_s, 0, taus, chans, out=R), len(taus) * len(chans) * V)
    r.update({"unit": "averaged site-channels/s", "correlator_slices_per_step": 2 * len(taus),
              "outputs_finite": bool(torch.isfinite(R).all().item())})
    out["cpt_average"] = r
    del R

    quads = []
    for f in ("O-", "D++"):
        for l1 in (1, 2, 3):
            for l2 in (1, 2, 3):
                a, b = "%s(%d)" % (f, l1), "%s(%d)" % (f, l2)
                quads.append((a, b, a, b))
    quads += [("p2", "n2", "p2", "n2"), ("p2", "n", "p", "n2"), ("p", "n2", "p2", "n"), ("p2", "n2", "p", "n")]
    quads += [("O-(%d)" % l, "p", "O-(%d)" % l, "p") for l in (1, 2, 3)]
    quads += [("D+(%d)" % l,) * 4 for l in (1, 2, 3)]
    quads += [("S*0(%d)" % l, "p", "S*0(%d)" % l, "p") for l in (1, 2, 3)]
    gch = [bbc.channel_id(*q) for q in quads]
    C = torch.empty((T, len(gch), L, L, L, 16), dtype=torch.complex128, device=dev)
    r = timed(lambda: ctx.correlate(d_l, d_s, list(range(T)), gch, out=C), T * len(gch) * V)
    st = bbc.plan_stats(gch)
    r.update({"unit": "site-channels/s", "channels": len(gch), "block_components_per_site": st["components"],
              "iterations": st["iterations"], "outputs_finite": bool(torch.isfinite(C).all().item())})
    out["general_fields"] = r
    ctx.close()
    return {"metric": "CPT average and general-field correlators: site-channels/sec",
            "value": out["general_fields"]["value"], "unit": "site-channels/s", "n_gpus": 1, "steps": steps,
            "higher_is_better": True, "dtype": "f64", "data": "synthetic (seeded Gaussian propagators, "
            "exp(-m t) decay; the default job's inputs)",
            "config": {"workload": "16^3x32 FP64: CPT average (16 tau, 52 channels) and 31 general-field "
                                   "channels (decuplet Omega-/Delta++/Delta+/Sigma*0, {C, gamma_5} nucleon, "
                                   "Omega- p, Sigma*0 p)",
                       "lattice": [L, L, L], "T": T},
            "paths": out}


def device_correlated(torch, L, T, seed, dtype):
    """The 32^3 x 64 configuration's inputs, drawn on the device (seeded torch generator):
    S_f(x, t) = exp(-m_f t) (Z_f(x) + 1e-3 eta_f(x, t)), Z and eta complex Gaussian (re, im
    independent N(0, 1)), m = 0.5 (light), 0.7 (strange).  Drawn in FP32; the FP64 form
    takes the same values."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    out = []
    for m in (0.5, 0.7):
        Z = torch.randn((L, L, L, 12, 12), dtype=torch.complex64, device=dev, generator=g) * (2 ** 0.5)
        S = torch.empty((T, L, L, L, 12, 12), dtype=torch.complex64, device=dev)
        for t in range(T):
            eta = torch.randn((L, L, L, 12, 12), dtype=torch.complex64, device=dev, generator=g) * (2 ** 0.5)
            S[t] = (Z + 1e-3 * eta) * math.exp(-m * t)
        out.append(S if dtype == torch.complex64 else S.to(dtype))
    return out


def correlator_job(bbc, torch, d_l, d_s, L, fp32, steps, warmup, graph=False, channels=None, tuning=None):
    """Time `steps` whole jobs (every slice of d_l/d_s, all channels) after `warmup`
    untimed ones; per-stage device times from HIP events of the profiled steps.
    tuning: kernel variants for this request shape (default: the library's built-in choice)."""
    T = d_l.shape[0]
    channels = list(range(52)) if channels is None else channels
    n_ch = len(channels)
    dev = torch.device("cuda:0")
    out = torch.empty((T, n_ch, L, L, L, 16), dtype=torch.complex64 if fp32 else torch.complex128, device=dev)
    scale = torch.empty((T, n_ch), dtype=torch.float64, device=dev) if fp32 else None
    ctx = bbc.Context(0)
    t_list = list(range(T))
    if tuning is not None:
        ctx.set_tuning((L, L, L), channels, tuning, precision=bbc.F32 if fp32 else bbc.F64)
    tune = ctx.tuning((L, L, L), channels, precision=bbc.F32 if fp32 else bbc.F64)[0]
    # profiled calls run one slice at a time; when the job's tuning runs several
    # at once (or in graph mode) the timed steps are unprofiled and the stage
    # times come from one more, profiled, step
    separate = graph or (tune["slices"] > 0 and T > 1)
    if graph:
        ctx.graph_mode(True)
    for _ in range(warmup):
        ctx.correlate(d_l, d_s, t_list, channels, out=out, scale=scale)
    torch.cuda.synchronize()
    if not separate:
        ctx.profile(True)
        ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.correlate(d_l, d_s, t_list, channels, out=out, scale=scale)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof_steps = steps
    if separate:
        ctx.graph_mode(False)
        ctx.profile(True)
        ctx.profile_read()
        ctx.correlate(d_l, d_s, t_list, channels, out=out, scale=scale)
        torch.cuda.synchronize()
        prof_steps = 1
    prof = ctx.profile_read()
    ctx.close()
    ms_per_step = 1000.0 * el / steps
    site_ch = L ** 3 * T * n_ch
    st = bbc.plan_stats(channels)
    nc = st["components"] // 2
    csize = 8 if fp32 else 16
    peak = PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS
    stages = {}
    n_slices = T * prof_steps
    for name, (ms, launches) in prof.items():
        if launches == 0:
            continue                                 # stage without kernels on this path (fused)
        ms_slice = ms / n_slices
        stages[name] = {"ms_total": round(ms, 4), "kernels": int(launches), "ms_per_slice": round(ms_slice, 4)}
        nb = stage_model(name, L, nc, n_ch, csize)
        if nb is not None:
            stages[name]["alg_GBs"] = round(nb / (ms_slice * 1e-3) / 1e9, 1)
    dom = max(stages, key=lambda k: stages[k]["ms_total"])
    avg_s = stages[dom]["ms_total"] / 1000.0 / stages[dom]["kernels"]
    if dom == "contract":
        # the method's work: 16 complex MACs (8 flops each) per open-index item, all
        # channels; the pair products run on the matrix cores (peak of the dtype)
        flops = 8.0 * 16 * st["iterations"] * L ** 3
        achieved = flops / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4)}
    else:
        nbytes = stage_model(dom, L, nc, n_ch, csize) * n_slices / stages[dom]["kernels"]
        achieved = nbytes / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / PEAK_HBM_GBS, 4)}
    roof["kernel"] = dom
    roof["avg_launch_us"] = round(avg_s * 1e6, 2)
    roof["traffic"] = traffic_for(dom, "f32" if fp32 else "f64", L)
    roof["timed_in"] = ("a profiled step after the timed region (one slice at a time)" if separate
                        else "the timed region")
    return {"value": round(site_ch / (ms_per_step / 1000.0), 1), "ms_per_step": round(ms_per_step, 3),
            "site_channels_per_step": site_ch, "roofline": roof, "stages": stages, "tuning": tune,
            "block_components_per_site": st["components"], "iterations": st["iterations"]}, out, scale


def c1_job(bbc, torch, np, synth, steps):
    """8^3 x 8, channel 1 (p Lambda > p Lambda), FP64: eager launches and HIP-graph replay,
    with the library's built-in kernel variants and with those its autotuner picks for this
    request shape (tuned on one slice before the timed region)."""
    L, T = 8, 8
    dev = torch.device("cuda:0")
    Sl, Ss = synth.propagators(L, T, seed=synth.BASE_SEED)
    d_l, d_s = torch.from_numpy(Sl).to(dev), torch.from_numpy(Ss).to(dev)
    res = {}
    for mode in ("eager", "graph"):
        r, _, _ = correlator_job(bbc, torch, d_l, d_s, L, False, steps, 3, graph=mode == "graph", channels=[1])
        res[mode] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                     "stages_ms_per_slice": {k: v["ms_per_slice"] for k, v in r["stages"].items()}}
    ctx = bbc.Context(0)
    best, _ = ctx.autotune(d_l[0].contiguous(), d_s[0].contiguous(), [1], reps=5)
    ctx.close()
    tuned = {"variants": best}
    for mode in ("eager", "graph"):
        r, _, _ = correlator_job(bbc, torch, d_l, d_s, L, False, steps, 3, graph=mode == "graph", channels=[1],
                                 tuning=best)
        tuned[mode] = {"value": r["value"], "ms_per_step": r["ms_per_step"]}
    return {"workload": "8^3x8 lattice, channel 1 (p Lambda > p Lambda), FP64, all r, all t",
            "unit": "site-channels/s", "site_channels_per_step": L ** 3 * T, **res, "autotuned": tuned}


def c3_jobs(bbc, torch, np, steps):
    """32^3 x 64, 52 channels: the FP64 form and the FP32 form on the same (FP32-drawn)
    inputs, generated on the device; per-channel normwise error of the FP32 form against
    the FP64 form over every r at t = 0, 31, 63."""
    L, T = 32, 64
    res = {}
    d_l, d_s = device_correlated(torch, L, T, synth_seed_c3(), torch.complex64)
    r32, out32, scale32 = correlator_job(bbc, torch, d_l, d_s, L, True, steps, 1)
    res["f32"] = r32
    keep = [0, 31, 63]
    c32 = (out32[keep].to(torch.complex128) * scale32[keep].view(3, 52, 1, 1, 1, 1)).contiguous()
    del out32, scale32
    torch.cuda.empty_cache()
    d_l64, d_s64 = d_l.to(torch.complex128), d_s.to(torch.complex128)
    del d_l, d_s
    r64, out64, _ = correlator_job(bbc, torch, d_l64, d_s64, L, False, steps, 1)
    res["f64"] = r64
    c64 = out64[keep]
    err = ((c32 - c64).abs().amax(dim=(2, 3, 4, 5)) / c64.abs().amax(dim=(2, 3, 4, 5))).amax(dim=0)
    del out64, d_l64, d_s64, c32, c64
    torch.cuda.empty_cache()
    e = [float(x) for x in err.cpu()]
    return {"workload": "32^3x64 lattice, all 52 channels, inputs exp(-m t)(Z + 1e-3 eta_t) drawn on the device",
            "unit": "site-channels/s", "f32": res["f32"], "f64": res["f64"],
            "fp32_speedup": round(res["f32"]["value"] / res["f64"]["value"], 3),
            "fp32_vs_fp64_normwise_error": {"max": max(e), "per_channel": [float("%.3g" % x) for x in e],
                                            "slices": keep, "tolerance": 1e-5}}


def synth_seed_c3():
    return 1510009030 + 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the c1, c3 and serving measurements")
    ap.add_argument("--workload", default="16c32-f64",
                    choices=["16c32-f64", "32c64-f64", "32c64-f32", "serve-mix", "serve-small", "96c-f32-stream",
                             "post-16c32", "next-16c32", "8c8-plambda"],
                    help="16c32-f64: 16^3x32, 52 channels, FP64 (default, the paper's Table 5 job); "
                         "32c64-*: 32^3x64, 52 channels, correlated inputs, FP64 or FP32 form")
    ap.add_argument("--graph", action="store_true",
                    help="replay each job as a captured HIP graph (stage timings from one extra profiled step)")
    ap.add_argument("--slices", type=int, default=0,
                    help="time only the first N slices of the job (for profiling runs; 0 = all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 1 GiB (for scaling rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: runs on one GPU; the correlator of each time slice is independent, "
              "so several GPUs would each take a share of the slices. Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1510_00903_amd as bbc
    import synth

    if args.workload == "serve-mix":
        print(json.dumps(serve_sweep(bbc, torch, np)), flush=True)
        return
    if args.workload == "serve-small":
        print(json.dumps(serve_sweep(bbc, torch, np, n_jobs=256, lattices=SERVE_SMALL, max_t=8, presets=4)), flush=True)
        return
    if args.workload == "96c-f32-stream":
        print(json.dumps(stream96(bbc, torch, np, args.steps)), flush=True)
        return
    if args.workload == "post-16c32":
        print(json.dumps(postproc(bbc, torch, np, args.steps)), flush=True)
        return
    if args.workload == "next-16c32":
        print(json.dumps(next_rows(bbc, torch, np, synth, args.steps)), flush=True)
        return
    if args.workload == "8c8-plambda":
        print(json.dumps(c1_job(bbc, torch, np, synth, args.steps)), flush=True)
        return

    fp32 = args.workload.endswith("f32")
    L, T = (16, 32) if args.workload.startswith("16") else (32, 64)
    dev = torch.device("cuda:0")
    print("bench: generating %d^3 x %d propagators" % (L, T), file=sys.stderr, flush=True)
    if L == 16:
        Sl, Ss = synth.propagators(L, T, seed=synth.BASE_SEED + 1)
        d_l = torch.from_numpy(Sl).to(dev)
        d_s = torch.from_numpy(Ss).to(dev)
    else:
        Sl = Ss = None
        d_l, d_s = device_correlated(torch, L, T, synth_seed_c3(),
                                     torch.complex64 if fp32 else torch.complex128)
    if args.slices:
        T = min(T, args.slices)
        d_l, d_s = d_l[:T], d_s[:T]
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    print("bench: warmup %d, steps %d" % (args.warmup, args.steps), file=sys.stderr, flush=True)
    r, out, scale = correlator_job(bbc, torch, d_l, d_s, L, fp32, args.steps, args.warmup, graph=args.graph)
    del out, scale
    print("bench: timed %d steps, %.3f ms per step" % (args.steps, r["ms_per_step"]), file=sys.stderr, flush=True)
    n_ch = 52
    res = {
        "metric": "correlator site-channels/sec (C_ch(r,t))",
        "value": r["value"],
        "unit": "site-channels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": round(r["value"] / PAPER_SITE_CH_PER_S, 2) if L == 16 and not fp32 else None,
        "baseline_context": "paper Table 5, 16^3x32, 52 channels, 32 BlueGene/Q nodes, best layout 19 s"
                            if L == 16 else None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic (seeded Gaussian propagators, exp(-m t) decay)" if L == 16 else
                "synthetic (seeded t-independent Gaussian field + 1e-3 noise per slice, exp(-m t) decay, "
                "drawn on the device)",
        "config": {"workload": "%d^3x%d lattice, all 52 BB channels, %s, upper spins"
                               % (L, T, "FP32 form (power-of-two rescaled, FP32 blocks, forward FFT and "
                                        "matrix-core products, FP64 channel sums, compensated float-float "
                                        "inverse FFT)" if fp32 else "FP64 plain form"),
                   "lattice": [L, L, L], "T": T, "channels": n_ch, "site_channels_per_step": r["site_channels_per_step"],
                   "block_components_per_site": r["block_components_per_site"], "iterations": r["iterations"]},
        "roofline": r["roofline"],
        "stages": r["stages"],
        "tuning": r["tuning"],
        "hip_graph": bool(args.graph),
    }
    if L == 16 and not fp32 and not args.no_extras and not args.slices:
        del d_l, d_s
        torch.cuda.empty_cache()
        print("bench: c1 (8^3 x 8 p Lambda)", file=sys.stderr, flush=True)
        res["c1_8c8_plambda_f64"] = c1_job(bbc, torch, np, synth, 20)
        print("bench: c3 (32^3 x 64, FP32 and FP64)", file=sys.stderr, flush=True)
        res["c3_32c64"] = c3_jobs(bbc, torch, np, 2)
        print("bench: c4 (serving sweep)", file=sys.stderr, flush=True)
        res["c4_serving"] = serve_sweep(bbc, torch, np)
        print("bench: c4 small lattices (serving sweep)", file=sys.stderr, flush=True)
        res["c4_serving_small"] = serve_sweep(bbc, torch, np, n_jobs=256, lattices=SERVE_SMALL, max_t=8, presets=4)
    if not args.no_cpu_baseline and L == 16 and Sl is not None:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(Sl, Ss, 7)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
