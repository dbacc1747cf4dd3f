#!/usr/bin/env python3
"""Benchmark of the LArTPC signal-simulation hot path on one MI355X.

A step is one whole DepoTransform (arXiv:2304.01841, Sec. 2: rasterize with
fluctuation, scatter-add into the plane grid, FFT convolution with the
response) of one event whose depos are already resident in HBM.  The workload
is the detector-scale collection plane: 960 wires x 10 impact bins x 6,000
ticks, 500,000 depos on 200 straight tracks, Philox fluctuation, a 210 x 200
response, wire-resolution output.

Prints one JSON line: depos/s (the headline), planes/s and the p50/p99 event
latency, the per-stage times (the paper's per-kernel timers, Sec. 5.2), the
roofline of the dominant kernel measured live with HIP events on the stream
the library launches on, and the FP64 oracle timed on the host as a CPU
baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# VALU peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T
# 32-bit lane operations per second (an FMA counts as one operation).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic 32-bit operations of the fluctuating raster kernel:
#   per Philox4x32-10 call (4 bins): 10 rounds x (two 32x32->64 products = 4
#   multiplies, 4 xors) = 80; four uniforms (shift, convert, add, scale) = 16;
#   two Box-Muller pairs (log, scale, sqrt, sin, cos, 2 products) = 12;
#   per bin: p = Wp Wt, q p, 1 - p, q p (1 - p), sqrt, fma, clamp, patch sum,
#   rescale, LDS add = 10.
OPS_PER_PHILOX_CALL = 80 + 16 + 12
OPS_PER_BIN = 10
def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kind", choices=["wire", "pitch"], default="wire")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-event batched vs plain comparison")
    ap.add_argument("--batch-events", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served-form measurement")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--no-three-plane", action="store_true",
                    help="skip the three-plane (U/V/W, 2.4M depos) event measurement")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default schedules instead of autotuned ones")
    ap.add_argument("--schedule", type=str, default=None, metavar="K=V[,K=V]",
                    help="fixed schedule of the benchmark plane (no tuning), e.g. "
                         "fft_pitch=640,freq_chunk=16 (or the same as a JSON object)")
    ap.add_argument("--lifetime", type=float, default=0.0, metavar="US",
                    help="electron lifetime of the benchmark plane (an extension beyond the "
                         "paper; 0, the default, is the paper's workload without absorption)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (a plain copy kernel "
                         "whose HBM counters scale the kernels' FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def algorithmic_bytes(P, nout: int, n_depos: int) -> dict:
    """Minimum HBM bytes of each stage at the minimum transform sizes:
    H = floor((Nt + Rt - 1) / 2) + 1 frequencies per row; the grid written
    once; the spectrum written by the tick pass and read by the pitch pass;
    the kept rows written by the pitch pass and read by the inverse pass."""
    Np, Nt = P.npitch, P.nticks
    Rt = P._resp.shape[1]
    H = (Nt + Rt - 1) // 2 + 1
    L = P.info["fft_pitch"]
    return {
        "clear_grid": 4 * Np * Nt,
        "raster_tiles": 40 * n_depos + 4 * Np * Nt,
        "fft_ticks": 4 * Np * Nt + 8 * Np * H,
        "conv_pitch": 8 * Np * H + 8 * L * H + 8 * nout * H,
        "ifft_ticks": 8 * nout * H + 4 * nout * Nt,
    }


def raster_work(wcsim, P, dep) -> dict:
    """Bins and Philox calls of every patch, from the windows the library's
    own rasterizer returns (outside the timed region)."""
    pt = wcsim.rasterize(P, dep, 0)
    meta, offs, _ = pt.to_host()
    pt.destroy()
    lo_t, n_p, n_t = (meta[:, k].astype(np.int64) for k in (1, 2, 3))
    live = n_p > 0
    quads = np.where(live, np.floor_divide(lo_t + n_t - 1, 4) - np.floor_divide(lo_t, 4) + 1, 0)
    calls = int(np.sum(n_p * quads))
    bins = int(np.sum(n_p * n_t))
    return {"philox_calls": calls, "bins": bins,
            "ops": calls * OPS_PER_PHILOX_CALL + bins * OPS_PER_BIN}


# Schedule fields that change what each profiled kernel does (the raster
# kernel depends only on the tile shape, the FFT passes only on their sizes).
SCHEDULE_FIELDS = {"k_raster_tiles": ("tile",), "k_fill_records": ("tile",),
                   "k_rows_r2c": ("fft_ticks", "freq_chunk"),
                   "k_rows_c2r": ("fft_ticks", "freq_chunk"),
                   "k_pitch_conv": ("fft_ticks", "fft_pitch", "freq_chunk")}


def measured_traffic(kernel: str, schedule: dict):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy kernel), or None when
    the kernel's source changed since the counters were taken or they were
    taken under a schedule that runs the kernel differently."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic_collection.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get("kernels", {}).get(kernel)
    taken = rec.get("schedule") or {}
    fields = SCHEDULE_FIELDS.get(kernel, tuple(schedule))
    if not k or any(taken.get(f) != schedule.get(f) for f in fields):
        return None
    src = os.path.join(ROOT, k["source"])
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if digest != k["source_sha256"]:
        return None
    return k["bytes_per_launch"]


def cpu_baseline(w, kind_wire: bool) -> dict:
    """The FP64 oracle on one whole event, single-threaded."""
    from oracle import oracle as O

    pl, R, phys, dep = w["planes"][0], w["responses"][0], w["phys"], w["depos"]
    O.build()
    t0 = time.perf_counter()
    out = O.simulate_event(dep, phys, pl, R.astype(np.float64), R.shape[0] // 2, w["event_id"],
                           wire_output=kind_wire, workers=1)
    dt = time.perf_counter() - t0
    assert np.isfinite(out).all()
    return {"value": dep.shape[0] / dt, "unit": "depos/s", "cores": 1, "kind": "oracle",
            "sample": "one whole event (%d depos, %d x %d grid) in %.2f s, 1 thread"
                      % (dep.shape[0], pl["nwires"] * pl["nimpact"], pl["nticks"], dt)}


def batch_comparison(wcsim, W, dev, nevents: int, tuner=None, rounds: int = 3) -> dict:
    """The batch workload (uneven events: depo counts log-uniform in
    10^4..10^6, 100/480/800/960 wires x 6000 ticks): `nevents` plain
    per-event launches (library default schedules) against one captured batch
    (schedules from the autotuner, one per wire count, tuned on that wire
    count's median event), both timed over whole rounds with inputs resident
    in HBM."""
    import torch

    evs = W.batch_events(nevents=nevents)
    phys = W.physics(True)
    planes, tuned, schedules = {}, {}, {}
    for nw in sorted({e["plane"]["nwires"] for e in evs}):
        mine = sorted((e for e in evs if e["plane"]["nwires"] == nw),
                      key=lambda e: e["depos"].shape[0])
        e = mine[len(mine) // 2]
        planes[nw] = wcsim.Plane(e["plane"], phys, e["response"])
        sched = None
        if tuner is not None:
            sched = tuner.tune(e["plane"], phys, e["response"],
                               torch.from_numpy(e["depos"]).to(dev))
        schedules[nw] = sched or {}
        tuned[nw] = wcsim.Plane(e["plane"], phys, e["response"], schedule=sched)
    pl = [planes[e["plane"]["nwires"]] for e in evs]
    plb = [tuned[e["plane"]["nwires"]] for e in evs]
    deps = [torch.from_numpy(e["depos"]).to(dev) for e in evs]
    ids = [e["event_id"] for e in evs]
    outs = [torch.empty((p.nwires, p.nticks), dtype=torch.float32, device=dev) for p in pl]
    ntot = sum(d.shape[0] for d in deps)
    wsp = wcsim.simulate_workspace(pl[int(np.argmax([p.npitch * 10**7 + d.shape[0]
                                                     for p, d in zip(pl, deps)]))],
                                   max(d.shape[0] for d in deps), wcsim.OUT_WIRE, dev)
    # the largest workspace covers every event run in sequence
    need = max(wcsim._lib.wcsim_simulate_workspace_bytes(p.handle, d.shape[0], 0)
               for p, d in zip(pl, deps))
    if wsp.numel() < need:
        wsp = torch.empty(need, dtype=torch.uint8, device=dev)

    def plain():
        for p, d, i, o in zip(pl, deps, ids, outs):
            wcsim.simulate_event(p, d, i, out=o, workspace=wsp)

    batch = wcsim.Batch(plb, [d.shape[0] for d in deps])

    def batched():
        batch.run(deps, ids, outs)

    res = {}
    for name, fn in (("plain", plain), ("batched", batched)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(rounds):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / rounds
        res[name] = {"ms_per_batch": dt * 1e3, "depos_per_s": ntot / dt,
                     "planes_per_s": nevents / dt}
    batch.destroy()
    res["events"] = nevents
    res["depos"] = int(ntot)
    res["speedup"] = res["plain"]["ms_per_batch"] / res["batched"]["ms_per_batch"]
    res["batched_schedules"] = {str(k): v for k, v in schedules.items()}
    return res


def digitize_measurement(wcsim, out, reps: int = 20) -> dict:
    """Digitisation with white noise (an extension beyond the paper) of the
    benchmark event's output: time per call and HBM rate (4 B read + 2 B
    written per sample), HIP events on torch's current stream."""
    import torch

    codes = torch.empty(out.shape, dtype=torch.int16, device=out.device)
    for _ in range(3):
        wcsim.digitize(out, 1.0, 2048.0, 3.0, 12, seed=7, event_id=0, out=codes)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for e in range(reps):
        wcsim.digitize(out, 1.0, 2048.0, 3.0, 12, seed=7, event_id=e, out=codes)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    # coloured noise through a 64-tap filter
    fir = torch.exp(-torch.arange(64, dtype=torch.float32, device=out.device) / 9.0)
    for _ in range(3):
        wcsim.digitize(out, 1.0, 2048.0, 3.0, 12, seed=7, event_id=0, out=codes, fir=fir)
    t0.record()
    for e in range(reps):
        wcsim.digitize(out, 1.0, 2048.0, 3.0, 12, seed=7, event_id=e, out=codes, fir=fir)
    t1.record()
    torch.cuda.synchronize()
    ms_c = t0.elapsed_time(t1) / reps
    n = out.numel()
    return {"samples": int(n), "ms": ms, "hbm_gbs": 6.0 * n / (ms * 1e-3) / 1e9,
            "coloured_64tap_ms": ms_c}


def three_plane_measurement(wcsim, W, dev, tuner=None, steps: int = 10) -> dict:
    """The three-plane event (U/V/W 800/800/960 wires x 6000 ticks, 2,000,000
    track + 400,000 background depos, fluctuation on, wire output): the three
    planes run one after the other on one stream per step, depos resident."""
    import torch

    w = W.three_plane()
    dep = torch.from_numpy(w["depos"]).to(dev)
    n = dep.shape[0]
    planes, outs, wsps, scheds = [], [], [], []
    for pl, R in zip(w["planes"], w["responses"]):
        sched = tuner.tune(pl, w["phys"], R, dep) if tuner is not None else None
        P = wcsim.Plane(pl, w["phys"], R, schedule=sched)
        planes.append(P)
        scheds.append(sched or {})
        outs.append(torch.empty((P.nwires, P.nticks), dtype=torch.float32, device=dev))
        wsps.append(wcsim.simulate_workspace(P, n, wcsim.OUT_WIRE, dev))

    def step():
        for P, o, ws in zip(planes, outs, wsps):
            wcsim.simulate_event(P, dep, w["event_id"], out=o, workspace=ws)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for P in planes:
        P.destroy()
    return {"ms_per_event": dt * 1e3, "depos_per_s": n / dt, "depo_planes_per_s": 3 * n / dt,
            "planes_per_s": 3 / dt, "depos": int(n), "schedules": scheds}


def serve_measurement(W, nreq: int, tuner=None) -> dict:
    """The serving workload (requests of 1-3 planes of 100-960 wires x 6000
    ticks, depo counts log-uniform in 10^3..2x10^6): saturated throughput
    (all requests at t = 0), then Poisson arrivals at fractions of it.  With
    a tuner, one schedule tuned on a representative plane (480 wires, 200,000
    track depos) serves every plane of the same tick count and response
    shape, so that requests still group into one batch class."""
    import torch

    from paper_2304_01841_amd import serve

    reqs = W.serve_requests(nreq=nreq)
    phys = W.physics(True)
    schedule_for, sched = None, None
    if tuner is not None:
        rng = np.random.default_rng(6000)
        rep_plane = W.plane(480, 6000)
        rep_resp = W.response("unipolar")
        rep_dep = W.clipped_track_depos(rng, 200_000, (W.BOX_X, W.BOX_Y, 480 * W.PITCH))
        sched = tuner.tune(rep_plane, phys, rep_resp, torch.from_numpy(rep_dep).cuda())
        shape = (6000, rep_resp.shape)

        def schedule_for(desc, response):
            return sched if (desc["nticks"], np.shape(response)) == shape else None
    srv = serve.Server(phys, hbm_budget=64 << 30, slots=4, max_batch=8,
                       schedule_for=schedule_for)
    srv.serve(reqs)  # plane set-up and (pinned) allocator warm-up for every request size
    sat = serve.latency_summary(srv.serve(reqs))
    out = {"requests": nreq, "budget_gb": 64, "slots": 4, "max_group": 8, "schedule": sched,
           "depos": int(sum(r["depos"].shape[0] for r in reqs)),
           "planes": int(sum(len(r["planes"]) for r in reqs)), "saturated": sat}
    rate = sat["throughput_rps"]
    for frac in (0.5, 0.8, 0.95):
        arr = W.poisson_arrivals(77, nreq, frac * rate)
        out["qps_%.2f" % frac] = dict(serve.latency_summary(srv.serve(reqs, arr)),
                                      offered_rps=frac * rate)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (events and "
              "planes would shard with no communication); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2304_01841_amd import wcsim
    from paper_2304_01841_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.collection()
    if args.lifetime:
        w["phys"] = dict(w["phys"], lifetime=args.lifetime)
    pl, R = w["planes"][0], w["responses"][0]
    kind = wcsim.OUT_WIRE if args.kind == "wire" else wcsim.OUT_PITCH
    dep = torch.from_numpy(w["depos"]).to(dev)
    tuner, tuning, sched = None, None, None
    if args.schedule:
        if args.schedule.lstrip().startswith("{"):
            sched = json.loads(args.schedule)
        else:
            sched = {k: int(v) for k, v in (kv.split("=") for kv in args.schedule.split(","))}
    elif not args.no_tune:
        from paper_2304_01841_amd import autotune
        tuner = autotune.Tuner()
        sched = tuner.tune(pl, w["phys"], R, dep, kind=kind)
        key = autotune.cache_key(pl, R, R.shape[0] // 2, w["phys"]["fluctuate"], dep.shape[0],
                                 kind)
        tuning = dict(tuner.entry(key))
    P = wcsim.Plane(pl, w["phys"], R, schedule=sched)
    n = dep.shape[0]
    nout = P.out_rows(kind)
    out = torch.empty((nout, P.nticks), dtype=torch.float32, device=dev)
    wsp = wcsim.simulate_workspace(P, n, kind, dev)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for i in range(args.warmup):
        wcsim.simulate_event(P, dep, w["event_id"], out=out, kind=kind, workspace=wsp)
    torch.cuda.synchronize()

    K = args.steps
    ev = wcsim.HipEvents(K * wcsim.NUM_STAGE_EVENTS)
    NE = wcsim.NUM_STAGE_EVENTS
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        wcsim.simulate_event_profiled(P, dep, w["event_id"], out, kind, wsp,
                                      ev.handles[i * NE:(i + 1) * NE], stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    lat = np.array([ev.elapsed_ms(i * NE, i * NE + NE - 1) for i in range(K)])
    stages = {}
    for j, name in enumerate(wcsim.STAGE_NAMES):
        stages[name] = float(np.mean([ev.elapsed_ms(i * NE + j, i * NE + j + 1) for i in range(K)]))
    ev.destroy()

    ms_per_step = wall * 1e3 / K
    depos_per_s = n * K / wall
    planes_per_s = K / wall

    # Dominant stage: the longest.  The fluctuating raster kernel is bound by
    # plain VALU arithmetic (no stage is a dense contraction); the FFT passes
    # are reported against HBM.
    alg = algorithmic_bytes(P, nout, n)
    eff = {k: int(P.info[k]) for k in ("fft_ticks", "fft_pitch", "freq_chunk", "tile")}
    dom = max(("raster_tiles", "fft_ticks", "conv_pitch", "ifft_ticks"), key=lambda s: stages[s])
    kernel_of = {"raster_tiles": "k_raster_tiles", "fft_ticks": "k_rows_r2c",
                 "conv_pitch": "k_pitch_conv", "ifft_ticks": "k_rows_c2r"}
    if dom == "raster_tiles":
        work = raster_work(wcsim, P, dep)
        achieved = work["ops"] / (stages[dom] * 1e-3) / 1e12
        roofline = {"kernel": kernel_of[dom], "bound": "alu", "achieved": achieved,
                    "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS,
                    "traffic": measured_traffic(kernel_of[dom], eff), "algorithmic_ops": work["ops"],
                    "philox_calls": work["philox_calls"], "bins": work["bins"],
                    "avg_ms": stages[dom]}
    else:
        achieved = alg[dom] / (stages[dom] * 1e-3) / 1e9
        roofline = {"kernel": kernel_of[dom], "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic(kernel_of[dom], eff), "algorithmic_bytes": alg[dom],
                    "avg_ms": stages[dom]}
    per_stage_hbm = {s: alg[s] / (stages[s] * 1e-3) / 1e9 for s in alg if stages.get(s, 0) > 0}

    batch = None
    if not args.no_batch:
        batch = batch_comparison(wcsim, W, dev, args.batch_events, tuner)

    digit = digitize_measurement(wcsim, out)

    three = None
    if not args.no_three_plane:
        three = three_plane_measurement(wcsim, W, dev, tuner)

    served = None
    if not args.no_serve:
        served = serve_measurement(W, args.serve_requests, tuner)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, kind == wcsim.OUT_WIRE)

    line = {
        "metric": "depos/sec and planes/sec on 1 GPU (batched vs plain); p50/p99 event latency",
        "value": depos_per_s,
        "unit": "depos/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 windows)",
        "data": "synthetic",
        "config": {"workload": "collection plane 960 wires x 10 impact x 6000 ticks, 500000 "
                               "track depos, Philox fluctuation, 210x200 response, plain "
                               "per-event launch, %s output%s" % (
                                   args.kind, ", electron lifetime %g us" % args.lifetime
                                   if args.lifetime else ""),
                   "global_batch": 1, "depos_per_event": n,
                   "fft_ticks": P.info["fft_ticks"], "fft_pitch": P.info["fft_pitch"],
                   "freq_chunk": P.info["freq_chunk"], "tile": P.info["tile"],
                   "schedule": ("fixed" if args.schedule else
                                "autotuned" if tuning else "library default")},
        "tuning": tuning,
        "planes_per_s": planes_per_s,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(lat.mean())},
        "stage_ms": stages,
        "stage_hbm_gbs": per_stage_hbm,
        "roofline": roofline,
        "three_plane": three,
        "digitize": digit,
        "batch": batch,
        "serve": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    P.destroy()


if __name__ == "__main__":
    main()
