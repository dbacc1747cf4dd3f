#!/usr/bin/env python3
"""Benchmark of the LArTPC signal-simulation hot path on one MI355X.

A step is one batch of the batched workload (arXiv:2304.01841, Sec. 2: per
event, rasterize with fluctuation, scatter-add into the plane grid, FFT
convolution with the response, wire output): 64 single-plane events of uneven
size (depo counts log-uniform in 10^4..10^6, 100/480/800/960 wires x 10 impact
bins x 6000 ticks, track-structured depos, Philox fluctuation, 210 x 200
collection responses), all depos resident in HBM, run by the batched form
(``wcsim_simulate_batch``: chunks of events pipelined over two streams, with
autotuned schedules).  The headline is that form's depos/s; beside it the same
64 events as plain per-event launches on the same planes (one stream, same
schedules, so only batching differs), the captured-graph replay of the batch,
the detector-scale collection plane and the three-plane event as plain
events, the served form against its per-request baseline, digitisation, and
the FP64 oracle timed on the host.

Prints one JSON line.  The roofline of the dominant kernel of the step is
measured live: HIP events recorded on the stream each kernel is launched on,
around every launch in the timed steps (the paper's per-kernel timers,
Sec. 5.2), against the kernel's algorithmic work.
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
KERNEL_OF = {"raster_tiles": "k_raster_tiles", "fft_ticks": "k_rows_r2c",
             "conv_pitch": "k_pitch_conv", "ifft_ticks": "k_rows_c2r",
             "bin_depos": "k_fill_records"}
METRIC = "depos/sec and planes/sec on 1 GPU (batched vs plain); p50/p99 event latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed batches")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch-events", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form measurement")
    ap.add_argument("--serve-requests", type=int, default=64)
    ap.add_argument("--no-three-plane", action="store_true",
                    help="skip the three-plane (U/V/W, 2.4M depos) event measurement")
    ap.add_argument("--no-collection", action="store_true",
                    help="skip the collection-plane (960 wires, 500k depos) measurement")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain per-event run of the batch workload")
    ap.add_argument("--no-tune", action="store_true",
                    help="library default schedules instead of autotuned ones")
    ap.add_argument("--tune-cache", type=str, default=None,
                    help="JSON file of the schedule tuner (read, and written on a miss)")
    ap.add_argument("--lifetime", type=float, default=0.0, metavar="US",
                    help="electron lifetime (an extension beyond the paper; 0, the default, is "
                         "the paper's workload without absorption)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB (a plain copy kernel "
                         "whose HBM counters scale the kernels' FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# Algorithmic work of each kernel (per plane event)
# ---------------------------------------------------------------------------
def algorithmic_bytes(P, nout: int, n_depos: int) -> dict:
    """Minimum HBM bytes of each stage at the minimum transform sizes:
    H = floor((Nt + Rt - 1) / 2) + 1 frequencies per row; the grid written
    once; the spectrum written by the tick pass and read by the pitch pass;
    the kept rows written by the pitch pass and read by the inverse pass."""
    Np, Nt = P.npitch, P.nticks
    Rt = P._resp.shape[1]
    H = (Nt + Rt - 1) // 2 + 1
    # resident response spectrum read by the pitch pass: L rows per column for
    # the overlap-save blocks, nimpact phases of 128 for the polyphase wire pass
    if P.info["wire_polyphase"] and nout == P.nwires and nout != Np:
        spectrum_rows = P.info["nimpact"] * 128
    else:
        spectrum_rows = P.info["fft_pitch"]
    return {
        "raster_tiles": 40 * n_depos + 4 * Np * Nt,
        "fft_ticks": 4 * Np * Nt + 8 * Np * H,
        "conv_pitch": 8 * Np * H + 8 * spectrum_rows * H + 8 * nout * H,
        "ifft_ticks": 8 * nout * H + 4 * nout * Nt,
    }


def raster_work(wcsim, P, dep, event_id=0) -> dict:
    """Bins and Philox calls of every patch, from the windows the library's
    own rasterizer returns (outside the timed region)."""
    pt = wcsim.rasterize(P, dep, event_id)
    meta, offs, _ = pt.to_host(values=False)
    pt.destroy()
    lo_t, n_p, n_t = (meta[:, k].astype(np.int64) for k in (1, 2, 3))
    live = n_p > 0
    quads = np.where(live, np.floor_divide(lo_t + n_t - 1, 4) - np.floor_divide(lo_t, 4) + 1, 0)
    calls = int(np.sum(n_p * quads))
    bins = int(np.sum(n_p * n_t))
    return {"philox_calls": calls, "bins": bins,
            "ops": calls * OPS_PER_PHILOX_CALL + bins * OPS_PER_BIN}


def roofline_of(kernel_stage: str, total_ms: float, launches: int, work: dict) -> dict:
    """Roofline object of one kernel: its algorithmic work summed over the
    launches, over its summed event-measured duration."""
    kern = KERNEL_OF[kernel_stage]
    avg_ms = total_ms / max(launches, 1)
    if kernel_stage == "raster_tiles":
        ops = work["ops"]
        achieved = ops / (total_ms * 1e-3) / 1e12
        return {"kernel": kern, "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS, "traffic": None,
                "algorithmic_ops_per_launch": ops / max(launches, 1),
                "philox_calls": work["philox_calls"], "bins": work["bins"],
                "launches": launches, "avg_ms": avg_ms}
    nbytes = work["bytes"][kernel_stage]
    achieved = nbytes / (total_ms * 1e-3) / 1e9
    return {"kernel": kern, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": nbytes / max(launches, 1), "launches": launches,
            "avg_ms": avg_ms}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel), or None
    when it is missing or the kernel's source changed since it was taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    k = rec.get(workload, {}).get("kernels", {}).get(kernel)
    if not k:
        return None
    digest = hashlib.sha256(open(os.path.join(ROOT, k["source"]), "rb").read()).hexdigest()
    return k["bytes_per_launch"] if digest == k["source_sha256"] else None


# ---------------------------------------------------------------------------
# Workload set-up
# ---------------------------------------------------------------------------
def tuned_plane(wcsim, tuner, plane, phys, resp, dep):
    sched = tuner.tune(plane, phys, resp, dep) if tuner is not None else None
    return wcsim.Plane(plane, phys, resp, schedule=sched), (sched or {})


def batch_setup(wcsim, W, dev, nevents, phys, tuner):
    """The batch workload's events and one tuned plane per wire count, tuned on
    all of that wire count's events run together through the batched form."""
    import torch

    evs = W.batch_events(nevents=nevents)
    planes, schedules = {}, {}
    for nw in sorted({e["plane"]["nwires"] for e in evs}):
        mine = sorted((e for e in evs if e["plane"]["nwires"] == nw),
                      key=lambda e: e["depos"].shape[0])
        e = mine[len(mine) // 2]
        sched = None
        if tuner is not None:
            sched = tuner.tune_batch(e["plane"], phys, e["response"],
                                     [torch.from_numpy(x["depos"]).to(dev) for x in mine])
        planes[nw] = wcsim.Plane(e["plane"], phys, e["response"], schedule=sched)
        schedules[nw] = sched or {}
    pl = [planes[e["plane"]["nwires"]] for e in evs]
    deps = [torch.from_numpy(e["depos"]).to(dev) for e in evs]
    ids = [e["event_id"] for e in evs]
    return evs, planes, schedules, pl, deps, ids


# ---------------------------------------------------------------------------
# Measurements
# ---------------------------------------------------------------------------
def measure_batched(wcsim, pl, deps, ids, outs, steps, warmup):
    """The batched form, `steps` timed batches between synchronisations, with
    the per-chunk stage events; then the captured graph of the same batch."""
    import torch

    ns = [d.shape[0] for d in deps]
    nch = wcsim.batch_chunk_count(pl, ns)
    NE = wcsim.BATCH_STAGE_EVENTS
    wsp = wcsim.batch_workspace(pl, ns)
    ev = wcsim.HipEvents(steps * nch * NE)
    for _ in range(warmup):
        wcsim.simulate_batch(pl, deps, ids, outs, workspace=wsp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        wcsim.simulate_batch_profiled(pl, deps, ids, outs,
                                      ev.handles[s * nch * NE:(s + 1) * nch * NE], workspace=wsp)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # stage durations summed over chunks, averaged over steps
    names = {"bin_depos": (0, 1), "raster_tiles": (1, 2), "raster_large": (2, 3),
             "fft_ticks": (4, 5), "conv_pitch": (5, 6), "ifft_ticks": (8, 7)}
    stage = {k: 0.0 for k in names}
    step_ms = []
    for s in range(steps):
        base = s * nch * NE
        for c in range(nch):
            b = base + c * NE
            for k, (i, j) in names.items():
                stage[k] += ev.elapsed_ms(b + i, b + j)
        step_ms.append(ev.elapsed_ms(base, base + (nch - 1) * NE + 7))
    ev.destroy()
    stage = {k: v / steps for k, v in stage.items()}
    del wsp
    # the captured graph of the same batch
    batch = wcsim.Batch(pl, ns)
    for _ in range(max(warmup, 1)):
        batch.run(deps, ids, outs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        batch.run(deps, ids, outs)
    torch.cuda.synchronize()
    graph_wall = time.perf_counter() - t1
    batch.destroy()
    return {"wall_s": wall, "ms_per_step": wall * 1e3 / steps, "chunks": nch,
            "stage_ms_per_step": stage, "launches_per_step": nch,
            "event_ms_p50": float(np.percentile(step_ms, 50)),
            "graph_ms_per_step": graph_wall * 1e3 / steps}


def measure_plain(wcsim, pl, deps, ids, outs, rounds):
    """The same events as plain per-event launches on one stream (same planes
    and schedules), each event bracketed by HIP events for its latency."""
    import torch

    need = max(wcsim._lib.wcsim_simulate_workspace_bytes(p.handle, d.shape[0], 0)
               for p, d in zip(pl, deps))
    wsp = torch.empty(need, dtype=torch.uint8, device=deps[0].device)
    stream = torch.cuda.current_stream()
    NE = wcsim.NUM_STAGE_EVENTS
    ne = len(pl)
    for p, d, i, o in zip(pl, deps, ids, outs):
        wcsim.simulate_event(p, d, i, out=o, workspace=wsp)
    torch.cuda.synchronize()
    ev = wcsim.HipEvents(rounds * ne * NE)
    t0 = time.perf_counter()
    for r in range(rounds):
        for k, (p, d, i, o) in enumerate(zip(pl, deps, ids, outs)):
            h = ev.handles[(r * ne + k) * NE:(r * ne + k + 1) * NE]
            wcsim.simulate_event_profiled(p, d, i, o, 0, wsp, h, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([ev.elapsed_ms(j * NE, j * NE + NE - 1) for j in range(rounds * ne)])
    ev.destroy()
    return {"ms_per_batch": wall * 1e3 / rounds, "event_latency_ms":
            {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
             "mean": float(lat.mean())}}


def measure_event(wcsim, P, dep, event_id, steps, warmup, kind):
    """Plain events of one plane with the per-stage HIP events."""
    import torch

    n = dep.shape[0]
    out = torch.empty((P.out_rows(kind), P.nticks), dtype=torch.float32, device=dep.device)
    wsp = wcsim.simulate_workspace(P, n, kind, dep.device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        wcsim.simulate_event(P, dep, event_id, out=out, kind=kind, workspace=wsp)
    torch.cuda.synchronize()
    NE = wcsim.NUM_STAGE_EVENTS
    ev = wcsim.HipEvents(steps * NE)
    t0 = time.perf_counter()
    for i in range(steps):
        wcsim.simulate_event_profiled(P, dep, event_id, out, kind, wsp,
                                      ev.handles[i * NE:(i + 1) * NE], stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([ev.elapsed_ms(i * NE, i * NE + NE - 1) for i in range(steps)])
    stages = {name: float(np.mean([ev.elapsed_ms(i * NE + j, i * NE + j + 1)
                                   for i in range(steps)]))
              for j, name in enumerate(wcsim.STAGE_NAMES)}
    ev.destroy()
    return {"ms_per_event": wall * 1e3 / steps, "depos_per_s": n * steps / wall,
            "latency_ms": {"p50": float(np.percentile(lat, 50)),
                           "p99": float(np.percentile(lat, 99)), "mean": float(lat.mean())},
            "stage_ms": stages, "out": out}


def dominant(stages: dict) -> str:
    return max(("raster_tiles", "fft_ticks", "conv_pitch", "ifft_ticks", "bin_depos"),
               key=lambda s: stages.get(s, 0.0))


def event_roofline(wcsim, P, dep, event_id, stages, kind, workload):
    nout = P.out_rows(kind)
    dom = dominant(stages)
    work = {"bytes": algorithmic_bytes(P, nout, dep.shape[0])}
    if dom == "raster_tiles":
        work.update(raster_work(wcsim, P, dep, event_id))
    if dom == "bin_depos":
        dom = "raster_tiles" if stages["raster_tiles"] else "fft_ticks"
        if dom == "raster_tiles":
            work.update(raster_work(wcsim, P, dep, event_id))
    r = roofline_of(dom, stages[dom], 1, work)
    r["traffic"] = measured_traffic(r["kernel"], workload)
    return r


def digitize_measurement(wcsim, out, reps: int = 20) -> dict:
    """Digitisation with noise (an extension beyond the paper) of a collection
    plane's output: time per call and HBM rate (4 B read + 2 B written per
    sample), HIP events on torch's current stream."""
    import torch

    codes = torch.empty(out.shape, dtype=torch.int16, device=out.device)
    fir = torch.exp(-torch.arange(64, dtype=torch.float32, device=out.device) / 9.0)
    res = {}
    for name, f in (("white", None), ("coloured_64tap", fir)):
        for _ in range(3):
            wcsim.digitize(out, 1.0, 2048.0, 3.0, 12, seed=7, event_id=0, out=codes, fir=f)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for e in range(reps):
            wcsim.digitize(out, 1.0, 2048.0, 3.0, 12, seed=7, event_id=e, out=codes, fir=f)
        t1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = t0.elapsed_time(t1) / reps
    n = out.numel()
    res.update(samples=int(n), hbm_gbs=6.0 * n / (res["white_ms"] * 1e-3) / 1e9)
    return res


def three_plane_measurement(wcsim, W, dev, phys_over, tuner, steps=5) -> dict:
    """The three-plane event (U/V/W 800/800/960 wires x 6000 ticks, 2,000,000
    track + 400,000 background depos, fluctuation on, wire output): the planes
    one after the other on one stream, depos resident, with the roofline of
    the dominant kernel summed over the three planes; and the three planes as
    one batched call (wall time per event, median of `steps`)."""
    import torch

    w = W.three_plane()
    phys = dict(w["phys"], **phys_over)
    dep = torch.from_numpy(w["depos"]).to(dev)
    n = dep.shape[0]
    planes, scheds, per = [], [], []
    for pl, R in zip(w["planes"], w["responses"]):
        P, s = tuned_plane(wcsim, tuner, pl, phys, R, dep)
        planes.append(P)
        scheds.append(s)
    total_ms = 0.0
    stages = {}
    for P in planes:
        m = measure_event(wcsim, P, dep, w["event_id"], steps, 1, wcsim.OUT_WIRE)
        per.append(m["ms_per_event"])
        total_ms += m["ms_per_event"]
        for k, v in m["stage_ms"].items():
            stages[k] = stages.get(k, 0.0) + v
    dom = dominant(stages)
    work = {"bytes": {k: 0 for k in ("raster_tiles", "fft_ticks", "conv_pitch", "ifft_ticks")},
            "ops": 0, "philox_calls": 0, "bins": 0}
    for P in planes:
        for k, v in algorithmic_bytes(P, P.nwires, n).items():
            work["bytes"][k] += v
        if dom in ("raster_tiles", "bin_depos"):
            rw = raster_work(wcsim, P, dep, w["event_id"])
            for k in ("ops", "philox_calls", "bins"):
                work[k] += rw[k]
    if dom == "bin_depos":
        dom = "raster_tiles"
    roof = roofline_of(dom, stages[dom], 3, work)
    # the same event's three planes as one batched call (the depos shared)
    deps3, ids3 = [dep] * 3, [w["event_id"]] * 3
    outs = [torch.empty((P.nwires, P.nticks), dtype=torch.float32, device=dev) for P in planes]
    wsp = wcsim.batch_workspace(planes, [n] * 3)
    wcsim.simulate_batch(planes, deps3, ids3, outs, workspace=wsp)
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        wcsim.simulate_batch(planes, deps3, ids3, outs, workspace=wsp)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    bms = 1e3 * float(np.median(ts))
    del wsp, outs
    for P in planes:
        P.destroy()
    return {"ms_per_event": total_ms, "depos_per_s": n / (total_ms * 1e-3),
            "depo_planes_per_s": 3 * n / (total_ms * 1e-3), "planes_per_s": 3 / (total_ms * 1e-3),
            "ms_per_plane": per, "depos": int(n), "schedules": scheds, "stage_ms": stages,
            "roofline": roof,
            "batched": {"ms_per_event": bms, "depos_per_s": n / (bms * 1e-3),
                        "planes_per_s": 3 / (bms * 1e-3)}}


def serve_measurement(W, nreq: int, phys, tuner=None) -> dict:
    """The serving workload (requests of 1-3 planes of 100-960 wires x 6000
    ticks, depo counts log-uniform in 10^3..2x10^6): the per-request baseline
    and the continuous-batching server, saturated (all requests at t = 0) and
    under Poisson arrivals at fractions of the baseline's saturated rate (so
    that both serve the same offered load), p50/p99 latency beside depos/s."""
    import torch

    from paper_2304_01841_amd import serve

    reqs = W.serve_requests(nreq=nreq)
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
    srv.serve_plain(reqs[:4])
    out = {"requests": nreq, "budget_gb": 64, "slots": 4, "max_group": 8, "queue_depth": 2,
           "schedule": sched, "depos": int(sum(r["depos"].shape[0] for r in reqs)),
           "planes": int(sum(len(r["planes"]) for r in reqs))}
    plain = serve.latency_summary(srv.serve_plain(reqs), reqs)
    served = serve.latency_summary(srv.serve(reqs), reqs)
    out["saturated"] = {"plain": plain, "served": served,
                        "speedup": served["depos_per_s"] / plain["depos_per_s"]}
    rate = plain["throughput_rps"]
    for frac in (0.5, 0.8, 0.95):
        arr = W.poisson_arrivals(77, nreq, frac * rate)
        out["load_%.2f" % frac] = {
            "offered_rps": frac * rate,
            "plain": serve.latency_summary(srv.serve_plain(reqs, arr), reqs),
            "served": serve.latency_summary(srv.serve(reqs, arr), reqs)}
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on the host's cores
# ---------------------------------------------------------------------------
def cpu_baseline(W, phys_over, nevents: int) -> dict:
    """The FP64 oracle (rasterize + scatter in C, convolution with scipy) on a
    bounded sample of the batch workload: the first events of the batch until
    about 1.5 million depos.  The oracle is run as it stands: each event's
    depos are split into one contiguous part per core and rasterized by that
    many threads at once (the C calls release the interpreter lock; each part
    keyed by its depos' event indices, so the fluctuation is the event's), the
    patches scattered into one grid, and the convolution given every core.
    Also one core on the sample's first event."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as O

    O.build()
    cores = max(1, min(16, os.cpu_count() or 1))
    evs = W.batch_events(nevents=nevents)
    sample, tot = [], 0
    for e in evs:
        sample.append(e)
        tot += e["depos"].shape[0]
        if tot >= 1_500_000:
            break
    phys = dict(W.physics(True), **phys_over)
    with ThreadPoolExecutor(cores) as pool:
        t0 = time.perf_counter()
        for e in sample:
            dep, pl, R, ev = e["depos"], e["plane"], e["response"], e["event_id"]
            parts = np.array_split(np.arange(dep.shape[0]), cores)
            res = list(pool.map(lambda p: O.rasterize(dep[p], phys, pl, ev, ids=p), parts))
            shift = np.cumsum([0] + [v.size for _, v, _ in res[:-1]])
            meta = np.concatenate([m + np.array([0, 0, 0, 0, s]) for (m, _, _), s in
                                   zip(res, shift)])
            G = O.scatter(meta, np.concatenate([v for _, v, _ in res]), pl)
            out = O.wire_rows(O.convolve(G, R.astype(np.float64), R.shape[0] // 2,
                                         workers=cores), pl["nimpact"])
            assert np.isfinite(out).all()
        dt = time.perf_counter() - t0
    e = sample[0]
    t1 = time.perf_counter()
    O.simulate_event(e["depos"], phys, e["plane"], e["response"].astype(np.float64),
                     e["response"].shape[0] // 2, e["event_id"], wire_output=True, workers=1)
    dt1 = time.perf_counter() - t1
    return {"value": tot / dt, "unit": "depos/s", "cores": cores, "kind": "oracle",
            "sample": "first %d events of the 64-event batch workload (%d depos, %d planes) in "
                      "%.2f s: %d rasterizing threads (one depo part each), one scatter, a "
                      "%d-thread FFT; one core on the first event (%d depos): %.3g depos/s"
                      % (len(sample), tot, len(sample), dt, cores, cores,
                         e["depos"].shape[0], e["depos"].shape[0] / dt1),
            "single_core_depos_per_s": e["depos"].shape[0] / dt1}


# ---------------------------------------------------------------------------
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
    phys_over = {"lifetime": args.lifetime} if args.lifetime else {}
    phys = dict(W.physics(True), **phys_over)
    tuner = None
    if not args.no_tune:
        from paper_2304_01841_amd import autotune
        tuner = autotune.Tuner(args.tune_cache)

    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # -- headline: the batch workload, batched form -------------------------
    evs, planes, schedules, pl, deps, ids = batch_setup(wcsim, W, dev, args.batch_events, phys,
                                                        tuner)
    outs = [torch.empty((p.nwires, p.nticks), dtype=torch.float32, device=dev) for p in pl]
    ntot = int(sum(d.shape[0] for d in deps))
    K = args.steps
    bat = measure_batched(wcsim, pl, deps, ids, outs, K, args.warmup)
    ms_per_step = bat["ms_per_step"]
    value = ntot / (ms_per_step * 1e-3)

    # roofline of the step's dominant kernel over the timed batches
    st = bat["stage_ms_per_step"]
    dom = dominant(st)
    work = {"bytes": {k: 0 for k in ("raster_tiles", "fft_ticks", "conv_pitch", "ifft_ticks")}}
    for p, d in zip(pl, deps):
        for k, v in algorithmic_bytes(p, p.nwires, d.shape[0]).items():
            work["bytes"][k] += v
    if dom in ("raster_tiles", "bin_depos"):
        dom = "raster_tiles"
        work.update(ops=0, philox_calls=0, bins=0)
        for p, d, i in zip(pl, deps, ids):
            rw = raster_work(wcsim, p, d, i)
            for k in ("ops", "philox_calls", "bins"):
                work[k] += rw[k]
    roofline = roofline_of(dom, st[dom], bat["launches_per_step"], work)
    roofline["traffic"] = measured_traffic(roofline["kernel"], "batch")

    plain = None
    if not args.no_plain:
        plain = measure_plain(wcsim, pl, deps, ids, outs, max(2, K // 3))
        plain["depos_per_s"] = ntot / (plain["ms_per_batch"] * 1e-3)
        plain["planes_per_s"] = len(pl) / (plain["ms_per_batch"] * 1e-3)

    # -- the collection plane and the three-plane event (plain events) ------
    coll = None
    digit = None
    if not args.no_collection:
        w = W.collection()
        cphys = dict(w["phys"], **phys_over)
        cdep = torch.from_numpy(w["depos"]).to(dev)
        P, csched = tuned_plane(wcsim, tuner, w["planes"][0], cphys, w["responses"][0], cdep)
        m = measure_event(wcsim, P, cdep, w["event_id"], 20, 3, wcsim.OUT_WIRE)
        coll = {k: v for k, v in m.items() if k != "out"}
        coll.update(planes_per_s=1e3 / m["ms_per_event"], schedule=csched,
                    depos=int(cdep.shape[0]),
                    roofline=event_roofline(wcsim, P, cdep, w["event_id"], m["stage_ms"],
                                            wcsim.OUT_WIRE, "collection"))
        digit = digitize_measurement(wcsim, m["out"])
        P.destroy()
    three = None
    if not args.no_three_plane:
        three = three_plane_measurement(wcsim, W, dev, phys_over, tuner)
    served = None
    if not args.no_serve:
        served = serve_measurement(W, args.serve_requests, phys, tuner)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, phys_over, args.batch_events)

    batch = {"events": len(pl), "depos": ntot, "chunks": bat["chunks"],
             "batched": {"ms_per_batch": ms_per_step, "depos_per_s": value,
                         "planes_per_s": len(pl) / (ms_per_step * 1e-3),
                         "stage_ms_per_batch": st},
             "graph": {"ms_per_batch": bat["graph_ms_per_step"],
                       "depos_per_s": ntot / (bat["graph_ms_per_step"] * 1e-3)},
             "plain": plain,
             "speedup_vs_plain": (plain["ms_per_batch"] / ms_per_step) if plain else None,
             "schedules": {str(k): v for k, v in schedules.items()}}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "depos/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (f64 windows, erf weights, normalisation and patch totals)",
        "data": "synthetic",
        "config": {"workload": "batch of 64 single-plane events: depo counts log-uniform in "
                               "1e4-1e6 (%d depos), 100/480/800/960 wires x 10 impact x 6000 "
                               "ticks, track depos, Philox fluctuation, 210x200 collection "
                               "response, wire output, batched form (chunks pipelined over two "
                               "streams), autotuned schedules%s" % (
                                   ntot, ", electron lifetime %g us" % args.lifetime
                                   if args.lifetime else ""),
                   "global_batch": len(pl), "depos_per_batch": ntot,
                   "schedule": "library default" if args.no_tune else "autotuned"},
        "planes_per_s": len(pl) / (ms_per_step * 1e-3),
        "latency_ms": {"batch_p50": bat["event_ms_p50"],
                       "plain_event": plain["event_latency_ms"] if plain else None},
        "roofline": roofline,
        "batch": batch,
        "collection": coll,
        "three_plane": three,
        "digitize": digit,
        "serve": served,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
