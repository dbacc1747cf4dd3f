"""Continuous-batching server for DepoTransform requests on one GPU.

A request is a depo set and 1-3 planes (each with its response); its result is
the wire waveform of every plane.  The server keeps one plane object per
(wire count, plane id, response) resident, all planes of one response sharing
one resident response spectrum, and runs a scheduling loop:

* requests join a FIFO at their arrival time;
* a request whose depos the library would reject (non-finite fields,
  negative charge, behind a plane or unable to reach it) fails alone at
  arrival, before it can spoil a group;
* whenever a stream slot has room (fewer than `depth` groups queued on it),
  every arrived request that fits the HBM budget (its workspace, depos and
  outputs) is admitted, up to `max_batch`, and the whole group runs as one
  batched launch sequence (``wcsim_simulate_batch``) on that slot's stream,
  followed by the copies of its outputs to pinned host memory.  With
  `depth` = 2 the next group is already queued on the device behind the
  running one, so the device never waits for the host to notice a completion;
* slots and budget are released when a group's completion event fires;
* a client may cancel a request: before admission it leaves the queue, after
  admission its results are dropped when its group completes.

Groups on different slots overlap on the device, and a request that arrives
while others run is admitted as soon as a slot and memory free up.  Latency is
measured from a request's arrival to its results being in host memory.  All
device memory comes from torch's caching allocator on the slot's stream.

``serve_plain`` is the per-request baseline on the same request stream: one
request at a time in arrival order, each plane one ``wcsim_simulate_event``
on one stream.
"""
from __future__ import annotations

import hashlib
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import wcsim


@dataclass
class Result:
    rid: int
    outputs: list = field(default_factory=list)  # numpy [nwires][nticks] per plane
    arrival: float = 0.0
    admitted: float = 0.0
    done: float = 0.0
    error: str | None = None
    group_size: int = 0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def validate_request(req: dict, phys: dict) -> str | None:
    """Why the library would reject this request's host depos on one of its
    planes (the checks ``wcsim_simulate_event`` makes on host depos), or None."""
    d = np.asarray(req["depos"], np.float64)
    if d.ndim != 2 or d.shape[1] != 5:
        return "depos must be [n, 5]"
    if not np.isfinite(d).all():
        return "a depo has a non-finite field"
    if (d[:, 4] < 0).any():
        return "a depo has negative charge"
    v, a = float(phys["drift_speed"]), float(phys.get("drift_accel", 0.0))
    for pl in req["planes"]:
        L = d[:, 0] - float(pl["plane_x"])
        if (L < 0).any():
            return "a depo lies behind plane %d" % pl["plane_id"]
        if (v * v - 2.0 * a * L < 0).any():
            return "a depo cannot reach plane %d" % pl["plane_id"]
    return None


class Server:
    def __init__(self, phys: dict, device="cuda", hbm_budget: int = 64 << 30, slots: int = 4,
                 max_batch: int = 8, kind: int = wcsim.OUT_WIRE, schedule_for=None,
                 depth: int = 2):
        self.phys = dict(phys)
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.depth = int(depth)  # groups queued per slot
        self.kind = kind
        # default-priority streams, one per slot
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        # schedule_for(desc, response) -> schedule dict or None (library default),
        # e.g. from the autotuner's cache
        self.schedule_for = schedule_for
        self._planes: dict = {}
        self._donors: dict = {}
        self.stats = {"groups": 0, "max_group": 0, "max_inflight_groups": 0,
                      "max_inflight_bytes": 0}

    # -- resident planes ----------------------------------------------------
    def plane(self, desc: dict, response: np.ndarray) -> wcsim.Plane:
        rkey = hashlib.sha1(np.ascontiguousarray(response, np.float32).tobytes()).hexdigest()
        key = (rkey, desc["nwires"], desc["nimpact"], desc["nticks"], desc["plane_id"],
               desc["pitch"], desc["tick"], desc["t0"], desc["plane_x"], desc["dir_y"],
               desc["dir_z"], desc["pitch_origin"])
        p = self._planes.get(key)
        if p is None:
            sched = self.schedule_for(desc, response) if self.schedule_for else None
            # planes share a response spectrum only under the same schedule
            dkey = (rkey, tuple(sorted((sched or {}).items())))
            donor = self._donors.get(dkey)
            if donor is not None:
                p = wcsim.Plane(desc, self.phys, response, share=donor)
            else:
                p = wcsim.Plane(desc, self.phys, response, schedule=sched)
                self._donors[dkey] = p
            self._planes[key] = p
        return p

    def request_bytes(self, planes, n: int) -> int:
        """HBM the request holds while in flight: its share of the batch
        workspace, its depos and its device outputs."""
        arr_p = (wcsim.ctypes.c_void_p * len(planes))(*[p.handle.value for p in planes])
        arr_n = (wcsim.ctypes.c_int64 * len(planes))(*([n] * len(planes)))
        ws = wcsim._lib.wcsim_batch_workspace_bytes(arr_p, arr_n, len(planes), self.kind)
        outs = sum(4 * p.out_rows(self.kind) * p.nticks for p in planes)
        return int(ws + 40 * n + outs)

    # -- scheduling loop ----------------------------------------------------
    def serve(self, requests: list[dict], arrivals=None, poll_s: float = 20e-6,
              cancel_at: dict | None = None) -> list[Result]:
        """Run `requests` (dicts with planes, responses, depos, event_id)
        arriving at `arrivals` seconds after the start (None: all at once).
        `cancel_at` maps request ids to the time their client cancels."""
        nreq = len(requests)
        if arrivals is None:
            arrivals = np.zeros(nreq)
        cancel_at = dict(cancel_at or {})
        order = np.argsort(arrivals, kind="stable")
        # resolve planes and sizes up front (plane set-up is not serving work)
        prepared = []
        for r in requests:
            planes = [self.plane(d, R) for d, R in zip(r["planes"], r["responses"])]
            n = int(r["depos"].shape[0])
            prepared.append((planes, n, self.request_bytes(planes, n),
                             validate_request(r, self.phys)))
        results = [Result(rid=i) for i in range(nreq)]
        pending = []  # request ids that have arrived, FIFO
        nxt = 0       # next index into `order` not yet arrived
        inflight = []  # (event, slot, rids, bytes, keep), in launch order per slot
        queued = [0] * len(self.streams)
        used = 0
        finished = 0
        cancelled, arrived = set(), set()
        t0 = time.perf_counter()
        while finished < nreq:
            now = time.perf_counter() - t0
            while nxt < nreq and arrivals[order[nxt]] <= now:
                rid = int(order[nxt])
                arrived.add(rid)
                results[rid].arrival = float(arrivals[rid])
                err = prepared[rid][3]
                if err is None and prepared[rid][2] > self.budget:
                    err = "request needs more HBM than the budget"
                if err is not None:
                    results[rid].error = err
                    results[rid].done = now
                    finished += 1
                else:
                    pending.append(rid)
                nxt += 1
            # client cancellations (of arrived requests that have not finished)
            for rid, tc in list(cancel_at.items()):
                if tc > now or rid not in arrived:
                    continue
                del cancel_at[rid]
                if results[rid].error is not None or results[rid].done > 0:
                    continue
                cancelled.add(rid)
                if rid in pending:
                    pending.remove(rid)
                    results[rid].error = "cancelled"
                    results[rid].done = now
                    finished += 1
            # completions
            still = []
            for ev, slot, rids, nbytes, keep in inflight:
                if ev.query():
                    tdone = time.perf_counter() - t0
                    for rid, host in zip(rids, keep["host"]):
                        if rid in cancelled:
                            results[rid].error = "cancelled"
                        else:
                            results[rid].outputs = [h.numpy() for h in host]
                        results[rid].done = tdone
                    finished += len(rids)
                    used -= nbytes
                    queued[slot] -= 1
                else:
                    still.append((ev, slot, rids, nbytes, keep))
            inflight = still
            # admission: one group per slot with room in its queue
            while pending:
                slot = min(range(len(queued)), key=lambda k: queued[k])
                if queued[slot] >= self.depth:
                    break
                group, gbytes = [], 0
                for rid in pending:
                    b = prepared[rid][2]
                    if used + gbytes + b > self.budget:
                        break
                    group.append(rid)
                    gbytes += b
                    if len(group) == self.max_batch:
                        break
                if not group:
                    break
                pending = pending[len(group):]
                tadm = time.perf_counter() - t0
                for rid in group:
                    results[rid].admitted = tadm
                    results[rid].group_size = len(group)
                ev, keep = self._launch(group, requests, prepared, self.streams[slot])
                inflight.append((ev, slot, group, gbytes, keep))
                queued[slot] += 1
                used += gbytes
                self.stats["groups"] += 1
                self.stats["max_group"] = max(self.stats["max_group"], len(group))
                self.stats["max_inflight_groups"] = max(self.stats["max_inflight_groups"],
                                                        len(inflight))
                self.stats["max_inflight_bytes"] = max(self.stats["max_inflight_bytes"], used)
            if finished < nreq:
                time.sleep(poll_s)
        return results

    def serve_plain(self, requests: list[dict], arrivals=None) -> list[Result]:
        """Baseline on the same request stream: each request alone, in arrival
        order, its planes one wcsim_simulate_event each on one stream, results
        copied to pinned host memory before the next request starts."""
        nreq = len(requests)
        if arrivals is None:
            arrivals = np.zeros(nreq)
        order = np.argsort(arrivals, kind="stable")
        stream = self.streams[0]
        results = [Result(rid=i) for i in range(nreq)]
        prepared = [[self.plane(d, R) for d, R in zip(r["planes"], r["responses"])]
                    for r in requests]
        t0 = time.perf_counter()
        for rid in (int(k) for k in order):
            r = requests[rid]
            results[rid].arrival = float(arrivals[rid])
            while time.perf_counter() - t0 < arrivals[rid]:
                time.sleep(20e-6)
            results[rid].admitted = time.perf_counter() - t0
            err = validate_request(r, self.phys)
            if err is not None:
                results[rid].error = err
                results[rid].done = time.perf_counter() - t0
                continue
            with torch.cuda.stream(stream):
                hdep = torch.from_numpy(np.ascontiguousarray(r["depos"])).pin_memory()
                ddep = hdep.to(self.device, non_blocking=True)
                hosts = []
                for p in prepared[rid]:
                    o = wcsim.simulate_event(p, ddep, r["event_id"], kind=self.kind,
                                             stream=stream, device=self.device)
                    h = torch.empty(o.shape, dtype=torch.float32, pin_memory=True)
                    h.copy_(o, non_blocking=True)
                    hosts.append(h)
            stream.synchronize()
            results[rid].outputs = [h.numpy() for h in hosts]
            results[rid].done = time.perf_counter() - t0
            results[rid].group_size = 1
        return results

    def _launch(self, group, requests, prepared, stream):
        planes, deps, ids, outs, hosts = [], [], [], [], []
        with torch.cuda.stream(stream):
            for rid in group:
                r = requests[rid]
                pl = prepared[rid][0]
                hdep = torch.from_numpy(np.ascontiguousarray(r["depos"])).pin_memory()
                ddep = hdep.to(self.device, non_blocking=True)
                host = []
                for p in pl:
                    o = torch.empty((p.out_rows(self.kind), p.nticks), dtype=torch.float32,
                                    device=self.device)
                    planes.append(p)
                    deps.append(ddep)
                    ids.append(r["event_id"])
                    outs.append(o)
                    host.append(torch.empty(o.shape, dtype=torch.float32, pin_memory=True))
                hosts.append(host)
            ws = wcsim.batch_workspace(planes, [d.shape[0] for d in deps], self.kind, self.device)
            wcsim.simulate_batch(planes, deps, ids, outs, kind=self.kind, workspace=ws,
                                 stream=stream)
            k = 0
            for host in hosts:
                for h in host:
                    h.copy_(outs[k], non_blocking=True)
                    k += 1
            ev = torch.cuda.Event()
            ev.record(stream)
        # device tensors stay referenced until the group completes
        return ev, {"host": hosts, "dev": (deps, outs, ws)}


def latency_summary(results: list[Result], requests: list[dict] | None = None) -> dict:
    """p50/p99/mean latency and throughput of the successful requests; with
    `requests`, also depos/s and planes/s over the span from the first arrival
    to the last completion."""
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok])
    if lat.size == 0:
        return {}
    span = max(r.done for r in results) - min(r.arrival for r in results)
    out = {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
           "throughput_rps": float(lat.size / span) if span > 0 else None}
    if requests is not None and span > 0:
        out["depos_per_s"] = float(sum(requests[r.rid]["depos"].shape[0] for r in ok) / span)
        out["planes_per_s"] = float(sum(len(requests[r.rid]["planes"]) for r in ok) / span)
    return out
