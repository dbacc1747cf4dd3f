"""Continuous-batching server for DepoTransform requests on one GPU.

A request is a depo set and 1-3 planes (each with its response); its result is
the wire waveform of every plane.  The server keeps one plane object per
(wire count, plane id, response) resident, all planes of one response sharing
one resident response spectrum, and runs a scheduling loop:

* requests join a FIFO at their arrival time;
* whenever a stream slot is free, every arrived request that fits the HBM
  budget (its workspace, depos and outputs) is admitted, up to `max_batch`,
  and the whole group runs as one batched launch sequence
  (``wcsim_simulate_batch``) on that slot's stream, followed by the copies of
  its outputs to pinned host memory;
* slots and budget are released when a group's completion event fires.

Groups on different slots overlap on the device, and a request that arrives
while others run is admitted as soon as a slot and memory free up.  Latency is
measured from a request's arrival to its results being in host memory.  All
device memory comes from torch's caching allocator on the slot's stream.
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


class Server:
    def __init__(self, phys: dict, device="cuda", hbm_budget: int = 64 << 30, slots: int = 4,
                 max_batch: int = 8, kind: int = wcsim.OUT_WIRE, schedule_for=None):
        self.phys = dict(phys)
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
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
    def serve(self, requests: list[dict], arrivals=None, poll_s: float = 20e-6) -> list[Result]:
        """Run `requests` (dicts with planes, responses, depos, event_id)
        arriving at `arrivals` seconds after the start (None: all at once)."""
        nreq = len(requests)
        if arrivals is None:
            arrivals = np.zeros(nreq)
        order = np.argsort(arrivals, kind="stable")
        # resolve planes and sizes up front (plane set-up is not serving work)
        prepared = []
        for r in requests:
            planes = [self.plane(d, R) for d, R in zip(r["planes"], r["responses"])]
            n = int(r["depos"].shape[0])
            prepared.append((planes, n, self.request_bytes(planes, n)))
        results = [Result(rid=i) for i in range(nreq)]
        pending = []  # request ids that have arrived, FIFO
        nxt = 0       # next index into `order` not yet arrived
        inflight = []  # (event, slot, rids, bytes, keep)
        free_slots = list(range(len(self.streams)))
        used = 0
        finished = 0
        t0 = time.perf_counter()
        while finished < nreq:
            now = time.perf_counter() - t0
            while nxt < nreq and arrivals[order[nxt]] <= now:
                rid = int(order[nxt])
                results[rid].arrival = float(arrivals[rid])
                if prepared[rid][2] > self.budget:
                    results[rid].error = "request needs more HBM than the budget"
                    results[rid].done = now
                    finished += 1
                else:
                    pending.append(rid)
                nxt += 1
            # completions
            still = []
            for ev, slot, rids, nbytes, keep in inflight:
                if ev.query():
                    tdone = time.perf_counter() - t0
                    for rid, host in zip(rids, keep["host"]):
                        results[rid].outputs = [h.numpy() for h in host]
                        results[rid].done = tdone
                    finished += len(rids)
                    used -= nbytes
                    free_slots.append(slot)
                else:
                    still.append((ev, slot, rids, nbytes, keep))
            inflight = still
            # admission: one group per free slot
            while free_slots and pending:
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
                slot = free_slots.pop(0)
                tadm = time.perf_counter() - t0
                for rid in group:
                    results[rid].admitted = tadm
                    results[rid].group_size = len(group)
                ev, keep = self._launch(group, requests, prepared, self.streams[slot])
                inflight.append((ev, slot, group, gbytes, keep))
                used += gbytes
                self.stats["groups"] += 1
                self.stats["max_group"] = max(self.stats["max_group"], len(group))
                self.stats["max_inflight_groups"] = max(self.stats["max_inflight_groups"],
                                                        len(inflight))
                self.stats["max_inflight_bytes"] = max(self.stats["max_inflight_bytes"], used)
            if finished < nreq:
                time.sleep(poll_s)
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


def latency_summary(results: list[Result]) -> dict:
    lat = np.array([r.latency for r in results if r.error is None])
    if lat.size == 0:
        return {}
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"requests": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_rps": float(lat.size / span) if span > 0 else None}
