"""Schedule autotuner for the plane kernels.

The schedule of a plane (padded tick-transform length, pitch block length and
frequency-chunk width of the overlap-save pass, LDS tile shape of the
rasterizer) changes only the speed of the path, never its result beyond the
stated tolerances.  Which schedule is fastest depends on the plane shape, the
response size and the depo density (the paper likewise treats launch geometry
as a tuning parameter, Sec. 5.3).  The tuner times a fixed candidate list with
the library's own timing entry point (`wcsim_tune_schedules`, HIP events on
the device) and keeps the winner in a JSON cache keyed by device architecture,
plane shape, response shape, fluctuation and the depo count's power of two.
"""
from __future__ import annotations

import json
import math
import os
import threading

import numpy as np
import torch

from . import wcsim

# Candidate schedules: the library default first, then the polyphase wire
# pass over 16- and 8-column chunks, then the compiled overlap-save block
# variants (block length x chunk width; 640 and 960 allow the folded
# wire-output inverse), crossed with the raster tile shapes.  The block
# length also sets the pitch-output pass of every candidate.
PITCH_CHOICES = ({}, {"freq_chunk": 16}, {"freq_chunk": 8},
                 {"fft_pitch": 512, "freq_chunk": 16, "wire_mode": 2},
                 {"fft_pitch": 1024, "freq_chunk": 16, "wire_mode": 2},
                 {"fft_pitch": 1024, "freq_chunk": 8, "wire_mode": 2},
                 {"fft_pitch": 640, "freq_chunk": 16, "wire_mode": 2},
                 {"fft_pitch": 960, "freq_chunk": 16, "wire_mode": 2})
TILE_CHOICES = (0, 1, 2)
TIE = 0.02  # relative timing difference treated as a tie


def candidates() -> list:
    out = []
    for p in PITCH_CHOICES:
        for t in TILE_CHOICES:
            c = dict(p)
            if t:
                c["tile"] = t
            out.append(c)
    return out


def arch() -> str:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def cache_key(plane: dict, response: np.ndarray, r0: int, fluctuate: bool, ndepos: int,
              kind: int, device_arch: str | None = None) -> str:
    Rp, Rt = np.shape(response)
    elec = plane.get("elec_response")
    if elec is not None and np.size(elec) > 0:
        Rt += int(np.size(elec)) - 1  # the plane convolves with response x electronics
    bucket = int(math.log2(ndepos)) if ndepos > 0 else -1
    return "%s|%dx%dx%d|R%dx%d@%d|fl%d|n2^%d|out%d" % (
        device_arch or arch(), int(plane["nwires"]), int(plane["nimpact"]), int(plane["nticks"]), Rp, Rt,
        int(r0), int(bool(fluctuate)), bucket, int(kind))


class Tuner:
    """Schedule cache (optionally backed by a JSON file) that tunes on a miss."""

    def __init__(self, path: str | None = None, reps: int = 9):
        self.path = path
        self.reps = reps
        self.table: dict = {}
        self._lock = threading.Lock()
        if path and os.path.exists(path):
            with open(path) as f:
                self.table = json.load(f)

    def lookup(self, plane: dict, response: np.ndarray, r0: int, fluctuate: bool, ndepos: int,
               kind: int = wcsim.OUT_WIRE) -> dict | None:
        e = self.table.get(cache_key(plane, response, r0, fluctuate, ndepos, kind))
        return None if e is None else dict(e["schedule"])

    def tune(self, plane: dict, phys: dict, response: np.ndarray, depos: torch.Tensor,
             r0: int | None = None, kind: int = wcsim.OUT_WIRE, stream=None) -> dict:
        """Best schedule for this plane shape and depo count (cached)."""
        if r0 is None:
            r0 = np.shape(response)[0] // 2
        key = cache_key(plane, response, r0, phys["fluctuate"], int(depos.shape[0]), kind)
        with self._lock:
            if key in self.table:
                return dict(self.table[key]["schedule"])
        cands = candidates()
        ms = wcsim.tune_schedules(plane, phys, response, depos, cands, r0=r0, kind=kind,
                                  reps=self.reps, stream=stream)
        return self._keep(key, cands, ms)

    def tune_batch(self, plane: dict, phys: dict, response: np.ndarray, depos_list: list,
                   r0: int | None = None, kind: int = wcsim.OUT_WIRE) -> dict:
        """Best schedule for a class of events of one plane shape that run together
        through the batched form (cached).  A single event can pick a schedule that
        fills the GPU alone but wastes it beside other events (a small plane's
        pitch pass, say); here every candidate's plane runs the whole class as one
        wcsim_simulate_batch and the median of `reps` runs, timed with HIP events
        on the current stream, decides."""
        if r0 is None:
            r0 = np.shape(response)[0] // 2
        ns = [int(d.shape[0]) for d in depos_list]
        key = "batch%d|" % len(ns) + cache_key(plane, response, r0, phys["fluctuate"], sum(ns), kind)
        with self._lock:
            if key in self.table:
                return dict(self.table[key]["schedule"])
        cands = candidates()
        ids = list(range(len(ns)))
        dev = depos_list[0].device
        ms = []
        for c in cands:
            try:
                P = wcsim.Plane(plane, phys, response, r0=r0, schedule=c)
            except wcsim.WcsimError:
                ms.append(-1.0)
                continue
            planes = [P] * len(ns)
            outs = [torch.empty((P.out_rows(kind), P.nticks), dtype=torch.float32, device=dev)
                    for _ in ns]
            ws = wcsim.batch_workspace(planes, ns, kind)
            wcsim.simulate_batch(planes, depos_list, ids, outs, kind=kind, workspace=ws)
            times = []
            for _ in range(self.reps):
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record()
                wcsim.simulate_batch(planes, depos_list, ids, outs, kind=kind, workspace=ws)
                t1.record()
                t1.synchronize()
                times.append(t0.elapsed_time(t1))
            ms.append(float(np.median(times)))
            del outs, ws
            P.destroy()
        return self._keep(key, cands, ms)

    def _keep(self, key: str, cands: list, ms: list) -> dict:
        # the first candidate (in list order) within TIE of the fastest, so that
        # timing noise does not flip between near-equal schedules
        timed = [(t, i) for i, t in enumerate(ms) if t >= 0.0]
        fastest = min(t for t, _ in timed)
        best_t, best_i = next((t, i) for t, i in timed if t <= fastest * (1.0 + TIE))
        entry = {"schedule": cands[best_i], "ms": best_t,
                 "default_ms": ms[0] if ms[0] >= 0.0 else None,
                 "candidates": [{"schedule": c, "ms": t} for c, t in zip(cands, ms)]}
        with self._lock:
            self.table[key] = entry
            if self.path:
                tmp = self.path + ".tmp"
                with open(tmp, "w") as f:
                    json.dump(self.table, f, indent=1, sort_keys=True)
                os.replace(tmp, self.path)
        return dict(entry["schedule"])

    def entry(self, key: str) -> dict | None:
        return self.table.get(key)
