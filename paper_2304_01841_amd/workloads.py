"""Seeded synthetic inputs for the LArTPC signal-simulation hot path.

This module only draws inputs: depo sets (rows of x, y, z, t, q in mm, us and
electrons), plane descriptors, physics constants and synthetic field responses.
It holds none of the simulation's arithmetic and is shared by the tests, the
benchmark, the HIP binding's callers and the oracle's callers alike.

The paper (Sec. 2) states only the orders of magnitude of the problem: patches
of about 20 x 20 bins, a grid of about 10^4 x 10^4 bins and a response of about
100 x 100 bins.  Its input depo sets and detector parameters are not published,
so every workload here is synthetic:

* ``small``     one plane of 100 wires x 10 impact bins x 1000 ticks, 1,000
                uniform depos with log-normal charge, no fluctuation;
* ``collection`` one collection plane of 960 wires x 10 impact bins x 6,000
                ticks, 500,000 depos on 200 straight 1.25 m tracks, fluctuation;
* ``three_plane`` U/V/W planes of 800/800/960 wires x 6,000 ticks, 2,000,000
                track depos plus 400,000 low-charge background depos;
* ``batch``     64 single-plane events of uneven depo count and wire count;
* ``serve``     a Poisson request stream of uneven sizes.
"""
from __future__ import annotations

import math

import numpy as np

# Physics common to every workload (units: mm, us, electrons).
DRIFT_SPEED = 1.6          # mm/us
D_L = 4.0e-4               # mm^2/us  (4 cm^2/s)
D_T = 8.8e-4               # mm^2/us  (8.8 cm^2/s)
NSIGMA = 3.0
PITCH = 5.0                # mm
NIMPACT = 10
TICK = 0.5                 # us
PHILOX_SEED = 0x2304018410
RESP_NPITCH, RESP_NTICKS, RESP_ORIGIN = 210, 200, 105

# Detector box of the track workloads (mm): x is the drift coordinate.
BOX_X, BOX_Y, BOX_Z = 4000.0, 1848.0, 4800.0

# Charge of a 0.5 mm step of a minimum-ionising track: 2.1 MeV/cm x 0.05 cm
# / 23.6 eV per pair x 0.8 recombination survival.
TRACK_DEPO_CHARGE = 0.105e6 / 23.6 * 0.8
TRACK_STEP = 0.5
TRACK_LENGTH = 1250.0


def physics(fluctuate: bool, seed: int = PHILOX_SEED) -> dict:
    return dict(drift_speed=DRIFT_SPEED, DL=D_L, DT=D_T, nsigma=NSIGMA,
                fluctuate=int(bool(fluctuate)), seed=int(seed))


def plane(nwires: int, nticks: int, plane_id: int = 0, dir_y: float = 0.0, dir_z: float = 1.0,
          pitch_origin: float = 0.0, nimpact: int = NIMPACT) -> dict:
    return dict(plane_id=int(plane_id), nwires=int(nwires), nimpact=int(nimpact),
                nticks=int(nticks), pitch=PITCH, tick=TICK, t0=0.0, plane_x=0.0,
                dir_y=float(dir_y), dir_z=float(dir_z), pitch_origin=float(pitch_origin))


def response(kind: str, sigma_t: float = 10.0, Rp: int = RESP_NPITCH, Rt: int = RESP_NTICKS,
             r0: int = RESP_ORIGIN, sigma_p: float = 10.0) -> np.ndarray:
    """Synthetic field response [Rp][Rt] (float32): a Gaussian in pitch times a
    bipolar (derivative-of-Gaussian, induction) or unipolar (Gaussian, unit
    sum, collection) shape in time."""
    r = np.arange(Rp, dtype=np.float64)[:, None]
    s = np.arange(Rt, dtype=np.float64)[None, :]
    c = Rt // 2
    pitch_prof = np.exp(-(r - r0) ** 2 / (2.0 * sigma_p ** 2))
    if kind == "bipolar":
        time_prof = -(s - c) / sigma_t * np.exp(-(s - c) ** 2 / (2.0 * sigma_t ** 2))
    elif kind == "unipolar":
        time_prof = np.exp(-(s - c) ** 2 / (2.0 * 8.0 ** 2))
        time_prof = time_prof / time_prof.sum()
    else:
        raise ValueError(kind)
    return np.ascontiguousarray((pitch_prof * time_prof).astype(np.float32))


def random_response(rng: np.random.Generator, Rp: int, Rt: int) -> np.ndarray:
    """Non-separable, non-symmetric response (for convolution tests)."""
    return np.ascontiguousarray(rng.standard_normal((Rp, Rt)).astype(np.float32))


# ---------------------------------------------------------------------------
# Depo generators
# ---------------------------------------------------------------------------
def uniform_depos(rng: np.random.Generator, n: int, z_range, t_window, max_drift_time=2500.0,
                  q_median=5000.0, q_sigma_ln=0.5, y_range=(0.0, BOX_Y)) -> np.ndarray:
    """Uniform depos: drift time uniform in [0, max_drift_time] (sets x), arrival
    time uniform in the readout window (sets t = arrival - drift time),
    log-normal charge."""
    T = rng.uniform(0.0, max_drift_time, n)
    x = DRIFT_SPEED * T
    y = rng.uniform(y_range[0], y_range[1], n)
    z = rng.uniform(z_range[0], z_range[1], n)
    arrival = rng.uniform(t_window[0], t_window[1], n)
    t = arrival - x / DRIFT_SPEED
    q = q_median * np.exp(q_sigma_ln * rng.standard_normal(n))
    return np.ascontiguousarray(np.stack([x, y, z, t, q], axis=1))


def track_depos(rng: np.random.Generator, nseg: int, per_seg: int = 2500,
                box=(BOX_X, BOX_Y, BOX_Z), step: float = TRACK_STEP,
                q: float = TRACK_DEPO_CHARGE) -> np.ndarray:
    """Straight segments of per_seg depos at `step` spacing (step midpoints),
    start uniform in the box, isotropic direction; segments that leave the box
    are redrawn.  All depos at t = 0."""
    length = per_seg * step
    bx, by, bz = box
    out = np.empty((nseg * per_seg, 5), np.float64)
    k = 0
    offs = (np.arange(per_seg, dtype=np.float64) + 0.5) * step
    while k < nseg:
        start = rng.uniform([0.0, 0.0, 0.0], [bx, by, bz])
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        end = start + length * v
        if not (0.0 <= end[0] <= bx and 0.0 <= end[1] < by and 0.0 <= end[2] < bz):
            continue
        pts = start[None, :] + offs[:, None] * v[None, :]
        sl = slice(k * per_seg, (k + 1) * per_seg)
        out[sl, 0:3] = pts
        out[sl, 3] = 0.0
        out[sl, 4] = q
        k += 1
    return out


def clipped_track_depos(rng: np.random.Generator, n: int, box, step: float = TRACK_STEP,
                        q: float = TRACK_DEPO_CHARGE, seg_len: float = TRACK_LENGTH) -> np.ndarray:
    """Exactly n track-structured depos in `box`: segments up to seg_len are
    clipped at the box faces and drawn until n depos exist."""
    bx, by, bz = box
    chunks = []
    have = 0
    while have < n:
        start = rng.uniform([0.0, 0.0, 0.0], [bx, by, bz])
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        # distance to the box boundary along v
        tmax = seg_len
        for a, hi in enumerate((bx, by, bz)):
            if v[a] > 0:
                tmax = min(tmax, (hi - start[a]) / v[a])
            elif v[a] < 0:
                tmax = min(tmax, -start[a] / v[a])
        m = int(tmax / step)
        if m <= 0:
            continue
        m = min(m, n - have)
        offs = (np.arange(m, dtype=np.float64) + 0.5) * step
        pts = start[None, :] + offs[:, None] * v[None, :]
        pts[:, 1] = np.minimum(pts[:, 1], np.nextafter(by, 0))
        pts[:, 2] = np.minimum(pts[:, 2], np.nextafter(bz, 0))
        c = np.empty((m, 5))
        c[:, 0:3] = pts
        c[:, 3] = 0.0
        c[:, 4] = q
        chunks.append(c)
        have += m
    return np.ascontiguousarray(np.concatenate(chunks, axis=0)[:n])


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------
def small(seed: int = 1000) -> dict:
    """1 plane, 100 wires x 10 impact bins = 1000 pitch bins x 1000 ticks,
    1,000 uniform depos, log-normal charge (median 5,000 e-), no fluctuation,
    bipolar response 210 x 200."""
    rng = np.random.default_rng(seed)
    pl = plane(100, 1000)
    dep = uniform_depos(rng, 1000, (0.0, 500.0), (0.0, 500.0))
    return dict(name="small", phys=physics(False), planes=[pl],
                responses=[response("bipolar")], depos=dep, event_id=0)


def collection(seed: int = 2000, nseg: int = 200, per_seg: int = 2500) -> dict:
    """1 collection plane, 960 wires x 10 impact bins x 6,000 ticks, 500,000
    track depos (200 segments of 1.25 m, 0.5 mm steps), fluctuation on,
    unipolar response 210 x 200."""
    rng = np.random.default_rng(seed)
    pl = plane(960, 6000)
    dep = track_depos(rng, nseg, per_seg)
    return dict(name="collection", phys=physics(True), planes=[pl],
                responses=[response("unipolar")], depos=dep, event_id=0)


def three_plane(seed: int = 3000, nseg: int = 800, nbkg: int = 400_000) -> dict:
    """U/V/W planes of 800/800/960 wires x 6,000 ticks (pitch directions +60,
    -60 and 0 degrees from z), 2,000,000 track depos plus 400,000 uniform
    background depos (median 300 e-), fluctuation on."""
    rng = np.random.default_rng(seed)
    c, s = math.cos(math.radians(60.0)), math.sin(math.radians(60.0))
    planes = [plane(800, 6000, 0, dir_y=s, dir_z=c, pitch_origin=0.0),
              plane(800, 6000, 1, dir_y=-s, dir_z=c, pitch_origin=-BOX_Y * s),
              plane(960, 6000, 2, dir_y=0.0, dir_z=1.0, pitch_origin=0.0)]
    resp = [response("bipolar", sigma_t=10.0), response("bipolar", sigma_t=12.0),
            response("unipolar")]
    trk = track_depos(rng, nseg)
    bkg = uniform_depos(rng, nbkg, (0.0, BOX_Z), (0.0, 2500.0), q_median=300.0)
    bkg[:, 0] = rng.uniform(0.0, BOX_X, nbkg)
    bkg[:, 3] = 0.0
    dep = np.ascontiguousarray(np.concatenate([trk, bkg], axis=0))
    return dict(name="three_plane", phys=physics(True), planes=planes, responses=resp,
                depos=dep, event_id=0)


def batch_events(seed: int = 4000, nevents: int = 64, lo: float = 4.0, hi: float = 6.0,
                 wires=(100, 480, 800, 960), nticks: int = 6000) -> list[dict]:
    """Uneven single-plane events: depo count log-uniform in [10^lo, 10^hi],
    wire count uniform over `wires`, clipped tracks inside the plane's extent."""
    out = []
    for e in range(nevents):
        rng = np.random.default_rng(seed + e)
        n = int(round(10.0 ** rng.uniform(lo, hi)))
        nw = int(rng.choice(wires))
        box = (BOX_X, BOX_Y, nw * PITCH)
        dep = clipped_track_depos(rng, n, box)
        out.append(dict(plane=plane(nw, nticks), response=response("unipolar"), depos=dep,
                        event_id=e))
    return out


def serve_requests(seed: int = 5000, nreq: int = 64, lo: float = 3.0,
                   hi: float = math.log10(2e6), nticks: int = 6000) -> list[dict]:
    """Requests of 1-3 planes (last one collection, the others induction) with
    100..960 wires and log-uniform depo counts."""
    out = []
    for r in range(nreq):
        rng = np.random.default_rng(seed + r)
        n = int(round(10.0 ** rng.uniform(lo, hi)))
        nplanes = int(rng.integers(1, 4))
        nws = [int(rng.integers(100, 961)) for _ in range(nplanes)]
        box = (BOX_X, BOX_Y, max(nws) * PITCH)
        dep = clipped_track_depos(rng, n, box)
        planes, resps = [], []
        for k, nw in enumerate(nws):
            planes.append(plane(nw, nticks, plane_id=k))
            resps.append(response("unipolar" if k == nplanes - 1 else "bipolar"))
        out.append(dict(planes=planes, responses=resps, depos=dep, event_id=r))
    return out


def poisson_arrivals(seed: int, n: int, qps: float) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, n))
