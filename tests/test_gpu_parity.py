"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (normwise, max|gpu - oracle| / max|oracle| over the array):
  * patch values and the plane grid: 1e-5 (FP32 outer product and
    fluctuation; bin weights and their normalisation in FP64 on both the fused
    and the generic path, rounded once to float32; FP64 patch totals for the
    fluctuation's rescaling);
  * convolved output: 1e-4 (FP32 FFTs of length up to ~10^4);
  * integer window bounds, the Philox words and ADC codes: bit-exact.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2304_01841_amd import workloads as W

pytestmark = pytest.mark.gpu

GRID_TOL = 1e-5
CONV_TOL = 1e-4


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_01841_amd import wcsim
    return wcsim


def normwise(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    got = np.asarray(got, dtype=np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        return np.abs(got).max()
    return np.abs(got - ref).max() / scale


def log(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# Philox
# ---------------------------------------------------------------------------
def test_philox_bitwise(ws):
    log("case: philox sweep")
    rng = np.random.default_rng(1)
    n = 200_000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0; key[0] = 0; ctr[1] = 0xFFFFFFFF; key[1] = 0xFFFFFFFF
    ref = O.philox4x32_10(ctr, key)
    got = ws.philox4x32_10(torch.from_numpy(ctr.view(np.int32)).cuda(),
                           torch.from_numpy(key.view(np.int32)).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint32), ref)


# ---------------------------------------------------------------------------
# Rasterization (patch sets)
# ---------------------------------------------------------------------------
def _compare_patches(ws, plane, phys, depos, event_id=0, mem="device"):
    R = W.response("bipolar")
    P = ws.Plane(plane, phys, R)
    dep = torch.from_numpy(depos).cuda() if mem == "device" else depos
    pt = ws.rasterize(P, dep, event_id)
    meta, offs, vals = pt.to_host()
    ometa, ovals, ost = O.rasterize(depos, phys, plane, event_id)
    # windows: bit-exact
    assert np.array_equal(meta[:, 0], ometa[:, 0])
    assert np.array_equal(meta[:, 1], ometa[:, 1])
    assert np.array_equal(meta[:, 2], ometa[:, 2])
    assert np.array_equal(meta[:, 3], ometa[:, 3])
    assert np.array_equal(offs[:-1], ometa[:, 4])
    assert offs[-1] == ovals.size
    # values: per patch, normwise
    worst = 0.0
    for d in range(depos.shape[0]):
        o, n = ometa[d, 4], ometa[d, 2] * ometa[d, 3]
        if n:
            worst = max(worst, normwise(vals[o:o + n], ovals[o:o + n]))
    assert worst <= GRID_TOL, worst
    pt.destroy()
    P.destroy()
    return meta, offs, vals


def test_rasterize_small_no_fluct(ws):
    log("case: rasterize small workload, no fluctuation")
    w = W.small()
    _compare_patches(ws, w["planes"][0], w["phys"], w["depos"])


def test_rasterize_small_fluct_host_depos(ws):
    log("case: rasterize small workload, fluctuation, host depos")
    w = W.small()
    _compare_patches(ws, w["planes"][0], W.physics(True), w["depos"], event_id=77, mem="host")


def test_rasterize_edges_and_large_windows(ws):
    """Depos straddling the grid edges (negative lo), missing the grid, at zero
    drift, and with windows beyond the one-wave path (long diffusion)."""
    log("case: rasterize edges and long windows")
    pl = W.plane(20, 300)
    rng = np.random.default_rng(9)
    dep = W.uniform_depos(rng, 300, (-5.0, 105.0), (-10.0, 160.0))
    dep[0] = [0.0, 0.0, 50.0, 70.0, 100.0]          # zero drift
    dep[1] = [100.0, 0.0, 5000.0, 0.0, 100.0]       # misses the grid
    for fl in (False, True):
        _compare_patches(ws, pl, W.physics(fl), dep, event_id=3)
    phys = W.physics(True)
    phys["DT"] = phys["DT"] * 40     # pitch windows ~ 110 bins
    phys["DL"] = phys["DL"] * 40
    _compare_patches(ws, pl, phys, dep[:60], event_id=4)


# ---------------------------------------------------------------------------
# Scatter-Add
# ---------------------------------------------------------------------------
def test_scatter_add_small(ws):
    log("case: scatter-add small")
    w = W.small()
    for fl in (False, True):
        phys = W.physics(fl)
        P = ws.Plane(w["planes"][0], phys, w["responses"][0])
        pt = ws.rasterize(P, torch.from_numpy(w["depos"]).cuda(), 5)
        grid = torch.full((P.npitch, P.nticks), 7.0, device="cuda")
        ws.scatter_add(P, pt, grid, zero_first=True)
        G = O.grid(w["depos"], phys, w["planes"][0], 5)
        assert normwise(grid.cpu().numpy(), G) <= GRID_TOL
        # accumulate twice without zeroing
        ws.scatter_add(P, pt, grid, zero_first=False)
        assert normwise(grid.cpu().numpy(), 2 * G) <= GRID_TOL
        if not fl:
            assert grid.sum().item() == pytest.approx(2 * G.sum(), rel=1e-5)


# ---------------------------------------------------------------------------
# Convolution
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nw,nimp,nt,Rp,Rt,r0", [
    (7, 3, 50, 5, 9, 2),        # odd everything
    (16, 4, 64, 8, 8, 0),
    (13, 10, 333, 21, 40, 20),   # ragged tail in pitch and ticks
    (30, 10, 1000, 210, 200, 105),
    (5, 10, 601, 60, 31, 59),
])
def test_convolve_random_response(ws, nw, nimp, nt, Rp, Rt, r0):
    log("case: convolve %s" % ((nw, nimp, nt, Rp, Rt, r0),))
    rng = np.random.default_rng(nw * 1000 + nt)
    pl = W.plane(nw, nt, nimpact=nimp)
    R = W.random_response(rng, Rp, Rt)
    P = ws.Plane(pl, W.physics(False), R, r0=r0)
    G = rng.standard_normal((nw * nimp, nt)).astype(np.float32)
    ref = O.convolve(G.astype(np.float64), R.astype(np.float64), r0)
    g = torch.from_numpy(G).cuda()
    out = ws.convolve(P, g, kind=ws.OUT_PITCH)
    assert normwise(out.cpu().numpy(), ref) <= CONV_TOL
    outw = ws.convolve(P, g, kind=ws.OUT_WIRE)
    assert normwise(outw.cpu().numpy(), O.wire_rows(ref, nimp)) <= CONV_TOL


def test_convolve_schedules_agree(ws):
    """The result does not depend on the FFT schedule (padded sizes, chunk
    width, pitch block length, column split of the pitch pass, the folded
    wire-output inverse when the block length is a multiple of the impact
    count, and the polyphase wire pass against the overlap-save blocks):
    pitch and wire output against the oracle."""
    log("case: convolve schedules")
    rng = np.random.default_rng(5)
    pl = W.plane(40, 900)
    nimp = pl["nimpact"]
    R = W.random_response(rng, 50, 60)
    G = rng.standard_normal((400, 900)).astype(np.float32)
    ref = O.convolve(G.astype(np.float64), R.astype(np.float64), 25)
    refw = O.wire_rows(ref, nimp)
    g = torch.from_numpy(G).cuda()
    for sc in ({}, {"fft_ticks": 1024}, {"fft_ticks": 1000, "freq_chunk": 8},
               {"fft_pitch": 512, "freq_chunk": 16}, {"fft_ticks": 1250},
               {"fft_pitch": 128}, {"fft_pitch": 1024, "freq_chunk": 8}, {"fft_pitch": 240},
               {"fft_pitch": 1024, "freq_chunk": 16}, {"fft_ticks": 6250}, {"fft_ticks": 1200},
               {"fft_pitch": 640, "freq_chunk": 16}, {"fft_pitch": 960, "freq_chunk": 16},
               {"fft_pitch": 640, "freq_chunk": 8}, {"fft_pitch": 100}, {"fft_pitch": 320}):
        for wm in (0, 2):
            P = ws.Plane(pl, W.physics(False), R, r0=25, schedule=dict(sc, wire_mode=wm))
            assert P.info["wire_polyphase"] == (1 if wm == 0 else 0)
            out = ws.convolve(P, g, kind=ws.OUT_PITCH)
            assert normwise(out.cpu().numpy(), ref) <= CONV_TOL, sc
            outw = ws.convolve(P, g, kind=ws.OUT_WIRE)
            assert normwise(outw.cpu().numpy(), refw) <= CONV_TOL, ("wire", sc, wm)
    # the polyphase pass asked for where it cannot apply
    with pytest.raises(ws.WcsimError):
        ws.Plane(W.plane(40, 900, nimpact=1), W.physics(False), R, r0=25,
                 schedule={"wire_mode": 1})
    Rlong = W.random_response(rng, 700, 20)  # ceil(700 / 10) = 70 taps per phase
    with pytest.raises(ws.WcsimError):
        ws.Plane(pl, W.physics(False), Rlong, r0=350, schedule={"wire_mode": 1})
    assert ws.Plane(pl, W.physics(False), Rlong, r0=350).info["wire_polyphase"] == 0


def test_convolve_delta_response_identity(ws):
    log("case: convolve delta")
    rng = np.random.default_rng(6)
    pl = W.plane(20, 500)
    R = np.zeros((31, 17), np.float32)
    R[15, 0] = 1.0
    P = ws.Plane(pl, W.physics(False), R, r0=15)
    G = rng.standard_normal((200, 500)).astype(np.float32)
    out = ws.convolve(P, torch.from_numpy(G).cuda(), kind=ws.OUT_PITCH)
    assert normwise(out.cpu().numpy(), G) <= 1e-6


# ---------------------------------------------------------------------------
# Whole path
# ---------------------------------------------------------------------------
def _sim_and_compare(ws, w, fl=None, kinds=(0, 1), out_mem="device", event_id=None,
                     schedules=(None,)):
    pl, R = w["planes"][0], w["responses"][0]
    phys = w["phys"] if fl is None else W.physics(fl)
    ev = w["event_id"] if event_id is None else event_id
    dep = torch.from_numpy(w["depos"]).cuda()
    G = O.grid(w["depos"], phys, pl, ev)
    full = O.convolve(G, R.astype(np.float64), R.shape[0] // 2)
    for sched in schedules:
        log("  schedule %s" % (sched,))
        P = ws.Plane(pl, phys, R, schedule=sched)
        for kind in kinds:
            wsp = ws.simulate_workspace(P, dep.shape[0], kind)
            if out_mem == "device":
                out = ws.simulate_event(P, dep, ev, kind=kind, workspace=wsp).cpu().numpy()
            else:
                out = np.zeros((P.out_rows(kind), P.nticks), np.float32)
                ws.simulate_event(P, dep, ev, out=out, kind=kind, workspace=wsp)
            grid = ws.workspace_grid(P, wsp, dep.shape[0]).cpu().numpy()
            assert normwise(grid, G) <= GRID_TOL, sched
            ref = full if kind == ws.OUT_PITCH else O.wire_rows(full, pl["nimpact"])
            assert normwise(out, ref) <= CONV_TOL, (kind, sched)
            assert ws.workspace_invalid_count(wsp) == 0
    return P


def test_simulate_small(ws):
    log("case: simulate small workload")
    w = W.small()
    _sim_and_compare(ws, w)
    _sim_and_compare(ws, w, fl=True, out_mem="host", event_id=12)


def test_simulate_small_every_tile_shape(ws):
    """Every raster tile shape (32 x 8, 32 x 32, 64 x 8 bins x ticks) gives the
    oracle's grid and output, with and without fluctuation."""
    log("case: simulate small workload, every tile shape")
    shapes = [{"tile": t} for t in range(3)]
    w = W.small()
    for fl in (False, True):
        _sim_and_compare(ws, w, fl=fl, kinds=(ws.OUT_PITCH,), schedules=shapes)
    # depos straddling every grid edge (windows starting before pitch bin 0 and
    # tick 0, or running past the last ones) on the fused tile path
    rng = np.random.default_rng(19)
    dep = W.uniform_depos(rng, 600, (-5.0, 105.0), (-10.0, 160.0))
    edges = dict(planes=[W.plane(20, 300)], responses=[W.response("bipolar")], depos=dep,
                 phys=W.physics(True), event_id=6)
    _sim_and_compare(ws, edges, kinds=(ws.OUT_PITCH,), schedules=shapes)


def test_unreached_grid_blocks_are_neither_cleared_nor_read(ws):
    """Only the grid blocks (32 pitch rows x 2^k ticks) that some depo window
    reaches are cleared and read: on a workspace full of NaN (all-one bytes),
    and then after a dense event left its data behind, a sparse event gives
    the oracle's output; its grid keeps the stale contents outside the reached
    blocks until completed, and then equals the oracle's grid.  Also on a
    ragged plane (130 pitch rows: a partial last band; 997 ticks: rows of an
    odd length, cleared and read float by float)."""
    log("case: unreached grid blocks")
    w = W.small()
    rng = np.random.default_rng(41)
    ragged = (W.plane(13, 997), W.uniform_depos(rng, 400, (0.0, 65.0), (0.0, 480.0)))
    for pl, dense in ((w["planes"][0], w["depos"]), ragged):
        R = w["responses"][0]
        phys = W.physics(True)
        P = ws.Plane(pl, phys, R)
        sparse = np.ascontiguousarray(dense[:25])
        wsp = ws.simulate_workspace(P, dense.shape[0], ws.OUT_PITCH)
        wsp.fill_(0xFF)
        for dep, ev in ((sparse, 3), (dense, 4), (sparse, 5)):
            log("  plane %d x %d, %d depos" % (P.npitch, P.nticks, dep.shape[0]))
            G = O.grid(dep, phys, pl, ev)
            ref = O.convolve(G, R.astype(np.float64), R.shape[0] // 2)
            out = ws.simulate_event(P, torch.from_numpy(dep).cuda(), ev, kind=ws.OUT_PITCH,
                                    workspace=wsp).cpu().numpy()
            assert np.isfinite(out).all()
            assert normwise(out, ref) <= CONV_TOL, ev
            n = dep.shape[0]
            if ev == 3:  # NaN where no window reached, values wherever charge landed
                stale = ws.workspace_grid(P, wsp, n, complete=False).cpu().numpy()
                assert np.isnan(stale).any()
                assert np.isfinite(stale[G != 0.0]).all()
            grid = ws.workspace_grid(P, wsp, n).cpu().numpy()
            assert normwise(grid, G) <= GRID_TOL, ev


def test_simulate_collection_full_size(ws):
    """Detector-scale collection plane (960 wires x 10 impact x 6000 ticks,
    500,000 track depos, fluctuation) in every launch configuration the
    benchmark's schedule tuner can pick: the whole grid and output against
    the oracle."""
    from paper_2304_01841_amd import autotune
    log("case: simulate collection plane, full size")
    w = W.collection()
    _sim_and_compare(ws, w, kinds=(ws.OUT_WIRE,), schedules=autotune.candidates())


def test_lifetime_absorption(ws):
    """Electron-lifetime absorption (an extension beyond the paper): patch
    sets, the fused path's grid and the convolved output agree with the
    oracle with and without fluctuation, on the small workload (drift times
    up to 2.5 ms against a 1.5 ms lifetime) and on the full collection plane;
    a negative lifetime is rejected."""
    log("case: lifetime absorption")
    w = W.small()
    for fl in (False, True):
        ph = W.physics(fl)
        ph["lifetime"] = 1500.0
        _compare_patches(ws, w["planes"][0], ph, w["depos"], event_id=4)
        _sim_and_compare(ws, dict(w, phys=ph), kinds=(ws.OUT_PITCH, ws.OUT_WIRE), event_id=4)
    ph = W.physics(True)
    ph["lifetime"] = 3000.0
    log("  collection plane, full size")
    _sim_and_compare(ws, dict(W.collection(), phys=ph), kinds=(ws.OUT_WIRE,))
    ph["lifetime"] = -1.0
    with pytest.raises(ws.WcsimError):
        ws.Plane(w["planes"][0], ph, w["responses"][0])


def test_lifetime_draw_shared_by_planes(ws):
    """The surviving charge of a depo is drawn once per depo and event, not
    per plane: with fluctuation and a lifetime on, the GPU patch of each depo
    integrates to the same count on the U, V and W planes of one event, equal
    to the oracle's count."""
    log("case: lifetime draw shared by the planes")
    w = W.three_plane()
    rng = np.random.default_rng(17)
    dep = W.uniform_depos(rng, 3000, (1500.0, 3300.0), (100.0, 2000.0), y_range=(600.0, 1200.0))
    ph = dict(W.physics(True), lifetime=1500.0)
    totals = []
    for pl in w["planes"]:
        P = ws.Plane(pl, ph, W.response("bipolar"))
        meta, offs, vals = ws.rasterize(P, torch.from_numpy(dep).cuda(), 4).to_host()
        assert (meta[:, 2] > 0).all()
        t = np.add.reduceat(vals.astype(np.float64), offs[:-1])
        totals.append(t)
        om, ov, _ = O.rasterize(dep, ph, pl, event_id=4)
        ot = np.array([ov[m[4]:m[4] + m[2] * m[3]].sum() for m in om])
        assert np.abs(t - ot).max() <= 1e-5 * ot.max()
    for t in totals[1:]:
        assert np.abs(t - totals[0]).max() <= 1e-5 * totals[0].max()


def test_drift_accel(ws):
    """A drift speed changing linearly with drift time (an extension beyond
    the paper): windows bit-exact, patch sets, grid and output against the
    oracle for accelerating and decelerating drifts (with a lifetime), on the
    small workload and on the full collection plane; host depos that cannot
    reach the plane are rejected, device ones counted and dropped."""
    log("case: drift acceleration")
    w = W.small()
    for a in (-3e-4, 2e-4):
        for fl in (False, True):
            ph = dict(W.physics(fl), drift_accel=a, lifetime=2000.0 if fl else 0.0)
            _compare_patches(ws, w["planes"][0], ph, w["depos"], event_id=8)
            _sim_and_compare(ws, dict(w, phys=ph), kinds=(ws.OUT_PITCH,), event_id=8)
    log("  collection plane, full size")
    ph = dict(W.physics(True), drift_accel=1e-4)
    _sim_and_compare(ws, dict(W.collection(), phys=ph), kinds=(ws.OUT_WIRE,))
    # a depo beyond reach: 1.6^2 / (2 a) = 1280 mm at a = 1e-3
    ph = dict(W.physics(False), drift_accel=1e-3)
    P = ws.Plane(w["planes"][0], ph, w["responses"][0])
    bad = np.array([[1300.0, 0.0, 100.0, -500.0, 100.0], [100.0, 0.0, 100.0, 10.0, 100.0]])
    with pytest.raises(ws.WcsimError):
        ws.simulate_event(P, bad, 0)
    wsp = ws.simulate_workspace(P, 2)
    ws.simulate_event(P, torch.from_numpy(bad).cuda(), 0, workspace=wsp)
    assert ws.workspace_invalid_count(wsp) == 1


def _pitch_bins(depos, pl):
    """Mean pitch bin of each depo (projection of (y, z) on the pitch
    direction); used only to pick a superset of the depos that can reach
    given grid rows."""
    dp = pl["pitch"] / pl["nimpact"]
    return ((depos[:, 1] * pl["dir_y"] + depos[:, 2] * pl["dir_z"]) - pl["pitch_origin"]) / dp


def test_simulate_three_plane_full_size_sampled(ws):
    """The three-plane event (U/V/W 800/800/960 wires x 6000 ticks, bipolar
    and unipolar responses, 2,400,000 depos, fluctuation on) at its full size,
    under the library default and the tuned pitch schedule: sampled wire
    waveforms against the oracle.  For each sampled wire the oracle takes
    every depo whose window can reach the response's reach of that wire (a
    superset chosen by mean pitch bin plus 40 bins), keyed by its index in
    the event, and evaluates the defining convolution sum at the sampled
    ticks."""
    log("case: simulate three planes, full size, sampled")
    w = W.three_plane()
    dep_np, ph, ev = w["depos"], w["phys"], w["event_id"]
    dep = torch.from_numpy(dep_np).cuda()
    rng = np.random.default_rng(31)
    for pl, R in zip(w["planes"], w["responses"]):
        Rp = R.shape[0]
        r0 = Rp // 2
        nimp = pl["nimpact"]
        mu = _pitch_bins(dep_np, pl)
        for sched in (None, {"fft_pitch": 640, "freq_chunk": 16}):
            log("  plane %d schedule %s" % (pl["plane_id"], sched))
            P = ws.Plane(pl, ph, R, schedule=sched)
            wsp = ws.simulate_workspace(P, dep.shape[0], ws.OUT_WIRE)
            out = ws.simulate_event(P, dep, ev, kind=ws.OUT_WIRE, workspace=wsp).cpu().numpy()
            assert ws.workspace_invalid_count(wsp) == 0
            scale = np.abs(out).max()
            assert scale > 0
            # the two wires with the largest signal and two at random
            wires = list(np.argsort(-np.abs(out).max(axis=1))[:2])
            wires += list(rng.integers(0, pl["nwires"], 2))
            ticks = np.arange(0, pl["nticks"], 7)
            for wi in wires:
                p = int(wi) * nimp + nimp // 2
                lo, hi = p + r0 - (Rp - 1), p + r0
                idx = np.nonzero((mu >= lo - 40) & (mu <= hi + 40))[0]
                G = O.grid(dep_np[idx], ph, pl, ev, ids=idx)
                pts = np.stack([np.full(ticks.shape, p), ticks], axis=1)
                ref = O.convolve_points(G, R.astype(np.float64), r0, pts)
                err = np.abs(out[int(wi), ticks] - ref).max() / scale
                assert err <= CONV_TOL, (pl["plane_id"], sched, int(wi), err)
            P.destroy()


def test_simulate_empty_and_invalid(ws):
    log("case: simulate empty / invalid")
    pl = W.plane(10, 200)
    R = W.response("bipolar", Rp=21, Rt=20, r0=10)
    P = ws.Plane(pl, W.physics(True), R, r0=10)
    dep = torch.zeros((0, 5), dtype=torch.float64, device="cuda")
    wsp = ws.simulate_workspace(P, 0, ws.OUT_WIRE)
    out = ws.simulate_event(P, dep, 0, workspace=wsp)
    assert float(out.abs().max()) == 0.0
    bad = np.array([[-1.0, 0, 10, 0, 5.0], [10.0, 0, 10, 0, -5.0], [np.nan, 0, 1, 0, 1.0],
                    [10.0, 0, 10, 0, 5.0]])
    with pytest.raises(ws.WcsimError) as ei:
        ws.simulate_event(P, bad, 0)
    assert ei.value.status == ws.E_INVALID
    dev = torch.from_numpy(bad).cuda()
    wsp = ws.simulate_workspace(P, 4, ws.OUT_WIRE)
    out = ws.simulate_event(P, dev, 0, workspace=wsp)
    assert ws.workspace_invalid_count(wsp) == 3
    ref = O.wire_rows(O.convolve(O.grid(bad[3:], W.physics(True), pl, 0), R.astype(float), 10), 10)
    # the valid depo keeps its index 3 in the Philox key
    G = O.grid(bad, W.physics(True), pl, 0)
    ref = O.wire_rows(O.convolve(G, R.astype(float), 10), 10)
    assert normwise(out.cpu().numpy(), ref) <= CONV_TOL


def test_simulate_long_windows_use_generic_path(ws):
    log("case: simulate long windows")
    pl = W.plane(30, 800)
    rng = np.random.default_rng(31)
    dep = W.uniform_depos(rng, 400, (0.0, 150.0), (0.0, 400.0))
    phys = W.physics(True)
    phys["DT"] *= 30
    phys["DL"] *= 30
    w = dict(planes=[pl], responses=[W.response("bipolar")], depos=dep, phys=phys, event_id=2)
    _sim_and_compare(ws, w)
    # the generic path applies electron-lifetime absorption as the tile path does
    _sim_and_compare(ws, dict(w, phys=dict(phys, lifetime=1200.0)), kinds=(ws.OUT_PITCH,))


# ---------------------------------------------------------------------------
# Digitisation with white noise (an extension beyond the paper)
# ---------------------------------------------------------------------------
def _digitize_wave(rng, nrows, ncols):
    """Seeded float32 waveform spanning negative values, exact halves after
    the gain, and values past the top code."""
    w = rng.normal(0.0, 600.0, (nrows, ncols)).astype(np.float32)
    w[:, ::7] = (np.rint(w[:, ::7]) + 0.25).astype(np.float32)  # x 2 + 100: exact .5
    edge = np.array([-1e6, 1e6, 0.25, 0.75, 1997.75], np.float32)[:ncols]
    w[0, :edge.size] = edge
    return w


def test_digitize_bit_exact_without_noise(ws):
    """Codes of a seeded waveform (ragged sizes) equal the oracle's exactly,
    including halves and both clamps; empty input is a no-op and bad
    parameters are rejected."""
    log("case: digitize without noise")
    rng = np.random.default_rng(23)
    for nrows, ncols in [(7, 1001), (96, 6000), (1, 3)]:
        w = _digitize_wave(rng, nrows, ncols)
        got = ws.digitize(torch.from_numpy(w).cuda(), 2.0, 100.0, 0.0, 12).cpu().numpy()
        ref = O.digitize(w, 2.0, 100.0, 0.0, 12, 0, 0)
        assert np.array_equal(got.view(np.uint16), ref), (nrows, ncols)
    empty = torch.zeros((0, 5), dtype=torch.float32, device="cuda")
    assert ws.digitize(empty, 1.0, 0.0).shape == (0, 5)
    w = torch.zeros((2, 2), dtype=torch.float32, device="cuda")
    for bad in [dict(bits=0), dict(bits=17), dict(sigma=-1.0), dict(gain=float("nan"))]:
        kw = dict(gain=1.0, pedestal=0.0, sigma=0.0, bits=12)
        kw.update(bad)
        with pytest.raises(ws.WcsimError):
            ws.digitize(w, **kw)


def test_digitize_with_noise_and_simulated_output(ws):
    """With white noise the codes equal the oracle's exactly on identical
    input waveforms (the deviates are evaluated in FP64 on both sides and
    rounded once to float32; the decision is the same float32 arithmetic), on
    ragged sizes with more than 1024 columns; the digitised simulate output
    agrees with the digitised oracle output to one code (their inputs differ:
    float32 simulation against FP64)."""
    log("case: digitize with noise")
    rng = np.random.default_rng(29)
    seed = 0x0123_4567_89AB_CDEF
    for nrows, ncols, ev in [(64, 3001, 11), (5, 1027, 3), (3, 6000, 0x1_0000_0007)]:
        w = _digitize_wave(rng, nrows, ncols)
        got = ws.digitize(torch.from_numpy(w).cuda(), 1.5, 800.0, 2.5, 14, seed, ev).cpu().numpy()
        ref = O.digitize(w, 1.5, 800.0, 2.5, 14, seed, ev)
        assert np.array_equal(got.view(np.uint16), ref), (nrows, ncols)
    wk = W.small()
    pl, R = wk["planes"][0], wk["responses"][0]
    P = ws.Plane(pl, wk["phys"], R)
    out = ws.simulate_event(P, torch.from_numpy(wk["depos"]).cuda(), wk["event_id"])
    full = O.convolve(O.grid(wk["depos"], wk["phys"], pl, wk["event_id"]), R.astype(float),
                      R.shape[0] // 2)
    oref = O.wire_rows(full, pl["nimpact"])
    gain = 1500.0 / np.abs(oref).max()
    got = ws.digitize(out, gain, 2048.0, 0.0, 12).cpu().numpy().view(np.uint16)
    ref = O.digitize(oref.astype(np.float32), gain, 2048.0, 0.0, 12, 0, 0)
    assert np.abs(got.astype(np.int64) - ref.astype(np.int64)).max() <= 1
    # the GPU's own float32 output digitised by both sides: identical codes
    o32 = out.cpu().numpy()
    got = ws.digitize(out, gain, 2048.0, 3.0, 12, seed, 5).cpu().numpy().view(np.uint16)
    assert np.array_equal(got, O.digitize(o32, gain, 2048.0, 3.0, 12, seed, 5))


# ---------------------------------------------------------------------------
# Electronics response (an extension beyond the paper)
# ---------------------------------------------------------------------------
def test_electronics_response(ws):
    """A plane with an electronics response convolves with R (x) E: simulated
    output (pitch and wire) and the convolve entry point agree with the
    oracle; a plane sharing the same detector response but another
    electronics response does not share its spectrum; non-finite samples are
    rejected."""
    log("case: electronics response")
    w = W.small()
    rng = np.random.default_rng(61)
    E = (np.exp(-np.arange(60) / 12.0) * np.sin(np.arange(60) / 5.0)).astype(np.float32)
    pl = dict(w["planes"][0], elec_response=E)
    R = w["responses"][0]
    Rc = O.combined_response(R.astype(np.float64), E.astype(np.float64))
    ev = w["event_id"]
    G = O.grid(w["depos"], w["phys"], pl, ev)
    full = O.convolve(G, Rc, R.shape[0] // 2)
    P = ws.Plane(pl, w["phys"], R)
    assert P.info["fft_ticks"] >= pl["nticks"] + Rc.shape[1] - 1
    dep = torch.from_numpy(w["depos"]).cuda()
    for kind in (ws.OUT_PITCH, ws.OUT_WIRE):
        out = ws.simulate_event(P, dep, ev, kind=kind).cpu().numpy()
        ref = full if kind == ws.OUT_PITCH else O.wire_rows(full, pl["nimpact"])
        assert normwise(out, ref) <= CONV_TOL, kind
    Gr = rng.normal(size=G.shape).astype(np.float32)
    out = ws.convolve(P, torch.from_numpy(Gr).cuda(), kind=ws.OUT_PITCH).cpu().numpy()
    assert normwise(out, O.convolve(Gr.astype(np.float64), Rc, R.shape[0] // 2)) <= CONV_TOL
    # same detector response, another electronics response: its own spectrum
    E2 = E[::-1].copy()
    pl2 = dict(w["planes"][0], elec_response=E2)
    P2 = ws.Plane(pl2, w["phys"], R, share=P)
    out2 = ws.simulate_event(P2, dep, ev, kind=ws.OUT_PITCH).cpu().numpy()
    full2 = O.convolve(G, O.combined_response(R.astype(np.float64), E2.astype(np.float64)),
                       R.shape[0] // 2)
    assert normwise(out2, full2) <= CONV_TOL
    bad = dict(w["planes"][0], elec_response=np.array([1.0, np.nan], np.float32))
    with pytest.raises(ws.WcsimError):
        ws.Plane(bad, w["phys"], R)


def test_digitize_coloured_noise(ws):
    """FIR-coloured noise: fir = {1} gives exactly the white-noise codes; 64-
    and 1024-tap filters (the longest, whose history spans a whole 1024-column
    tile) give exactly the oracle's codes (FP64 deviates and FP64 filter sums
    on both sides, rounded once to float32) on ragged sizes spanning several
    tiles; bad filters are rejected."""
    log("case: digitize with coloured noise")
    rng = np.random.default_rng(31)
    seed = 0xFEED_F00D
    for nrows, ncols in [(9, 2500), (2, 1025), (3, 4097)]:
        w = _digitize_wave(rng, nrows, ncols)
        wt = torch.from_numpy(w).cuda()
        white = ws.digitize(wt, 1.5, 800.0, 2.5, 14, seed, 4).cpu().numpy()
        one = torch.ones(1, dtype=torch.float32, device="cuda")
        same = ws.digitize(wt, 1.5, 800.0, 2.5, 14, seed, 4, fir=one).cpu().numpy()
        assert np.array_equal(same, white)
        for nfir in (64, 1024):
            k = np.arange(nfir)
            h = (np.exp(-k / (nfir / 7.0)) * np.cos(k / 3.0)).astype(np.float32)
            h /= np.float32(np.sqrt(np.sum(h.astype(np.float64) ** 2)))
            got = ws.digitize(wt, 1.5, 800.0, 2.5, 14, seed, 4,
                              fir=torch.from_numpy(h).cuda()).cpu().numpy().view(np.uint16)
            ref = O.digitize(w, 1.5, 800.0, 2.5, 14, seed, 4, fir=h.astype(np.float64))
            assert np.array_equal(got, ref), (nrows, ncols, nfir)
    long_h = torch.ones(1025, dtype=torch.float32, device="cuda")
    with pytest.raises(ws.WcsimError):
        ws.digitize(wt, 1.0, 0.0, 1.0, 12, fir=long_h)
