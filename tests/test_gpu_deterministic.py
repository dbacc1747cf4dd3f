"""Reproducible sums (wcsim_schedule.deterministic = 1): depos listed per tile
in depo order, the owner flush (tiles in colour phases whose LDS regions are
disjoint, plain read-add-writes) and the large patches added one after
another.  The grid and output must repeat bit for bit, whatever the
workspace held and whether the event runs alone or in a batch, and agree
with the float-atomic path and the oracle to the usual tolerances (grid 1e-5,
convolved output 1e-4, normwise).

The mix below stresses what makes the atomic path vary: 31 depos per
occupied 32 x 8 tile on average and up to 127 (several work items per tile, a
tile's depos spread over many binning wavefronts by the shuffle), and
long-drift depos whose windows exceed a tile region (the large-patch path)."""
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
    ref = np.asarray(ref, np.float64)
    return np.abs(np.asarray(got, np.float64) - ref).max() / max(np.abs(ref).max(), 1e-300)


def log(msg):
    print(msg, flush=True)


def _mix(seed=5, fluct=True):
    pl = W.plane(30, 1000)  # 300 pitch bins x 1000 ticks
    rng = np.random.default_rng(seed)
    dense = W.uniform_depos(rng, 20000, (0.0, 60.0), (100.0, 350.0), max_drift_time=300.0)
    spread = W.uniform_depos(rng, 600, (-5.0, 155.0), (-10.0, 520.0))
    dep = np.concatenate([dense, spread])
    dep = np.ascontiguousarray(dep[rng.permutation(dep.shape[0])])
    phys = W.physics(fluct)
    phys["DT"] *= 6.0  # long drifts: windows beyond a tile region
    phys["DL"] *= 6.0
    return pl, phys, dep


def _large_count(pl, phys, dep):
    """Depos whose window exceeds what a tile region takes (32 pitch bins,
    17 ticks): those take the large-patch path."""
    n = 0
    for d in dep:
        st, _, (_, _, n_p, n_t) = O.depo_window(d, phys, pl)
        n += st == 0 and (n_p > 32 or n_t > 17)
    return n


def _run(ws, P, dep, ev, fill):
    wsp = ws.simulate_workspace(P, dep.shape[0], ws.OUT_PITCH)
    wsp.fill_(fill)
    out = ws.simulate_event(P, torch.from_numpy(dep).cuda(), ev, kind=ws.OUT_PITCH,
                            workspace=wsp).cpu().numpy()
    grid = ws.workspace_grid(P, wsp, dep.shape[0]).cpu().numpy()
    return grid, out


def test_mix_reaches_both_raster_paths():
    pl, phys, dep = _mix()
    assert _large_count(pl, phys, dep[:8000]) >= 20


@pytest.mark.parametrize("tile", [0, 1, 2])
def test_deterministic_repeats_bit_for_bit(ws, tile):
    log("case: deterministic repeats, tile shape %d" % tile)
    pl, phys, dep = _mix()
    R = W.response("bipolar")
    P = ws.Plane(pl, phys, R, schedule={"tile": tile, "deterministic": 1})
    assert P.info["deterministic"] == 1
    g0, o0 = _run(ws, P, dep, 9, 0xFF)  # a workspace full of NaN
    for fill in (0x00, 0x3C):
        g, o = _run(ws, P, dep, 9, fill)
        assert np.array_equal(g, g0), fill
        assert np.array_equal(o, o0), fill
    # a fresh plane of the same schedule gives the same bits
    Q = ws.Plane(pl, phys, R, schedule={"tile": tile, "deterministic": 1})
    g, o = _run(ws, Q, dep, 9, 0x00)
    assert np.array_equal(g, g0) and np.array_equal(o, o0)


@pytest.mark.parametrize("fluct", [True, False])
def test_deterministic_against_atomic_and_oracle(ws, fluct):
    log("case: deterministic vs atomic vs oracle, fluctuation %s" % fluct)
    pl, phys, dep = _mix(seed=6, fluct=fluct)
    R = W.response("bipolar")
    G = O.grid(dep, phys, pl, 11)
    ref = O.convolve(G, R.astype(np.float64), R.shape[0] // 2)
    Pd = ws.Plane(pl, phys, R, schedule={"deterministic": 1})
    Pa = ws.Plane(pl, phys, R)
    assert Pa.info["deterministic"] == 0
    gd, od = _run(ws, Pd, dep, 11, 0xFF)
    ga, oa = _run(ws, Pa, dep, 11, 0xFF)
    assert normwise(gd, G) <= GRID_TOL
    assert normwise(ga, G) <= GRID_TOL
    assert normwise(gd, ga) <= GRID_TOL
    assert normwise(od, ref) <= CONV_TOL
    assert normwise(od, oa) <= CONV_TOL


def test_deterministic_with_lifetime_and_drift_accel(ws):
    """The extensions that change a record's charge and window (electron
    lifetime with fluctuation, an accelerating drift): repeats bit for bit and
    agrees with the oracle."""
    log("case: deterministic with lifetime and drift acceleration")
    pl, phys, dep = _mix(seed=9)
    phys = dict(phys, lifetime=1800.0, drift_accel=2e-4)
    R = W.response("bipolar")
    P = ws.Plane(pl, phys, R, schedule={"deterministic": 1})
    g0, o0 = _run(ws, P, dep, 13, 0xFF)
    g1, o1 = _run(ws, P, dep, 13, 0x00)
    assert np.array_equal(g0, g1) and np.array_equal(o0, o1)
    G = O.grid(dep, phys, pl, 13)
    assert normwise(g0, G) <= GRID_TOL
    assert normwise(o0, O.convolve(G, R.astype(np.float64), R.shape[0] // 2)) <= CONV_TOL


def test_deterministic_batch_equals_single_bit_for_bit(ws):
    """Events of different planes and sizes (one empty, one ragged) in one
    batched call and in two replays of its captured graph: each output equals
    the event's own single run bit for bit, and the oracle's to the output
    tolerance."""
    log("case: deterministic batch vs single")
    pl, phys, dep = _mix(seed=7)
    R = W.response("bipolar")
    rng = np.random.default_rng(8)
    evs = [(pl, dep, 21),
           (W.plane(13, 1000), W.uniform_depos(rng, 500, (0.0, 65.0), (0.0, 480.0)), 22),
           (W.plane(20, 1000), np.zeros((0, 5)), 23),
           (W.plane(30, 1000, plane_id=1), dep[:5000].copy(), 24)]
    sched = {"deterministic": 1}
    planes = [ws.Plane(p, phys, R, schedule=sched) for p, _, _ in evs]
    deps = [torch.from_numpy(np.ascontiguousarray(d)).cuda() for _, d, _ in evs]
    outs = [torch.full((P.out_rows(ws.OUT_WIRE), P.nticks), 3.0, device="cuda") for P in planes]
    wsp = ws.batch_workspace(planes, [d.shape[0] for d in deps], ws.OUT_WIRE)
    wsp.fill_(0xFF)
    ws.simulate_batch(planes, deps, [e for _, _, e in evs], outs, workspace=wsp)
    torch.cuda.synchronize()
    # the captured graph of the same batch, replayed twice
    gouts = [torch.full_like(o, -2.0) for o in outs]
    b = ws.Batch(planes, [d.shape[0] for d in deps])
    for _ in range(2):
        b.run(deps, [e for _, _, e in evs], gouts)
        torch.cuda.synchronize()
        for o, g in zip(outs, gouts):
            assert torch.equal(o, g)
    b.destroy()
    for P, (p, d, e), dd, o in zip(planes, evs, deps, outs):
        single = ws.simulate_event(P, dd, e, kind=ws.OUT_WIRE).cpu().numpy()
        got = o.cpu().numpy()
        assert np.array_equal(got, single), e
        if d.shape[0] == 0:
            assert np.abs(got).max() == 0.0
            continue
        full = O.convolve(O.grid(d, phys, p, e), R.astype(np.float64), R.shape[0] // 2)
        assert normwise(got, O.wire_rows(full, p["nimpact"])) <= CONV_TOL, e


def test_deterministic_collection_plane(ws):
    """Full collection plane (500,000 track depos, fluctuation): two runs give
    the same bits, and the wire output matches the atomic path's."""
    log("case: deterministic collection plane")
    w = W.collection()
    pl, R, dep = w["planes"][0], w["responses"][0], w["depos"]
    d = torch.from_numpy(dep).cuda()
    Pd = ws.Plane(pl, w["phys"], R, schedule={"deterministic": 1})
    Pa = ws.Plane(pl, w["phys"], R)
    o1 = ws.simulate_event(Pd, d, w["event_id"]).cpu().numpy()
    o2 = ws.simulate_event(Pd, d, w["event_id"]).cpu().numpy()
    oa = ws.simulate_event(Pa, d, w["event_id"]).cpu().numpy()
    assert np.array_equal(o1, o2)
    assert normwise(o1, oa) <= GRID_TOL
