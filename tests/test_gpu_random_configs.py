"""Seeded sweep of small random configurations through the whole path, each
against the oracle: odd and even wire and tick counts, 1, 3 or 10 impact
bins, random response sizes and origins, every raster tile shape, both
wire-output pitch passes, fluctuation on and off, reproducible sums on and
off, depos spilling over every grid edge.  Grid within 1e-5 and output
within 1e-4 (normwise); with reproducible sums two runs give the same bits."""
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


def _config(seed):
    rng = np.random.default_rng(seed)
    nwires = int(rng.integers(3, 60))
    nimpact = int(rng.choice([1, 3, 10]))
    nticks = int(rng.integers(60, 1500))
    pl = W.plane(nwires, nticks, plane_id=int(rng.integers(0, 3)), nimpact=nimpact)
    Rp = int(rng.integers(1, 60))
    Rt = int(rng.integers(1, 90))
    r0 = int(rng.integers(0, Rp))
    R = rng.normal(0.0, 1.0, (Rp, Rt)).astype(np.float32)
    span_p = nwires * W.PITCH
    span_t = nticks * W.TICK
    n = int(rng.integers(1, 2500))
    dep = W.uniform_depos(rng, n, (-0.1 * span_p, 1.1 * span_p), (-0.1 * span_t, 1.1 * span_t),
                          max_drift_time=float(rng.uniform(50.0, 2500.0)))
    phys = W.physics(bool(rng.integers(0, 2)))
    sched = {"tile": int(rng.integers(0, 3)), "deterministic": int(rng.integers(0, 2)),
             "wire_mode": 2 if rng.integers(0, 2) else 0}
    return pl, R, r0, dep, phys, sched


@pytest.mark.parametrize("seed", list(range(4000, 4040)))
def test_random_configuration_against_oracle(ws, seed):
    pl, R, r0, dep, phys, sched = _config(seed)
    print("case: seed %d, %d wires x %d impact x %d ticks, R %s @%d, %d depos, fluct %d, %s"
          % (seed, pl["nwires"], pl["nimpact"], pl["nticks"], R.shape, r0, dep.shape[0],
             phys["fluctuate"], sched), flush=True)
    P = ws.Plane(pl, phys, R, r0=r0, schedule=sched)
    d = torch.from_numpy(dep).cuda()
    G = O.grid(dep, phys, pl, seed)
    full = O.convolve(G, R.astype(np.float64), r0)
    for kind, ref in ((ws.OUT_PITCH, full), (ws.OUT_WIRE, O.wire_rows(full, pl["nimpact"]))):
        wsp = ws.simulate_workspace(P, dep.shape[0], kind)
        wsp.fill_(0xFF)
        out = ws.simulate_event(P, d, seed, kind=kind, workspace=wsp).cpu().numpy()
        grid = ws.workspace_grid(P, wsp, dep.shape[0]).cpu().numpy()
        assert np.isfinite(out).all()
        if np.abs(G).max() > 0:
            assert normwise(grid, G) <= GRID_TOL, kind
        else:
            assert np.abs(grid).max() == 0.0
        if np.abs(ref).max() > 0:
            assert normwise(out, ref) <= CONV_TOL, kind
        if sched["deterministic"]:
            again = ws.simulate_event(P, d, seed, kind=kind, workspace=wsp).cpu().numpy()
            assert np.array_equal(again, out), kind


def test_random_configurations_in_one_batch(ws):
    """Twelve of the random configurations (their planes fall in several
    schedule classes) in one batched call and two replays of its captured
    graph: each event equals its single run (1e-5; bit for bit when its plane
    has reproducible sums) and the oracle (1e-4)."""
    print("case: random configurations in one batch", flush=True)
    cfgs = [_config(s) for s in range(4100, 4112)]
    planes = [ws.Plane(pl, phys, R, r0=r0, schedule=sched) for pl, R, r0, dep, phys, sched in cfgs]
    deps = [torch.from_numpy(c[3]).cuda() for c in cfgs]
    ids = list(range(4100, 4112))
    outs = [torch.full((P.nwires, P.nticks), 7.0, device="cuda") for P in planes]
    ws.simulate_batch(planes, deps, ids, outs)
    b = ws.Batch(planes, [d.shape[0] for d in deps])
    gouts = [torch.full_like(o, -7.0) for o in outs]
    for _ in range(2):
        b.run(deps, ids, gouts)
        torch.cuda.synchronize()
        for o, g in zip(outs, gouts):
            assert normwise(g.cpu().numpy(), o.cpu().numpy()) <= 1e-5
    b.destroy()
    for (pl, R, r0, dep, phys, sched), P, d, e, o in zip(cfgs, planes, deps, ids, outs):
        got = o.cpu().numpy()
        single = ws.simulate_event(P, d, e).cpu().numpy()
        if sched["deterministic"]:
            assert np.array_equal(got, single), e
        elif np.abs(single).max() > 0:
            assert normwise(got, single) <= 1e-5, e
        ref = O.wire_rows(O.convolve(O.grid(dep, phys, pl, e), R.astype(np.float64), r0),
                          pl["nimpact"])
        if np.abs(ref).max() > 0:
            assert normwise(got, ref) <= CONV_TOL, e


@pytest.mark.parametrize("seed", list(range(4200, 4212)))
def test_random_patch_sets_scatter_and_convolve(ws, seed):
    """The other entry points on the same random configurations: patch sets
    (windows and offsets bit-exact, values per patch within 1e-5), their
    scatter-add (1e-5) and the convolution of a random grid (1e-4), against the
    oracle."""
    pl, R, r0, dep, phys, sched = _config(seed)
    print("case: seed %d patch sets / scatter / convolve" % seed, flush=True)
    P = ws.Plane(pl, phys, R, r0=r0, schedule=sched)
    pt = ws.rasterize(P, torch.from_numpy(dep).cuda(), seed)
    meta, offs, vals = pt.to_host()
    ometa, ovals, _ = O.rasterize(dep, phys, pl, seed)
    for c in range(4):
        assert np.array_equal(meta[:, c], ometa[:, c]), c
    assert np.array_equal(offs[:-1], ometa[:, 4]) and offs[-1] == ovals.size
    for d in range(dep.shape[0]):
        o, n = ometa[d, 4], ometa[d, 2] * ometa[d, 3]
        if n and np.abs(ovals[o:o + n]).max() > 0:
            assert normwise(vals[o:o + n], ovals[o:o + n]) <= GRID_TOL, d
    grid = torch.full((P.npitch, P.nticks), 5.0, device="cuda")
    ws.scatter_add(P, pt, grid, zero_first=True)
    G = O.grid(dep, phys, pl, seed)
    if np.abs(G).max() > 0:
        assert normwise(grid.cpu().numpy(), G) <= GRID_TOL
    pt.destroy()
    rng = np.random.default_rng(seed)
    g = rng.normal(0.0, 1.0, (P.npitch, P.nticks)).astype(np.float32)
    full = O.convolve(g.astype(np.float64), R.astype(np.float64), r0)
    out = ws.convolve(P, torch.from_numpy(g).cuda(), kind=ws.OUT_PITCH).cpu().numpy()
    assert normwise(out, full) <= CONV_TOL
    outw = ws.convolve(P, torch.from_numpy(g).cuda(), kind=ws.OUT_WIRE).cpu().numpy()
    assert normwise(outw, O.wire_rows(full, pl["nimpact"])) <= CONV_TOL
