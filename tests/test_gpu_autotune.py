"""GPU: the schedule tuner times candidate schedules through the C ABI, flags
invalid ones, and the schedule it picks gives the oracle's result."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2304_01841_amd import workloads as W

pytestmark = pytest.mark.gpu

CONV_TOL = 1e-4


@pytest.fixture(scope="module")
def ws():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2304_01841_amd import wcsim
    return wcsim


def normwise(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(np.asarray(got, np.float64) - ref).max() / np.abs(ref).max()


def test_tune_schedules_times_valid_and_flags_invalid(ws):
    print("case: tune_schedules small plane", flush=True)
    w = W.small()
    pl, R = w["planes"][0], w["responses"][0]
    dep = torch.from_numpy(w["depos"]).cuda()
    cands = [{}, {"fft_pitch": 512, "freq_chunk": 16}, {"fft_pitch": 100}, {"freq_chunk": 12},
             {"tile": 2}]
    ms = ws.tune_schedules(pl, W.physics(True), R, dep, cands, reps=2)
    assert ms[0] > 0 and ms[1] > 0 and ms[4] > 0
    assert ms[2] == -1.0 and ms[3] == -1.0
    with pytest.raises(ws.WcsimError):
        ws.tune_schedules(pl, W.physics(True), R, dep, [{"fft_pitch": 100}], reps=1)


def test_tuned_schedule_matches_oracle_and_is_cached(ws, tmp_path):
    from paper_2304_01841_amd import autotune
    print("case: tuner small plane", flush=True)
    w = W.small()
    pl, R = w["planes"][0], w["responses"][0]
    phys = W.physics(True)
    dep = torch.from_numpy(w["depos"]).cuda()
    path = str(tmp_path / "tune.json")
    t = autotune.Tuner(path, reps=2)
    sched = t.tune(pl, phys, R, dep)
    assert sched in autotune.candidates()
    P = ws.Plane(pl, phys, R, schedule=sched)
    out = ws.simulate_event(P, dep, 3, kind=ws.OUT_WIRE).cpu().numpy()
    ref = O.simulate_event(w["depos"], phys, pl, R.astype(np.float64), P.r0, 3,
                           wire_output=True)
    assert normwise(out, ref) <= CONV_TOL
    # a second tuner reads the file and needs no timing
    t2 = autotune.Tuner(path)
    assert t2.lookup(pl, R, P.r0, True, dep.shape[0]) == sched
    P.destroy()


def test_batch_tuned_schedule_matches_oracle_and_is_cached(ws, tmp_path):
    """tune_batch times every candidate on a class of events run as one batch:
    the schedule it picks is a candidate, gives every event the oracle's
    output through the batched form, and is cached under the class's key."""
    from paper_2304_01841_amd import autotune
    print("case: batch tuner, small planes", flush=True)
    w = W.small()
    pl, R = w["planes"][0], w["responses"][0]
    phys = W.physics(True)
    rng = np.random.default_rng(12)
    deps_np = [w["depos"], W.uniform_depos(rng, 300, (0.0, 400.0), (0.0, 450.0))]
    deps = [torch.from_numpy(np.ascontiguousarray(d)).cuda() for d in deps_np]
    path = str(tmp_path / "tune.json")
    t = autotune.Tuner(path, reps=2)
    sched = t.tune_batch(pl, phys, R, deps)
    assert sched in autotune.candidates()
    key = next(k for k in t.table if k.startswith("batch2|"))
    assert sum(c["ms"] > 0 for c in t.entry(key)["candidates"]) >= 2
    P = ws.Plane(pl, phys, R, schedule=sched)
    outs = [torch.empty((P.nwires, P.nticks), device="cuda") for _ in deps]
    ws.simulate_batch([P, P], deps, [5, 6], outs)
    for d, e, o in zip(deps_np, (5, 6), outs):
        ref = O.simulate_event(d, phys, pl, R.astype(np.float64), P.r0, e, wire_output=True)
        assert normwise(o.cpu().numpy(), ref) <= CONV_TOL
    assert autotune.Tuner(path).tune_batch(pl, phys, R, deps) == sched  # from the file
