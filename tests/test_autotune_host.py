"""Host-side logic of the schedule autotuner (no GPU): candidate list, cache
keys and the JSON cache file."""
import json

import numpy as np
import pytest

from paper_2304_01841_amd import workloads as W

autotune = pytest.importorskip("paper_2304_01841_amd.autotune")


def test_candidates_start_with_the_default_and_are_distinct():
    c = autotune.candidates()
    assert c[0] == {}
    keys = {json.dumps(x, sort_keys=True) for x in c}
    assert len(keys) == len(c)
    for x in c:
        assert set(x) <= {"fft_ticks", "fft_pitch", "freq_chunk", "tile", "wire_mode"}


def test_cache_key_separates_shapes_and_depo_scales():
    pl = W.plane(960, 6000)
    R = np.zeros((210, 200), np.float32)
    k = autotune.cache_key(pl, R, 105, True, 500000, 0, device_arch="gfx950")
    assert k == autotune.cache_key(pl, R, 105, True, 400000, 0, device_arch="gfx950")
    assert k != autotune.cache_key(pl, R, 105, True, 100000, 0, device_arch="gfx950")
    assert k != autotune.cache_key(W.plane(800, 6000), R, 105, True, 500000, 0,
                                   device_arch="gfx950")
    assert k != autotune.cache_key(pl, R, 105, False, 500000, 0, device_arch="gfx950")
    assert k != autotune.cache_key(pl, R, 105, True, 500000, 1, device_arch="gfx950")
    assert k.startswith("gfx950|")


def test_cache_file_is_loaded(tmp_path):
    pl = W.plane(100, 1000)
    R = np.zeros((31, 17), np.float32)
    key = autotune.cache_key(pl, R, 15, False, 1000, 0, device_arch="gfx950")
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({key: {"schedule": {"fft_pitch": 512, "freq_chunk": 16},
                                      "ms": 1.0}}))
    t = autotune.Tuner(str(path))
    assert t.entry(key)["schedule"] == {"fft_pitch": 512, "freq_chunk": 16}
