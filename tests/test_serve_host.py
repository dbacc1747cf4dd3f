"""Host-side request checks of the server (no GPU): a request the library
would reject is recognised before admission, so it can fail alone."""
import numpy as np

from paper_2304_01841_amd import workloads as W


def test_validate_request_flags_what_the_library_rejects():
    from paper_2304_01841_amd import serve
    phys = W.physics(True)
    ok = W.serve_requests(seed=1, nreq=1, lo=3.0, hi=3.2, nticks=600)[0]
    assert serve.validate_request(ok, phys) is None
    for field, value, what in [(1, np.inf, "non-finite"), (4, -1.0, "negative"),
                               (0, -0.5, "behind")]:
        r = dict(ok, depos=ok["depos"].copy())
        r["depos"][3, field] = value
        assert what in serve.validate_request(r, phys)
    far = dict(ok, depos=ok["depos"].copy())
    far["depos"][0, 0] = 3000.0
    assert serve.validate_request(far, dict(phys, drift_accel=1e-3)) is not None
    assert serve.validate_request(far, phys) is None
