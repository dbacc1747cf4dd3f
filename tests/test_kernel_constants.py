"""Constants typed into the HIP sources, checked on the CPU against the
mathematics they stand for."""
import os
import re

import numpy as np
from scipy import special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RASTER = os.path.join(ROOT, "paper_2304_01841_amd", "csrc", "raster.hip")
FFT = os.path.join(ROOT, "paper_2304_01841_amd", "csrc", "fft.hip")


def _array(path, name):
    src = open(path).read()
    m = re.search(name + r"\[\d+\]\s*=\s*\{([^}]*)\}", src)
    assert m, name
    return np.array([float(v) for v in m.group(1).replace("\n", " ").split(",") if v.strip()])


def test_record_erfc_tail_matches_erfc():
    """The record kernel's erfc(x) = exp(-x^2) * sum_j m_j u^j,
    u = 9 / (3 + min(x, 6)) - 2, evaluated by the same Horner rule in float64
    (the reciprocal rounded once, as the kernel's Newton-refined reciprocal
    gives it to within an ulp), is within 4e-15 of erfc on [0, 6] (relative)
    and within 1e-17 of it beyond (absolute); and the coefficients are
    well conditioned for Horner's rule (their magnitudes sum to about 1)."""
    m = _array(RASTER, "kErfcxPoly")
    assert m.size == 19
    assert np.abs(m).sum() < 1.001

    def tail(x):
        u = 9.0 * (1.0 / (3.0 + np.minimum(x, 6.0))) - 2.0
        p = np.full_like(x, m[18])
        for k in range(17, -1, -1):
            p = p * u + m[k]
        return np.exp(-x * x) * p

    x = np.linspace(0.0, 6.0, 60001)
    ref = special.erfc(x)
    assert np.max(np.abs(tail(x) / ref - 1.0)) < 4e-15
    xb = np.linspace(6.0, 40.0, 3401)
    assert np.max(np.abs(tail(xb) - special.erfc(xb))) < 1e-17


def test_record_reciprocal_refinement_reaches_double_precision():
    """Two Newton steps r <- r + r (1 - d r) from a reciprocal good to 2^-22
    (worse than the hardware's) give 1 / d to within 2 ulp for d in [3, 9]:
    each step squares the relative error.  Checked in float64 with the FMA
    residual formed exactly in 40-digit arithmetic."""
    import mpmath as mp
    mp.mp.dps = 40
    rng = np.random.default_rng(3)
    for d in np.concatenate([[3.0, 9.0, 4.5], rng.uniform(3.0, 9.0, 400)]):
        r = (1.0 / d) * (1.0 + float(rng.choice([-1, 1])) * 2.0 ** -22)
        for _ in range(2):
            e = float(1 - mp.mpf(d) * mp.mpf(r))  # fma(-d, r, 1)
            r = float(mp.mpf(r) * mp.mpf(e) + mp.mpf(r))  # fma(r, e, r)
        exact = mp.mpf(1) / mp.mpf(d)
        assert abs(mp.mpf(r) - exact) <= 2 * np.spacing(1.0 / d), d


def test_butterfly_constants_match_their_trig_values():
    """Every constexpr float of the FFT butterflies that names the value it
    stands for in a trailing comment (cos(2 pi / 5), sin(pi/8), ...) equals
    that value to the 20 digits printed (evaluated in 30-digit arithmetic)."""
    import mpmath as mp
    mp.mp.dps = 30
    src = open(FFT).read()
    found = re.findall(r"constexpr float \w+ = (-?[0-9.]+)f;\s*//\s*((?:cos|sin)\([^)]*\))", src)
    assert len(found) >= 8
    for value, expr in found:
        fn, arg = re.match(r"(cos|sin)\((.*)\)", expr).groups()
        num, _, den = arg.replace(" ", "").partition("/")
        k = mp.mpf(num.replace("pi", "") or 1)
        want = getattr(mp, fn)(k * mp.pi / mp.mpf(den or 1))
        assert abs(mp.mpf(value) - want) < mp.mpf("1e-19"), (value, expr)
    # the 8-point butterfly's cos(pi/4)
    m = re.search(r"constexpr float c = (0\.[0-9]+)f;", src)
    assert m and abs(mp.mpf(m.group(1)) - mp.sqrt(mp.mpf(1) / 2)) < mp.mpf("1e-19")
