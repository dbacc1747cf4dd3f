"""FP64 CPU oracle of the LArTPC signal-simulation hot path (arXiv:2304.01841).

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg import it; the product path never does.  It shares
no code with the GPU library: the per-depo arithmetic lives in
``wcsim_oracle.c`` (built here with gcc), and the convolution uses numpy/scipy
in float64.

Paper coverage (Sec. 2 lists the three steps of ``DepoTransform``):
  * Rasterization (Sec. 2 step 1)  -> :func:`rasterize`
  * Scatter-Add   (Sec. 2 step 2)  -> :func:`scatter`
  * Convolution   (Sec. 2 step 3)  -> :func:`convolve` (library FFT of the
    defining linear convolution) and :func:`convolve_points` /
    :func:`convolve_direct` (the defining double sum itself)
  * the wire waveform (Sec. 1: current induced in the wires) -> :func:`wire_rows`
The fluctuation random numbers follow the random123 Philox4x32-10 generator the
paper names for CPUs (Sec. 4.1; Salmon et al., SC'11).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wcsim_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libwcsim_oracle.so")

STATUS_OK, STATUS_INVALID, STATUS_EMPTY = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no FMA contraction, no fast math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                               "-fno-fast-math", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32
        lib.oracle_philox_batch.argtypes = [i64, P, P, P]
        lib.oracle_normal.argtypes = [i64, i64, i64, u64, u64, i32]
        lib.oracle_normal.restype = ctypes.c_double
        lib.oracle_surviving_charge.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                i32, i64, u64, u64]
        lib.oracle_surviving_charge.restype = ctypes.c_double
        lib.oracle_depo_window.argtypes = [P, P, P, P, P, P]
        lib.oracle_depo_window.restype = ctypes.c_int
        lib.oracle_axis_weights.argtypes = [i64, i64, ctypes.c_double, ctypes.c_double, P]
        lib.oracle_rasterize.argtypes = [P, i64, P, i32, u64, P, P, u64, P, P, P, i64, P]
        lib.oracle_rasterize.restype = i64
        lib.oracle_scatter.argtypes = [P, P, i64, i64, i64, P]
        lib.oracle_convolve_points.argtypes = [P, i64, i64, P, i64, i64, i64, P, i64, P]
        lib.oracle_convolve_direct.argtypes = [P, i64, i64, P, i64, i64, i64, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Problem description helpers (plain dictionaries, same fields as the C ABI)
# ---------------------------------------------------------------------------
def _phys_arr(phys: dict) -> np.ndarray:
    return np.array([phys["drift_speed"], phys["DL"], phys["DT"], phys["nsigma"],
                     phys.get("lifetime", 0.0), phys.get("drift_accel", 0.0)], dtype=np.float64)


def _geom_arr(plane: dict) -> np.ndarray:
    return np.array([plane["pitch"], plane["tick"], plane["t0"], plane["plane_x"], plane["dir_y"],
                     plane["dir_z"], plane["pitch_origin"]], dtype=np.float64)


def _dims_arr(plane: dict) -> np.ndarray:
    return np.array([plane["plane_id"], plane["nwires"], plane["nimpact"], plane["nticks"]],
                    dtype=np.int32)


def grid_shape(plane: dict) -> tuple[int, int]:
    return plane["nwires"] * plane["nimpact"], plane["nticks"]


# ---------------------------------------------------------------------------
# Philox4x32-10 and the normal deviates it feeds
# ---------------------------------------------------------------------------
def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr: (n, 4) uint32, key: (n, 2) uint32 -> (n, 4) uint32."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    assert ctr.shape[0] == key.shape[0]
    out = np.empty_like(ctr)
    _load().oracle_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def normal(I: int, J: int, d: int, event_id: int, seed: int, plane_id: int) -> float:
    """Standard normal deviate that fluctuates absolute bin (I, J) of depo d."""
    return _load().oracle_normal(I, J, d, event_id & (2**64 - 1), seed & (2**64 - 1), plane_id)


def surviving_charge(q: float, T: float, tau: float, fluctuate: bool, d: int, event_id: int,
                     seed: int) -> float:
    """Electrons of a depo that survive drift time T with electron lifetime
    tau (0: no absorption); see oracle_surviving_charge.  The draw depends on
    the depo and the event only, never on a plane."""
    return _load().oracle_surviving_charge(q, T, tau, int(bool(fluctuate)), d,
                                           event_id & (2**64 - 1), seed & (2**64 - 1))


def combined_response(R: np.ndarray, E) -> np.ndarray:
    """Detector response followed by an electronics response along ticks (an
    extension beyond the paper): each response row convolved with E, FP64,
    Rp x (Rt + len(E) - 1); E empty or None leaves R unchanged."""
    R = np.asarray(R, np.float64)
    if E is None or np.size(E) == 0:
        return R.copy()
    E = np.asarray(E, np.float64).reshape(-1)
    return np.stack([np.convolve(R[r], E) for r in range(R.shape[0])])


# ---------------------------------------------------------------------------
# Digitisation with white noise (an extension beyond the paper, which ends at
# the current induced on the wires)
# ---------------------------------------------------------------------------
DIGITIZE_KEY_XOR = 0x6E6F6973  # XORed into the seed's low word for the noise stream


def digitize_normals(nrows: int, ncols: int, seed: int, event_id: int) -> np.ndarray:
    """Standard normal per sample (row, col): Philox4x32-10 under the key
    (seed low word ^ 0x6e6f6973, seed high word) at counter (col // 4, row, 0,
    event low word); words (0,1) serve columns with col % 4 in {0,1}, words
    (2,3) the others, each pair through Box-Muller (cosine branch to the even
    column), the uniform of a word r being ((r >> 9) + 1/2) 2^-23.  FP64."""
    nq = (ncols + 3) // 4
    q, r = np.meshgrid(np.arange(nq), np.arange(nrows))
    ctr = np.stack([q.ravel(), r.ravel(), np.zeros(q.size, np.int64),
                    np.full(q.size, event_id & 0xFFFFFFFF)], axis=1).astype(np.uint32)
    key = np.tile(np.array([(seed & 0xFFFFFFFF) ^ DIGITIZE_KEY_XOR, (seed >> 32) & 0xFFFFFFFF],
                           np.uint32), (q.size, 1))
    words = philox4x32_10(ctr, key).astype(np.float64).reshape(nrows, nq, 4)
    u = (np.floor(words / 512.0) + 0.5) * 2.0 ** -23
    z = np.empty((nrows, nq, 4))
    for a in (0, 2):
        rho = np.sqrt(-2.0 * np.log(u[..., a]))
        theta = 2.0 * np.pi * u[..., a + 1]
        z[..., a] = rho * np.cos(theta)
        z[..., a + 1] = rho * np.sin(theta)
    return z.reshape(nrows, 4 * nq)[:, :ncols]


def coloured_noise(nrows: int, ncols: int, seed: int, event_id: int, fir) -> np.ndarray:
    """White deviates (digitize_normals) filtered by the causal FIR `fir`:
    n[r][c] = sum_k fir[k] z[r][c - k], no white noise before column 0. FP64."""
    z = digitize_normals(nrows, ncols, seed, event_id)
    h = np.asarray(fir, np.float64).reshape(-1)
    return np.stack([np.convolve(z[r], h)[:ncols] for r in range(nrows)]) if nrows else z


def digitize(wave: np.ndarray, gain: float, pedestal: float, sigma: float, bits: int, seed: int,
             event_id: int, fir=None) -> np.ndarray:
    """ADC codes min(max(rint(((w gain) + pedestal) + sigma n), 0), 2^bits - 1)
    as uint16, with float32 arithmetic in that order (each operation rounded,
    no fused multiply-add) and rint rounding half to even; n is the white
    deviate, or with `fir` the coloured noise."""
    w = np.asarray(wave, np.float32)
    f32 = np.float32
    v = w * f32(gain)
    v = v + f32(pedestal)
    if sigma > 0:
        if fir is None:
            z = digitize_normals(w.shape[0], w.shape[1], seed, event_id).astype(np.float32)
        else:
            z = coloured_noise(w.shape[0], w.shape[1], seed, event_id, fir).astype(np.float32)
        v = v + f32(sigma) * z
    v = np.rint(v)
    v = np.minimum(np.maximum(v, f32(0.0)), f32(2 ** bits - 1))
    return v.astype(np.uint16)


# ---------------------------------------------------------------------------
# Rasterization and Scatter-Add (Sec. 2 steps 1 and 2)
# ---------------------------------------------------------------------------
def _window(depo, phys: dict, plane: dict):
    d = np.ascontiguousarray(depo, dtype=np.float64).reshape(5)
    od = np.zeros(5, np.float64)
    oi = np.zeros(4, np.int64)
    st = _load().oracle_depo_window(_ptr(d), _ptr(_phys_arr(phys)), _ptr(_geom_arr(plane)),
                                    _ptr(_dims_arr(plane)), _ptr(od), _ptr(oi))
    return st, od, oi


def depo_window(depo, phys: dict, plane: dict):
    """(status, (mu_p, s_p, mu_t, s_t), (lo_p, lo_t, n_p, n_t)) of one depo."""
    st, od, oi = _window(depo, phys, plane)
    return st, tuple(od[:4].tolist()), tuple(int(v) for v in oi)


def drift_time(depo, phys: dict, plane: dict) -> float:
    """Drift time T (us) of one depo to the response plane (0 for an invalid
    depo)."""
    st, od, _ = _window(depo, phys, plane)
    return float(od[4]) if st != STATUS_INVALID else 0.0


def axis_weights(lo: int, n: int, mu: float, s: float) -> np.ndarray:
    W = np.zeros(n, np.float64)
    _load().oracle_axis_weights(lo, n, mu, s, _ptr(W))
    return W


def rasterize(depos: np.ndarray, phys: dict, plane: dict, event_id: int = 0, ids=None):
    """Patches of all depos.

    Returns (meta, values, status): meta is (n, 5) int64 rows
    (lo_p, lo_t, n_p, n_t, offset); values the flat float64 patch values
    (row-major n_p x n_t per depo, at its offset); status per depo
    (0 ok, 1 invalid, 2 window misses the grid).  `ids`: the depos' indices
    in their event (default 0..n-1), which key the fluctuation."""
    depos = np.ascontiguousarray(depos, dtype=np.float64).reshape(-1, 5)
    n = depos.shape[0]
    ids_arr = None if ids is None else np.ascontiguousarray(ids, dtype=np.int64).reshape(n)
    meta = np.zeros((n, 5), np.int64)
    status = np.zeros(n, np.int32)
    lib = _load()
    args = (_ptr(_phys_arr(phys)), int(phys["fluctuate"]), int(phys["seed"]) & (2**64 - 1),
            _ptr(_geom_arr(plane)), _ptr(_dims_arr(plane)), int(event_id) & (2**64 - 1))
    cap = max(1, 400 * n)
    while True:
        values = np.zeros(cap, np.float64)
        got = lib.oracle_rasterize(_ptr(depos), n, args[0], args[1], args[2], args[3], args[4],
                                   args[5], None if ids_arr is None else _ptr(ids_arr), _ptr(meta),
                                   _ptr(values), cap, _ptr(status))
        if got >= 0:
            return meta, values[:got], status
        cap = -got


def scatter(meta: np.ndarray, values: np.ndarray, plane: dict) -> np.ndarray:
    Np, Nt = grid_shape(plane)
    meta = np.ascontiguousarray(meta, dtype=np.int64)
    values = np.ascontiguousarray(values, dtype=np.float64)
    G = np.zeros((Np, Nt), np.float64)
    _load().oracle_scatter(_ptr(meta), _ptr(values), meta.shape[0], Np, Nt, _ptr(G))
    return G


def grid(depos: np.ndarray, phys: dict, plane: dict, event_id: int = 0, ids=None) -> np.ndarray:
    meta, values, _ = rasterize(depos, phys, plane, event_id, ids)
    return scatter(meta, values, plane)


# ---------------------------------------------------------------------------
# Convolution (Sec. 2 step 3)
# ---------------------------------------------------------------------------
def convolve_points(G: np.ndarray, R: np.ndarray, r0: int, pts) -> np.ndarray:
    """Defining double sum at the listed (p, t) points."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.int64).reshape(-1, 2)
    out = np.zeros(pts.shape[0], np.float64)
    _load().oracle_convolve_points(_ptr(G), G.shape[0], G.shape[1], _ptr(R), R.shape[0],
                                   R.shape[1], r0, _ptr(pts), pts.shape[0], _ptr(out))
    return out


def convolve_direct(G: np.ndarray, R: np.ndarray, r0: int) -> np.ndarray:
    """Defining double sum over the whole grid (tiny grids only)."""
    G = np.ascontiguousarray(G, dtype=np.float64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    O = np.zeros_like(G)
    _load().oracle_convolve_direct(_ptr(G), G.shape[0], G.shape[1], _ptr(R), R.shape[0],
                                   R.shape[1], r0, _ptr(O))
    return O


def convolve(G: np.ndarray, R: np.ndarray, r0: int, workers: int = 1) -> np.ndarray:
    """Linear 2-D convolution of the grid with the response, float64.

    The full linear convolution is taken with a library FFT (zero padding to at
    least (Np + Rp - 1) x (Nt + Rt - 1), so no wrap-around) and cropped to the
    grid: output row p takes full-convolution row p + r0 (response row r0 is
    aligned with the output row) and output tick t takes full tick t (causal)."""
    import scipy.fft as sfft

    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    Np, Nt = G.shape
    Rp, Rt = R.shape
    M = sfft.next_fast_len(Np + Rp - 1, real=True)
    N = sfft.next_fast_len(Nt + Rt - 1, real=True)
    Gh = sfft.rfft2(G, s=(M, N), workers=workers)
    Rh = sfft.rfft2(R, s=(M, N), workers=workers)
    full = sfft.irfft2(Gh * Rh, s=(M, N), workers=workers)
    return np.ascontiguousarray(full[r0:r0 + Np, :Nt])


def wire_rows(O: np.ndarray, nimpact: int) -> np.ndarray:
    """Wire waveforms: the impact row at the centre of each wire's pitch cell."""
    return np.ascontiguousarray(O[nimpact // 2::nimpact])


def simulate_event(depos: np.ndarray, phys: dict, plane: dict, response: np.ndarray, r0: int,
                   event_id: int = 0, wire_output: bool = True, workers: int = 1):
    """Whole DepoTransform path: patches -> grid -> convolved plane (-> wires)."""
    G = grid(depos, phys, plane, event_id)
    O = convolve(G, response, r0, workers=workers)
    return wire_rows(O, plane["nimpact"]) if wire_output else O
