"""Thin ctypes binding of ``libbnlat.so`` (the C ABI in include/bnlat.h).

Every function here only marshals arguments: the computation runs in the
library's gfx950 kernels.  Names match the C entry points without the
``bn_`` prefix.  Failures raise :class:`BnlatError` carrying the status and
the library's message.  The module refuses to work without the built
library; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BNLAT_LIB names another build of the same library (e.g. a host-sanitized test build)
LIB_PATH = os.environ.get("BNLAT_LIB") or os.path.join(HERE, "libbnlat.so")

BN_OK, BN_EINVAL, BN_ENOMEM, BN_EHIP, BN_ESTATE, BN_EUNSUPPORTED, BN_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
BN_FP32, BN_BF16 = 0, 1
BN_REDRAW, BN_SWAP = 0, 1
BN_ROWS_ALL, BN_ROWS_HEAVISIDE, BN_ROWS_GAUSSIAN = 0, 1, 2
BN_PEAK_HBM_COPY, BN_PEAK_VALU_DOT2, BN_PEAK_MFMA_BF16 = 0, 1, 2


class BnlatError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: status {status}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("n", C.c_uint32), ("g", C.c_uint32 * 2), ("width", C.c_uint32),
                ("height", C.c_uint32), ("t_heaviside", C.c_uint32), ("t_gauss", C.c_uint32),
                ("sigma", C.c_double), ("radius", C.c_uint32), ("colour_k", C.c_uint32),
                ("objective", C.c_int32), ("seed", C.c_uint64), ("problem_id", C.c_uint32),
                ("precision", C.c_int), ("move", C.c_int)]


class Heaviside(C.Structure):
    _fields_ = [("nx", C.c_int16), ("ny", C.c_int16), ("cx", C.c_uint16), ("cy", C.c_uint16)]


class SweepStats(C.Structure):
    _fields_ = [("proposals", C.c_uint64), ("accepts", C.c_uint64), ("bf16_vetoes", C.c_uint64),
                ("sweep_index", C.c_uint64)]


class ProfileStats(C.Structure):
    _fields_ = [("recount_launches", C.c_uint64), ("recount_ms", C.c_double), ("phases", C.c_uint64),
                ("evaluate_ms", C.c_double), ("commit_ms", C.c_double)]


HEAVISIDE_DTYPE = np.dtype([("nx", "<i2"), ("ny", "<i2"), ("cx", "<u2"), ("cy", "<u2")])
GAUSSIAN_DTYPE = np.dtype([("mx", "<f8"), ("my", "<f8"), ("s", "<f8")])


class DeviceBuffers(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("counts", C.c_void_p), ("errors", C.c_void_p)]


class Gaussian(C.Structure):
    _fields_ = [("mx", C.c_double), ("my", C.c_double), ("s", C.c_double)]

_P = C.c_void_p
_SIGNATURES = {
    "bn_create_problem": [C.POINTER(Config), _P, _P, _P, C.POINTER(_P)],
    "bn_destroy_problem": [_P],
    "bn_create_problem_ext": [C.POINTER(Config), _P, _P, _P, _P, C.POINTER(_P)],
    "bn_init_offsets": [_P, _P],
    "bn_compute_errors": [_P],
    "bn_sweep": [_P, C.c_uint32, C.POINTER(SweepStats)],
    "bn_energy": [_P, C.POINTER(C.c_double)],
    "bn_energy_bf16": [_P, C.POINTER(C.c_double)],
    "bn_get_phase_bf16": [_P, _P],
    "bn_quality_metric": [_P, _P, C.c_uint32, _P],
    "bn_quality_metric_family": [_P, C.c_int, _P, C.c_uint32, _P],
    "bn_error_spectrum": [_P, C.c_int, C.c_uint32, _P, _P],
    "bn_get_offsets": [_P, _P],
    "bn_get_counts": [_P, _P],
    "bn_get_errors": [_P, _P],
    "bn_get_integrands": [_P, _P, _P, _P, _P],
    "bn_get_points": [_P, C.c_uint32, _P],
    "bn_delta_energy": [_P, _P, _P, C.c_uint32, _P, _P],
    "bn_delta_energy_noalloc": [_P, _P, _P, C.c_uint32, _P, _P],
    "bn_get_sweep_index": [_P, C.POINTER(C.c_uint64)],
    "bn_set_sweep_index": [_P, C.c_uint64],
    "bn_set_profiling": [_P, C.c_int],
    "bn_set_recount_blocks": [_P, C.c_uint32],
    "bn_get_profile": [_P, C.POINTER(ProfileStats)],
    "bn_phase_propose": [_P, C.c_uint32],
    "bn_phase_evaluate": [_P, C.c_uint32],
    "bn_phase_commit": [_P, C.c_uint32],
    "bn_phase_advance": [_P],
    "bn_get_phase": [_P, _P, _P, _P, _P],
    "bn_get_swap_pass": [_P, _P, _P, _P, _P],
    "bn_sample": [_P, C.c_uint32, _P, _P, _P, C.c_uint32, _P],
    "bn_sample_device": [_P, C.c_uint32, _P, _P, _P, C.c_uint32, _P, _P],
    "bn_create_batch": [_P, C.c_uint32, C.c_char_p, C.POINTER(_P)],
    "bn_batch_sweep": [_P, C.c_uint32],
    "bn_destroy_batch": [_P],
    "bn_batch_tuning": [_P, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)],
    "bn_validate_config": [C.POINTER(Config)],
    "bn_swap_permutation": [C.POINTER(Config), _P],
    "bn_window_classes": [C.POINTER(Config), C.POINTER(C.c_uint32), _P, _P],
    "bn_heaviside_area": [C.POINTER(Heaviside), C.POINTER(C.c_double)],
    "bn_draw_heavisides": [C.c_uint64, C.c_uint32, C.c_uint32, _P],
    "bn_draw_gaussians": [C.c_uint64, C.c_uint32, C.c_uint32, _P],
    "bn_gaussian_integral": [C.POINTER(Gaussian), C.POINTER(C.c_double)],
    "bn_measure_peak": [C.c_int, C.c_uint64, C.c_uint32, C.POINTER(C.c_double)],
}

_lib = None


def lib():
    """Load ``libbnlat.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2105_12620_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.bn_status_string.argtypes = [C.c_int]
        L.bn_status_string.restype = C.c_char_p
        L.bn_last_error.argtypes = []
        L.bn_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _call(name, *args):
    st = getattr(lib(), name)(*args)
    if st != BN_OK:
        raise BnlatError(st, name, lib().bn_last_error().decode(errors="replace"))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_config(n, g, width, height, t_heaviside, sigma=2.1, radius=3, colour_k=2, objective=1,
                seed=0, problem_id=0, t_gauss=0, precision=BN_FP32, move=BN_REDRAW, **_ignored) -> Config:
    c = Config()
    c.n, c.width, c.height = n, width, height
    c.g[0], c.g[1] = int(g[0]), int(g[1])
    c.t_heaviside, c.t_gauss, c.sigma, c.radius = t_heaviside, t_gauss, sigma, radius
    c.colour_k, c.objective, c.seed, c.problem_id = colour_k, objective, seed, problem_id
    c.precision, c.move = precision, move
    return c


def heaviside_array(table: dict) -> np.ndarray:
    """synthgen Heaviside table -> packed bn_heaviside array."""
    out = np.empty(len(table["nx"]), dtype=HEAVISIDE_DTYPE)
    for k in ("nx", "ny", "cx", "cy"):
        out[k] = table[k]
    return out


# ------------------------------------------------------------ host-only calls
def validate_config(cfg: Config) -> None:
    _call("bn_validate_config", C.byref(cfg))


def swap_permutation(cfg: Config) -> np.ndarray:
    """Pixel permutation of the swap mutation (host computation)."""
    out = np.zeros(cfg.width * cfg.height, dtype=np.uint32)
    _call("bn_swap_permutation", C.byref(cfg), _ptr(out))
    return out


def window_classes(cfg: Config):
    n = C.c_uint32(0)
    _call("bn_window_classes", C.byref(cfg), C.byref(n), None, None)
    d = np.zeros(n.value, dtype=np.uint32)
    w = np.zeros(n.value, dtype=np.float64)
    _call("bn_window_classes", C.byref(cfg), C.byref(n), _ptr(d), _ptr(w))
    return d, w


def heaviside_area(nx, ny, cx, cy) -> float:
    h = Heaviside(int(nx), int(ny), int(cx), int(cy))
    out = C.c_double()
    _call("bn_heaviside_area", C.byref(h), C.byref(out))
    return out.value


def draw_heavisides(seed: int, problem_id: int, t: int) -> np.ndarray:
    out = np.zeros(t, dtype=HEAVISIDE_DTYPE)
    _call("bn_draw_heavisides", seed, problem_id, t, _ptr(out))
    return out


def gaussian_array(table: dict) -> np.ndarray:
    """synthgen Gaussian table -> packed bn_gaussian array."""
    out = np.empty(len(table["mx"]), dtype=GAUSSIAN_DTYPE)
    for k in ("mx", "my", "s"):
        out[k] = table[k]
    return out


def draw_gaussians(seed: int, problem_id: int, t: int) -> np.ndarray:
    out = np.zeros(t, dtype=GAUSSIAN_DTYPE)
    _call("bn_draw_gaussians", seed, problem_id, t, _ptr(out))
    return out


def gaussian_integral(mx, my, s) -> float:
    g = Gaussian(float(mx), float(my), float(s))
    out = C.c_double()
    _call("bn_gaussian_integral", C.byref(g), C.byref(out))
    return out.value


def measure_peak(kind: int, nbytes: int = 0, reps: int = 5) -> float:
    """Best rate of a plain device loop: bytes/s (copy), lane-ops/s (dot2) or flop/s (BF16 MFMA)."""
    out = C.c_double()
    _call("bn_measure_peak", kind, nbytes, reps, C.byref(out))
    return out.value


# ------------------------------------------------------------------- problems
class Problem:
    """Owns one ``bn_problem`` handle."""

    def __init__(self, cfg: Config, heavisides: np.ndarray | None = None, stream: int | None = None,
                 gaussians: np.ndarray | None = None, buffers: tuple | None = None):
        """buffers: optional (offsets, counts, errors) device addresses the
        caller owns (bn_create_problem_ext); None entries are allocated by
        the library."""
        self.cfg = cfg
        self.P = cfg.width * cfg.height
        self.T = cfg.t_heaviside
        self.TG = cfg.t_gauss
        self.M = self.P // (cfg.colour_k * cfg.colour_k)
        h = None if heavisides is None else np.ascontiguousarray(heavisides, dtype=HEAVISIDE_DTYPE)
        if h is not None and h.shape[0] != cfg.t_heaviside:
            raise ValueError("heaviside table length differs from t_heaviside")
        g = None if gaussians is None else np.ascontiguousarray(gaussians, dtype=GAUSSIAN_DTYPE)
        if g is not None and g.shape[0] != cfg.t_gauss:
            raise ValueError("gaussian table length differs from t_gauss")
        handle = C.c_void_p()
        if buffers is None:
            _call("bn_create_problem", C.byref(cfg), _ptr(h), _ptr(g), C.c_void_p(stream or 0), C.byref(handle))
        else:
            b = DeviceBuffers(*[C.c_void_p(x) if x else None for x in buffers])
            _call("bn_create_problem_ext", C.byref(cfg), _ptr(h), _ptr(g), C.c_void_p(stream or 0),
                  C.byref(b), C.byref(handle))
        self.handle = handle

    def close(self):
        if getattr(self, "handle", None):
            _call("bn_destroy_problem", self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # lifecycle
    def init_offsets(self, u: np.ndarray | None = None):
        a = None if u is None else np.ascontiguousarray(u, dtype=np.uint16).reshape(self.cfg.height, self.cfg.width, 2)
        _call("bn_init_offsets", self.handle, _ptr(a))

    def compute_errors(self):
        _call("bn_compute_errors", self.handle)

    def sweep(self, k: int = 1, stats: bool = False):
        st = SweepStats() if stats else None
        _call("bn_sweep", self.handle, k, C.byref(st) if st is not None else None)
        if st is not None:
            return {"proposals": st.proposals, "accepts": st.accepts,
                    "bf16_vetoes": st.bf16_vetoes, "sweep_index": st.sweep_index}
        return None

    def energy(self) -> float:
        out = C.c_double()
        _call("bn_energy", self.handle, C.byref(out))
        return out.value

    def energy_bf16(self) -> float:
        """Eq. (1) from the BF16 field (BF16 precision form only)."""
        out = C.c_double()
        _call("bn_energy_bf16", self.handle, C.byref(out))
        return out.value

    def quality_metric(self, sigmas, rows: int = 0) -> np.ndarray:
        """Blur criterion per sigma over all rows (0), Heaviside rows (1) or Gaussian rows (2)."""
        s = np.ascontiguousarray(sigmas, dtype=np.float64)
        out = np.zeros_like(s)
        if rows:
            _call("bn_quality_metric_family", self.handle, rows, _ptr(s), s.shape[0], _ptr(out))
        else:
            _call("bn_quality_metric", self.handle, _ptr(s), s.shape[0], _ptr(out))
        return out

    def error_spectrum(self, nbins: int, rows: int = 0):
        """Radially averaged |DFT2(e_t)|^2 / P: (mean power [nbins], frequencies per bin)."""
        out = np.zeros(nbins, dtype=np.float64)
        cnt = np.zeros(nbins, dtype=np.uint32)
        _call("bn_error_spectrum", self.handle, rows, nbins, _ptr(out), _ptr(cnt))
        return out, cnt

    def get_offsets(self) -> np.ndarray:
        out = np.zeros((self.cfg.height, self.cfg.width, 2), dtype=np.uint16)
        _call("bn_get_offsets", self.handle, _ptr(out))
        return out

    # inspection
    def get_counts(self) -> np.ndarray:
        out = np.zeros((self.P, self.T), dtype=np.uint16)
        _call("bn_get_counts", self.handle, _ptr(out))
        return out

    def get_errors(self) -> np.ndarray:
        """float32 [P, T + T_G]: Heaviside rows, then Gaussian rows."""
        out = np.zeros((self.P, self.T + self.TG), dtype=np.float32)
        _call("bn_get_errors", self.handle, _ptr(out))
        return out

    def get_integrands(self, gaussians: bool = False):
        h = np.zeros(self.T, dtype=HEAVISIDE_DTYPE)
        a = np.zeros(self.T, dtype=np.float64)
        g = np.zeros(self.TG, dtype=GAUSSIAN_DTYPE)
        gi = np.zeros(self.TG, dtype=np.float64)
        _call("bn_get_integrands", self.handle, _ptr(h), _ptr(a), _ptr(g), _ptr(gi))
        return (h, a, g, gi) if gaussians else (h, a)

    def get_points(self, pixel: int) -> np.ndarray:
        out = np.zeros((self.cfg.n, 2), dtype=np.uint16)
        _call("bn_get_points", self.handle, pixel, _ptr(out))
        return out

    def delta_energy(self, pixels, proposals, counts: bool = False):
        px = np.ascontiguousarray(pixels, dtype=np.uint32)
        pr = np.ascontiguousarray(proposals, dtype=np.uint16).reshape(-1, 2)
        m = px.shape[0]
        de = np.zeros(m, dtype=np.float64)
        cn = np.zeros((m, self.T), dtype=np.uint16) if counts else None
        _call("bn_delta_energy", self.handle, _ptr(px), _ptr(pr), m, _ptr(de), _ptr(cn))
        return (de, cn) if counts else de

    def delta_energy_noalloc(self, pixels, proposals, counts: bool = False):
        """bn_delta_energy_noalloc: the same as delta_energy, with its list
        buffers in the library's fixed per-GPU scratch array."""
        px = np.ascontiguousarray(pixels, dtype=np.uint32)
        pr = np.ascontiguousarray(proposals, dtype=np.uint16).reshape(-1, 2)
        m = px.shape[0]
        de = np.zeros(m, dtype=np.float64)
        cn = np.zeros((m, self.T), dtype=np.uint16) if counts else None
        _call("bn_delta_energy_noalloc", self.handle, _ptr(px), _ptr(pr), m, _ptr(de), _ptr(cn))
        return (de, cn) if counts else de

    def get_sweep_index(self) -> int:
        out = C.c_uint64()
        _call("bn_get_sweep_index", self.handle, C.byref(out))
        return out.value

    def set_sweep_index(self, s: int):
        _call("bn_set_sweep_index", self.handle, s)

    def set_profiling(self, enable: bool):
        _call("bn_set_profiling", self.handle, 1 if enable else 0)

    def set_recount_blocks(self, blocks: int):
        _call("bn_set_recount_blocks", self.handle, blocks)

    def get_profile(self) -> dict:
        st = ProfileStats()
        _call("bn_get_profile", self.handle, C.byref(st))
        return {k: getattr(st, k) for k, _ in ProfileStats._fields_}

    # phase steps
    def phase_propose(self, kappa: int):
        _call("bn_phase_propose", self.handle, kappa)

    def phase_evaluate(self, kappa: int):
        _call("bn_phase_evaluate", self.handle, kappa)

    def phase_commit(self, kappa: int):
        _call("bn_phase_commit", self.handle, kappa)

    def phase_advance(self):
        _call("bn_phase_advance", self.handle)

    def get_phase(self):
        u = np.zeros((self.M, 2), dtype=np.uint16)
        c = np.zeros((self.M, self.T), dtype=np.uint16)
        d = np.zeros(self.M, dtype=np.float64)
        a = np.zeros(self.M, dtype=np.uint8)
        _call("bn_get_phase", self.handle, _ptr(u), _ptr(c), _ptr(d), _ptr(a))
        return {"u_new": u, "c_new": c, "delta": d, "accept": a.astype(bool)}

    def get_phase_bf16(self) -> np.ndarray:
        """Energy changes of the last phase from the BF16 matrix-core pass."""
        d = np.zeros(self.M, dtype=np.float64)
        _call("bn_get_phase_bf16", self.handle, _ptr(d))
        return d

    def get_swap_pass(self):
        """Couples of the last evaluated swap pass: pixels a, b, delta, accept."""
        half = self.M // 2
        a = np.zeros(half, dtype=np.uint32)
        b = np.zeros(half, dtype=np.uint32)
        d = np.zeros(half, dtype=np.float64)
        acc = np.zeros(half, dtype=np.uint8)
        _call("bn_get_swap_pass", self.handle, _ptr(a), _ptr(b), _ptr(d), _ptr(acc))
        return {"a": a, "b": b, "delta": d, "accept": acc.astype(bool)}


def sample(problems, x, y, k) -> np.ndarray:
    """Padded sampler query: float32 [m, 2 * len(problems)], dimension 2d + a
    = component a of problems[d]'s scrambled lattice sample k at pixel (x, y)."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    y = np.ascontiguousarray(y, dtype=np.uint32)
    k = np.ascontiguousarray(k, dtype=np.uint32)
    if not (x.shape == y.shape == k.shape and x.ndim == 1):
        raise ValueError("x, y, k must be 1-D arrays of one length")
    out = np.zeros((x.shape[0], 2 * len(problems)), dtype=np.float32)
    arr = (C.c_void_p * len(problems))(*[p.handle.value for p in problems])
    _call("bn_sample", arr, len(problems), _ptr(x), _ptr(y), _ptr(k), x.shape[0], _ptr(out))
    return out


class Batch:
    """Owns one ``bn_batch`` over existing problems (which must outlive it)."""

    def __init__(self, problems, tune_cache: str | None = None):
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[p.handle.value for p in self.problems])
        handle = C.c_void_p()
        _call("bn_create_batch", arr, len(self.problems),
              None if tune_cache is None else tune_cache.encode(), C.byref(handle))
        self.handle = handle

    def sweep(self, k: int = 1):
        _call("bn_batch_sweep", self.handle, k)

    def tuning(self):
        a, b, c = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _call("bn_batch_tuning", self.handle, C.byref(a), C.byref(b), C.byref(c))
        return {"tch": a.value, "slice_target": b.value, "stage_shape": c.value}

    def close(self):
        if getattr(self, "handle", None):
            _call("bn_destroy_batch", self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def create_problem(workload: dict, heavisides=None, stream=None, gaussians=None, buffers=None,
                   **overrides) -> Problem:
    """Create a problem from a workload description (synthgen format)."""
    w = dict(workload)
    w.update(overrides)
    return Problem(make_config(**w), heavisides, stream, gaussians, buffers)
