"""ctypes wrapper over the PLAS CPU oracle (``plas_oracle.c``).

TEST INFRASTRUCTURE ONLY. The oracle checks the GPU library; only the test
suite, the smoke check and the CPU-baseline leg of the benchmark use it. It
shares no code with the GPU library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "plas_oracle.c")
LIBRARY = os.path.join(HERE, "libplas_oracle.so")

LAYOUTS = {"cn": 0, "nc": 1}
OK, INVALID, NONFINITE = 0, -1, -5

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
          "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE float32, no contraction)."""
    if force or not os.path.exists(LIBRARY):
        tmp = LIBRARY + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SOURCE, "-o", tmp, "-lm"])
        os.replace(tmp, LIBRARY)
    return LIBRARY


class State(ctypes.Structure):
    """Where a sort stopped (plas_ref_state): resume it with this state and
    the stopped sort's permutation as init_perm."""
    _fields_ = [
        ("k", ctypes.c_int64),
        ("j", ctypes.c_uint64),
        ("level", ctypes.c_int32),
        ("levels_run", ctypes.c_int32),
        ("dy", ctypes.c_int32),
        ("dx", ctypes.c_int32),
        ("has_prev", ctypes.c_int32),
        ("just_shifted", ctypes.c_int32),
        ("E_prev", ctypes.c_uint64),
        ("E_last", ctypes.c_uint64),
        ("level_reorders", ctypes.c_int64),
        ("level_moved", ctypes.c_uint64),
        ("done", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Control(ctypes.Structure):
    """The progress-control state of one radius level (plas_ref_ctl)."""
    _fields_ = [
        ("has_prev", ctypes.c_int32),
        ("just_shifted", ctypes.c_int32),
        ("E_prev", ctypes.c_uint64),
    ]


# Actions of plas_ref_control.
CTL_KEEP, CTL_SHIFT, CTL_END = 0, 1, 2


class _Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("radius_decay", ctypes.c_double),
        ("inv_threshold", ctypes.c_uint32),
        ("min_block", ctypes.c_int32),
        ("start_radius", ctypes.c_double),
        ("max_reorders", ctypes.c_int64),
        ("init_perm", ctypes.c_void_p),
        ("storage_bf16", ctypes.c_int32),
        ("filter", ctypes.c_int32),
        ("resume", ctypes.POINTER(State)),
    ]


# The target's low-pass filter: one box pass per axis, or three (a
# Gaussian-like filter of variance r(r+1) per axis).
FILTERS = {"box": 0, "box3": 1}


class _Level(ctypes.Structure):
    _fields_ = [
        ("phi", ctypes.c_double),
        ("r", ctypes.c_int32),
        ("beta", ctypes.c_int32),
        ("reorders", ctypes.c_int64),
        ("energy", ctypes.c_uint64),
        ("moved", ctypes.c_uint64),
    ]


class _Result(ctypes.Structure):
    _fields_ = [
        ("reorders", ctypes.c_int64),
        ("levels", ctypes.c_int32),
        ("scale_shift", ctypes.c_int32),
        ("energy", ctypes.c_uint64),
        ("energy_mean", ctypes.c_double),
        ("trace", ctypes.POINTER(_Level)),
        ("trace_cap", ctypes.c_int32),
        ("trace_len", ctypes.c_int32),
        ("reorder_energy", ctypes.POINTER(ctypes.c_uint64)),
        ("reorder_energy_cap", ctypes.c_int64),
        ("state", ctypes.POINTER(State)),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIBRARY):
            build(force=False)
        L = ctypes.CDLL(LIBRARY)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        vp = ctypes.c_void_p
        sig = {
            "plas_ref_philox4x64_10": (None, [u64p, u64p, u64p]),
            "plas_ref_draw": (None, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u64p]),
            "plas_ref_fmix64": (ctypes.c_uint64, [ctypes.c_uint64]),
            "plas_ref_bijection": (ctypes.c_uint64, [ctypes.c_uint64, u64p, ctypes.c_uint64]),
            "plas_ref_bijection_table": (None, [ctypes.c_uint64, u64p, vp]),
            "plas_ref_shift": (None, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32, i32p, i32p]),
            "plas_ref_scale_shift": (ctypes.c_int32, [vp, ctypes.c_int64, ctypes.c_int32,
                                                      ctypes.c_int32, i32p,
                                                      ctypes.POINTER(ctypes.c_double)]),
            "plas_ref_blur": (ctypes.c_int32, [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
            "plas_ref_blur_storage": (ctypes.c_int32, [vp, vp, ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.c_int32, ctypes.c_int32]),
            "plas_ref_round_bf16": (ctypes.c_float, [ctypes.c_float]),
            "plas_ref_blur_filter": (ctypes.c_int32, [vp, vp, ctypes.c_int32, ctypes.c_int32,
                                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
            "plas_ref_grid_energy_storage": (ctypes.c_int32, [vp, vp, ctypes.c_int64, ctypes.c_int32,
                                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                              ctypes.c_int32, u64p, i32p,
                                                              ctypes.POINTER(ctypes.c_double)]),
            "plas_ref_distance": (ctypes.c_float, [vp, vp, ctypes.c_int32]),
            "plas_ref_quantise": (ctypes.c_uint64, [ctypes.c_float, ctypes.c_int32]),
            "plas_ref_energy_fixed": (ctypes.c_uint64, [vp, vp, ctypes.c_int64, ctypes.c_int32,
                                                        ctypes.c_int32]),
            "plas_ref_perms24": (None, [vp]),
            "plas_ref_assign": (ctypes.c_uint64, [vp, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                  u64p, ctypes.c_int32, u64p]),
            "plas_ref_schedule": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                                   ctypes.c_double, vp, vp, vp, ctypes.c_int32]),
            "plas_ref_gather": (ctypes.c_int32, [vp, vp, ctypes.c_int64, ctypes.c_int32,
                                                 ctypes.c_int32, vp]),
            "plas_ref_sort": (ctypes.c_int32, [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.POINTER(_Params), vp,
                                               ctypes.POINTER(_Result)]),
            "plas_ref_grid_energy": (ctypes.c_int32, [vp, vp, ctypes.c_int64, ctypes.c_int32,
                                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                      u64p, i32p, ctypes.POINTER(ctypes.c_double)]),
            "plas_ref_grid_energy_f64": (ctypes.c_double, [vp, vp, ctypes.c_int64, ctypes.c_int32,
                                                           ctypes.c_int32, ctypes.c_int32,
                                                           ctypes.c_int32]),
            "plas_ref_vad": (ctypes.c_double, [vp, vp, ctypes.c_int64, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_int32]),
            "plas_ref_set_threads": (ctypes.c_int32, [ctypes.c_int32]),
            "plas_ref_improved": (ctypes.c_int32, [ctypes.c_uint64, ctypes.c_uint64,
                                                   ctypes.c_int32, ctypes.c_uint32]),
            "plas_ref_control": (ctypes.c_int32, [ctypes.POINTER(Control), ctypes.c_uint64,
                                                  ctypes.c_uint32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _u64(values) -> ctypes.Array:
    arr = (ctypes.c_uint64 * len(values))()
    for i, v in enumerate(values):
        arr[i] = int(v) & 0xFFFFFFFFFFFFFFFF
    return arr


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------- primitives

def philox4x64_10(ctr, key) -> list[int]:
    out = (ctypes.c_uint64 * 4)()
    lib().plas_ref_philox4x64_10(_u64(ctr), _u64(key), out)
    return [int(v) for v in out]


def draw(seed: int, purpose: int, index: int) -> list[int]:
    out = (ctypes.c_uint64 * 4)()
    lib().plas_ref_draw(seed, purpose, index, out)
    return [int(v) for v in out]


def fmix64(k: int) -> int:
    return int(lib().plas_ref_fmix64(k & 0xFFFFFFFFFFFFFFFF))


def bijection(n: int, round_keys, i: int) -> int:
    return int(lib().plas_ref_bijection(n, _u64(round_keys), i))


def bijection_table(n: int, round_keys) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    lib().plas_ref_bijection_table(n, _u64(round_keys), _ptr(out))
    return out


def shift(seed: int, j: int, w: int) -> tuple[int, int]:
    dy, dx = ctypes.c_int32(), ctypes.c_int32()
    lib().plas_ref_shift(seed, j, w, ctypes.byref(dy), ctypes.byref(dx))
    return dy.value, dx.value


def scale_shift(F: np.ndarray, layout: str = "cn") -> tuple[int, int, float]:
    """Returns (status, s, D_max)."""
    F = _f32(F)
    n, d = _nd(F, layout)
    s, dmax = ctypes.c_int32(), ctypes.c_double()
    st = lib().plas_ref_scale_shift(_ptr(F), n, d, LAYOUTS[layout], ctypes.byref(s), ctypes.byref(dmax))
    return int(st), s.value, dmax.value


def blur(G: np.ndarray, side: int, r: int, storage_bf16: bool = False, filter: str = "box") -> np.ndarray:
    """G is [N][d] (cell-major); returns T [N][d]."""
    G = _f32(G)
    N, d = G.shape
    assert N == side * side
    T = np.empty_like(G)
    st = lib().plas_ref_blur_filter(_ptr(G), _ptr(T), side, d, r, 1 if storage_bf16 else 0, FILTERS[filter])
    if st != OK:
        raise ValueError(f"plas_ref_blur failed: {st}")
    return T


def round_bf16(x) -> np.ndarray:
    """Elementwise round-to-nearest-even to bfloat16, as float32."""
    a = np.asarray(x, dtype=np.float32)
    f = lib().plas_ref_round_bf16
    return np.array([f(float(v)) for v in a.ravel()], dtype=np.float32).reshape(a.shape)


def distance(a, b) -> np.float32:
    a, b = _f32(a), _f32(b)
    assert a.shape == b.shape and a.ndim == 1
    return np.float32(lib().plas_ref_distance(_ptr(a), _ptr(b), a.shape[0]))


def quantise(dist: float, s: int) -> int:
    return int(lib().plas_ref_quantise(float(np.float32(dist)), s))


def energy_fixed(G: np.ndarray, T: np.ndarray, s: int) -> int:
    G, T = _f32(G), _f32(T)
    N, d = G.shape
    return int(lib().plas_ref_energy_fixed(_ptr(G), _ptr(T), N, d, s))


def perms24() -> np.ndarray:
    out = np.empty((24, 4), dtype=np.int32)
    lib().plas_ref_perms24(_ptr(out))
    return out


def assign(G: np.ndarray, T: np.ndarray, P: np.ndarray, side: int, beta: int, dy: int, dx: int,
           round_keys, s: int) -> tuple[int, int]:
    """One reorder in place on G ([N][d] float32) and P (int32). Returns
    (energy, moved)."""
    assert G.dtype == np.float32 and G.flags.c_contiguous
    assert P.dtype == np.int32 and P.flags.c_contiguous
    T = _f32(T)
    N, d = G.shape
    moved = ctypes.c_uint64()
    E = lib().plas_ref_assign(_ptr(G), _ptr(T), _ptr(P), side, d, beta, dy, dx,
                              _u64(round_keys), s, ctypes.byref(moved))
    return int(E), int(moved.value)


def schedule(w: int, decay: float = 0.95, min_block: int = 16, start_radius: float = 0.0):
    n = lib().plas_ref_schedule(w, decay, min_block, start_radius, None, None, None, 0)
    if n < 0:
        raise ValueError("bad schedule arguments")
    phi = np.empty(n, dtype=np.float64)
    r = np.empty(n, dtype=np.int32)
    beta = np.empty(n, dtype=np.int32)
    lib().plas_ref_schedule(w, decay, min_block, start_radius, _ptr(phi), _ptr(r), _ptr(beta), n)
    return phi, r, beta


def gather(F: np.ndarray, perm: np.ndarray | None, layout: str = "cn") -> np.ndarray:
    F = _f32(F)
    n, d = _nd(F, layout)
    G = np.empty((n, d), dtype=np.float32)
    p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    st = lib().plas_ref_gather(_ptr(F), _ptr(p), n, d, LAYOUTS[layout], _ptr(G))
    if st != OK:
        raise ValueError("bad gather arguments")
    return G


def _nd(F: np.ndarray, layout: str) -> tuple[int, int]:
    if layout == "cn":
        d, n = F.shape
    elif layout == "nc":
        n, d = F.shape
    else:
        raise ValueError(layout)
    return n, d


# -------------------------------------------------------------------- sort

@dataclass
class SortResult:
    status: int
    perm: np.ndarray
    reorders: int = 0
    levels: int = 0
    scale_shift: int = 0
    energy: int = 0
    energy_mean: float = 0.0
    trace: list = field(default_factory=list)
    reorder_energy: np.ndarray | None = None
    state: State | None = None  # where the sort stopped


def sort(F: np.ndarray, side: int, seed: int, layout: str = "cn", *, radius_decay: float = 0.95,
         inv_threshold: int = 10000, min_block: int = 16, start_radius: float = 0.0,
         max_reorders: int = 0, init_perm: np.ndarray | None = None,
         energy_cap: int = 0, storage_bf16: bool = False, filter: str = "box",
         resume: State | None = None) -> SortResult:
    """The whole sort (or its continuation from `resume`, with init_perm the
    stopped sort's permutation). The result's `state` says where it stopped."""
    F = _f32(F)
    n, d = _nd(F, layout)
    ip = None if init_perm is None else np.ascontiguousarray(init_perm, dtype=np.int32)
    prm = _Params(seed & 0xFFFFFFFFFFFFFFFF, radius_decay, inv_threshold, min_block,
                  start_radius, max_reorders, None if ip is None else ip.ctypes.data,
                  1 if storage_bf16 else 0, FILTERS[filter],
                  None if resume is None else ctypes.pointer(resume))
    cap = 4096
    trace = (_Level * cap)()
    energies = np.zeros(max(energy_cap, 1), dtype=np.uint64)
    res = _Result()
    res.trace = ctypes.cast(trace, ctypes.POINTER(_Level))
    res.trace_cap = cap
    res.reorder_energy = energies.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if energy_cap else None
    res.reorder_energy_cap = energy_cap
    state = State()
    res.state = ctypes.pointer(state)
    perm = np.empty(n, dtype=np.int32)
    st = lib().plas_ref_sort(_ptr(F), n, d, side, LAYOUTS[layout], ctypes.byref(prm), _ptr(perm),
                             ctypes.byref(res))
    out = SortResult(status=int(st), perm=perm)
    if st != OK:
        return out
    out.state = state
    out.reorders = res.reorders
    out.levels = res.levels
    out.scale_shift = res.scale_shift
    out.energy = int(res.energy)
    out.energy_mean = res.energy_mean
    out.trace = [dict(phi=t.phi, r=t.r, beta=t.beta, reorders=t.reorders, energy=int(t.energy),
                      moved=int(t.moved)) for t in trace[: res.trace_len]]
    if energy_cap:
        out.reorder_energy = energies[: min(energy_cap, res.reorders)].copy()
    return out


def grid_energy(F: np.ndarray, perm: np.ndarray | None, side: int, r: int,
                layout: str = "cn", storage_bf16: bool = False) -> tuple[int, int, int, float]:
    """Returns (status, E, s, mean)."""
    F = _f32(F)
    n, d = _nd(F, layout)
    p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    E, s, mean = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_double()
    st = lib().plas_ref_grid_energy_storage(_ptr(F), _ptr(p), n, d, side, LAYOUTS[layout], r,
                                            1 if storage_bf16 else 0, ctypes.byref(E),
                                            ctypes.byref(s), ctypes.byref(mean))
    return int(st), int(E.value), s.value, mean.value


def grid_energy_f64(F: np.ndarray, perm: np.ndarray | None, side: int, r: int,
                    layout: str = "cn") -> float:
    F = _f32(F)
    n, d = _nd(F, layout)
    p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    return float(lib().plas_ref_grid_energy_f64(_ptr(F), _ptr(p), n, d, side, LAYOUTS[layout], r))


def vad(F: np.ndarray, perm: np.ndarray | None, side: int, layout: str = "cn") -> float:
    F = _f32(F)
    n, d = _nd(F, layout)
    p = None if perm is None else np.ascontiguousarray(perm, dtype=np.int32)
    return float(lib().plas_ref_vad(_ptr(F), _ptr(p), n, d, side, LAYOUTS[layout]))


def improved(E: int, E_prev: int, has_prev: bool, M: int) -> bool:
    """The oracle's improvement test for one reorder's energy E."""
    return bool(lib().plas_ref_improved(E, E_prev, 1 if has_prev else 0, M))


def control(state: Control, E: int, M: int) -> int:
    """Applies E to the level's control state in place; returns CTL_KEEP,
    CTL_SHIFT or CTL_END."""
    return int(lib().plas_ref_control(ctypes.byref(state), E, M))


def set_threads(threads: int) -> int:
    return int(lib().plas_ref_set_threads(threads))
