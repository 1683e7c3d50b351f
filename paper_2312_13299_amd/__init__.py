"""Python binding of libplas.so, the MI355X (gfx950) implementation of
Parallel Linear Assignment Sorting (PLAS), the sort of Sec. 3.1 of
"Compact 3D Scene Representation via Self-Organizing Gaussian Grids"
(arXiv 2312.13299).

This module only marshals arguments: torch tensors are passed to the C ABI
(include/plas.h) as device pointers and the current HIP stream, and every
step of the sort runs in the library's HIP kernels. There is no fallback: if
libplas.so is missing or cannot be loaded, every entry point raises.

    perm, stats = paper_2312_13299_amd.sort(features_cn, side=1024, seed=0x5EED)
    arranged = features_cn[:, perm]          # channel-major grid, row-major cells
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(HERE, "libplas.so")

OK = 0
ERR_INVALID_ARGUMENT = -1
ERR_UNSUPPORTED = -2
ERR_OUT_OF_MEMORY = -3
ERR_HIP = -4
ERR_NONFINITE = -5

LAYOUT_CN = 0
LAYOUT_NC = 1
DTYPE_F32 = 0
DTYPE_BF16 = 1
STORAGE_F32 = 0
STORAGE_BF16 = 1
STORAGES = {"f32": STORAGE_F32, "bf16": STORAGE_BF16}
FILTERS = {"box": 0, "box3": 1}  # PLAS_FILTER_BOX, PLAS_FILTER_BOX3
ABI_VERSION = 2  # PLAS_ABI_VERSION of include/plas.h
MAX_CHANNELS = 64

# Every symbol declared in include/plas.h, include/plas_stages.h and
# include/plas_batch.h.
EXPORTS = (
    "plas_get_abi_version", "plas_sort_params_init", "plas_create", "plas_destroy",
    "plas_set_stream", "plas_sort", "plas_grid_energy", "plas_grid_energy_noalloc", "plas_status_string",
    "plas_last_error",
    "plas_vad", "plas_stage_blur", "plas_stage_group_table", "plas_stage_assign", "plas_stage_energy",
    "plas_stage_bijection", "plas_philox4x64_10", "plas_draw", "plas_schedule",
    "plas_scale_shift_from_ranges",
    "plas_batch_config_init", "plas_sort_batch", "plas_autotune_batch",
    "plas_job_footprint", "plas_server_create", "plas_server_submit", "plas_server_step",
    "plas_server_poll", "plas_server_destroy",
)


class PlasError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"PLAS status {status}: {message}")
        self.status = status


class Checkpoint(ctypes.Structure):
    """plas_sort_checkpoint: where a sort stopped. Pass it back as
    Context.sort(..., resume=cp, init_perm=perm) to continue."""
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("done", ctypes.c_int32),
        ("reorders", ctypes.c_int64),
        ("shift_draws", ctypes.c_uint64),
        ("level", ctypes.c_int32),
        ("levels_done", ctypes.c_int32),
        ("dy", ctypes.c_int32),
        ("dx", ctypes.c_int32),
        ("has_prev", ctypes.c_int32),
        ("just_shifted", ctypes.c_int32),
        ("energy_prev", ctypes.c_uint64),
        ("energy_last", ctypes.c_uint64),
        ("level_reorders", ctypes.c_int64),
        ("level_moved", ctypes.c_uint64),
    ]


class SortParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("inv_threshold", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("radius_decay", ctypes.c_double),
        ("start_radius", ctypes.c_double),
        ("max_reorders", ctypes.c_int64),
        ("init_perm", ctypes.c_void_p),
        ("min_block", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("reorders_per_sync", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("filter", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("resume", ctypes.POINTER(Checkpoint)),
    ]


class LevelStat(ctypes.Structure):
    _fields_ = [
        ("phi", ctypes.c_double),
        ("r", ctypes.c_int32),
        ("beta", ctypes.c_int32),
        ("reorders", ctypes.c_int64),
        ("energy_fixed", ctypes.c_uint64),
        ("moved", ctypes.c_uint64),
    ]


class SortStats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("levels", ctypes.c_int32),
        ("reorders", ctypes.c_int64),
        ("energy_fixed", ctypes.c_uint64),
        ("scale_shift", ctypes.c_int32),
        ("trace_len", ctypes.c_int32),
        ("energy", ctypes.c_double),
        ("trace", ctypes.POINTER(LevelStat)),
        ("trace_cap", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("blur_ms", ctypes.c_double),
        ("blur_launches", ctypes.c_int64),
        ("assign_ms", ctypes.c_double),
        ("assign_launches", ctypes.c_int64),
        ("total_ms", ctypes.c_double),
        ("checkpoint", ctypes.POINTER(Checkpoint)),
    ]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("features", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int32),
        ("side", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("init_perm", ctypes.c_void_p),
        ("perm_out", ctypes.c_void_p),
        ("stats", ctypes.POINTER(SortStats)),
    ]


class TuneEntry(ctypes.Structure):
    _fields_ = [
        ("side_lo", ctypes.c_int32),
        ("side_hi", ctypes.c_int32),
        ("blur_waves_per_block", ctypes.c_int32),
        ("assign_blocks", ctypes.c_int32),
    ]


class BatchConfig(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("graph", ctypes.c_int32),
        ("reorders_per_sync", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("tune_count", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("tune", ctypes.POINTER(TuneEntry)),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("sorts", ctypes.c_int32),
        ("chunks", ctypes.c_int64),
        ("reorder_slots", ctypes.c_int64),
        ("graph_builds", ctypes.c_int64),
        ("launches", ctypes.c_int64),
        ("prepare_ms", ctypes.c_double),
        ("loop_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("step_ms", ctypes.c_double),
        ("blur_ms", ctypes.c_double),
        ("assign_ms", ctypes.c_double),
    ]


_lib = None


def library() -> ctypes.CDLL:
    """Load libplas.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBRARY):
        raise ImportError(f"{LIBRARY} is missing: build it with paper_2312_13299_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIBRARY)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    sigs = {
        "plas_get_abi_version": (i32, []),
        "plas_sort_params_init": (i32, [ctypes.POINTER(SortParams)]),
        "plas_create": (i32, [ctypes.POINTER(vp), i32]),
        "plas_destroy": (i32, [vp]),
        "plas_set_stream": (i32, [vp, vp]),
        "plas_sort": (i32, [vp, vp, i64, i32, i32, i32, i32, ctypes.POINTER(SortParams), vp,
                            ctypes.POINTER(SortStats)]),
        "plas_grid_energy": (i32, [vp, vp, vp, i64, i32, i32, i32, i32, i32, i32, u64p, i32p,
                                   ctypes.POINTER(ctypes.c_double)]),
        "plas_grid_energy_noalloc": (i32, [vp, vp, vp, i64, i32, i32, i32, i32, i32, i32, u64p, i32p,
                                           ctypes.POINTER(ctypes.c_double)]),
        "plas_vad": (i32, [vp, vp, vp, i64, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_double)]),
        "plas_status_string": (ctypes.c_char_p, [i32]),
        "plas_last_error": (ctypes.c_char_p, [vp]),
        "plas_stage_blur": (i32, [vp, vp, vp, i32, i32, i32, i32]),
        "plas_stage_group_table": (i32, [vp, i32, u64p, vp]),
        "plas_stage_assign": (i32, [vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, u64p, i32, u64p, u64p]),
        "plas_stage_energy": (i32, [vp, vp, vp, i32, i32, i32, i32, u64p]),
        "plas_stage_bijection": (i32, [vp, i64, u64p, vp]),
        "plas_philox4x64_10": (None, [u64p, u64p, u64p]),
        "plas_draw": (None, [u64, u64, u64, u64p]),
        "plas_schedule": (i32, [i32, ctypes.c_double, i32, ctypes.c_double, vp, vp, vp, i32]),
        "plas_scale_shift_from_ranges": (i32, [vp, vp, i32, i64, i32p]),
        "plas_batch_config_init": (i32, [ctypes.POINTER(BatchConfig)]),
        "plas_sort_batch": (i32, [vp, ctypes.POINTER(BatchItem), i32, ctypes.POINTER(SortParams),
                                  ctypes.POINTER(BatchConfig), ctypes.POINTER(BatchStats)]),
        "plas_autotune_batch": (i32, [vp, ctypes.POINTER(BatchItem), i32, ctypes.POINTER(SortParams), i32,
                                      ctypes.POINTER(TuneEntry), i32, i32p]),
        "plas_job_footprint": (i64, [i32, i32, i32, ctypes.POINTER(SortParams)]),
        "plas_server_create": (i32, [vp, ctypes.POINTER(SortParams), ctypes.POINTER(BatchConfig), i64,
                                     ctypes.POINTER(vp)]),
        "plas_server_submit": (i32, [vp, ctypes.POINTER(BatchItem), ctypes.POINTER(ctypes.c_int64)]),
        "plas_server_step": (i32, [vp, i32p, i32p]),
        "plas_server_poll": (i32, [vp, ctypes.POINTER(ctypes.c_int64), i32p, i32, i32p]),
        "plas_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.plas_get_abi_version() != ABI_VERSION:
        raise ImportError(f"libplas.so ABI version {L.plas_get_abi_version()}, this binding needs {ABI_VERSION}")
    _lib = L
    return L


def _u64x4(values):
    arr = (ctypes.c_uint64 * 4)()
    for i, v in enumerate(values):
        arr[i] = int(v) & 0xFFFFFFFFFFFFFFFF
    return arr


# --------------------------------------------------------- host-side helpers

def philox4x64_10(ctr, key) -> list[int]:
    out = (ctypes.c_uint64 * 4)()
    k = (ctypes.c_uint64 * 2)(*(int(v) & 0xFFFFFFFFFFFFFFFF for v in key))
    library().plas_philox4x64_10(_u64x4(ctr), k, out)
    return [int(v) for v in out]


def draw(seed: int, purpose: int, index: int) -> list[int]:
    out = (ctypes.c_uint64 * 4)()
    library().plas_draw(seed & 0xFFFFFFFFFFFFFFFF, purpose, index, out)
    return [int(v) for v in out]


def schedule(side: int, decay: float = 0.95, min_block: int = 16, start_radius: float = 0.0):
    L = library()
    count = L.plas_schedule(side, decay, min_block, start_radius, None, None, None, 0)
    if count < 0:
        raise PlasError(count, "bad schedule arguments")
    phi = (ctypes.c_double * count)()
    r = (ctypes.c_int32 * count)()
    beta = (ctypes.c_int32 * count)()
    L.plas_schedule(side, decay, min_block, start_radius, phi, r, beta, count)
    return list(phi), list(r), list(beta)


def scale_shift_from_ranges(mins, maxs, n: int) -> int:
    d = len(mins)
    lo = (ctypes.c_float * d)(*mins)
    hi = (ctypes.c_float * d)(*maxs)
    s = ctypes.c_int32()
    st = library().plas_scale_shift_from_ranges(lo, hi, d, n, ctypes.byref(s))
    if st != OK:
        raise PlasError(st, "bad ranges")
    return s.value


def status_string(status: int) -> str:
    return library().plas_status_string(status).decode()


# ------------------------------------------------------------------ context

def padded_channels(d: int) -> int:
    dp = 4
    while dp < d:
        dp *= 2
    return dp


class Context:
    """A library context on one device. Work goes to torch's current stream
    of that device at each call."""

    def __init__(self, device: int = 0):
        self._h = ctypes.c_void_p()
        self.device = device
        st = library().plas_create(ctypes.byref(self._h), device)
        if st != OK:
            raise PlasError(st, f"plas_create failed on device {device}: {status_string(st)}")

    def close(self):
        if self._h:
            library().plas_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != OK:
            msg = library().plas_last_error(self._h).decode() or status_string(st)
            raise PlasError(st, f"{what}: {msg}")

    def _bind_stream(self):
        import torch
        stream = torch.cuda.current_stream(self.device).cuda_stream
        library().plas_set_stream(self._h, ctypes.c_void_p(stream))

    # ---- whole sort

    def sort(self, features, side: int | None = None, seed: int = 0x5EED, layout: str = "cn", *,
             radius_decay: float = 0.95, inv_threshold: int = 10000, min_block: int = 16,
             start_radius: float = 0.0, max_reorders: int = 0, init_perm=None,
             profile: bool = False, reorders_per_sync: int = 0, storage: str = "f32", out=None,
             filter: str = "box", resume: Checkpoint | None = None):
        """Sort device features ([d][n] for layout "cn", [n][d] for "nc",
        float32 or bfloat16, contiguous) onto a side x side grid, with the
        working grids stored as float32 ("f32") or bfloat16 ("bf16") and the
        target filtered by one box pass per axis ("box") or three ("box3",
        Gaussian-like). Returns (perm, stats): perm is an int32 device tensor
        in gather form, stats a SortResult whose checkpoint says where the
        sort stopped; pass it as resume, with perm as init_perm, to go on."""
        import torch
        dtype = _feature_dtype(features)
        if layout == "cn":
            d, n = features.shape
            lay = LAYOUT_CN
        elif layout == "nc":
            n, d = features.shape
            lay = LAYOUT_NC
        else:
            raise ValueError(f"unknown layout {layout!r}")
        if side is None:
            side = int(round(n ** 0.5))
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=features.device)
        _check_tensor(out, torch.int32)
        prm = _sort_params(seed=seed, radius_decay=radius_decay, inv_threshold=inv_threshold,
                           min_block=min_block, start_radius=start_radius, max_reorders=max_reorders,
                           profile=profile, reorders_per_sync=reorders_per_sync, storage=storage,
                           filter=filter)
        if init_perm is not None:
            _check_tensor(init_perm, torch.int32)
            prm.init_perm = init_perm.data_ptr()
        if resume is not None:
            prm.resume = ctypes.pointer(resume)
        stats, trace = _new_stats()
        self._bind_stream()
        st = library().plas_sort(self._h, ctypes.c_void_p(features.data_ptr()), n, d, side, lay,
                                 dtype, ctypes.byref(prm), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.byref(stats))
        self._check(st, "plas_sort")
        return out, _result(stats, trace)

    # ---- batches

    def _batch_items(self, features_list, sides, seeds, layouts, storages, init_perms, outs):
        import torch
        count = len(features_list)
        def per(v, name):
            if isinstance(v, (list, tuple)):
                if len(v) != count:
                    raise ValueError(f"{name}: {len(v)} values for {count} sorts")
                return list(v)
            return [v] * count
        sides, seeds, layouts = per(sides, "sides"), per(seeds, "seeds"), per(layouts, "layouts")
        storages, init_perms = per(storages, "storages"), per(init_perms, "init_perms")
        outs = per(outs, "out")
        items = (BatchItem * max(count, 1))()
        keep = []
        for i, f in enumerate(features_list):
            dtype = _feature_dtype(f)
            if layouts[i] == "cn":
                d, n = f.shape
                lay = LAYOUT_CN
            elif layouts[i] == "nc":
                n, d = f.shape
                lay = LAYOUT_NC
            else:
                raise ValueError(f"unknown layout {layouts[i]!r}")
            side = sides[i] if sides[i] is not None else int(round(n ** 0.5))
            out = outs[i]
            if out is None:
                out = torch.empty(n, dtype=torch.int32, device=f.device)
            _check_tensor(out, torch.int32)
            stats, trace = _new_stats()
            it = items[i]
            it.features = f.data_ptr()
            it.n, it.d, it.side, it.layout, it.dtype = n, d, side, lay, dtype
            it.storage = STORAGES[storages[i]]
            it.seed = int(seeds[i]) & 0xFFFFFFFFFFFFFFFF
            if init_perms[i] is not None:
                _check_tensor(init_perms[i], torch.int32)
                it.init_perm = init_perms[i].data_ptr()
            it.perm_out = out.data_ptr()
            it.stats = ctypes.pointer(stats)
            keep.append((out, stats, trace))
        return items, keep

    def sort_batch(self, features_list, sides=None, seeds=0x5EED, layouts="cn", storages="f32",
                   init_perms=None, *, graph: bool = False, tune=None, reorders_per_sync: int = 0,
                   profile: bool = False, radius_decay: float = 0.95, inv_threshold: int = 10000,
                   min_block: int = 16, start_radius: float = 0.0, max_reorders: int = 0, out=None,
                   filter: str = "box"):
        """Sort several grids together (plas_sort_batch). Per-sort arguments
        (sides, seeds, layouts, storages, init_perms, out) take one value for
        all or a list. tune: list of dicts with side_lo, side_hi,
        blur_waves_per_block, assign_blocks (as autotune_batch returns).
        Returns (perms, results, BatchResult)."""
        count = len(features_list)
        items, keep = self._batch_items(features_list, sides, seeds, layouts, storages, init_perms, out)
        prm = _sort_params(radius_decay=radius_decay, inv_threshold=inv_threshold, min_block=min_block,
                           start_radius=start_radius, max_reorders=max_reorders, filter=filter)
        cfg, table = _batch_config(graph, reorders_per_sync, profile, tune)
        bstats = BatchStats()
        bstats.struct_size = ctypes.sizeof(BatchStats)
        self._bind_stream()
        st = library().plas_sort_batch(self._h, items, count, ctypes.byref(prm), ctypes.byref(cfg),
                                       ctypes.byref(bstats))
        self._check(st, "plas_sort_batch")
        perms = [k[0] for k in keep]
        results = [_result(k[1], k[2]) for k in keep]
        b = BatchResult(**{name: getattr(bstats, name) for name, _ in BatchStats._fields_
                           if name != "struct_size"})
        return perms, results, b

    def autotune_batch(self, features_list, sides=None, seeds=0x5EED, layouts="cn", storages="f32", *,
                       graph: bool = False, radius_decay: float = 0.95, inv_threshold: int = 10000,
                       min_block: int = 16):
        """Measured launch shapes per side bucket for these grids
        (plas_autotune_batch): a list of dicts for sort_batch(tune=...)."""
        count = len(features_list)
        items, keep = self._batch_items(features_list, sides, seeds, layouts, storages, None, None)
        prm = _sort_params(radius_decay=radius_decay, inv_threshold=inv_threshold, min_block=min_block)
        cap = 64
        table = (TuneEntry * cap)()
        entries = ctypes.c_int32()
        self._bind_stream()
        st = library().plas_autotune_batch(self._h, items, count, ctypes.byref(prm), 1 if graph else 0, table,
                                           cap, ctypes.byref(entries))
        self._check(st, "plas_autotune_batch")
        return [dict(side_lo=t.side_lo, side_hi=t.side_hi, blur_waves_per_block=t.blur_waves_per_block,
                     assign_blocks=t.assign_blocks) for t in table[: entries.value]]

    def grid_energy(self, features, perm=None, side: int | None = None, radius: int = 1,
                    layout: str = "cn", storage: str = "f32", noalloc: bool = False):
        """(energy_fixed, scale_shift, energy_mean) of features[perm] at radius.
        noalloc: through plas_grid_energy_noalloc (n <= 65536, no device
        allocation)."""
        import torch
        dtype = _feature_dtype(features)
        if layout == "cn":
            d, n = features.shape
            lay = LAYOUT_CN
        else:
            n, d = features.shape
            lay = LAYOUT_NC
        if side is None:
            side = int(round(n ** 0.5))
        p = None
        if perm is not None:
            _check_tensor(perm, torch.int32)
            p = ctypes.c_void_p(perm.data_ptr())
        E, s, mean = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_double()
        self._bind_stream()
        name = "plas_grid_energy_noalloc" if noalloc else "plas_grid_energy"
        st = getattr(library(), name)(self._h, ctypes.c_void_p(features.data_ptr()), p, n, d, side,
                                      lay, dtype, STORAGES[storage], radius, ctypes.byref(E),
                                      ctypes.byref(s), ctypes.byref(mean))
        self._check(st, name)
        return int(E.value), s.value, mean.value

    def vad(self, features, perm=None, side: int | None = None, layout: str = "cn") -> float:
        """VAD (App. C) of features[perm] on the side x side grid."""
        import torch
        dtype = _feature_dtype(features)
        if layout == "cn":
            d, n = features.shape
            lay = LAYOUT_CN
        else:
            n, d = features.shape
            lay = LAYOUT_NC
        if side is None:
            side = int(round(n ** 0.5))
        p = None
        if perm is not None:
            _check_tensor(perm, torch.int32)
            p = ctypes.c_void_p(perm.data_ptr())
        v = ctypes.c_double()
        self._bind_stream()
        st = library().plas_vad(self._h, ctypes.c_void_p(features.data_ptr()), p, n, d, side, lay, dtype,
                                ctypes.byref(v))
        self._check(st, "plas_vad")
        return v.value

    # ---- stages (working layout [n][dp] float32)

    def stage_blur(self, grid, side: int, radius: int, target=None):
        """grid: device [n][dp] float32 or bfloat16 (the storage)."""
        import torch
        storage = _grid_storage(grid)
        dp = grid.shape[1]
        if target is None:
            target = torch.empty_like(grid)
        self._bind_stream()
        self._check(library().plas_stage_blur(self._h, ctypes.c_void_p(grid.data_ptr()),
                                              ctypes.c_void_p(target.data_ptr()), side, dp, storage,
                                              radius), "plas_stage_blur")
        return target

    def stage_group_table(self, beta: int, round_keys):
        import torch
        table = torch.empty(beta * beta, dtype=torch.int32, device=f"cuda:{self.device}")
        self._bind_stream()
        self._check(library().plas_stage_group_table(self._h, beta, _u64x4(round_keys),
                                                     ctypes.c_void_p(table.data_ptr())),
                    "plas_stage_group_table")
        return table

    def stage_assign(self, grid, target, perm, side: int, beta: int, dy: int, dx: int, round_keys,
                     scale_shift: int):
        """One reorder in place on grid ([n][dp]) and perm. Returns (energy, moved)."""
        import torch
        storage = _grid_storage(grid)
        if target.dtype != grid.dtype:
            raise ValueError("grid and target must have the same storage")
        _check_tensor(perm, torch.int32)
        E, M = ctypes.c_uint64(), ctypes.c_uint64()
        self._bind_stream()
        self._check(library().plas_stage_assign(
            self._h, ctypes.c_void_p(grid.data_ptr()), ctypes.c_void_p(target.data_ptr()),
            ctypes.c_void_p(perm.data_ptr()), side, grid.shape[1], storage, beta, dy, dx,
            _u64x4(round_keys), scale_shift, ctypes.byref(E), ctypes.byref(M)), "plas_stage_assign")
        return int(E.value), int(M.value)

    def stage_energy(self, grid, target, side: int, scale_shift: int) -> int:
        storage = _grid_storage(grid)
        if target.dtype != grid.dtype:
            raise ValueError("grid and target must have the same storage")
        E = ctypes.c_uint64()
        self._bind_stream()
        self._check(library().plas_stage_energy(self._h, ctypes.c_void_p(grid.data_ptr()),
                                                ctypes.c_void_p(target.data_ptr()), side,
                                                grid.shape[1], storage, scale_shift, ctypes.byref(E)),
                    "plas_stage_energy")
        return int(E.value)

    def stage_bijection(self, n: int, round_keys):
        import torch
        out = torch.empty(n, dtype=torch.int32, device=f"cuda:{self.device}")
        self._bind_stream()
        self._check(library().plas_stage_bijection(self._h, n, _u64x4(round_keys),
                                                   ctypes.c_void_p(out.data_ptr())),
                    "plas_stage_bijection")
        return out


@dataclass
class SortResult:
    reorders: int
    levels: int
    energy_fixed: int
    scale_shift: int
    energy: float
    trace: list = field(default_factory=list)
    blur_ms: float = 0.0
    blur_launches: int = 0
    assign_ms: float = 0.0
    assign_launches: int = 0
    total_ms: float = 0.0
    checkpoint: Checkpoint | None = None  # where the sort stopped


def _batch_config(graph: bool, reorders_per_sync: int, profile: bool, tune):
    cfg = BatchConfig()
    library().plas_batch_config_init(ctypes.byref(cfg))
    cfg.graph = 1 if graph else 0
    cfg.reorders_per_sync = reorders_per_sync
    cfg.profile = 1 if profile else 0
    table = None
    if tune:
        table = (TuneEntry * len(tune))()
        for i, e in enumerate(tune):
            table[i].side_lo, table[i].side_hi = e["side_lo"], e["side_hi"]
            table[i].blur_waves_per_block = e.get("blur_waves_per_block", 0)
            table[i].assign_blocks = e.get("assign_blocks", 0)
        cfg.tune = ctypes.cast(table, ctypes.POINTER(TuneEntry))
        cfg.tune_count = len(tune)
    return cfg, table


def job_footprint(side: int, d: int, storage: str = "f32", **params) -> int:
    """Device bytes one served job holds while it runs."""
    prm = _sort_params(**params)
    v = library().plas_job_footprint(side, d, STORAGES[storage], ctypes.byref(prm))
    if v < 0:
        raise PlasError(int(v), "bad job arguments")
    return int(v)


class Server:
    """Continuous-batching sort server on a Context (plas_server_*): submit
    jobs at any time; each step() admits waiting jobs whose device memory
    fits in the budget, runs one chunk of reorders of every running job and
    collects finished ones; poll() returns them."""

    def __init__(self, ctx: "Context", memory_budget: int, *, graph: bool = False, reorders_per_sync: int = 0,
                 tune=None, radius_decay: float = 0.95, inv_threshold: int = 10000, min_block: int = 16,
                 start_radius: float = 0.0, max_reorders: int = 0, filter: str = "box"):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        prm = _sort_params(radius_decay=radius_decay, inv_threshold=inv_threshold, min_block=min_block,
                           start_radius=start_radius, max_reorders=max_reorders, filter=filter)
        cfg, self._table = _batch_config(graph, reorders_per_sync, False, tune)
        ctx._bind_stream()
        st = library().plas_server_create(ctx._h, ctypes.byref(prm), ctypes.byref(cfg), int(memory_budget),
                                          ctypes.byref(self._h))
        ctx._check(st, "plas_server_create")
        self._jobs = {}

    def submit(self, features, side: int | None = None, seed: int = 0x5EED, layout: str = "cn",
               storage: str = "f32", init_perm=None, out=None) -> int:
        items, keep = self.ctx._batch_items([features], [side], [seed], [layout], [storage], [init_perm], [out])
        job = ctypes.c_int64()
        st = library().plas_server_submit(self._h, ctypes.byref(items[0]), ctypes.byref(job))
        self.ctx._check(st, "plas_server_submit")
        # The buffers stay referenced until the job is polled.
        self._jobs[job.value] = (features, init_perm, items, keep[0])
        return job.value

    def step(self) -> tuple[int, int]:
        running, waiting = ctypes.c_int32(), ctypes.c_int32()
        self.ctx._bind_stream()
        st = library().plas_server_step(self._h, ctypes.byref(running), ctypes.byref(waiting))
        self.ctx._check(st, "plas_server_step")
        return running.value, waiting.value

    def poll(self):
        """[(job_id, status, perm, SortResult or None)] of the jobs finished
        or failed since the last poll."""
        cap = 256
        ids = (ctypes.c_int64 * cap)()
        sts = (ctypes.c_int32 * cap)()
        out = []
        while True:
            n = ctypes.c_int32()
            st = library().plas_server_poll(self._h, ids, sts, cap, ctypes.byref(n))
            self.ctx._check(st, "plas_server_poll")
            for i in range(n.value):
                _, _, _, (perm, stats, trace) = self._jobs.pop(ids[i])
                ok = sts[i] == OK
                out.append((ids[i], sts[i], perm if ok else None, _result(stats, trace) if ok else None))
            if n.value < cap:
                return out

    def close(self):
        if self._h:
            library().plas_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._jobs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class BatchResult:
    sorts: int
    chunks: int
    reorder_slots: int
    graph_builds: int
    launches: int
    prepare_ms: float
    loop_ms: float
    total_ms: float
    step_ms: float
    blur_ms: float
    assign_ms: float


def _sort_params(seed: int = 0x5EED, radius_decay: float = 0.95, inv_threshold: int = 10000,
                 min_block: int = 16, start_radius: float = 0.0, max_reorders: int = 0,
                 profile: bool = False, reorders_per_sync: int = 0, storage: str = "f32",
                 filter: str = "box") -> SortParams:
    prm = SortParams()
    library().plas_sort_params_init(ctypes.byref(prm))
    prm.seed = seed & 0xFFFFFFFFFFFFFFFF
    prm.radius_decay = radius_decay
    prm.inv_threshold = inv_threshold
    prm.min_block = min_block
    prm.start_radius = start_radius
    prm.max_reorders = max_reorders
    prm.profile = 1 if profile else 0
    prm.reorders_per_sync = reorders_per_sync
    prm.storage = STORAGES[storage]
    prm.filter = FILTERS[filter]
    return prm


TRACE_CAP = 4096


def _new_stats():
    trace = (LevelStat * TRACE_CAP)()
    stats = SortStats()
    stats.struct_size = ctypes.sizeof(SortStats)
    stats.trace = ctypes.cast(trace, ctypes.POINTER(LevelStat))
    stats.trace_cap = TRACE_CAP
    stats._checkpoint = Checkpoint()  # kept alive with the stats
    stats.checkpoint = ctypes.pointer(stats._checkpoint)
    return stats, trace


def _result(stats: SortStats, trace) -> SortResult:
    return SortResult(
        reorders=stats.reorders, levels=stats.levels, energy_fixed=int(stats.energy_fixed),
        scale_shift=stats.scale_shift, energy=stats.energy,
        trace=[dict(phi=t.phi, r=t.r, beta=t.beta, reorders=t.reorders,
                    energy=int(t.energy_fixed), moved=int(t.moved))
               for t in trace[: stats.trace_len]],
        blur_ms=stats.blur_ms, blur_launches=stats.blur_launches,
        assign_ms=stats.assign_ms, assign_launches=stats.assign_launches,
        total_ms=stats.total_ms, checkpoint=Checkpoint.from_buffer_copy(stats._checkpoint))


def _feature_dtype(t) -> int:
    import torch
    if t.dtype == torch.float32:
        _check_tensor(t, torch.float32)
        return DTYPE_F32
    if t.dtype == torch.bfloat16:
        _check_tensor(t, torch.bfloat16)
        return DTYPE_BF16
    raise ValueError(f"features must be float32 or bfloat16, got {t.dtype}")


def _grid_storage(t) -> int:
    import torch
    if t.dtype == torch.float32:
        _check_tensor(t, torch.float32)
        return STORAGE_F32
    if t.dtype == torch.bfloat16:
        _check_tensor(t, torch.bfloat16)
        return STORAGE_BF16
    raise ValueError(f"grids are float32 or bfloat16, got {t.dtype}")


def _check_tensor(t, dtype):
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")


_contexts: dict[int, Context] = {}


def context(device: int = 0) -> Context:
    if device not in _contexts:
        _contexts[device] = Context(device)
    return _contexts[device]


def sort(features, side: int | None = None, seed: int = 0x5EED, layout: str = "cn", **kw):
    """Module-level shortcut of Context.sort on the tensor's device."""
    return context(features.device.index or 0).sort(features, side, seed, layout, **kw)


def grid_energy(features, perm=None, side: int | None = None, radius: int = 1, layout: str = "cn"):
    return context(features.device.index or 0).grid_energy(features, perm, side, radius, layout)
