"""CPU checks of libplas.so: it loads, it exports every function that
include/*.h declares, and its host-side logic (random draws, schedule,
energy scale, status strings) agrees with the paper's definitions and with
numpy. No device work is started here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(INCLUDE)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(INCLUDE, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(plas_[a-z0-9_]+)\s*\(",
                            text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def plas():
    import paper_2312_13299_amd as plas
    if not os.path.exists(plas.LIBRARY):
        pytest.skip("libplas.so not built")
    plas.library()
    return plas


def test_every_declared_symbol_is_exported(plas):
    names = declared_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(plas.LIBRARY)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(plas.EXPORTS)


def test_abi_version_and_status_strings(plas):
    assert plas.library().plas_get_abi_version() == 2
    for st in (0, -1, -2, -3, -4, -5):
        assert plas.status_string(st) not in ("", "unknown status")
    assert plas.status_string(-99) == "unknown status"


def test_params_defaults_follow_the_paper(plas):
    p = plas.SortParams()
    assert plas.library().plas_sort_params_init(ctypes.byref(p)) == 0
    assert p.struct_size == ctypes.sizeof(plas.SortParams)
    assert p.radius_decay == 0.95 and p.inv_threshold == 10000 and p.min_block == 16
    assert p.start_radius == 0.0 and p.max_reorders == 0 and not p.init_perm


def test_struct_layouts(plas):
    assert ctypes.sizeof(plas.LevelStat) == 40
    assert ctypes.sizeof(plas.SortParams) == 80
    assert ctypes.sizeof(plas.SortStats) == 104
    assert ctypes.sizeof(plas.Checkpoint) == 80


def test_library_philox_matches_numpy(plas):
    from test_oracle_rng import numpy_philox_block
    rng = np.random.default_rng(3)
    for _ in range(40):
        ctr = [int(v) for v in rng.integers(0, 1 << 63, 4, dtype=np.uint64)]
        key = [int(v) for v in rng.integers(0, 1 << 63, 2, dtype=np.uint64)]
        assert plas.philox4x64_10(ctr, key) == numpy_philox_block(ctr, key)
    assert plas.draw(0x5EED, 2, 17) == numpy_philox_block((2, 17, 0, 0), (0x5EED, 0))


@pytest.mark.parametrize("w,expect", [(2, 1), (3, 1), (64, 67), (512, 109), (1024, 122), (1448, 129)])
def test_library_schedule(plas, ref, w, expect):
    phi, r, beta = plas.schedule(w)
    assert len(phi) == expect
    phi_ref, r_ref, beta_ref = ref.schedule(w)
    assert phi == list(phi_ref) and r == list(r_ref) and beta == list(beta_ref)
    if w >= 4:
        assert len(phi) == 1 + math.floor(math.log(w / 2 - 1) / math.log(1 / 0.95))


def test_library_scale_shift(plas, ref):
    import synthetic
    F = synthetic.gaussian_attributes(4096, 1)
    _, s_ref, _ = ref.scale_shift(F)
    s = plas.scale_shift_from_ranges(F.min(axis=1).tolist(), F.max(axis=1).tolist(), 4096)
    assert s == s_ref
    assert plas.scale_shift_from_ranges([1.0, 2.0], [1.0, 2.0], 16) == 0


def test_create_without_gpu_fails_cleanly(plas):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    st = plas.library().plas_create(ctypes.byref(h), 0)
    assert st in (plas.ERR_HIP, plas.ERR_INVALID_ARGUMENT) and not h.value


def test_null_handle_is_rejected(plas):
    L = plas.library()
    assert L.plas_destroy(None) == 0
    assert L.plas_set_stream(None, None) == plas.ERR_INVALID_ARGUMENT
    stats = plas.SortStats()
    stats.struct_size = ctypes.sizeof(stats)
    assert L.plas_sort(None, None, 4, 1, 2, 0, 0, None, None, ctypes.byref(stats)) == plas.ERR_INVALID_ARGUMENT
    assert L.plas_last_error(None) == b""


def test_batch_structs_and_defaults(plas):
    # plas_batch_item: 8 + 8 + 6*4 + 8 + 3 pointers; the config ends in a pointer.
    assert ctypes.sizeof(plas.BatchItem) == 72
    assert ctypes.sizeof(plas.TuneEntry) == 16
    assert ctypes.sizeof(plas.BatchConfig) == 32
    assert ctypes.sizeof(plas.BatchStats) == 88
    c = plas.BatchConfig()
    assert plas.library().plas_batch_config_init(ctypes.byref(c)) == 0
    assert c.struct_size == ctypes.sizeof(plas.BatchConfig)
    assert c.graph == 0 and c.reorders_per_sync == 0 and c.profile == 0 and c.tune_count == 0
    assert plas.library().plas_batch_config_init(None) == plas.ERR_INVALID_ARGUMENT


def test_batch_null_handle_is_rejected(plas):
    L = plas.library()
    items = (plas.BatchItem * 1)()
    assert L.plas_sort_batch(None, items, 1, None, None, None) == plas.ERR_INVALID_ARGUMENT
    table = (plas.TuneEntry * 4)()
    n = ctypes.c_int32()
    assert L.plas_autotune_batch(None, items, 1, None, 0, table, 4, ctypes.byref(n)) == plas.ERR_INVALID_ARGUMENT


def test_job_footprint(plas):
    # Three grids of n * dp elements dominate; the permutation, grouping table
    # and small tables add about 4 bytes per cell plus the table of the
    # largest block (beta = side/2 at the first level).
    for side, d, storage, elem in ((256, 59, "f32", 4), (1024, 59, "bf16", 2), (100, 3, "f32", 4)):
        n = side * side
        dp = plas.padded_channels(d)
        f = plas.job_footprint(side, d, storage)
        beta = max(16, side // 2)
        low = 3 * n * dp * elem + 4 * n + 4 * beta * beta
        assert low <= f <= low + 64 * 1024
    with pytest.raises(plas.PlasError):
        plas.job_footprint(1, 59)
    with pytest.raises(plas.PlasError):
        plas.job_footprint(64, 65)


def test_server_null_arguments(plas):
    L = plas.library()
    h = ctypes.c_void_p()
    assert L.plas_server_create(None, None, None, 1 << 30, ctypes.byref(h)) == plas.ERR_INVALID_ARGUMENT
    assert L.plas_server_destroy(None) == 0
    assert L.plas_server_step(None, None, None) == plas.ERR_INVALID_ARGUMENT
    n = ctypes.c_int32()
    assert L.plas_server_poll(None, None, None, 0, ctypes.byref(n)) == plas.ERR_INVALID_ARGUMENT
