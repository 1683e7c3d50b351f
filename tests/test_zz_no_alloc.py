"""GPU test of plas_grid_energy_noalloc, the energy query that allocates no
device memory: through the C ABI, its results equal plas_grid_energy's bit
for bit, on consecutive calls whose second input is smaller than the first
(the shared device scratch keeps the earlier call's data), in both storages,
with and without a permutation; inputs above its limit are refused."""
import ctypes

import numpy as np
import pytest

import synthetic
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _call(plas, ctx, name, f, perm, side, d, radius, storage, dtype):
    L = plas.library()
    E, s, mean = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_double()
    p = None if perm is None else ctypes.c_void_p(perm.data_ptr())
    ctx._bind_stream()
    st = getattr(L, name)(ctx._h, ctypes.c_void_p(f.data_ptr()), p, side * side, d, side, plas.LAYOUT_CN,
                          dtype, plas.STORAGES[storage], radius, ctypes.byref(E), ctypes.byref(s),
                          ctypes.byref(mean))
    return st, int(E.value), s.value, mean.value


def test_noalloc_energy_equals_the_allocating_query():
    torch, plas = require_gpu()
    ctx = plas.Context(0)
    cases = [  # (side, d, radius, storage, with perm): each a smaller input than the one before
        (256, 59, 1, "f32", True), (200, 59, 3, "bf16", True), (64, 14, 2, "f32", False),
        (33, 3, 1, "bf16", True), (16, 59, 0, "f32", True), (2, 4, 1, "bf16", False),
    ]
    for side, d, radius, storage, with_perm in cases:
        n = side * side
        F = synthetic.random_features(n, d, 7 + side, "cn", -2.0, 2.0)
        f = torch.from_numpy(F).cuda()
        perm = torch.from_numpy(synthetic.random_permutation(n, side)).cuda() if with_perm else None
        want = _call(plas, ctx, "plas_grid_energy", f, perm, side, d, radius, storage, plas.DTYPE_F32)
        got = _call(plas, ctx, "plas_grid_energy_noalloc", f, perm, side, d, radius, storage, plas.DTYPE_F32)
        assert want[0] == plas.OK and got[0] == plas.OK, (side, d, storage)
        assert got[1:3] == want[1:3], (side, d, radius, storage, got, want)
        assert got[3] == want[3]


def test_noalloc_energy_two_calls_in_a_row_second_smaller():
    torch, plas = require_gpu()
    ctx = plas.Context(0)
    out = []
    for side in (240, 48):
        n = side * side
        f = torch.from_numpy(synthetic.gaussian_attributes(n, side)).cuda()
        perm = torch.from_numpy(synthetic.random_permutation(n, side + 1)).cuda()
        want = ctx.grid_energy(f, perm, side, 1)
        got = ctx.grid_energy(f, perm, side, 1, noalloc=True)
        assert got == want, side
        out.append(got)
    assert out[0] != out[1]


def test_noalloc_energy_limits_and_errors():
    torch, plas = require_gpu()
    ctx = plas.Context(0)
    side = 257  # 66,049 cells: above the limit
    f = torch.zeros(3, side * side, device="cuda")
    st = _call(plas, ctx, "plas_grid_energy_noalloc", f, None, side, 3, 1, "f32", plas.DTYPE_F32)[0]
    assert st == plas.ERR_INVALID_ARGUMENT
    # Non-finite features and a bad permutation are reported as by plas_grid_energy.
    side = 20
    f = torch.from_numpy(synthetic.gaussian_attributes(side * side, 3)).cuda()
    bad = f.clone()
    bad[4, 9] = float("nan")
    assert _call(plas, ctx, "plas_grid_energy_noalloc", bad, None, side, 59, 1, "f32",
                 plas.DTYPE_F32)[0] == plas.ERR_NONFINITE
    perm = torch.zeros(side * side, dtype=torch.int32, device="cuda")
    assert _call(plas, ctx, "plas_grid_energy_noalloc", f, perm, side, 59, 1, "f32",
                 plas.DTYPE_F32)[0] == plas.ERR_INVALID_ARGUMENT
    # The query still works afterwards and agrees with the allocating one.
    assert ctx.grid_energy(f, None, side, 2, noalloc=True) == ctx.grid_energy(f, None, side, 2)
