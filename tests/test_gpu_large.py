"""GPU parity at a size where element offsets pass 2^31: a 5800 x 5800 grid of
64-channel cells holds 2.15e9 elements per working grid, so any 32-bit
element offset in ingest, blur, gather or assignment would address the wrong
cell. The first two reorders of the sort (the coarsest level, block side
2900) must equal the oracle's bit for bit."""
import numpy as np
import pytest

import synthetic
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def test_side_5800_first_reorders_match_oracle(ref):
    torch, plas = require_gpu()
    side, d = 5800, 59
    n = side * side
    assert n * plas.padded_channels(d) > 2 ** 31
    F = synthetic.random_features(n, d, 21, "cn", -1.0, 1.0)
    ctx = plas.Context(0)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, 5, max_reorders=2)
    want = ref.sort(F, side, 5, max_reorders=2)
    assert want.status == 0
    assert res.reorders == want.reorders == 2
    assert res.energy_fixed == want.energy and res.scale_shift == want.scale_shift
    p = perm.cpu().numpy()
    assert np.array_equal(p, want.perm)
    assert np.array_equal(np.bincount(p, minlength=n), np.ones(n, dtype=np.int64))
