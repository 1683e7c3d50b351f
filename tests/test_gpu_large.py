"""GPU parity on large grids. At side 5800, 64-channel cells hold 2.15e9
elements per working grid, so any 32-bit element offset in ingest, blur,
gather or assignment would address the wrong cell; at side 2091 the grid has
the size of App. C's largest scene. The first two reorders of each sort (the
coarsest level) must equal the oracle's bit for bit."""
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


@pytest.mark.parametrize("channels", [59, 14])
def test_side_2091_first_reorders_match_oracle(ref, channels):
    """The scene scale of App. C's largest scene (4.37 M Gaussians, side
    2091): the first two reorders of the sort, with D = 59 and with the 14
    channels before the higher SH coefficients, equal the oracle's."""
    torch, plas = require_gpu()
    side = synthetic.GARDEN_SIDE
    n = side * side
    F = (synthetic.gaussian_attributes(n, synthetic.DATA_SEED_GARDEN) if channels == 59
         else synthetic.scene_attributes_14(n, synthetic.DATA_SEED_GARDEN))
    ctx = plas.Context(0)
    perm, res = ctx.sort(torch.from_numpy(F).cuda(), side, synthetic.SORT_SEED, max_reorders=2)
    want = ref.sort(F, side, synthetic.SORT_SEED, max_reorders=2)
    assert want.status == 0
    assert res.reorders == want.reorders == 2
    assert res.energy_fixed == want.energy and res.scale_shift == want.scale_shift
    assert np.array_equal(perm.cpu().numpy(), want.perm)
