"""Helpers shared by the GPU tests (marshalling only)."""
import numpy as np


def require_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2312_13299_amd as plas
    plas.library()  # raises if libplas.so is missing: no silent fallback
    return torch, plas


def to_working_layout(torch, G: np.ndarray, dp: int):
    """[N][d] float32 (numpy) -> device [N][dp] with zero padding."""
    N, d = G.shape
    out = np.zeros((N, dp), dtype=np.float32)
    out[:, :d] = G
    return torch.from_numpy(out).cuda()


def from_working_layout(t, d: int) -> np.ndarray:
    return t.cpu().numpy()[:, :d].copy()


def bits(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
