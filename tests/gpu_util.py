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


def to_working_layout(torch, G: np.ndarray, dp: int, storage: str = "f32"):
    """[N][d] float32 (numpy) -> device [N][dp] with zero padding, held as
    float32 or bfloat16 (the values must then be bfloat16 values already)."""
    N, d = G.shape
    out = np.zeros((N, dp), dtype=np.float32)
    out[:, :d] = G
    t = torch.from_numpy(out)
    if storage == "bf16":
        b = t.to(torch.bfloat16)
        assert torch.equal(b.to(torch.float32), t), "values are not bfloat16 values"
        t = b
    return t.cuda()


def from_working_layout(t, d: int) -> np.ndarray:
    return t.float().cpu().numpy()[:, :d].copy()


def bits(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
