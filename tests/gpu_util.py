"""Shared helpers of the GPU tests: device buffers in the library's layouts."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def ctx():
    from paper_2312_13051_amd import Context
    return Context(0)


def colmajor(n_mat, rows, cols, ld, dtype=torch.complex128, fill=None):
    """Device buffer of n_mat column-major rows x cols matrices with leading dimension ld.

    Returned tensor has shape (n_mat, cols, ld); element (r, c) of matrix q is t[q, c, r].
    """
    t = torch.empty((n_mat, cols, ld), dtype=dtype, device="cuda")
    if fill is not None:
        t.fill_(fill)
    return t


def to_np(t, rows):
    """(n_mat, cols, ld) device tensor -> numpy (n_mat, rows, cols)."""
    a = t.detach().cpu().numpy()
    return np.ascontiguousarray(np.swapaxes(a[:, :, :rows], 1, 2))


def from_np(a, ld, dtype=torch.complex128):
    """numpy (n_mat, rows, cols) -> device (n_mat, cols, ld)."""
    n_mat, rows, cols = a.shape
    buf = np.zeros((n_mat, cols, ld), dtype=np.complex128)
    buf[:, :, :rows] = np.swapaxes(a, 1, 2)
    return torch.from_numpy(buf).to(device="cuda", dtype=dtype)
