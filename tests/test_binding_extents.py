"""Host logic of the binding's buffer checks: the extent of a batch of
column-major matrices, and the bytes a tensor's allocation holds from its
first element on (CPU tensors; the device check needs a GPU)."""
import pytest
import torch

from paper_2312_13051_amd import _lib as L


def test_span_of_matrix_batches():
    # 3 matrices of 4 x 2, leading dimension 5, 12 elements apart:
    # last matrix starts at 24, its last column at 24 + 5, ends at 24 + 5 + 4
    assert L._span(3, 12, 4, 2, 5) == 33
    assert L._span(1, 0, 4, 4, 4) == 16
    assert L._span(5, 0, 4, 4, 4) == 16          # stride 0: one matrix read five times
    for n, rows, cols in ((0, 4, 4), (2, 0, 4), (2, 4, 0), (2, 4, -1)):
        assert L._span(n, 16, rows, cols, 4) == 0


def test_require_counts_the_allocation_from_the_first_element():
    t = torch.zeros(10, dtype=torch.complex128)
    L._require(t, "t", 160)                 # exactly the allocation
    with pytest.raises(L.BerryError, match="t: the call accesses 161 bytes"):
        L._require(t, "t", 161)
    L._require(t[:2], "v", 160)             # a view: the allocation behind it counts
    with pytest.raises(L.BerryError, match="holds 144"):
        L._require(t[1:], "v", 160)         # starts one element in
    L._require(None, "absent", 10)          # left to the library's null-pointer check
    L._require(t, "nothing", 0)


def test_require_checks_the_device():
    with pytest.raises(L.BerryError, match="must be a tensor on cuda:0"):
        L._require(torch.zeros(4), "x", 8, device=0)
