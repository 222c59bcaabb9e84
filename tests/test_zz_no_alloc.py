"""The plaquette flux without device allocation (be_plaquette_flux_noalloc,
for callers that cannot allocate): through the C ABI, its outputs equal
be_plaquette_flux's on the same inputs, on two calls in a row, the second
with a smaller input (the fixed scratch keeps the first call's contents);
one system larger than the fixed scratch is refused before any launch."""
import ctypes as C

import numpy as np
import pytest

from tests import gpu_util as gu

torch = gu.torch
pytestmark = pytest.mark.gpu


def grid(seed, n_sys, n_perp, n_par, N, m):
    """Random orthonormal bases, U-grid layout (n_mat, m, N) on the device."""
    rng = np.random.default_rng(seed)
    g = np.linalg.qr(rng.standard_normal((n_sys * n_perp * n_par, N, m)) +
                     1j * rng.standard_normal((n_sys * n_perp * n_par, N, m)))[0]
    return gu.from_np(g, N)


def outputs(n_sys, n_perp, n_par, fill):
    return (torch.full((n_sys, n_perp, n_par), fill, dtype=torch.float64, device="cuda"),
            torch.full((n_sys,), -7, dtype=torch.int32, device="cuda"),
            torch.full((n_sys,), fill, dtype=torch.float64, device="cuda"),
            torch.full((n_sys,), -7, dtype=torch.int32, device="cuda"))


def call(c, fn, U, N, m, n_sys, n_par, n_perp, out):
    from paper_2312_13051_amd import _lib as L
    f, ch, tot, st = out
    return getattr(c.lib, fn)(c.handle, L._ptr(U), N, m, N, U.stride(0), n_sys, n_par, n_perp, L._ptr(f), L._ptr(ch),
                              L._ptr(tot), L._ptr(st), L._stream())


def test_noalloc_flux_equals_flux_twice_then_smaller():
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    c = gu.ctx()
    lib = c.lib
    lib.be_plaquette_flux_noalloc.argtypes = lib.be_plaquette_flux.argtypes
    lib.be_plaquette_flux_noalloc.restype = C.c_int
    # (n_sys, n_perp, n_par, N, m): 90 links of order 140 (workgroup LU), then
    # a smaller input in every respect: 12 links of order 40 (one-wave LU)
    for seed, (n_sys, n_perp, n_par, N, m) in ((1, (3, 5, 6, 300, 140)), (2, (1, 3, 4, 80, 40))):
        U = grid([41, seed], n_sys, n_perp, n_par, N, m)
        ref = outputs(n_sys, n_perp, n_par, 9.0)
        got = outputs(n_sys, n_perp, n_par, -9.0)
        assert call(c, "be_plaquette_flux", U, N, m, n_sys, n_par, n_perp, ref) == L.BE_OK
        ws = c.workspace_bytes
        assert call(c, "be_plaquette_flux_noalloc", U, N, m, n_sys, n_par, n_perp, got) == L.BE_OK
        torch.cuda.synchronize()
        assert c.workspace_bytes == ws
        for a, b in zip(ref, got):
            assert torch.equal(a, b)
        assert np.isfinite(got[0].cpu().numpy()).all()


def test_noalloc_flux_refuses_a_system_beyond_the_scratch():
    gu.need_gpu()
    from paper_2312_13051_amd import _lib as L
    c = gu.ctx()
    lib = c.lib
    lib.be_plaquette_flux_noalloc.argtypes = lib.be_plaquette_flux.argtypes
    lib.be_plaquette_flux_noalloc.restype = C.c_int
    # one system of 8 x 8 links of order 1200: 1.47 GB of links > 128 MiB
    N, m = 1200, 1200
    U = torch.zeros((1, m, N), dtype=torch.complex128, device="cuda")
    f = torch.zeros((1, 8, 8), dtype=torch.float64, device="cuda")
    i = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc = lib.be_plaquette_flux_noalloc(c.handle, L._ptr(U), N, m, N, m * N, 1, 8, 8, L._ptr(f), L._ptr(i), L._ptr(f),
                                       L._ptr(i), L._stream())
    assert rc == L.BE_EINVAL
    assert "scratch" in lib.be_last_error(c.handle).decode()
