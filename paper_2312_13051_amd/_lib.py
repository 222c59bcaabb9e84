"""ctypes binding of libberryhip (argument marshalling only).

Every function here forwards device pointers, sizes and the current torch
stream to the C ABI declared in ``include/berryhip.h``; all computation runs in
the library's HIP kernels. PyTorch provides device memory and streams only.
The library must have been built (``paper_2312_13051_amd/build.py``); there is
no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libberryhip.so")

BE_OK, BE_EINVAL, BE_ENOMEM, BE_EHIP, BE_ENOTIMPL = 0, -1, -2, -3, -4
BE_C128, BE_C64 = 0, 1
BE_FP64, BE_MIXED_FP32, BE_MIXED_FP32_REFINED, BE_MIXED_BF16X = 0, 1, 2, 3


def c64_input(precision: int) -> bool:
    """The eigensolver takes c64 Hamiltonians for this precision (the mixed
    paths that reduce in FP32 from an FP32 input), else c128."""
    return precision in (BE_MIXED_FP32, BE_MIXED_BF16X)
BE_OVL_POLAR, BE_OVL_RAW = 0, 1
ST_GAP_CLOSED, ST_OVERLAP_SINGULAR, ST_WINDING_UNRESOLVED = 1, 2, 4
ST_PSO_GAP, ST_WANNIER_GAP, ST_NONCONVERGED, ST_NAN_INF = 8, 16, 32, 64

EXPORTS = [
    "be_create", "be_destroy", "be_last_error", "be_workspace_bytes",
    "be_hk_plan_create", "be_hk_plan_destroy", "be_hk_plan_N",
    "be_build_hk", "be_eigh_batched", "be_wilson_loop", "be_nested_wilson",
    "be_spin_resolved_wilson", "be_plaquette_flux", "be_plaquette_flux_noalloc", "be_spin_sectors",
    "be_zgemm_strided",
    "be_profile_enable", "be_profile_query", "be_profile_names", "be_tune_set", "be_tune_get",
    "be_tune_set_orders", "be_tune_clear", "be_eigh_round",
]


class be_hoplist(C.Structure):
    _fields_ = [("N", C.c_int32), ("dim", C.c_int32), ("nnz", C.c_int64),
                ("i", C.c_void_p), ("j", C.c_void_p), ("R", C.c_void_p), ("t", C.c_void_p)]


class BerryError(RuntimeError):
    pass


_lib = None


def load():
    """Load libberryhip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise BerryError(f"{LIB_PATH} is missing: run `python paper_2312_13051_amd/build.py` first")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, f64p = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.be_create.argtypes = [C.POINTER(vp), C.c_int]
    lib.be_destroy.argtypes = [vp]
    lib.be_last_error.argtypes = [vp]
    lib.be_last_error.restype = C.c_char_p
    lib.be_workspace_bytes.argtypes = [vp]
    lib.be_workspace_bytes.restype = C.c_size_t
    lib.be_hk_plan_create.argtypes = [vp, C.POINTER(be_hoplist), i32, C.POINTER(vp)]
    lib.be_hk_plan_destroy.argtypes = [vp]
    lib.be_hk_plan_N.argtypes = [vp, i32]
    lib.be_hk_plan_N.restype = i32
    lib.be_build_hk.argtypes = [vp, vp, i32, i32, vp, i32, vp, i64, i32, i32, vp]
    lib.be_eigh_batched.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, i32, i32, vp, vp, i32, i64, vp, vp]
    lib.be_wilson_loop.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.be_nested_wilson.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, i32, i32, C.c_double, C.c_double,
                                     vp, vp, vp, C.POINTER(i32), vp, vp]
    lib.be_spin_resolved_wilson.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, i32, i32, i32, vp,
                                            vp, vp, vp, vp, vp, vp, C.POINTER(i32), vp, vp]
    lib.be_plaquette_flux.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, i32, vp, vp, vp, vp, vp]
    lib.be_plaquette_flux_noalloc.argtypes = lib.be_plaquette_flux.argtypes
    lib.be_spin_sectors.argtypes = [vp, vp, i32, i32, i32, i64, i32, i32, i32, vp, vp, vp, i32, i64,
                                    C.POINTER(i32), vp, vp]
    lib.be_zgemm_strided.argtypes = [vp, C.c_char, C.c_char, i32, i32, i32, f64p, vp, i32, i64, vp, i32, i64,
                                     f64p, vp, i32, i64, i32, vp]
    lib.be_profile_enable.argtypes = [vp, C.c_int]
    lib.be_profile_query.argtypes = [vp, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.be_profile_names.argtypes = [vp, C.c_char_p, C.c_size_t]
    lib.be_tune_set.argtypes = [vp, C.c_char_p, i32]
    lib.be_tune_get.argtypes = [vp, C.c_char_p, C.POINTER(i32)]
    lib.be_tune_set_orders.argtypes = [vp, C.c_char_p, i32, i32, i32, i32]
    lib.be_tune_clear.argtypes = [vp, C.c_char_p]
    lib.be_eigh_round.argtypes = [vp, i32, i32, C.POINTER(C.c_int64)]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype if name in (
            "be_last_error", "be_workspace_bytes", "be_hk_plan_N") else C.c_int
    _lib = lib
    return lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _span(n, stride, rows, cols, ld):
    """Elements from the start of the first to the end of the last of n
    column-major rows x cols matrices (matrix q at q*stride, leading
    dimension ld); 0 when nothing is accessed."""
    if n <= 0 or rows <= 0 or cols <= 0:
        return 0
    return (int(n) - 1) * int(stride) + (int(cols) - 1) * int(ld) + int(rows)


def _require(t, name, nbytes, device=None):
    """The library accesses nbytes bytes through t's pointer: t's storage
    must hold that many from t's first element on (whatever t's own shape and
    strides), and, with device given, t must live on that HIP device. Checked
    on the host before the call, so a too-small buffer is an error here, not
    a device memory fault. A missing tensor is left to the library (its
    BE_EINVAL for a null pointer)."""
    if t is None or nbytes <= 0:
        return
    if device is not None and (not t.is_cuda or t.device.index != device):
        raise BerryError(f"{name}: must be a tensor on cuda:{device}, got one on {t.device}")
    avail = t.untyped_storage().nbytes() - t.storage_offset() * t.element_size()
    if avail < nbytes:
        raise BerryError(f"{name}: the call accesses {nbytes} bytes from its first element, its storage holds {avail}")


class HkPlan:
    """Device copy of packed hopping lists (be_hk_plan)."""

    def __init__(self, ctx: "Context", hoplists):
        self.ctx = ctx
        self._keep = []
        arr = (be_hoplist * len(hoplists))()
        for k, h in enumerate(hoplists):
            i = np.ascontiguousarray(h.i, dtype=np.int32)
            j = np.ascontiguousarray(h.j, dtype=np.int32)
            R = np.ascontiguousarray(h.R, dtype=np.int32)
            t = np.ascontiguousarray(np.asarray(h.t, dtype=np.complex128).view(np.float64))
            self._keep += [i, j, R, t]
            arr[k] = be_hoplist(int(h.N), int(h.dim), int(h.t.shape[0]), i.ctypes.data, j.ctypes.data,
                                R.ctypes.data, t.ctypes.data)
        self.handle = C.c_void_p()
        ctx._check(ctx.lib.be_hk_plan_create(ctx.handle, arr, len(hoplists), C.byref(self.handle)))
        self.N = [int(ctx.lib.be_hk_plan_N(self.handle, k)) for k in range(len(hoplists))]

    def close(self):
        if self.handle:
            self.ctx.lib.be_hk_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Per-order settings measured on an MI355X by tune.py (applied by default)
DEFAULT_TUNING = os.path.join(_HERE, "tuning_mi355x.json")


class Context:
    """One be_ctx on a HIP device. tuning: "default" applies DEFAULT_TUNING
    (when present), None leaves the library's defaults, or a table / path."""

    def __init__(self, device: int = 0, tuning="default"):
        self.lib = load()
        try:  # torch provides the streams and device memory: let it initialize the device first
            import torch
            torch.cuda.init()
        except Exception:  # noqa: BLE001 - be_create reports a missing device itself
            pass
        self.handle = C.c_void_p()
        self.device = int(device)
        rc = self.lib.be_create(C.byref(self.handle), self.device)
        if rc != BE_OK:
            raise BerryError(f"be_create failed ({rc})")
        self.tuning = None
        if tuning == "default":
            if os.path.exists(DEFAULT_TUNING):
                self.load_tuning(DEFAULT_TUNING)
                self.tuning = os.path.basename(DEFAULT_TUNING)
        elif tuning is not None:
            self.load_tuning(tuning)
            self.tuning = tuning if isinstance(tuning, str) else "table"

    def _check(self, rc):
        if rc != BE_OK:
            raise BerryError(f"berryhip error {rc}: {self.lib.be_last_error(self.handle).decode()}")

    def close(self):
        if self.handle:
            self.lib.be_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.be_workspace_bytes(self.handle))

    # ------------------------------------------------------------ calls
    def hk_plan(self, hoplists) -> HkPlan:
        return HkPlan(self, hoplists)

    def _req(self, t, name, n_elems, elem_bytes):
        _require(t, name, int(n_elems) * elem_bytes, self.device)

    def _ugrid(self, U, N, m, ldu, u_stride, n_mats, name="U"):
        self._req(U, name, _span(n_mats, u_stride, N, m, ldu), 16)

    def build_hk(self, plan: HkPlan, sys_first: int, n_sys: int, kappa, H, mat_stride: int, ld: int, dtype: int):
        n_kap = kappa.shape[0]
        N = int(self.lib.be_hk_plan_N(plan.handle, int(sys_first)))
        self._req(kappa, "kappa", n_kap * 3, 8)
        self._req(H, "H", _span(n_sys * n_kap, mat_stride, N, N, ld), 16 if dtype == BE_C128 else 8)
        self._check(self.lib.be_build_hk(self.handle, plan.handle, sys_first, n_sys, _ptr(kappa), kappa.shape[0],
                                         _ptr(H), mat_stride, ld, dtype, _stream()))

    def eigh_batched(self, H, dtype, N, ld, mat_stride, n_mat, lo, hi, precision, evals, U, ldu, u_stride, status):
        m = hi - lo
        self._req(H, "H", _span(n_mat, mat_stride, N, N, ld), 16 if dtype == BE_C128 else 8)
        self._req(evals, "evals", n_mat * (m + 2), 8)
        self._ugrid(U, N, m, ldu, u_stride, n_mat)
        self._req(status, "status", n_mat, 4)
        self._check(self.lib.be_eigh_batched(self.handle, _ptr(H), dtype, N, ld, mat_stride, n_mat, lo, hi,
                                             precision, _ptr(evals), _ptr(U), ldu, u_stride, _ptr(status),
                                             _stream()))

    def wilson_loop(self, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, mode, theta, phi, winding, status):
        self._ugrid(U, N, m, ldu, u_stride, n_sys * n_perp * n_par)
        self._req(theta, "theta", n_sys * n_perp * m, 8)
        self._req(phi, "phi", n_sys * n_perp, 8)
        self._req(winding, "winding", n_sys, 4)
        self._req(status, "status", n_sys, 4)
        self._check(self.lib.be_wilson_loop(self.handle, _ptr(U), N, m, ldu, u_stride, n_sys, n_par, n_perp, mode,
                                            _ptr(theta), _ptr(phi), _ptr(winding), _ptr(status), _stream()))

    def nested_wilson(self, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, mode, win_lo, win_hi, nested_theta, p,
                      p_mean, status):
        self._ugrid(U, N, m, ldu, u_stride, n_sys * n_perp * n_par)
        self._req(nested_theta, "nested_theta", n_sys * n_par * m, 8)
        self._req(p, "p", n_sys * n_par, 8)
        self._req(p_mean, "p_mean", n_sys, 8)
        self._req(status, "status", n_sys, 4)
        s_out = (C.c_int32 * n_sys)()
        self._check(self.lib.be_nested_wilson(self.handle, _ptr(U), N, m, ldu, u_stride, n_sys, n_par, n_perp, mode,
                                              win_lo, win_hi, _ptr(nested_theta), _ptr(p), _ptr(p_mean), s_out,
                                              _ptr(status), _stream()))
        return [int(x) for x in s_out]

    def spin_resolved_wilson(self, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, mode, spin_diag, pso_evals,
                             theta_dn, theta_up, C_dn, C_up, C_s, status, precision=BE_FP64, m_dn_in=None):
        """m_dn_in: sector sizes to pass in (required while the stream is
        being captured into a graph)."""
        self._ugrid(U, N, m, ldu, u_stride, n_sys * n_perp * n_par)
        self._req(spin_diag, "spin_diag", n_sys * N, 8)
        self._req(pso_evals, "pso_evals", n_sys * n_perp * n_par * m, 8)
        for t, name in ((theta_dn, "theta_dn"), (theta_up, "theta_up")):
            self._req(t, name, n_sys * n_perp * m, 8)
        for t, name in ((C_dn, "C_dn"), (C_up, "C_up"), (status, "status")):
            self._req(t, name, n_sys, 4)
        self._req(C_s, "C_s", n_sys, 8)
        m_dn = (C.c_int32 * n_sys)(*(m_dn_in or []))
        self._check(self.lib.be_spin_resolved_wilson(self.handle, _ptr(U), N, m, ldu, u_stride, n_sys, n_par, n_perp,
                                                     mode, precision, _ptr(spin_diag), _ptr(pso_evals), _ptr(theta_dn),
                                                     _ptr(theta_up), _ptr(C_dn), _ptr(C_up), _ptr(C_s), m_dn,
                                                     _ptr(status), _stream()))
        return [int(x) for x in m_dn]

    def _flux_args(self, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status):
        self._ugrid(U, N, m, ldu, u_stride, n_sys * n_perp * n_par)
        self._req(flux, "flux", n_sys * n_perp * n_par, 8)
        self._req(chern, "chern", n_sys, 4)
        self._req(total, "total", n_sys, 8)
        self._req(status, "status", n_sys, 4)

    def plaquette_flux(self, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status):
        self._flux_args(U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status)
        self._check(self.lib.be_plaquette_flux(self.handle, _ptr(U), N, m, ldu, u_stride, n_sys, n_par, n_perp,
                                               _ptr(flux), _ptr(chern), _ptr(total), _ptr(status), _stream()))

    def plaquette_flux_noalloc(self, U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status):
        self._flux_args(U, N, m, ldu, u_stride, n_sys, n_par, n_perp, flux, chern, total, status)
        self._check(self.lib.be_plaquette_flux_noalloc(self.handle, _ptr(U), N, m, ldu, u_stride, n_sys, n_par,
                                                       n_perp, _ptr(flux), _ptr(chern), _ptr(total), _ptr(status),
                                                       _stream()))

    def spin_sectors(self, U, N, m, ldu, u_stride, n_sys, n_k_sys, spin_diag, pso_evals, V, ldv, v_stride, status,
                     precision=BE_FP64):
        self._ugrid(U, N, m, ldu, u_stride, n_sys * n_k_sys)
        self._req(spin_diag, "spin_diag", n_sys * N, 8)
        self._req(pso_evals, "pso_evals", n_sys * n_k_sys * m, 8)
        self._ugrid(V, N, m, ldv, v_stride, n_sys * n_k_sys, "V")
        self._req(status, "status", n_sys, 4)
        m_dn = (C.c_int32 * n_sys)()
        self._check(self.lib.be_spin_sectors(self.handle, _ptr(U), N, m, ldu, u_stride, n_sys, n_k_sys, precision,
                                             _ptr(spin_diag), _ptr(pso_evals), _ptr(V), ldv, v_stride, m_dn,
                                             _ptr(status), _stream()))
        return [int(x) for x in m_dn]

    def tune_set(self, knob: str, value: int):
        self._check(self.lib.be_tune_set(self.handle, knob.encode(), int(value)))

    def tune_get(self, knob: str) -> int:
        v = C.c_int32()
        self._check(self.lib.be_tune_get(self.handle, knob.encode(), C.byref(v)))
        return v.value

    def tune_set_orders(self, knob: str, n_lo: int, n_hi: int, precision: int, value: int):
        self._check(self.lib.be_tune_set_orders(self.handle, knob.encode(), int(n_lo), int(n_hi), int(precision),
                                                int(value)))

    def eigh_round(self, N: int, precision: int) -> int:
        """Matrices of order N the eigensolver runs at once on the device."""
        r = C.c_int64()
        self._check(self.lib.be_eigh_round(self.handle, int(N), int(precision), C.byref(r)))
        return int(r.value)

    def tune_clear(self, knob: str):
        self._check(self.lib.be_tune_clear(self.handle, knob.encode()))

    def load_tuning(self, table):
        """Apply a tuning table (a dict, or the path of its JSON file, as
        tune.py writes it): {"knobs": {knob: [{"n_lo", "n_hi", "precision",
        "value"}, ...]}}. Returns the table."""
        if isinstance(table, (str, os.PathLike)):
            import json
            with open(table) as f:
                table = json.load(f)
        for knob, rows in table.get("knobs", {}).items():
            self.tune_clear(knob)
            for r in rows:
                self.tune_set_orders(knob, r["n_lo"], r["n_hi"], r["precision"], r["value"])
        return table

    def profile_enable(self, on=True):
        self._check(self.lib.be_profile_enable(self.handle, 1 if on else 0))

    def profile(self):
        """{name: (total_ms, launches)} of the launches recorded since profile_enable."""
        buf = C.create_string_buffer(8192)
        self._check(self.lib.be_profile_names(self.handle, buf, 8192))
        out = {}
        for name in filter(None, buf.value.decode().split(",")):
            ms, n = C.c_double(), C.c_int64()
            self._check(self.lib.be_profile_query(self.handle, name.encode(), C.byref(ms), C.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def zgemm_strided(self, opA, opB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, Cm, ldc, sC, batch):
        a = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        b = (C.c_double * 2)(complex(beta).real, complex(beta).imag)
        ra, ca = (M, K) if opA == "N" else (K, M)
        rb, cb = (K, N) if opB == "N" else (N, K)
        self._req(A, "A", _span(batch, sA, ra, ca, lda), 16)
        self._req(B, "B", _span(batch, sB, rb, cb, ldb), 16)
        self._req(Cm, "C", _span(batch, sC, M, N, ldc), 16)
        self._check(self.lib.be_zgemm_strided(self.handle, opA.encode(), opB.encode(), M, N, K, a, _ptr(A), lda, sA,
                                              _ptr(B), ldb, sB, b, _ptr(Cm), ldc, sC, batch, _stream()))
