"""Thin ctypes binding of libgw.so.

Argument marshalling only: every step of the screened-interaction path runs
in the library's HIP kernels.  Function names match include/gw.h.  Device
buffers are torch tensors on the GPU (only their data pointers cross the ABI);
streams are torch.cuda streams (their HIP handle crosses the ABI).

If libgw.so has not been built this module raises on import: there is no
fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgw.so")

GW_OK, GW_PENDING = 0, 1
GW_E_INVALID, GW_E_OOM, GW_E_DEVICE, GW_E_NOCONV, GW_E_RANGE, GW_E_STATE = -1, -2, -3, -4, -5, -6
GW_FP64, GW_FP32_IR, GW_BF16X_IR = 0, 1, 2

STATUS_NAMES = {
    0: "GW_OK", 1: "GW_PENDING", -1: "GW_E_INVALID", -2: "GW_E_OOM", -3: "GW_E_DEVICE",
    -4: "GW_E_NOCONV", -5: "GW_E_RANGE", -6: "GW_E_STATE",
}


class gw_molecule(ctypes.Structure):
    _fields_ = [
        ("n_orb", ctypes.c_int32), ("n_occ", ctypes.c_int32), ("n_prod", ctypes.c_int32),
        ("eig", ctypes.c_void_p), ("X", ctypes.c_void_p), ("n_blk", ctypes.c_int32),
        ("blk_prod", ctypes.c_void_p), ("blk_orb", ctypes.c_void_p), ("orb_idx", ctypes.c_void_p),
        ("blk_val", ctypes.c_void_p), ("vals", ctypes.c_void_p),
    ]


class gw_grid(ctypes.Structure):
    _fields_ = [
        ("n_omega", ctypes.c_int32), ("omega_min", ctypes.c_double), ("omega_max", ctypes.c_double),
        ("eps", ctypes.c_double), ("frac_bits", ctypes.c_int32),
    ]


class gw_report(ctypes.Structure):
    _fields_ = [
        ("n_hbins", ctypes.c_int32), ("frac_bits_used", ctypes.c_int32),
        ("n_dropped_pairs", ctypes.c_int64), ("n_solved", ctypes.c_int32),
        ("n_fallback", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("max_rel_update", ctypes.c_double),
    ]


class gw_sizes(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int64), ("n_hbins", ctypes.c_int32), ("n_upper", ctypes.c_int64),
        ("hist_bytes", ctypes.c_int64), ("chi0_bytes", ctypes.c_int64),
    ]


class gw_kernel_stat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
        ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
    ]


_P = ctypes.c_void_p
_SIGS = {
    "gw_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "gw_destroy": (ctypes.c_int, [_P]),
    "gw_last_error": (ctypes.c_char_p, [_P]),
    "gw_query_sizes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                      ctypes.POINTER(gw_grid), ctypes.c_int32, ctypes.POINTER(gw_sizes)]),
    "gw_build_chi0": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), ctypes.POINTER(gw_grid), _P,
                                     ctypes.c_int32, _P, _P, _P, ctypes.POINTER(gw_report)]),
    "gw_build_chi0_2w": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), ctypes.POINTER(gw_grid),
                                        ctypes.POINTER(gw_grid), _P, ctypes.c_int32, _P, _P, _P,
                                        ctypes.POINTER(gw_report)]),
    "gw_build_chi0_time": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), ctypes.POINTER(gw_grid), _P, _P, _P,
                                          ctypes.POINTER(gw_report)]),
    "gw_build_A_time": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), _P, ctypes.POINTER(gw_grid), _P, _P, _P,
                                       ctypes.POINTER(gw_report)]),
    "gw_self_energy": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), _P, ctypes.POINTER(gw_grid), _P, _P, _P, _P,
                                      _P, ctypes.POINTER(gw_report)]),
    "gw_dyson_dos": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), ctypes.POINTER(gw_grid), _P, _P, _P, _P, _P,
                                    _P, ctypes.POINTER(gw_report)]),
    "gw_solve_W": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                  ctypes.c_int, ctypes.c_double, _P, _P, ctypes.POINTER(gw_report)]),
    "gw_solve_W_A": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32,
                                    ctypes.c_int, ctypes.c_double, _P, _P, ctypes.POINTER(gw_report)]),
    "gw_solve_W_A_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32, _P, _P,
                                            ctypes.POINTER(gw_report)]),
    "gw_build_A": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), _P, ctypes.POINTER(gw_grid), _P, _P,
                                  ctypes.POINTER(gw_report)]),
    "gw_build_A_compressed": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), _P, _P, ctypes.c_int32,
                                             ctypes.POINTER(gw_grid), _P, _P, ctypes.POINTER(gw_report)]),
    "gw_compress_basis": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "gw_decompress": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P]),
    "gw_pair_basis": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), _P, ctypes.c_double, ctypes.c_int32, _P, _P,
                                     _P, _P, ctypes.POINTER(ctypes.c_int64)]),
    "gw_submit": (ctypes.c_int, [_P, ctypes.POINTER(gw_molecule), _P, ctypes.POINTER(gw_grid),
                                 ctypes.c_int32, ctypes.c_int, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "gw_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_P), ctypes.POINTER(gw_report)]),
    "gw_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "gw_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(gw_molecule), ctypes.POINTER(_P),
                                       ctypes.POINTER(gw_grid), ctypes.c_int, ctypes.c_double, ctypes.c_int32, _P,
                                       ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    "gw_batch_run": (ctypes.c_int, [_P, _P, ctypes.POINTER(gw_report)]),
    "gw_batch_destroy": (ctypes.c_int, [_P]),
    "gw_batch_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "gw_profile_begin": (ctypes.c_int, [_P]),
    "gw_profile_read": (ctypes.c_int, [_P, ctypes.POINTER(gw_kernel_stat), ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]),
    "gw_profile_end": (ctypes.c_int, [_P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libgw.so is not built (%s). Run `python -m paper_1101_2065_amd.build` "
            "(hipcc --offload-arch=gfx950); there is no fallback path." % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class GwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Context:
    """Owns one gw_ctx (device workspace) on one GPU."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = _P()
        st = lib.gw_create(device, budget_bytes, ctypes.byref(h))
        if st != GW_OK:
            raise GwError(st, "gw_create(device=%d) failed" % device)
        self.h = h

    def close(self):
        if self.h:
            lib.gw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str) -> int:
        if st < 0:
            raise GwError(st, "%s: %s" % (what, lib.gw_last_error(self.h).decode()))
        return st

    def build_chi0(self, mol: "gw_molecule", grid: "gw_grid", chi0_out, hist_out=None, basis=None,
                   k: int = 0, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_build_chi0(self.h, ctypes.byref(mol), ctypes.byref(grid), _ptr(basis), k,
                               _stream_handle(stream), _ptr(hist_out), _ptr(chi0_out),
                               ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_build_chi0")
        return rep

    def build_chi0_2w(self, mol: "gw_molecule", g_small: "gw_grid", g_large: "gw_grid", chi_small_out,
                      chi_large_out, basis=None, k: int = 0, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_build_chi0_2w(self.h, ctypes.byref(mol), ctypes.byref(g_small), ctypes.byref(g_large),
                                  _ptr(basis), k, _stream_handle(stream), _ptr(chi_small_out), _ptr(chi_large_out),
                                  ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_build_chi0_2w")
        return rep

    def build_chi0_time(self, mol: "gw_molecule", grid: "gw_grid", chi0_out, a_out=None, stream=None,
                        report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_build_chi0_time(self.h, ctypes.byref(mol), ctypes.byref(grid), _stream_handle(stream),
                                    _ptr(a_out), _ptr(chi0_out), ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_build_chi0_time")
        return rep

    def build_A_time(self, mol: "gw_molecule", v, grid: "gw_grid", A_out, a_out=None, stream=None,
                     report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_build_A_time(self.h, ctypes.byref(mol), _ptr(v), ctypes.byref(grid), _stream_handle(stream),
                                 _ptr(a_out), _ptr(A_out), ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_build_A_time")
        return rep

    def self_energy(self, mol: "gw_molecule", grid: "gw_grid", W, Sigma_out, v=None, sigma_out=None,
                    Sigma_x_out=None, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_self_energy(self.h, ctypes.byref(mol), _ptr(v), ctypes.byref(grid), _ptr(W),
                                _stream_handle(stream), _ptr(sigma_out), _ptr(Sigma_out), _ptr(Sigma_x_out),
                                ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_self_energy")
        return rep

    def dyson_dos(self, mol: "gw_molecule", grid: "gw_grid", dos_out, Sigma_c=None, Sigma_x=None, Vxc=None,
                  G_out=None, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_dyson_dos(self.h, ctypes.byref(mol), ctypes.byref(grid), _ptr(Sigma_c), _ptr(Sigma_x), _ptr(Vxc),
                              _stream_handle(stream), _ptr(dos_out), _ptr(G_out),
                              ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_dyson_dos")
        return rep

    def solve_W(self, v, n: int, chi0, n_omega: int, W_out, prec: int = GW_FP64, tol: float = 1e-7,
                v_is_diag: bool = False, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_solve_W(self.h, _ptr(v), int(v_is_diag), n, _ptr(chi0), n_omega, prec, tol,
                            _stream_handle(stream), _ptr(W_out),
                            ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_solve_W")
        return rep

    def build_A(self, mol: "gw_molecule", v, grid: "gw_grid", A_out, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_build_A(self.h, ctypes.byref(mol), _ptr(v), ctypes.byref(grid), _stream_handle(stream),
                            _ptr(A_out), ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_build_A")
        return rep

    def build_A_compressed(self, mol: "gw_molecule", S, basis, k: int, grid: "gw_grid", A_out, stream=None,
                           report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_build_A_compressed(self.h, ctypes.byref(mol), _ptr(S), _ptr(basis), k, ctypes.byref(grid),
                                       _stream_handle(stream), _ptr(A_out),
                                       ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_build_A_compressed")
        return rep

    def solve_W_A(self, v, n: int, A, n_omega: int, W_out, prec: int = GW_FP64, tol: float = 1e-7,
                  v_is_diag: bool = False, stream=None, report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_solve_W_A(self.h, _ptr(v), int(v_is_diag), n, _ptr(A), n_omega, prec, tol,
                              _stream_handle(stream), _ptr(W_out),
                              ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_solve_W_A")
        return rep

    def solve_W_A_noalloc(self, v, n: int, A, n_omega: int, W_out, v_is_diag: bool = False, stream=None,
                          report: bool = True):
        rep = gw_report() if report else None
        st = lib.gw_solve_W_A_noalloc(self.h, _ptr(v), int(v_is_diag), n, _ptr(A), n_omega, _stream_handle(stream),
                                      _ptr(W_out), ctypes.byref(rep) if rep is not None else None)
        self._check(st, "gw_solve_W_A_noalloc")
        return rep

    def compress_basis(self, v, n: int, k: int, Q_out, S_out, stream=None):
        st = lib.gw_compress_basis(self.h, _ptr(v), n, k, _stream_handle(stream), _ptr(Q_out), _ptr(S_out))
        self._check(st, "gw_compress_basis")

    def decompress(self, U, n: int, k: int, X, W_out, R=None, stream=None):
        st = lib.gw_decompress(self.h, _ptr(U), n, k, _ptr(X), _ptr(R), _stream_handle(stream), _ptr(W_out))
        self._check(st, "gw_decompress")

    def pair_basis(self, mol: "gw_molecule", v, e_threshold: float, k: int, Z_out, U_out, R_out=None,
                   stream=None) -> int:
        """Returns N_rank, the number of generating pairs."""
        nr = ctypes.c_int64()
        st = lib.gw_pair_basis(self.h, ctypes.byref(mol), _ptr(v), e_threshold, k, _stream_handle(stream),
                               _ptr(Z_out), _ptr(U_out), _ptr(R_out), ctypes.byref(nr))
        self._check(st, "gw_pair_basis")
        return nr.value

    def submit(self, mol: "gw_molecule", v, grid: "gw_grid", k_compress: int = 0, prec: int = GW_FP64,
               tol: float = 1e-7) -> int:
        t = ctypes.c_uint64()
        st = lib.gw_submit(self.h, ctypes.byref(mol), _ptr(v), ctypes.byref(grid), k_compress, prec, tol,
                           ctypes.byref(t))
        self._check(st, "gw_submit")
        return t.value

    def poll(self, ticket: int):
        """None while pending, else (device pointer, report)."""
        p = _P()
        rep = gw_report()
        st = lib.gw_poll(self.h, ticket, ctypes.byref(p), ctypes.byref(rep))
        if st == GW_PENDING:
            return None
        self._check(st, "gw_poll")
        return p.value, rep

    def release(self, ticket: int):
        self._check(lib.gw_release(self.h, ticket), "gw_release")

    def profile_begin(self):
        self._check(lib.gw_profile_begin(self.h), "gw_profile_begin")

    def profile_read(self):
        """Per kernel class: dict(name, launches, ms, flops, bytes)."""
        cap = 64
        arr = (gw_kernel_stat * cap)()
        n = ctypes.c_int32()
        self._check(lib.gw_profile_read(self.h, arr, cap, ctypes.byref(n)), "gw_profile_read")
        return [{"name": a.name.decode(), "launches": a.launches, "ms": a.ms, "flops": a.flops, "bytes": a.bytes}
                for a in arr[: min(n.value, cap)]]

    def profile_end(self):
        self._check(lib.gw_profile_end(self.h), "gw_profile_end")

    def batch_create(self, mols, vs, grid: "gw_grid", chi0_outs, W_outs, prec: int = GW_FP64,
                     tol: float = 1e-7, n_refine: int = 2, stream=None) -> "Batch":
        n = len(mols)
        arr = (gw_molecule * n)(*mols)
        pv = (_P * n)(*[_ptr(v) for v in vs])
        pc = (_P * n)(*[_ptr(c) for c in chi0_outs])
        pw = (_P * n)(*[_ptr(w) for w in W_outs])
        h = _P()
        st = lib.gw_batch_create(self.h, n, arr, pv, ctypes.byref(grid), prec, tol, n_refine,
                                 _stream_handle(stream), pc, pw, ctypes.byref(h))
        self._check(st, "gw_batch_create")
        return Batch(self, h, n)


class Batch:
    """A recorded batch (hipGraph) of molecules; run() replays it."""

    def __init__(self, ctx: "Context", h, n: int):
        self.ctx, self.h, self.n = ctx, h, n

    def run(self, stream=None, report: bool = True):
        reps = (gw_report * self.n)() if report else None
        st = lib.gw_batch_run(self.h, _stream_handle(stream), reps)
        self.ctx._check(st, "gw_batch_run")
        return list(reps) if report else None

    def stats(self):
        """dict(mode, steps, launches, products): how the batch was recorded
        (mode 0 molecules on branches, 1 lock steps aligned at the end, 2 at
        the start)."""
        m = ctypes.c_int32()
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.ctx._check(lib.gw_batch_stats(self.h, ctypes.byref(m), ctypes.byref(a), ctypes.byref(b),
                                           ctypes.byref(c)), "gw_batch_stats")
        return {"mode": m.value, "steps": a.value, "launches": b.value, "products": c.value}

    def close(self):
        if self.h:
            lib.gw_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_sizes(n_orb: int, n_occ: int, n_prod: int, eig_host, grid: "gw_grid", k: int = 0) -> gw_sizes:
    """eig_host: a C-contiguous float64 numpy array (host memory)."""
    out = gw_sizes()
    st = lib.gw_query_sizes(n_orb, n_occ, n_prod, eig_host.ctypes.data, ctypes.byref(grid), k,
                            ctypes.byref(out))
    if st != GW_OK:
        raise GwError(st, "gw_query_sizes")
    return out


def make_grid(n_omega: int, omega_min: float, omega_max: float, eps: float, frac_bits: int = -1) -> gw_grid:
    return gw_grid(n_omega, omega_min, omega_max, eps, frac_bits)


class DeviceMolecule:
    """Device copies (torch tensors) of a molecule's arrays plus the gw_molecule
    struct pointing at them.  `src` is any object with the fields of
    gw_molecule as host arrays (n_orb, n_occ, eig, X, blk_prod, blk_orb,
    orb_idx, blk_val, vals) and the Coulomb metric v."""

    def __init__(self, src, device="cuda"):
        import numpy as np
        import torch

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)

        self.eig = up(src.eig, np.float64)
        self.X = up(src.X, np.float64)
        self.blk_prod = up(src.blk_prod, np.int32)
        self.blk_orb = up(src.blk_orb, np.int32)
        self.orb_idx = up(src.orb_idx, np.int32)
        self.blk_val = up(src.blk_val, np.int64)
        self.vals = up(src.vals, np.float64)
        self.v = up(src.v, np.float64)
        self.n_orb = int(src.n_orb)
        self.n_occ = int(src.n_occ)
        self.n_prod = int(src.blk_prod[-1])
        self.struct = gw_molecule(
            self.n_orb, self.n_occ, self.n_prod, self.eig.data_ptr(), self.X.data_ptr(),
            len(src.blk_prod) - 1, self.blk_prod.data_ptr(), self.blk_orb.data_ptr(),
            self.orb_idx.data_ptr(), self.blk_val.data_ptr(), self.vals.data_ptr(),
        )
