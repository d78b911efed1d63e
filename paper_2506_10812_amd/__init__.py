"""MI355X (gfx950) library for the exact thin-disc self-gravity kernel of
arXiv 2506.10812 -- Python binding.

This module only marshals arguments to the C ABI of ``libsg.so`` (declared in
``include/sg.h``); every step of the computation runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  If the
library has not been built the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg.so")

OK, ERR_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_WORKSPACE, ERR_TABLE, ERR_SCRATCH = range(7)
NOALLOC_SCRATCH_BYTES = 64 << 20
F32, F64 = 0, 1
SELF_CELL_EXCLUDE = 1
WITH_DH = 2
INDIRECT = 4
SEMI_SPECTRAL = 8
SS_FULL = 16
POTENTIAL = 32
LINEAR_R = 64
SECOND_ORDER = 128


class SGError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


class Grid(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("r_min", ctypes.c_double), ("r_max", ctypes.c_double)]


class Fluids(ctypes.Structure):
    _fields_ = [("n_fluids", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("h", ctypes.c_double * 4)]


class Disc(ctypes.Structure):
    _fields_ = [("grid", Grid), ("fluids", Fluids), ("flags", ctypes.c_uint32),
                ("n_species", ctypes.c_int32), ("sigma", ctypes.c_void_p), ("g_r", ctypes.c_void_p),
                ("g_phi", ctypes.c_void_p), ("table", ctypes.c_void_p),
                ("species_group", ctypes.c_uint8 * 8)]


class TuneResult(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "pass_", "length", "n_fluids", "n_jobs", "small_radix_first", "groups_per_wg", "cluster",
        "candidates", "rejected")] + [(n, ctypes.c_float) for n in ("rel_best", "ms_default", "ms_best")]


def grid(n_r, n_phi, r_min, r_max) -> Grid:
    return Grid(int(n_r), int(n_phi), float(r_min), float(r_max))


def fluids(h) -> Fluids:
    h = [float(v) for v in (h if hasattr(h, "__len__") else [h])]
    arr = (ctypes.c_double * 4)(*(h + [0.0] * (4 - len(h))))
    return Fluids(len(h), 0, arr)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: the HIP library has not been built "
            "(run __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, u32, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int, ctypes.c_int64
    GP, FP, DP = ctypes.POINTER(Grid), ctypes.POINTER(Fluids), ctypes.POINTER(Disc)
    dp = ctypes.POINTER(ctypes.c_double)
    sigs = {
        "sg_kernel_table_bytes": (sz, [GP, FP, u32]),
        "sg_kernel_table_workspace_bytes": (sz, [GP, FP, u32]),
        "sg_kernel_table": (i32, [GP, FP, u32, vp, vp, sz, vp]),
        "sg_ss_table_bytes": (sz, [GP, i32, u32]),
        "sg_ss_table_workspace_bytes": (sz, [GP, i32]),
        "sg_ss_table": (i32, [GP, i32, vp, u32, vp, vp, sz, vp]),
        "sg_field_fft_workspace_bytes": (sz, [DP, i32]),
        "sg_field_fft": (i32, [DP, i32, vp, sz, vp]),
        "sg_field_fft_profile": (i32, [DP, i32, vp, sz, vp, i32, ctypes.POINTER(ctypes.c_float)]),
        "sg_field_fft_tune": (i32, [DP, i32, vp, sz, vp, ctypes.POINTER(TuneResult), i32,
                                    ctypes.POINTER(ctypes.c_int)]),
        "sg_field_direct_workspace_bytes": (sz, [GP, i32, i32, i32]),
        "sg_field_direct": (i32, [GP, i32, dp, vp, vp, vp, vp, i32, u32, vp, sz, vp]),
        "sg_field_direct_noalloc": (i32, [GP, i32, dp, vp, vp, vp, vp, i32, u32, vp]),
        "sg_field_adjoint_workspace_bytes": (sz, [DP]),
        "sg_field_adjoint": (i32, [DP, vp, vp, vp, vp, vp, sz, vp]),
        "sg_ss_grad_H_workspace_bytes": (sz, [DP]),
        "sg_ss_grad_H": (i32, [DP, vp, vp, vp, vp, vp, sz, vp]),
        "sg_eval_F": (i32, [vp, vp, vp, i64, i32, vp]),
        "sg_eval_G0": (i32, [vp, vp, i64, i32, vp]),
        "sg_hsg": (i32, [i64, i32, vp, vp, vp, vp]),
        "sg_potential_direct_workspace_bytes": (sz, [GP, i32, i32, i32]),
        "sg_potential_direct": (i32, [GP, i32, dp, vp, vp, vp, i32, u32, vp, sz, vp]),
        "sg_self_cell": (i32, [GP, dp, dp, i32, i32, vp, vp]),
        "sg_release": (None, []),
        "sg_field_fft_cache_entries": (i32, []),
        "sg_status_string": (ctypes.c_char_p, [i32]),
        "sg_version": (i32, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_lib = _load()
EXPORTED = (
    "sg_kernel_table_bytes", "sg_kernel_table_workspace_bytes", "sg_kernel_table",
    "sg_ss_table_bytes", "sg_ss_table_workspace_bytes", "sg_ss_table",
    "sg_field_fft_workspace_bytes", "sg_field_fft", "sg_field_fft_profile", "sg_field_fft_tune",
    "sg_field_direct_workspace_bytes",
    "sg_field_direct", "sg_field_direct_noalloc", "sg_potential_direct_workspace_bytes",
    "sg_potential_direct",
    "sg_field_adjoint_workspace_bytes", "sg_field_adjoint", "sg_ss_grad_H_workspace_bytes",
    "sg_ss_grad_H", "sg_eval_F", "sg_eval_G0", "sg_hsg",
    "sg_self_cell", "sg_release", "sg_field_fft_cache_entries", "sg_status_string", "sg_version")


def lib():
    return _lib


def status_string(s: int) -> str:
    return _lib.sg_status_string(int(s)).decode()


def version() -> int:
    return int(_lib.sg_version())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(st, where):
    if st != OK:
        raise SGError(st, where)


# ------------------------------------------------------------------ sizes
def kernel_table_bytes(g: Grid, f: Fluids, flags: int = 0) -> int:
    return int(_lib.sg_kernel_table_bytes(ctypes.byref(g), ctypes.byref(f), flags))


def kernel_table_workspace_bytes(g: Grid, f: Fluids, flags: int = 0) -> int:
    return int(_lib.sg_kernel_table_workspace_bytes(ctypes.byref(g), ctypes.byref(f), flags))


def ss_table_bytes(g: Grid, n_fluids: int, flags: int = 0) -> int:
    return int(_lib.sg_ss_table_bytes(ctypes.byref(g), int(n_fluids), int(flags)))


def ss_table_workspace_bytes(g: Grid, n_fluids: int) -> int:
    return int(_lib.sg_ss_table_workspace_bytes(ctypes.byref(g), int(n_fluids)))


def _disc_array(discs):
    arr = (Disc * len(discs))(*discs)
    return arr


def field_fft_workspace_bytes(discs) -> int:
    arr = _disc_array(discs)
    return int(_lib.sg_field_fft_workspace_bytes(arr, len(discs)))


def field_direct_workspace_bytes(g: Grid, n_fluids: int, dtype: int, per_cell_H: bool) -> int:
    return int(_lib.sg_field_direct_workspace_bytes(ctypes.byref(g), n_fluids, dtype,
                                                    1 if per_cell_H else 0))


def field_adjoint_workspace_bytes(disc: Disc) -> int:
    return int(_lib.sg_field_adjoint_workspace_bytes(ctypes.byref(disc)))


def ss_grad_H_workspace_bytes(disc: Disc) -> int:
    return int(_lib.sg_ss_grad_H_workspace_bytes(ctypes.byref(disc)))


# ------------------------------------------------------------------ calls
def kernel_table(g: Grid, f: Fluids, flags, table, ws, ws_bytes=None, stream=None):
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_kernel_table(ctypes.byref(g), ctypes.byref(f), flags, _ptr(table), _ptr(ws),
                                ws_bytes, _stream(stream)), "sg_kernel_table")


def ss_table(g: Grid, n_fluids, H, flags, table, ws, ws_bytes=None, stream=None):
    """H: device float64 [n_fluids][n_r], the scale heights at the ring centres."""
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_ss_table(ctypes.byref(g), int(n_fluids), _ptr(H), flags, _ptr(table), _ptr(ws),
                            ws_bytes, _stream(stream)), "sg_ss_table")


def make_disc(g: Grid, f: Fluids, flags, sigma, g_r, g_phi, table, species_group=None) -> Disc:
    """species_group: kernel group of each species of sigma ([S][n_r][n_phi]),
    or None for one density per fluid."""
    sp = list(species_group) if species_group is not None else []
    grp = (ctypes.c_uint8 * 8)(*(sp + [0] * (8 - len(sp))))
    return Disc(g, f, flags, len(sp), _ptr(sigma), _ptr(g_r), _ptr(g_phi), _ptr(table), grp)


def field_fft(discs, ws, ws_bytes=None, stream=None):
    arr = _disc_array(discs)
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_field_fft(arr, len(discs), _ptr(ws), ws_bytes, _stream(stream)), "sg_field_fft")


def field_fft_profile(discs, ws, reps, ws_bytes=None, stream=None):
    """Mean ms of the three passes over `reps` event-timed launches."""
    arr = _disc_array(discs)
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    ms = (ctypes.c_float * 3)()
    _check(_lib.sg_field_fft_profile(arr, len(discs), _ptr(ws), ws_bytes, _stream(stream), reps, ms),
           "sg_field_fft_profile")
    return [float(v) for v in ms]


def field_fft_tune(discs, ws, ws_bytes=None, stream=None, capacity=256):
    """Autotunes the batch's launch classes; returns one dict per class."""
    arr = _disc_array(discs)
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    res = (TuneResult * capacity)()
    n = ctypes.c_int(0)
    _check(_lib.sg_field_fft_tune(arr, len(discs), _ptr(ws), ws_bytes, _stream(stream), res, capacity,
                                  ctypes.byref(n)), "sg_field_fft_tune")
    out = []
    for r in res[:min(n.value, capacity)]:
        d = {k: getattr(r, k) for k, _ in TuneResult._fields_}
        d["pass"] = d.pop("pass_")
        out.append(d)
    return out


def field_direct(g: Grid, n_fluids, h, sigma, H, g_r, g_phi, dtype, flags, ws, ws_bytes=None,
                 stream=None):
    harr = (ctypes.c_double * 4)(*([float(v) for v in h] + [0.0] * (4 - len(h)))) if h is not None else None
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_field_direct(ctypes.byref(g), n_fluids,
                                ctypes.cast(harr, ctypes.POINTER(ctypes.c_double)) if harr else None,
                                _ptr(sigma), _ptr(H), _ptr(g_r), _ptr(g_phi), dtype, flags,
                                _ptr(ws), ws_bytes, _stream(stream)), "sg_field_direct")


def field_direct_noalloc(g: Grid, n_fluids, h, sigma, H, g_r, g_phi, dtype, flags, stream=None):
    """sg_field_direct on the library's static scratch array (no workspace)."""
    harr = (ctypes.c_double * 4)(*([float(v) for v in h] + [0.0] * (4 - len(h)))) if h is not None else None
    _check(_lib.sg_field_direct_noalloc(ctypes.byref(g), n_fluids,
                                        ctypes.cast(harr, ctypes.POINTER(ctypes.c_double)) if harr else None,
                                        _ptr(sigma), _ptr(H), _ptr(g_r), _ptr(g_phi), dtype, flags,
                                        _stream(stream)), "sg_field_direct_noalloc")


def potential_direct_workspace_bytes(g: Grid, n_fluids, dtype, per_cell_H) -> int:
    return int(_lib.sg_potential_direct_workspace_bytes(ctypes.byref(g), n_fluids, dtype,
                                                        1 if per_cell_H else 0))


def potential_direct(g: Grid, n_fluids, h, sigma, H, pot, dtype, flags, ws, ws_bytes=None, stream=None):
    harr = (ctypes.c_double * 4)(*([float(v) for v in h] + [0.0] * (4 - len(h)))) if h is not None else None
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_potential_direct(ctypes.byref(g), n_fluids,
                                    ctypes.cast(harr, ctypes.POINTER(ctypes.c_double)) if harr else None,
                                    _ptr(sigma), _ptr(H), _ptr(pot), dtype, flags, _ptr(ws), ws_bytes,
                                    _stream(stream)), "sg_potential_direct")


def hsg(H, Q, out, stream=None):
    """sg_hsg on [F][n] float64 device tensors."""
    nf, n = H.shape
    _check(_lib.sg_hsg(n, nf, _ptr(H), _ptr(Q), _ptr(out), _stream(stream)), "sg_hsg")


def eval_G0(x, G, dtype, stream=None):
    _check(_lib.sg_eval_G0(_ptr(x), _ptr(G), x.numel(), dtype, _stream(stream)), "sg_eval_G0")


def field_adjoint(disc: Disc, lam_r, lam_phi, dsigma, dh, ws, ws_bytes=None, stream=None):
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_field_adjoint(ctypes.byref(disc), _ptr(lam_r), _ptr(lam_phi), _ptr(dsigma),
                                 _ptr(dh), _ptr(ws), ws_bytes, _stream(stream)),
           "sg_field_adjoint")


def ss_grad_H(disc: Disc, H, lam_r, lam_phi, dH, ws, ws_bytes=None, stream=None):
    ws_bytes = ws.numel() * ws.element_size() if ws_bytes is None else ws_bytes
    _check(_lib.sg_ss_grad_H(ctypes.byref(disc), _ptr(H), _ptr(lam_r), _ptr(lam_phi), _ptr(dH),
                             _ptr(ws), ws_bytes, _stream(stream)),
           "sg_ss_grad_H")


def eval_F(x, F, dF=None, dtype=F64, stream=None):
    _check(_lib.sg_eval_F(_ptr(x), _ptr(F), _ptr(dF), x.numel(), dtype, _stream(stream)),
           "sg_eval_F")


def self_cell(g: Grid, ha, hb, which, out, stream=None):
    n = len(ha)
    a = (ctypes.c_double * n)(*[float(v) for v in ha])
    b = (ctypes.c_double * n)(*[float(v) for v in hb])
    _check(_lib.sg_self_cell(ctypes.byref(g), a, b, n, which, _ptr(out), _stream(stream)),
           "sg_self_cell")


def field_fft_cache_entries() -> int:
    """Batch signatures whose plan (and graph, where used) sg_field_fft keeps cached."""
    return int(_lib.sg_field_fft_cache_entries())


def release():
    _lib.sg_release()
