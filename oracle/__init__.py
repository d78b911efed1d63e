"""CPU FP64 oracle for the exact thin-disc self-gravity kernel (arXiv 2506.10812).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything in this directory, and this module never imports the
product package.  The arithmetic lives in ``sg_oracle.c`` (plain C, double
precision, OpenMP over target cells); this file only marshals numpy arrays.

Array layout everywhere: ``[fluid][i_r][j_phi]`` with phi fastest, fluid 0 =
gas, 1 = dust.  Flags: bit 0 excludes the self-cell term; bit 1 selects a
uniform radial grid (centres r_min + (i + 1/2) dr, cell areas r_i dr dphi)
instead of the log-spaced one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EXCLUDE_SELF = 1
LINEAR_R = 2
SECOND_ORDER = 4  # table mode: hat-weighted (piecewise-bilinear source) offsets

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build() -> str:
    """Compile the oracle with gcc (portable x86-64 AVX2 code, OpenMP)."""
    cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-fopenmp", "-fPIC", "-shared",
           "-Wall", _SRC, "-o", _LIB, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        L.sg_oracle_F.restype = ctypes.c_double
        L.sg_oracle_F.argtypes = [ctypes.c_double]
        L.sg_oracle_dF.restype = ctypes.c_double
        L.sg_oracle_dF.argtypes = [ctypes.c_double]
        L.sg_oracle_D.restype = ctypes.c_double
        L.sg_oracle_D.argtypes = [ctypes.c_double]
        L.sg_oracle_kernel.restype = ctypes.c_double
        L.sg_oracle_kernel.argtypes = [ctypes.c_double] * 3
        L.sg_oracle_conv_kernels.restype = None
        L.sg_oracle_conv_kernels.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.sg_oracle_self_cell.restype = ctypes.c_double
        L.sg_oracle_self_cell.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int]
        L.sg_oracle_field_pairwise.restype = ctypes.c_int
        L.sg_oracle_field_pairwise.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            _dp, _dp, _dp, ctypes.c_int64, _i64p, ctypes.c_uint, _dp, _dp]
        L.sg_oracle_field_table.restype = ctypes.c_int
        L.sg_oracle_field_table.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            _dp, _dp, ctypes.c_int64, _i64p, ctypes.c_uint, ctypes.c_int, _dp]
        L.sg_oracle_adjoint_sigma.restype = ctypes.c_int
        L.sg_oracle_adjoint_sigma.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            _dp, _dp, ctypes.c_int64, _i64p, ctypes.c_uint, _dp]
        L.sg_oracle_G0.restype = ctypes.c_double
        L.sg_oracle_G0.argtypes = [ctypes.c_double]
        L.sg_oracle_potential_kernel.restype = ctypes.c_double
        L.sg_oracle_potential_kernel.argtypes = [ctypes.c_double] * 3
        L.sg_oracle_potential_self.restype = ctypes.c_double
        L.sg_oracle_potential_self.argtypes = [ctypes.c_double] * 5
        L.sg_oracle_potential_self_range.restype = ctypes.c_double
        L.sg_oracle_potential_self_range.argtypes = [ctypes.c_double] * 6
        L.sg_oracle_self_cell_range.restype = ctypes.c_double
        L.sg_oracle_self_cell_range.argtypes = [ctypes.c_double] * 5
        L.sg_oracle_potential_pairwise.restype = ctypes.c_int
        L.sg_oracle_potential_pairwise.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            _dp, _dp, _dp, ctypes.c_int64, _i64p, ctypes.c_uint, _dp]
        L.sg_oracle_point_fields.restype = ctypes.c_int
        L.sg_oracle_point_fields.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, _dp, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp]
        L.sg_oracle_hsg.restype = None
        L.sg_oracle_hsg.argtypes = [ctypes.c_int64, ctypes.c_int, _dp, _dp, _dp]
        L.sg_oracle_indirect.restype = ctypes.c_int
        L.sg_oracle_indirect.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
            _dp, _dp, _dp, ctypes.c_uint, _dp]
        L.sg_oracle_hat_weight.restype = None
        L.sg_oracle_hat_weight.argtypes = [ctypes.c_int, ctypes.c_int] + [ctypes.c_double] * 4 + [ctypes.c_int, _dp]
        L.sg_oracle_field_ring_hat.restype = ctypes.c_int
        L.sg_oracle_field_ring_hat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_int, _dp, _dp, ctypes.c_int64, _i64p, _dp]
        L.sg_oracle_threads.restype = ctypes.c_int
        L.sg_oracle_threads.argtypes = []
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _iptr(a):
    return None if a is None else a.ctypes.data_as(_i64p)


def threads() -> int:
    return int(lib().sg_oracle_threads())


def F(x):
    """e^x [K1(x) - K0(x)] (App. A), elementwise."""
    x = np.atleast_1d(_d(x))
    return np.array([lib().sg_oracle_F(float(v)) for v in x.ravel()]).reshape(x.shape)


def dF(x):
    x = np.atleast_1d(_d(x))
    return np.array([lib().sg_oracle_dF(float(v)) for v in x.ravel()]).reshape(x.shape)


def D(x):
    """-x F'(x) - 3/2 F(x), the factor of the kernel's h derivative, from its
    cancellation-free integral (elementwise)."""
    x = np.atleast_1d(_d(x))
    return np.array([lib().sg_oracle_D(float(v)) for v in x.ravel()]).reshape(x.shape)


def kernel(s, Ha, Hb):
    """K_ab(s; H_a, H_b), Eq. 'SG force kernel exact' (Sect. 2.2)."""
    s, Ha, Hb = np.broadcast_arrays(_d(s), _d(Ha), _d(Hb))
    out = np.empty(s.shape)
    for idx in np.ndindex(s.shape):
        out[idx] = lib().sg_oracle_kernel(float(s[idx]), float(Ha[idx]), float(Hb[idx]))
    return out


def conv_kernels(X, phi, ha, hb, which=0):
    """App. C convolution kernels (K_r, K_phi) at offsets (X, phi).

    which = 0: the kernels; 1: d/dh_a; 2: d/dh_b."""
    X, phi = np.broadcast_arrays(_d(X), _d(phi))
    X, phi = _d(X), _d(phi)
    kr = np.empty(X.shape)
    kp = np.empty(X.shape)
    lib().sg_oracle_conv_kernels(X.size, _ptr(X), _ptr(phi), float(ha), float(hb), int(which),
                                 _ptr(kr), _ptr(kp))
    return kr, kp


def self_cell(ha, hb, du, dphi, which=0):
    """Principal-value cell average of K_r over the own cell (self term)."""
    return float(lib().sg_oracle_self_cell(float(ha), float(hb), float(du), float(dphi),
                                           int(which)))


def _targets(targets):
    if targets is None:
        return None
    return np.ascontiguousarray(targets, dtype=np.int64)


def field_pairwise(nr, nphi, rmin, rmax, h, sigma, H=None, targets=None, flags=0):
    """Plain pairwise Cartesian sum.  Returns (g_r, g_phi), each [nf][n_targets]."""
    sigma = _d(sigma)
    nf = sigma.shape[0]
    h = _d(np.atleast_1d(h))
    Hd = None if H is None else _d(H)
    t = _targets(targets)
    nt = nr * nphi if t is None else t.size
    gr = np.empty((nf, nt))
    gp = np.empty((nf, nt))
    rc = lib().sg_oracle_field_pairwise(nr, nphi, rmin, rmax, nf, _ptr(h), _ptr(Hd),
                                        _ptr(sigma), nt, _iptr(t), flags, _ptr(gr), _ptr(gp))
    if rc:
        raise RuntimeError(f"sg_oracle_field_pairwise failed ({rc})")
    return gr, gp


def field_table_pairs(nr, nphi, rmin, rmax, h, sigma, targets=None, flags=0, which=0):
    """Offset-table (App. C) sum per ordered pair: array [a][b][c][n_targets]."""
    sigma = _d(sigma)
    nf = sigma.shape[0]
    h = _d(np.atleast_1d(h))
    t = _targets(targets)
    nt = nr * nphi if t is None else t.size
    out = np.empty((nf, nf, 2, nt))
    rc = lib().sg_oracle_field_table(nr, nphi, rmin, rmax, nf, _ptr(h), _ptr(sigma), nt,
                                     _iptr(t), flags, which, _ptr(out))
    if rc:
        raise RuntimeError(f"sg_oracle_field_table failed ({rc})")
    return out


def hat_weight(P, Q, du, dphi, ha, hb, which=0):
    """Second-order offset weights (W_r, W_phi) of offset (P, Q) in cells, or
    their derivatives in h_a (which = 1) or h_b (which = 2)."""
    W = np.empty(2)
    lib().sg_oracle_hat_weight(int(P), int(Q), du, dphi, ha, hb, int(which), _ptr(W))
    return float(W[0]), float(W[1])


def field_ring_hat(nr, nphi, rmin, rmax, H, sigma, targets=None):
    """Second-order field for scale heights H [nf][nr] at the ring centres
    (hat weights with each ring pair's aspect ratios): (g_r, g_phi), each
    [nf][n_t], summed over source fluids."""
    sigma = _d(sigma)
    nf = sigma.shape[0]
    H = _d(H).reshape(nf, nr)
    t = _targets(targets)
    nt = nr * nphi if t is None else t.size
    out = np.empty((nf, 2, nt))
    rc = lib().sg_oracle_field_ring_hat(nr, nphi, rmin, rmax, nf, _ptr(H), _ptr(sigma), nt, _iptr(t),
                                        _ptr(out))
    if rc:
        raise RuntimeError(f"sg_oracle_field_ring_hat failed ({rc})")
    return out[:, 0, :].copy(), out[:, 1, :].copy()


def field_table(nr, nphi, rmin, rmax, h, sigma, targets=None, flags=0):
    """Offset-table field summed over source fluids: (g_r, g_phi), each [nf][n_t]."""
    out = field_table_pairs(nr, nphi, rmin, rmax, h, sigma, targets, flags, 0)
    g = out.sum(axis=0)  # over source fluid a -> [b][c][nt]
    return g[:, 0, :].copy(), g[:, 1, :].copy()


def adjoint_sigma(nr, nphi, rmin, rmax, h, lam_r, lam_phi, kidx=None, flags=0):
    """dL/dSigma from lam = dL/dg (transposed offset-table sum): [nf][n_k]."""
    lam_r = _d(lam_r)
    lam_phi = _d(lam_phi)
    nf = lam_r.shape[0]
    N = nr * nphi
    lam = np.empty((nf, 2, N))
    lam[:, 0] = lam_r.reshape(nf, N)
    lam[:, 1] = lam_phi.reshape(nf, N)
    h = _d(np.atleast_1d(h))
    k = _targets(kidx)
    nk = N if k is None else k.size
    out = np.empty((nf, nk))
    rc = lib().sg_oracle_adjoint_sigma(nr, nphi, rmin, rmax, nf, _ptr(h), _ptr(lam), nk,
                                       _iptr(k), flags, _ptr(out))
    if rc:
        raise RuntimeError(f"sg_oracle_adjoint_sigma failed ({rc})")
    return out


def adjoint_h(nr, nphi, rmin, rmax, h, sigma, lam_r, lam_phi, flags=0):
    """dL/dh_f for each fluid f from lam = dL/dg, by differentiating every
    offset-table entry (including the self-cell term) with respect to h_a
    (source) and h_b (target) and summing lam . (dK (*) Sigma) per pair."""
    sigma = _d(sigma)
    nf = sigma.shape[0]
    N = nr * nphi
    lam = np.stack([_d(lam_r).reshape(nf, N), _d(lam_phi).reshape(nf, N)], axis=1)  # [b][c][N]
    dh = np.zeros(nf)
    for which, role in ((1, "a"), (2, "b")):
        out = field_table_pairs(nr, nphi, rmin, rmax, h, sigma, None, flags, which)
        for a in range(nf):
            for b in range(nf):
                v = float(np.sum(lam[b] * out[a, b]))
                dh[a if role == "a" else b] += v
    return dh


def G0(y):
    """e^y K0(y) (vectorised)."""
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    L = lib()
    return np.array([L.sg_oracle_G0(float(v)) for v in y.ravel()]).reshape(y.shape)


def potential_kernel(s, Ha, Hb):
    return np.array([lib().sg_oracle_potential_kernel(float(v), float(Ha), float(Hb))
                     for v in np.atleast_1d(s)])


def potential_self(r, Ha, Hb, du, dphi):
    return lib().sg_oracle_potential_self(float(r), float(Ha), float(Hb), float(du), float(dphi))


def potential_self_range(r, Ha, Hb, xlo, xhi, dphi):
    """Own-cell integral of P over X = ln(r'/r) in [xlo, xhi], |phi| <= dphi/2."""
    return lib().sg_oracle_potential_self_range(float(r), float(Ha), float(Hb), float(xlo), float(xhi),
                                                float(dphi))


def self_cell_range(ha, hb, xlo, xhi, dphi):
    """Own-cell integral I of K_r over X in [xlo, xhi], |phi| <= dphi/2 (the
    field's own-cell term is -Sigma I)."""
    return lib().sg_oracle_self_cell_range(float(ha), float(hb), float(xlo), float(xhi), float(dphi))


def potential_pairwise(nr, nphi, rmin, rmax, h, sigma, H=None, targets=None, flags=0):
    """Potential at cell centres per target fluid: array [nf][n_targets]."""
    sigma = _d(sigma)
    nf = sigma.shape[0]
    h = _d(np.atleast_1d(h))
    Hd = None if H is None else _d(H)
    t = _targets(targets)
    nt = nr * nphi if t is None else t.size
    pot = np.empty((nf, nt))
    rc = lib().sg_oracle_potential_pairwise(nr, nphi, rmin, rmax, nf, _ptr(h), _ptr(Hd), _ptr(sigma),
                                            nt, _iptr(t), flags, _ptr(pot))
    if rc:
        raise RuntimeError(f"sg_oracle_potential_pairwise failed ({rc})")
    return pot


def point_fields(nr, nphi, rmin, rmax, Ha, Hb, sigma, px, py):
    """(Phi, g_x, g_y) of one source fluid at arbitrary points, constant H."""
    sigma = _d(sigma)
    px = _d(px)
    py = _d(py)
    n = px.size
    pot, gx, gy = np.empty(n), np.empty(n), np.empty(n)
    rc = lib().sg_oracle_point_fields(nr, nphi, rmin, rmax, Ha, Hb, _ptr(sigma), n, _ptr(px), _ptr(py),
                                      _ptr(pot), _ptr(gx), _ptr(gy))
    if rc:
        raise RuntimeError(f"sg_oracle_point_fields failed ({rc})")
    return pot, gx, gy


def hsg(H, Q):
    """Self-gravitating scale heights from H [F][n] and Toomre parameters Q [F][n]."""
    H = _d(np.atleast_2d(H))
    Q = _d(np.atleast_2d(Q))
    out = np.empty_like(H)
    lib().sg_oracle_hsg(H.shape[1], H.shape[0], _ptr(H), _ptr(Q), _ptr(out))
    return out


def indirect(nr, nphi, rmin, rmax, h, sigma, H=None, flags=0):
    """Indirect-term sums (A_a, B_a) per source fluid: array [nf][2]."""
    sigma = _d(sigma)
    nf = sigma.shape[0]
    h = _d(np.atleast_1d(h))
    Hd = None if H is None else _d(H)
    AB = np.empty((nf, 2))
    rc = lib().sg_oracle_indirect(nr, nphi, rmin, rmax, nf, _ptr(h), _ptr(Hd), _ptr(sigma), flags,
                                  _ptr(AB))
    if rc:
        raise RuntimeError(f"sg_oracle_indirect failed ({rc})")
    return AB


def indirect_field(nr, nphi, AB):
    """Acceleration -sum_a grad Phi_{a,ind} (the same for every target fluid),
    from the per-fluid sums of `indirect`: (g_r, g_phi), each [nr * nphi]."""
    A, B = np.asarray(AB).sum(axis=0)
    phi = (np.arange(nphi) + 0.5) * (2 * np.pi / nphi)
    gr = -(A * np.cos(phi) + B * np.sin(phi))
    gp = -(-A * np.sin(phi) + B * np.cos(phi))
    return np.tile(gr, nr), np.tile(gp, nr)


def grid(nr, nphi, rmin, rmax, flags=0):
    """Cell centres (r_i, phi_j) and widths (du, dphi) of the oracle's grid
    (with LINEAR_R: (r_i, phi_j, dr, dphi))."""
    dphi = 2.0 * np.pi / nphi
    phi = (np.arange(nphi) + 0.5) * dphi
    if flags & LINEAR_R:
        dr = (rmax - rmin) / nr
        return rmin + (np.arange(nr) + 0.5) * dr, phi, dr, dphi
    du = np.log(rmax / rmin) / nr
    r = np.exp(np.log(rmin) + (np.arange(nr) + 0.5) * du)
    return r, phi, du, dphi
