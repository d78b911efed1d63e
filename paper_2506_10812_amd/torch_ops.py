"""PyTorch-facing helpers over the C ABI: device buffers from torch, the
current stream, and a torch.autograd.Function whose backward is the
library's hand-written adjoint.  All arithmetic happens in libsg.so."""
from __future__ import annotations

import torch

import ctypes

from . import (F32, F64, INDIRECT, SELF_CELL_EXCLUDE, SEMI_SPECTRAL, WITH_DH, Fluids, field_adjoint,
               field_adjoint_workspace_bytes, field_fft_tune, potential_direct,
               potential_direct_workspace_bytes, field_direct, field_direct_workspace_bytes, field_fft,
               field_fft_workspace_bytes, fluids, grid, kernel_table, kernel_table_bytes,
               kernel_table_workspace_bytes, make_disc, ss_table, ss_table_bytes,
               ss_table_workspace_bytes)


def _dev(device):
    return torch.device(device if device is not None else "cuda")


def build_table(g, f, flags=0, device=None):
    """Kernel table (uint8 device tensor) for grid g, fluids f."""
    dev = _dev(device)
    nb = kernel_table_bytes(g, f, flags)
    if nb == 0:
        raise ValueError("unsupported grid / fluids for the FFT path")
    table = torch.empty(nb, dtype=torch.uint8, device=dev)
    ws = torch.empty(kernel_table_workspace_bytes(g, f, flags), dtype=torch.uint8, device=dev)
    kernel_table(g, f, flags, table, ws)
    torch.cuda.current_stream(dev).synchronize()
    del ws
    return table


class FFTField:
    """A fixed batch of discs for sg_field_fft with persistent tables,
    workspace and outputs (so the cached graph keeps stable addresses)."""

    def __init__(self, specs, flags=0, device=None):
        """specs: dicts with n_r, n_phi, r_min, r_max, h (one aspect ratio per
        kernel group) and optionally species_group (kernel group of each
        species; Sigma then holds one density per species)."""
        dev = _dev(device)
        self.device = dev
        self.specs = []
        self.tables, self.sigma, self.g_r, self.g_phi = [], [], [], []
        self.discs = []
        for s in specs:
            g = grid(s["n_r"], s["n_phi"], s["r_min"], s["r_max"])
            f = fluids(s["h"])
            nf = len(s["h"])
            groups = s.get("species_group")
            shape = (nf, s["n_r"], s["n_phi"])
            tab = build_table(g, f, flags, dev)
            ns = len(groups) if groups is not None else nf
            sig = torch.zeros((ns, s["n_r"], s["n_phi"]), dtype=torch.float32, device=dev)
            gr = torch.empty(shape, dtype=torch.float32, device=dev)
            gp = torch.empty(shape, dtype=torch.float32, device=dev)
            self.tables.append(tab)
            self.sigma.append(sig)
            self.g_r.append(gr)
            self.g_phi.append(gp)
            self.discs.append(make_disc(g, f, flags, sig, gr, gp, tab, groups))
            self.specs.append((g, f))
        self.ws = torch.empty(max(1, field_fft_workspace_bytes(self.discs)), dtype=torch.uint8,
                              device=dev)

    def set_sigma(self, i, sigma):
        self.sigma[i].copy_(torch.as_tensor(sigma, dtype=torch.float32))

    def run(self, stream=None):
        field_fft(self.discs, self.ws, stream=stream)

    def tune(self, stream=None):
        """Autotunes this batch (sg_field_fft_tune); later runs use the choices."""
        return field_fft_tune(self.discs, self.ws, stream=stream)


class SemiSpectral:
    """One disc on the semi-spectral path (any H_f(r)): a persistent table,
    Sigma and outputs.  refresh(H) rebuilds the radial operators for new
    scale heights in place (the cached graph stays valid); run() solves."""

    def __init__(self, n_r, n_phi, r_min, r_max, n_fluids, flags=0, device=None, species_group=None):
        dev = _dev(device)
        self.device = dev
        self.g = grid(n_r, n_phi, r_min, r_max)
        self.nf = int(n_fluids)
        self.flags = int(flags) & ~SEMI_SPECTRAL
        nb = ss_table_bytes(self.g, self.nf, self.flags)
        if nb == 0:
            raise ValueError("unsupported grid for the semi-spectral path")
        self.table = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.tws = None
        shape = (self.nf, n_r, n_phi)
        ns = len(species_group) if species_group is not None else self.nf
        self.sigma = torch.zeros((ns, n_r, n_phi), dtype=torch.float32, device=dev)
        self.g_r = torch.empty(shape, dtype=torch.float32, device=dev)
        self.g_phi = torch.empty(shape, dtype=torch.float32, device=dev)
        # the fluid count only (up to four groups here; h is not read)
        fl = Fluids(self.nf, 0, (ctypes.c_double * 4)(0.0, 0.0, 0.0, 0.0))
        self.disc = make_disc(self.g, fl, self.flags | SEMI_SPECTRAL, self.sigma, self.g_r, self.g_phi,
                              self.table, species_group)
        self.ws = torch.empty(max(1, field_fft_workspace_bytes([self.disc])), dtype=torch.uint8,
                              device=dev)

    def refresh(self, H, stream=None):
        """H: [n_fluids][n_r] scale heights at the ring centres (any dtype)."""
        Hd = torch.as_tensor(H, dtype=torch.float64).to(self.device).contiguous()
        if self.tws is None:
            self.tws = torch.empty(ss_table_workspace_bytes(self.g, self.nf), dtype=torch.uint8,
                                   device=self.device)
        self._H = Hd
        ss_table(self.g, self.nf, Hd, self.flags, self.table, self.tws, stream=stream)

    def release_workspace(self):
        self.tws = None

    def run(self, stream=None):
        field_fft([self.disc], self.ws, stream=stream)


def direct(g, h, sigma, H=None, flags=0, stream=None):
    """sg_field_direct on torch tensors (float32 or float64, same dtype)."""
    dt = F64 if sigma.dtype == torch.float64 else F32
    nf = sigma.shape[0]
    gr = torch.empty_like(sigma)
    gp = torch.empty_like(sigma)
    ws = torch.empty(field_direct_workspace_bytes(g, nf, dt, H is not None), dtype=torch.uint8,
                     device=sigma.device)
    field_direct(g, nf, list(h) if h is not None else None, sigma, H, gr, gp, dt, flags, ws,
                 stream=stream)
    return gr, gp


def potential(g, h, sigma, H=None, flags=0, stream=None):
    """sg_potential_direct on torch tensors (float32 or float64)."""
    dt = F64 if sigma.dtype == torch.float64 else F32
    nf = sigma.shape[0]
    pot = torch.empty_like(sigma)
    ws = torch.empty(potential_direct_workspace_bytes(g, nf, dt, H is not None), dtype=torch.uint8,
                     device=sigma.device)
    potential_direct(g, nf, list(h) if h is not None else None, sigma, H, pot, dt, flags, ws, stream=stream)
    return pot


class _TableCache:
    def __init__(self):
        self.key = None
        self.table = None

    def get(self, g, hs, flags, device):
        key = (g.n_r, g.n_phi, g.r_min, g.r_max, tuple(hs), flags, str(device))
        if key != self.key:
            self.table = build_table(g, fluids(list(hs)), flags, device)
            self.key = key
        return self.table


_cache = _TableCache()


class SGField(torch.autograd.Function):
    """g_r, g_phi = SGField.apply(sigma, h, n_r, n_phi, r_min, r_max[, indirect]).

    sigma: float32 CUDA tensor [F][n_r][n_phi]; h: float64 tensor [F] of
    aspect ratios; indirect: add the indirect term.  Forward: sg_field_fft.
    Backward: sg_field_adjoint (dL/dSigma and dL/dh)."""

    @staticmethod
    def forward(ctx, sigma, h, n_r, n_phi, r_min, r_max, indirect=False):
        g = grid(n_r, n_phi, r_min, r_max)
        hs = [float(v) for v in h.detach().cpu().tolist()]
        flags = WITH_DH | (INDIRECT if indirect else 0)
        table = _cache.get(g, hs, flags, sigma.device)
        sigma_c = sigma.detach().contiguous().to(torch.float32)
        gr = torch.empty_like(sigma_c)
        gp = torch.empty_like(sigma_c)
        f = fluids(hs)
        disc = make_disc(g, f, flags, sigma_c, gr, gp, table)
        ws = torch.empty(field_fft_workspace_bytes([disc]), dtype=torch.uint8, device=sigma.device)
        field_fft([disc], ws)
        ctx.save_for_backward(sigma_c, table)
        ctx.meta = (g, hs, flags, h.device, h.dtype, sigma.dtype)
        return gr, gp

    @staticmethod
    def backward(ctx, lam_r, lam_phi):
        sigma_c, table = ctx.saved_tensors
        g, hs, flags, h_device, h_dtype, s_dtype = ctx.meta
        f = fluids(hs)
        lam_r = (lam_r if lam_r is not None else torch.zeros_like(sigma_c)).contiguous().float()
        lam_phi = (lam_phi if lam_phi is not None else torch.zeros_like(sigma_c)).contiguous().float()
        dsig = torch.empty_like(sigma_c)
        dh = torch.empty(len(hs), dtype=torch.float64, device=sigma_c.device)
        disc = make_disc(g, f, flags, sigma_c, lam_r, lam_phi, table)  # g_r/g_phi unused
        ws = torch.empty(field_adjoint_workspace_bytes(disc), dtype=torch.uint8,
                         device=sigma_c.device)
        field_adjoint(disc, lam_r, lam_phi, dsig, dh, ws)
        # gradients in the dtype (and, for h, the device) of the inputs
        return dsig.to(s_dtype), dh.to(device=h_device, dtype=h_dtype), None, None, None, None, None
