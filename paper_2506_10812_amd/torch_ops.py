"""PyTorch-facing helpers over the C ABI: device buffers from torch, the
current stream, and a torch.autograd.Function whose backward is the
library's hand-written adjoint.  All arithmetic happens in libsg.so."""
from __future__ import annotations

import torch

import ctypes

from . import (F32, F64, INDIRECT, SECOND_ORDER, SELF_CELL_EXCLUDE, SEMI_SPECTRAL, WITH_DH, Fluids, field_adjoint,
               field_adjoint_workspace_bytes, field_fft_tune, potential_direct,
               potential_direct_workspace_bytes, field_direct, field_direct_workspace_bytes, field_fft,
               field_fft_workspace_bytes, fluids, grid, kernel_table, kernel_table_bytes,
               kernel_table_workspace_bytes, make_disc, ss_grad_H, ss_grad_H_workspace_bytes, ss_table,
               ss_table_bytes, ss_table_workspace_bytes)


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
    workspace and outputs (so the cached plan keeps stable addresses)."""

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
    scale heights in place (the cached plan stays valid); run() solves."""

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


class _Slot:
    """Persistent device state of SGField for one (device, grid, aspect ratios,
    flags): kernel table, input and output buffers, workspaces.  The library
    sees the same buffers on every call, so sg_field_fft reuses one cached
    plan and nothing is allocated on the device after the first forward and
    backward (returned tensors come from torch's caching allocator)."""

    def __init__(self, g, hs, flags, device):
        nf = len(hs)
        shape = (nf, g.n_r, g.n_phi)
        self.g, self.hs, self.flags, self.device = g, hs, flags, device
        self.f = fluids(hs)
        self.table = build_table(g, self.f, flags, device)
        self.sigma = torch.empty(shape, dtype=torch.float32, device=device)
        self.g_r = torch.empty(shape, dtype=torch.float32, device=device)
        self.g_phi = torch.empty(shape, dtype=torch.float32, device=device)
        self.disc = make_disc(g, self.f, flags, self.sigma, self.g_r, self.g_phi, self.table)
        self.ws = torch.empty(max(1, field_fft_workspace_bytes([self.disc])), dtype=torch.uint8,
                              device=device)
        self.adj = None  # reverse-mode buffers, made by the first backward

    def forward(self, sigma):
        self.sigma.copy_(sigma)
        field_fft([self.disc], self.ws)
        return self.g_r.clone(), self.g_phi.clone()

    def backward(self, sigma, lam_r, lam_phi):
        if self.adj is None:
            a_sig = torch.empty_like(self.sigma)
            a_disc = make_disc(self.g, self.f, self.flags, a_sig, self.g_r, self.g_phi, self.table)
            self.adj = dict(
                sigma=a_sig, disc=a_disc,
                lam_r=torch.empty_like(self.sigma), lam_phi=torch.empty_like(self.sigma),
                dsig=torch.empty_like(self.sigma),
                dh=torch.empty(len(self.hs), dtype=torch.float64, device=self.device),
                ws=torch.empty(max(1, field_adjoint_workspace_bytes(a_disc)), dtype=torch.uint8,
                               device=self.device))
        A = self.adj
        A["sigma"].copy_(sigma)
        if lam_r is None:
            A["lam_r"].zero_()
        else:
            A["lam_r"].copy_(lam_r)
        if lam_phi is None:
            A["lam_phi"].zero_()
        else:
            A["lam_phi"].copy_(lam_phi)
        field_adjoint(A["disc"], A["lam_r"], A["lam_phi"], A["dsig"], A["dh"], A["ws"])
        return A["dsig"].clone(), A["dh"].clone()


class _SlotCache:
    """The most recently used SGField slots (at most `size`)."""

    def __init__(self, size=8):
        self.size = size
        self.slots = {}

    def get(self, g, hs, flags, device):
        key = (str(device), g.n_r, g.n_phi, g.r_min, g.r_max, tuple(hs), flags)
        slot = self.slots.pop(key, None)
        if slot is None:
            slot = _Slot(g, list(hs), flags, device)
            if len(self.slots) >= self.size:
                self.slots.pop(next(iter(self.slots)))
        self.slots[key] = slot  # most recent last
        return slot


_slots = _SlotCache()


class SGField(torch.autograd.Function):
    """g_r, g_phi = SGField.apply(sigma, h, n_r, n_phi, r_min, r_max[, indirect[, second_order]]).

    sigma: float32 CUDA tensor [F][n_r][n_phi]; h: float64 tensor [F] of
    aspect ratios; indirect: add the indirect term; second_order: the
    hat-weighted kernel table (SG_SECOND_ORDER).  Forward: sg_field_fft.
    Backward: sg_field_adjoint (dL/dSigma and dL/dh).  Repeated calls with the
    same grid, aspect ratios and flags reuse one persistent slot (table,
    buffers, workspaces) and therefore one cached plan."""

    @staticmethod
    def forward(ctx, sigma, h, n_r, n_phi, r_min, r_max, indirect=False, second_order=False):
        g = grid(n_r, n_phi, r_min, r_max)
        hs = [float(v) for v in h.detach().cpu().tolist()]
        flags = WITH_DH | (INDIRECT if indirect else 0) | (SECOND_ORDER if second_order else 0)
        slot = _slots.get(g, hs, flags, sigma.device)
        sig = sigma.detach()
        gr, gp = slot.forward(sig)
        ctx.save_for_backward(sig)
        ctx.meta = (slot, h.device, h.dtype, sigma.dtype)
        return gr, gp

    @staticmethod
    def backward(ctx, lam_r, lam_phi):
        (sig,) = ctx.saved_tensors
        slot, h_device, h_dtype, s_dtype = ctx.meta
        dsig, dh = slot.backward(sig, lam_r, lam_phi)
        # gradients in the dtype (and, for h, the device) of the inputs
        return dsig.to(s_dtype), dh.to(device=h_device, dtype=h_dtype), None, None, None, None, None, None


class _SSSlot:
    """Persistent device state of SGFieldSS for one (device, grid, fluid
    count, flags): the semi-spectral disc (table, Sigma, outputs), the H its
    table was built for, and the reverse-mode buffers.  The table is rebuilt
    only when H changes, so a fit that holds H fixed solves at plan speed."""

    def __init__(self, g, nf, flags, device):
        self.nf, self.device = nf, device
        self.S = SemiSpectral(g.n_r, g.n_phi, g.r_min, g.r_max, nf, flags, device)
        self.H = None
        self.adj = None

    def _ensure(self, H):
        if self.H is None or not torch.equal(self.H, H):
            self.S.refresh(H)
            self.H = H.clone()

    def forward(self, sigma, H):
        self._ensure(H)
        self.S.sigma.copy_(sigma)
        self.S.run()
        return self.S.g_r.clone(), self.S.g_phi.clone()

    def backward(self, sigma, H, lam_r, lam_phi, need_sigma, need_H):
        S = self.S
        self._ensure(H)
        if self.adj is None:
            self.adj = dict(
                lam_r=torch.empty_like(S.g_r), lam_phi=torch.empty_like(S.g_phi),
                dsig=torch.empty_like(S.g_r),
                dH=torch.empty((self.nf, S.g.n_r), dtype=torch.float64, device=self.device),
                ws=torch.empty(max(1, field_adjoint_workspace_bytes(S.disc),
                                   ss_grad_H_workspace_bytes(S.disc)),
                               dtype=torch.uint8, device=self.device))
        A = self.adj
        for name, lam in (("lam_r", lam_r), ("lam_phi", lam_phi)):
            if lam is None:
                A[name].zero_()
            else:
                A[name].copy_(lam)
        S.sigma.copy_(sigma)
        dsig = dH = None
        if need_sigma:
            field_adjoint(S.disc, A["lam_r"], A["lam_phi"], A["dsig"], None, A["ws"])
            dsig = A["dsig"].clone()
        if need_H:
            ss_grad_H(S.disc, self.H, A["lam_r"], A["lam_phi"], A["dH"], A["ws"])
            dH = A["dH"].clone()
        return dsig, dH


class _SSSlotCache(_SlotCache):
    def get(self, g, nf, flags, device):
        key = (str(device), g.n_r, g.n_phi, g.r_min, g.r_max, nf, flags)
        slot = self.slots.pop(key, None)
        if slot is None:
            slot = _SSSlot(g, nf, flags, device)
            if len(self.slots) >= self.size:
                self.slots.pop(next(iter(self.slots)))
        self.slots[key] = slot
        return slot


_ss_slots = _SSSlotCache(size=4)


class SGFieldSS(torch.autograd.Function):
    """g_r, g_phi = SGFieldSS.apply(sigma, H, n_r, n_phi, r_min, r_max[, indirect[, second_order]]).

    The semi-spectral solve for scale heights that vary with radius (Sect. 5.2):
    sigma: float32 CUDA tensor [F][n_r][n_phi]; H: tensor [F][n_r] of scale
    heights at the ring centres (any float dtype).  Forward: sg_ss_table
    (only when H changed since the last call on this slot) and sg_field_fft.
    Backward: sg_field_adjoint for dL/dSigma and sg_ss_grad_H for dL/dH(r),
    each run only when that input needs a gradient."""

    @staticmethod
    def forward(ctx, sigma, H, n_r, n_phi, r_min, r_max, indirect=False, second_order=False):
        g = grid(n_r, n_phi, r_min, r_max)
        nf = sigma.shape[0]
        if tuple(H.shape) != (nf, n_r):
            raise ValueError(f"H must have shape ({nf}, {n_r}), got {tuple(H.shape)}")
        flags = (INDIRECT if indirect else 0) | (SECOND_ORDER if second_order else 0)
        slot = _ss_slots.get(g, nf, flags, sigma.device)
        sig = sigma.detach()
        Hd = H.detach().to(device=sigma.device, dtype=torch.float64).contiguous()
        gr, gp = slot.forward(sig, Hd)
        ctx.save_for_backward(sig, Hd)
        ctx.meta = (slot, H.device, H.dtype, sigma.dtype)
        return gr, gp

    @staticmethod
    def backward(ctx, lam_r, lam_phi):
        sig, Hd = ctx.saved_tensors
        slot, H_device, H_dtype, s_dtype = ctx.meta
        dsig, dH = slot.backward(sig, Hd, lam_r, lam_phi, ctx.needs_input_grad[0],
                                 ctx.needs_input_grad[1])
        if dsig is not None:
            dsig = dsig.to(s_dtype)
        if dH is not None:
            dH = dH.to(device=H_device, dtype=H_dtype)
        return dsig, dH, None, None, None, None, None, None
