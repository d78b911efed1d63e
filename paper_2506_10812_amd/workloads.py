"""Seeded synthetic inputs (surface densities and grid parameters).

This module only builds inputs; it contains none of the self-gravity
arithmetic.  Cell-centre coordinates are computed here solely to shape the
surface-density profiles.  The same arrays are handed to the HIP library and
to the CPU oracle.

Workloads (the paper's own experiments use log-r x uniform-phi grids with
H/r constant for the FFT method, Sect. 4 and Sect. 5.2):
  direct_fp64   64 x 128, r in [0.2, 2.5], Sigma = r^-1 (1 + 0.01 U(-1,1)), h = 0.05
  single_fft    512 x 1024, r in [0.2, 5], Sigma = r^-1 (1 + 0.1 cos(2 phi - 4 ln r))
                (1 + 0.01 U(-1,1)), h = 0.05
  bifluid_fft   1024 x 2048, r in [0.2, 5], gas as single_fft (h_g = 0.05), dust
                h_d = 0.005, Sigma_d = 0.01 Sigma_g (1 + sum of 20 Gaussian clumps of
                amplitude 5 and width 2 cells at seeded index-space centres,
                periodic in phi)
  batch64       64 single-fluid discs, n_r in {128,...,1024}, n_phi in {256,...,2048}
                (uniform over powers of two), h ~ U(0.03, 0.1), r in [0.2, 5],
                Sigma = r^-p (1 + sum_{m=1..4} A_m cos(m phi - 4 ln r + psi_m)),
                p ~ U(0.5, 1.5), A_m ~ U(0, 0.2), psi_m ~ U(0, 2 pi)
  adjoint       256 x 512 two-fluid, h_g = 0.05, h_d = 0.01 (H_d = 0.2 H_g); target
                Sigma* with the bifluid_fft recipe (seed A), evaluation
                Sigma = Sigma* (1 + 0.1 U(-1,1)) (seed B)
  flaring       the App. D setup for the semi-spectral path: r in [20, 250] (AU),
                r_0 = 100, Sigma = (r/r_0)^-1.5 (1 + 0.1 cos(2 phi - 4 ln r))
                (1 + 0.01 U(-1,1)); gas H_g/r = 0.05 (r/r_0)^p (power-law flaring)
                times sqrt(1 - 0.95 exp(-((r - r_0)/w)^2)) when a temperature gap of
                width w is asked for; optional dust with H_d = eta H_g and the
                clumpy recipe of bifluid_fft (up to three dust groups, eta, 3 eta
                and eta/3, each with its own seeded clumps).  Default 1200 x 2048 (App. D uses
                1200 x 2800; the azimuthal transforms take powers of two).  With
                linear_r the radial grid is uniform (centres r_min + (i + 1/2) dr), as in
                the NIRVANA runs of the paper.
  exponential   the Sect. 4.3 validation disc: Sigma = Sigma_0 exp(-r/r_0), Sigma_0 = 200,
                r_0 = 250, r in [0.01, 2500] (AU), axisymmetric; H/r^q = h with q = 1
                (H = h r, the FFT path) or q = 0 (H = h constant, the semi-spectral
                path).  The paper uses 1200 x 2800.
"""
from __future__ import annotations

import numpy as np


def centres(n_r, n_phi, r_min, r_max):
    du = np.log(r_max / r_min) / n_r
    r = np.exp(np.log(r_min) + (np.arange(n_r) + 0.5) * du)
    phi = (np.arange(n_phi) + 0.5) * (2 * np.pi / n_phi)
    return r, phi


def _spiral_gas(n_r, n_phi, r_min, r_max, rng, noise=0.01, amp=0.1):
    r, phi = centres(n_r, n_phi, r_min, r_max)
    R, P = np.meshgrid(r, phi, indexing="ij")
    sig = (1.0 / R) * (1 + amp * np.cos(2 * P - 4 * np.log(R)))
    return sig * (1 + noise * rng.uniform(-1, 1, sig.shape))


def _clumpy_dust(gas, rng, n_clumps=20, amp=5.0, width=2.0):
    n_r, n_phi = gas.shape
    ci = rng.uniform(0, n_r, n_clumps)
    cj = rng.uniform(0, n_phi, n_clumps)
    I, J = np.meshgrid(np.arange(n_r), np.arange(n_phi), indexing="ij")
    bump = np.zeros_like(gas)
    for a, b in zip(ci, cj):
        dj = np.abs(J - b)
        dj = np.minimum(dj, n_phi - dj)
        bump += amp * np.exp(-((I - a) ** 2 + dj ** 2) / (2 * width * width))
    return 0.01 * gas * (1 + bump)


def direct_fp64(seed=1):
    rng = np.random.default_rng(seed)
    n_r, n_phi, r_min, r_max = 64, 128, 0.2, 2.5
    r, _ = centres(n_r, n_phi, r_min, r_max)
    sig = (1.0 / r)[:, None] * (1 + 0.01 * rng.uniform(-1, 1, (n_r, n_phi)))
    return dict(name="direct_fp64", n_r=n_r, n_phi=n_phi, r_min=r_min, r_max=r_max,
                h=[0.05], sigma=sig[None])


def single_fft(seed=2, n_r=512, n_phi=1024):
    rng = np.random.default_rng(seed)
    r_min, r_max = 0.2, 5.0
    sig = _spiral_gas(n_r, n_phi, r_min, r_max, rng)
    return dict(name="single_fft", n_r=n_r, n_phi=n_phi, r_min=r_min, r_max=r_max, h=[0.05],
                sigma=sig[None])


def bifluid_fft(seed=3, n_r=1024, n_phi=2048, h_g=0.05, eta=0.1):
    rng = np.random.default_rng(seed)
    r_min, r_max = 0.2, 5.0
    gas = _spiral_gas(n_r, n_phi, r_min, r_max, rng)
    dust = _clumpy_dust(gas, rng)
    return dict(name="bifluid_fft", n_r=n_r, n_phi=n_phi, r_min=r_min, r_max=r_max,
                h=[h_g, eta * h_g], sigma=np.stack([gas, dust]))


def batch64(seed=4, n_discs=64):
    rng = np.random.default_rng(seed)
    discs = []
    for _ in range(n_discs):
        n_r = int(rng.choice([128, 256, 512, 1024]))
        n_phi = int(rng.choice([256, 512, 1024, 2048]))
        h = float(rng.uniform(0.03, 0.1))
        p = float(rng.uniform(0.5, 1.5))
        A = rng.uniform(0, 0.2, 4)
        psi = rng.uniform(0, 2 * np.pi, 4)
        r, phi = centres(n_r, n_phi, 0.2, 5.0)
        R, P = np.meshgrid(r, phi, indexing="ij")
        sig = R ** (-p) * (1 + sum(A[m - 1] * np.cos(m * P - 4 * np.log(R) + psi[m - 1])
                                   for m in range(1, 5)))
        discs.append(dict(n_r=n_r, n_phi=n_phi, r_min=0.2, r_max=5.0, h=[h], sigma=sig[None]))
    return discs


def adjoint(seed_a=5, seed_b=6, n_r=256, n_phi=512):
    tgt = bifluid_fft(seed=seed_a, n_r=n_r, n_phi=n_phi, h_g=0.05, eta=0.2)
    rng = np.random.default_rng(seed_b)
    sig = tgt["sigma"] * (1 + 0.1 * rng.uniform(-1, 1, tgt["sigma"].shape))
    d = dict(tgt)
    d["name"] = "adjoint"
    d["sigma_target"] = tgt["sigma"]
    d["sigma"] = sig
    return d


def sample_cells(n_r, n_phi, n, seed=7):
    """Seeded flat cell indices (without replacement) for sampled comparisons."""
    rng = np.random.default_rng(seed)
    N = n_r * n_phi
    return np.sort(rng.choice(N, size=min(n, N), replace=False)).astype(np.int64)


def flaring(seed=8, n_r=1200, n_phi=2048, p=0.25, gap_w=None, n_fluids=1, eta=0.1, linear_r=False):
    """Per-ring scale heights H [n_fluids][n_r] and Sigma [n_fluids][n_r][n_phi]."""
    rng = np.random.default_rng(seed)
    r_min, r_max, r0 = 20.0, 250.0, 100.0
    r, phi = centres(n_r, n_phi, r_min, r_max)
    if linear_r:
        r = r_min + (np.arange(n_r) + 0.5) * (r_max - r_min) / n_r
    R, P = np.meshgrid(r, phi, indexing="ij")
    gas = (R / r0) ** -1.5 * (1 + 0.1 * np.cos(2 * P - 4 * np.log(R)))
    gas = gas * (1 + 0.01 * rng.uniform(-1, 1, gas.shape))
    h = 0.05 * (r / r0) ** p
    if gap_w is not None:
        h = h * np.sqrt(1 - 0.95 * np.exp(-((r - r0) / gap_w) ** 2))
    H = [h * r]
    sig = [gas]
    for f in range(1, n_fluids):  # dust groups: eta, 3 eta, eta / 3
        sig.append(_clumpy_dust(gas, rng))
        H.append(eta * (1.0, 3.0, 1.0 / 3.0)[f - 1] * h * r)
    return dict(name="flaring", n_r=n_r, n_phi=n_phi, r_min=r_min, r_max=r_max, p=p, gap_w=gap_w,
                linear_r=linear_r, H=np.stack(H), sigma=np.stack(sig))


def exponential(n_r=1024, n_phi=2048, h=0.001, q=1):
    """Axisymmetric exponential disc; H [1][n_r] per ring (h r^q)."""
    r_min, r_max, r0, sig0 = 0.01, 2500.0, 250.0, 200.0
    r, _ = centres(n_r, n_phi, r_min, r_max)
    sig = np.repeat((sig0 * np.exp(-r / r0))[:, None], n_phi, axis=1)
    return dict(name="exponential", n_r=n_r, n_phi=n_phi, r_min=r_min, r_max=r_max, r0=r0,
                sigma0=sig0, h=[h], q=q, H=(h * r ** q)[None, :], sigma=sig[None])
