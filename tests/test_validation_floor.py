"""Continuum floor of the exponential-disc validation (Sect. 4.3), on the CPU.

Freeman's closed form is the field of a razor-thin disc; the exact kernel of
Sect. 2.2 describes Gaussian columns of height H = h r, so even in the
continuum limit the two differ by an amount that shrinks with h.  This test
measures that floor with an evaluation that has no discretisation error of
its own at the first order: for the axisymmetric disc the field is a 1-D
convolution in u = ln r of Sigma with the ring kernel R(X) = int K_r(X, phi)
dphi (the oracle's App. C kernel, integrated over phi by adaptive
quadrature), and the density is taken as its piecewise-linear interpolant on
the log grid, the ring kernel being integrated exactly against each hat
function within 16 cells of the target (point samples beyond, where the hat
average and the sample differ by (du^2/12) R'').  The error against Freeman
then converges with resolution to a floor close to h itself: the paper's
~1e-4 is therefore out of reach at h = 0.001 for this kernel (it is the
level its constant-H runs reach, where h = H/r is far smaller), and the
first-order error of the cell-centre sums on the GPU paths comes on top."""
import math
from functools import lru_cache

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

import oracle as O

R_MIN, R_MAX, R0, SIG0 = 0.01, 2500.0, 250.0, 200.0


def freeman(r):
    y = r / (2 * R0)
    return -2 * math.pi * SIG0 * y * (ss.i0e(y) * ss.k0e(y) - ss.i1e(y) * ss.k1e(y)), y


def ring_model_error(h, nr, M=16):
    @lru_cache(maxsize=None)
    def ring(X):
        f = lambda p: O.conv_kernels(np.array([X]), np.array([p]), h, h)[0][0]
        w = max(abs(X), 1e-12)
        pts = [p for p in (w, 10 * w, 100 * w) if p < math.pi]
        v, _ = si.quad(f, 0, math.pi, points=pts, limit=400, epsabs=0, epsrel=1e-11)
        return 2 * v

    du = math.log(R_MAX / R_MIN) / nr

    def hat(p):  # (1/du) int Lambda(X/du - p) R(X) dX
        if p == 0:  # the odd part cancels; the even part is log-singular at 0
            ev = lambda t: (1 - t) * 0.5 * (ring(du * t) + ring(-du * t))
            v, _ = si.quad(ev, 0, 1, limit=400, epsabs=0, epsrel=1e-10)
            return 2 * v
        g = lambda t: (1 - abs(t)) * ring(du * (p + t))
        v, _ = si.quad(g, -1, 1, points=[-p] if abs(p) <= 1 else None, limit=400, epsabs=0, epsrel=1e-10)
        return v

    r = np.exp(math.log(R_MIN) + (np.arange(nr) + 0.5) * du)
    sig = SIG0 * np.exp(-r / R0)
    R = np.array([hat(p) if abs(p) <= M else ring(p * du) for p in range(-(nr - 1), nr)])
    g = -du * np.convolve(sig, R, mode="full")[nr - 1:2 * nr - 1]
    ref, y = freeman(r)
    sel = (y >= 0.05) & (y <= 2.5)
    return float(np.median(np.abs(g[sel] - ref[sel]) / np.abs(ref[sel])))


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("h", [0.01, 0.001])
def test_bessel_kernel_continuum_floor_is_about_h(h):
    e1, e2 = ring_model_error(h, 128), ring_model_error(h, 256)
    # converged in resolution (the hat rule is second order) ...
    assert abs(e2 / e1 - 1) < 0.15, (e1, e2)
    # ... to a floor of the order of the aspect ratio (seen 1.0 h and 1.2 h)
    assert 0.7 * h < e2 < 1.5 * h, (h, e2)
