"""Pins of the CPU FP64 oracle against facts fixed by the paper and by mathematics.

None of these re-types an oracle formula: each compares the oracle with an
independent route (arbitrary-precision Bessel functions, brute-force
quadrature of the vertical double integral, closed-form limits printed in the
paper, conservation laws, brute-force sub-cell sums, a continuum closed form).
"""
import json
import math
from fractions import Fraction
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
mp.mp.dps = 40


def _F_mp(x):
    x = mp.mpf(x)
    return mp.e ** x * (mp.besselk(1, x) - mp.besselk(0, x))


def _dF_mp(x):
    x = mp.mpf(x)
    return mp.e ** x * (2 * mp.besselk(1, x) - 2 * mp.besselk(0, x) - mp.besselk(1, x) / x)


# --------------------------------------------------------------------- F(x)
def test_F_matches_arbitrary_precision_bessel():
    """F(x) = e^x [K1 - K0](x) (App. A) vs 40-digit mpmath Bessel functions."""
    for x in np.logspace(-12, 4.6, 45):
        ref = float(_F_mp(x))
        assert abs(O.F(x)[0] - ref) <= 2e-15 * ref, x


def test_dF_matches_arbitrary_precision_bessel():
    """F'(x) = e^x [2K1 - 2K0 - K1/x] (derivative of App. A's F) vs mpmath."""
    for x in np.logspace(-12, 4.6, 45):
        ref = float(_dF_mp(x))
        assert abs(O.dF(x)[0] - ref) <= 2e-15 * abs(ref), x


def test_D_matches_arbitrary_precision_bessel():
    """D(x) = -x F'(x) - 3/2 F(x), the factor of the kernel's h derivative,
    from the oracle's one-signed integral vs the two-term form at 40 digits
    (where its cancellation at large x costs nothing).  At large x it is
    O(x^-5/2) against terms of O(x^-3/2): in double the two-term form would
    lose up to log10(x) digits there."""
    for x in np.logspace(-12, 4.6, 45):
        ref = float(-mp.mpf(x) * _dF_mp(x) - mp.mpf(1.5) * _F_mp(x))
        assert abs(O.D(x)[0] - ref) <= 4e-15 * abs(ref), (x, O.D(x)[0], ref)


# ------------------------------------------------------------------- kernel
@pytest.mark.parametrize("s,Ha,Hb", [(0.7, 1.0, 1.0), (2.0, 1.0, 0.4), (5.0, 0.3, 1.2),
                                     (0.35, 0.5, 0.2), (9.0, 1.0, 1.0)])
def test_kernel_equals_vertical_double_integral(s, Ha, Hb):
    """Closed form (Sect. 2.2, Eq. 'SG force kernel exact') vs brute-force
    quadrature of the double integral over z, z' (Eq. 'SG force kernel general')."""
    # substitute z = Hb u, z' = Ha v: K = s/(2 pi) int int e^{-(u^2+v^2)/2}
    #                                        / (s^2 + (Hb u - Ha v)^2)^{3/2} du dv
    f = lambda v, u: math.exp(-0.5 * (u * u + v * v)) / (s * s + (Hb * u - Ha * v) ** 2) ** 1.5
    val, err = si.dblquad(f, -10, 10, -10, 10, epsabs=0, epsrel=1e-12)
    ref = s / (2 * math.pi) * val
    assert abs(O.kernel(s, Ha, Hb) - ref) <= 1e-9 * ref


def test_kernel_short_range_limit():
    """Light-disc singularity (Sect. 3.4): K ~ 1/(sqrt(pi) H s) as d -> 0."""
    H = 0.05
    for d in (1e-3, 1e-4, 1e-5):
        s = d * H
        k = O.kernel(s, H, H)
        assert abs(k * math.sqrt(math.pi) * H * s - 1.0) < 3.0 * d * d * abs(math.log(d)) + 1e-13


def test_kernel_razor_thin_limit():
    """H -> 0 gives the flat-disc kernel 1/s^2 (Sect. 4, razor-thin test)."""
    for s in (0.1, 1.0, 3.0):
        for H in (1e-4, 1e-6):
            assert abs(O.kernel(s, H, H) * s * s - 1.0) < 4.0 * (H / s) ** 2 + 1e-14


def test_kernel_large_distance_paper_expansion():
    """The three-term expansion printed in Sect. 5.3 (overflow fix) for x > 50;
    its error must be the next term, 525/1024 x^-3 relative."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        g = json.load(fh)["large_x_expansion"]
    c = [float(Fraction(t)) for t in g["coefficients"]]
    H = 1.0
    for x in (50.0, 88.0, 300.0, 5000.0):
        d = math.sqrt(8 * x)
        s = d * H
        series = (1 / (2 * math.sqrt(2))) * H ** -2 / d * (c[0] * x ** -0.5 + c[1] * x ** -1.5
                                                          + c[2] * x ** -2.5)
        k = O.kernel(s, H, H)
        rel = (series - k) / k
        nxt = 525.0 / 1024.0 / x ** 3
        assert abs(rel - nxt) < 0.05 * nxt + 1e-15, (x, rel, nxt)


def test_kernel_planet_special_case():
    """Planet as a fluid with zero thickness (Sect. 4): with H_a = 0 the kernel
    reproduces the printed planet-disc force, with c^2 = s^2/(4 H_g^2)."""
    Hg = 0.07
    for s in (0.01, 0.05, 0.2, 1.0):
        c2 = s * s / (4 * Hg * Hg)
        paper = (1 / s) * math.sqrt(2 / math.pi) / Hg * c2 * float(_F_mp(c2))
        assert abs(O.kernel(s, 0.0, Hg) - paper) < 1e-13 * paper


def test_kernel_dust_ratios():
    """Dust kernels (Sect. 3.3): K_dd/K_gg -> 1/eta and K_dg/K_gg -> sqrt(2/(1+eta^2))
    (-> sqrt 2) at d_g << eta; both -> 1 at large distance."""
    Hg = 1.0
    for eta in (0.3, 0.1, 0.01):
        s = 1e-4 * eta
        kgg = O.kernel(s, Hg, Hg)
        kdd = O.kernel(s, eta * Hg, eta * Hg)
        kdg = O.kernel(s, eta * Hg, Hg)
        assert abs(kdd / kgg * eta - 1) < 2e-3
        assert abs(kdg / kgg - math.sqrt(2 / (1 + eta * eta))) < 2e-3
        s = 300.0
        assert abs(O.kernel(s, eta, eta) / O.kernel(s, 1, 1) - 1) < 1e-4
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        lim = json.load(fh)["dust_gas_short_range_limit"]
    assert abs(O.kernel(1e-9, 1e-5, 1.0) / O.kernel(1e-9, 1.0, 1.0) - float(lim["value"])) < 1e-6


def test_kernel_symmetric_in_fluids():
    """Newton's third law between two columns (Sect. 2.2): K_ab = K_ba."""
    for s, a, b in ((0.3, 0.05, 0.01), (2.0, 0.2, 0.9)):
        assert O.kernel(s, a, b) == pytest.approx(O.kernel(s, b, a), rel=1e-15)


def test_conv_kernels_equal_cartesian_projection():
    """App. C convolution kernels vs the Cartesian kernel times the projection of
    e_s on e_r, e_phi and the source area factor r'^2 (pure geometry)."""
    rng = np.random.default_rng(5)
    ha, hb = 0.05, 0.005
    u = rng.uniform(-2, 2, 300)
    up = rng.uniform(-2, 2, 300)
    ph = rng.uniform(-np.pi, np.pi, 300)
    kr, kp = O.conv_kernels(u - up, ph, ha, hb)
    r, rp = np.exp(u), np.exp(up)
    xt = np.stack([r, np.zeros_like(r)])
    xs = np.stack([rp * np.cos(-ph), rp * np.sin(-ph)])
    dv = xt - xs
    s = np.hypot(dv[0], dv[1])
    K = O.kernel(s, ha * rp, hb * r)
    refr = K * dv[0] / s * rp ** 2
    refp = K * dv[1] / s * rp ** 2
    np.testing.assert_allclose(kr, refr, rtol=1e-10, atol=1e-12 * np.abs(refr).max())
    np.testing.assert_allclose(kp, refp, rtol=1e-10, atol=1e-12 * np.abs(refp).max())


def test_conv_kernel_h_derivatives_match_central_differences():
    """d/dh_a and d/dh_b of the App. C kernels vs central differences."""
    X = np.array([0.02, -0.3, 0.7, 1e-3])
    phi = np.array([0.01, 0.4, -1.0, 2e-3])
    ha, hb, e = 0.05, 0.01, 1e-6
    for which, (da, db) in ((1, (e, 0)), (2, (0, e))):
        d_r, d_p = O.conv_kernels(X, phi, ha, hb, which)
        p_r, p_p = O.conv_kernels(X, phi, ha + da, hb + db)
        m_r, m_p = O.conv_kernels(X, phi, ha - da, hb - db)
        np.testing.assert_allclose(d_r, (p_r - m_r) / (2 * e), rtol=1e-6)
        np.testing.assert_allclose(d_p, (p_p - m_p) / (2 * e), rtol=1e-6)


# ---------------------------------------------------------------- self cell
def _self_cell_bruteforce(ha, hb, du, dphi, n):
    """Midpoint rule on an n x n grid of the X-symmetrised quarter cell."""
    a, b = du / 2, dphi / 2
    X = (np.arange(n) + 0.5) * a / n
    P = (np.arange(n) + 0.5) * b / n
    XX, PP = np.meshgrid(X, P, indexing="ij")
    k1, _ = O.conv_kernels(XX.ravel(), PP.ravel(), ha, hb)
    k2, _ = O.conv_kernels(-XX.ravel(), PP.ravel(), ha, hb)
    return float(np.mean(0.5 * (k1 + k2)))


@pytest.mark.parametrize("ha,hb,du,dphi", [(0.05, 0.05, 0.0395, 0.0491),
                                            (0.05, 0.005, 0.00314, 0.00307),
                                            (0.01, 0.05, 0.02, 0.005)])
def test_self_cell_bruteforce(ha, hb, du, dphi):
    """Self-cell average (reading: PV cell average of K_r) vs brute-force
    midpoint sums, Richardson-extrapolated in the sub-cell count."""
    n1, n2 = 400, 800
    v1 = _self_cell_bruteforce(ha, hb, du, dphi, n1)
    v2 = _self_cell_bruteforce(ha, hb, du, dphi, n2)
    extrap = (4 * v2 - v1) / 3
    v = O.self_cell(ha, hb, du, dphi)
    assert abs(v - extrap) < 2e-5 * abs(v), (v, v1, v2, extrap)


@pytest.mark.parametrize("ha,hb,du,dphi", [(0.05, 0.05, 1e-6, 1e-6), (0.05, 0.005, 1e-7, 3e-7),
                                            (0.01, 0.04, 4e-7, 1e-7)])
def test_self_cell_small_cell_limit(ha, hb, du, dphi):
    """Closed form of the limit of tiny cells: with h0^2 = (h_a^2+h_b^2)/2 and
    c = (h_b^2-h_a^2)/(4 h0^2), Kbar -> (1/(sqrt(pi) h0)) [1/2 - (3/2+c) <cos^2>]
    where <cos^2> is the area mean of X^2/(X^2+phi^2) over the cell."""
    a, b = du / 2, dphi / 2
    cos2 = 0.5 + (a * a * math.atan(b / a) - b * b * math.atan(a / b)) / (2 * a * b)
    h0 = math.sqrt(0.5 * (ha * ha + hb * hb))
    c = (hb * hb - ha * ha) / (4 * h0 * h0)
    lim = (0.5 - (1.5 + c) * cos2) / (math.sqrt(math.pi) * h0)
    v = O.self_cell(ha, hb, du, dphi)
    assert abs(v - lim) < 1e-3 * abs(lim), (v, lim)


def _kr_scipy(X, phi, ha, hb):
    """K_r of the log-polar form rebuilt from the Cartesian geometry (target
    at r = 1, source at r' = e^-X, azimuth difference phi) with scipy's
    scaled Bessel functions for F(x) = e^x [K1(x) - K0(x)].  h may be
    complex (complex-step derivatives); nothing here calls the oracle."""
    rp = math.exp(-X)
    sx, sp = math.sinh(0.5 * X), math.sin(0.5 * phi)
    s2 = 2.0 * rp * (2.0 * sx * sx + 2.0 * sp * sp)  # |x - x'|^2 = 2 r r' (cosh X - cos phi)
    Hab2 = 0.5 * ((ha * rp) ** 2 + hb * hb)
    x = s2 / (8.0 * Hab2)
    F = ss.kve(1, x) - ss.kve(0, x)
    d = np.sqrt(s2 / Hab2)
    K = F * (d / 8.0) / (math.sqrt(math.pi) * Hab2)
    proj = rp * (math.expm1(X) + 2.0 * sp * sp) / math.sqrt(s2)  # e_s . e_r
    return K * proj * rp * rp  # times the source measure r'^2


def _self_cell_adaptive(ha, hb, du, dphi, part=lambda v: v):
    """Cell average of the X-symmetrised K_r by scipy's adaptive (QUADPACK)
    quadrature in polar coordinates about the cell centre, each quarter-cell
    triangle on its own (the symmetrised integrand is bounded)."""
    a, b = du / 2, dphi / 2
    f = lambda X, p: part(0.5 * (_kr_scipy(X, p, ha, hb) + _kr_scipy(-X, p, ha, hb)))
    th_c = math.atan2(b, a)
    tot = 0.0
    for th0, th1, edge in ((0.0, th_c, "a"), (th_c, math.pi / 2, "b")):
        def inner(th):
            c, s_ = math.cos(th), math.sin(th)
            rmax = a / c if edge == "a" else b / s_
            v, _ = si.quad(lambda rho: rho * f(rho * c, rho * s_), 0, rmax, epsabs=0,
                           epsrel=1e-13, limit=400)
            return v
        v, _ = si.quad(inner, th0, th1, epsabs=0, epsrel=1e-12, limit=400)
        tot += v
    return tot / (a * b)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("ha,hb,du,dphi", [
    (0.05, 0.05, math.log(2.5 / 0.2) / 64, 2 * math.pi / 128),   # 64 x 128 disc
    (0.05, 0.05, math.log(25.0) / 1024, 2 * math.pi / 2048),     # 1024 x 2048: gas-gas
    (0.005, 0.005, math.log(25.0) / 1024, 2 * math.pi / 2048),   # dust-dust
    (0.05, 0.005, math.log(25.0) / 1024, 2 * math.pi / 2048),    # gas source, dust target
    (0.005, 0.05, math.log(25.0) / 1024, 2 * math.pi / 2048),    # dust source, gas target
    (0.01, 0.01, 0.2, 0.3),                                       # cell much larger than h
    (0.03, 0.1, 0.05, 0.01)])
def test_self_cell_independent_adaptive_quadrature(ha, hb, du, dphi):
    """The own-cell average (reading: principal-value cell average of K_r) and
    its h_a, h_b derivatives against an independent evaluation: the kernel
    rebuilt from the Cartesian geometry with scipy's Bessel functions,
    integrated by adaptive quadrature; derivatives by the complex step
    (exact to rounding).  Bar 1e-10 relative (seen <= 7e-13)."""
    ref = _self_cell_adaptive(ha, hb, du, dphi)
    got = O.self_cell(ha, hb, du, dphi)
    assert abs(got / ref - 1) < 1e-10, (got, ref)
    e = 1e-30
    for which, (za, zb) in ((1, (ha + 1j * e, hb)), (2, (ha, hb + 1j * e))):
        dref = _self_cell_adaptive(za, zb, du, dphi, part=lambda v: v.imag / e)
        dgot = O.self_cell(ha, hb, du, dphi, which)
        assert abs(dgot / dref - 1) < 1e-10, (which, dgot, dref)


def _kphi_scipy(X, phi, ha, hb):
    """K_phi companion of _kr_scipy: the same Cartesian geometry projected on
    the target's e_phi (the source sits at azimuth -phi)."""
    rp = math.exp(-X)
    sx, sp = math.sinh(0.5 * X), math.sin(0.5 * phi)
    s2 = 2.0 * rp * (2.0 * sx * sx + 2.0 * sp * sp)
    Hab2 = 0.5 * ((ha * rp) ** 2 + hb * hb)
    x = s2 / (8.0 * Hab2)
    F = ss.kve(1, x) - ss.kve(0, x)
    d = np.sqrt(s2 / Hab2)
    K = F * (d / 8.0) / (math.sqrt(math.pi) * Hab2)
    return K * (rp * math.sin(phi) / math.sqrt(s2)) * rp * rp


def _hat_scipy(P, Q, du, dphi, ha, hb):
    """Second-order weights (W_r, W_phi) of offset (P, Q) by scipy's adaptive
    quadrature of Lambda(s) Lambda(t) K((P + s) du, (Q + t) dphi) over the
    four unit squares of the support.  A square with the kernel's singular
    point (-P, -Q) as a corner: iterated quad in polar coordinates about the
    corner, the hats taken from the corner (1 - x where the corner is at
    s = 0, x where it is at s = +-1); any other square: dblquad.  Nothing
    here calls the oracle."""
    tot = [0.0, 0.0]
    for s0 in (-1, 0):
        for t0 in (-1, 0):
            corner = (-P in (s0, s0 + 1)) and (-Q in (t0, t0 + 1))
            for comp, kf in enumerate((_kr_scipy, _kphi_scipy)):
                if corner:
                    sx = 1 if -P == s0 else -1
                    sy = 1 if -Q == t0 else -1

                    def inner(th):
                        c, sn = math.cos(th), math.sin(th)

                        def f(rho):
                            x, y = rho * c, rho * sn
                            w = (1 - x if P == 0 else x) * (1 - y if Q == 0 else y)
                            return rho * w * kf(sx * x * du, sy * y * dphi, ha, hb)
                        return si.quad(f, 0, 1 / max(c, sn), epsabs=0, epsrel=1e-13, limit=400)[0]
                    v = sum(si.quad(inner, a, b, epsabs=0, epsrel=1e-12, limit=400)[0]
                            for a, b in ((0, math.pi / 4), (math.pi / 4, math.pi / 2)))
                else:
                    def g(t, s):
                        return (1 - abs(s)) * (1 - abs(t)) * kf((P + s) * du, (Q + t) * dphi, ha, hb)
                    v = si.dblquad(g, s0, s0 + 1, t0, t0 + 1, epsabs=0, epsrel=1e-12)[0]
                tot[comp] += v
    return tot


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
@pytest.mark.parametrize("du,dphi,h", [
    (math.log(25.0) / 256, 2 * math.pi / 512, 0.05),    # 256 x 512 disc, gas
    (0.05, 2 * math.pi / 128, 1e-3),                     # cells much larger than H
    (0.02, 2 * math.pi / 64, 1e-4)])                     # elongated cells, nearly razor-thin
def test_hat_weights_independent_scipy_quadrature(du, dphi, h):
    """The second-order offset weights (reading: bilinear interpolant of the
    cell values integrated exactly against the App. C kernels) against an
    independent evaluation (scipy kernel and QUADPACK), for the nine
    offsets next to the singular point and a few regular ones.  Bar 1e-10
    relative to the entry's larger component."""
    for P, Q in ((0, 0), (1, 0), (0, -1), (1, 1), (-1, 1), (2, -1), (5, 3)):
        ref = _hat_scipy(P, Q, du, dphi, h, h)
        got = O.hat_weight(P, Q, du, dphi, h, h)
        sc = max(abs(ref[0]), abs(ref[1]))
        for c in range(2):
            assert abs(got[c] - ref[c]) < 1e-10 * sc, (P, Q, c, got, ref)


def test_hat_weights_far_field_expansion():
    """Far from the singular point the weight is the kernel plus the second
    moments of the hats: W = K + (du^2 K_XX + dphi^2 K_phiphi)/12 + O(cell^4)
    (int Lambda(s) s^2 ds = 1/6).  Checked on the correction W - K, which must
    match to 5% at 10-16 cells (the next term is ~(cell/distance)^2 smaller,
    seen up to 2.4%); derivatives by central differences of the kernel."""
    du, dphi, h = 0.02, 0.025, 0.01
    for P, Q in ((12, 3), (-10, 9), (4, -15), (16, 0)):
        X, ph = P * du, Q * dphi
        e1, e2 = 0.05 * du, 0.05 * dphi
        pts = [(X, ph), (X + e1, ph), (X - e1, ph), (X, ph + e2), (X, ph - e2)]
        kr, kp = O.conv_kernels(np.array([p[0] for p in pts]), np.array([p[1] for p in pts]), h, h)
        W = O.hat_weight(P, Q, du, dphi, h, h)
        for c, k in enumerate((kr, kp)):
            kxx = (k[1] - 2 * k[0] + k[2]) / e1 ** 2
            kpp = (k[3] - 2 * k[0] + k[4]) / e2 ** 2
            corr = (du * du * kxx + dphi * dphi * kpp) / 12.0
            if Q == 0 and c == 1:  # K_phi odd in phi: the weight vanishes too
                assert abs(W[1]) <= 1e-12 * abs(W[0]), (P, W)
                continue
            assert abs((W[c] - k[0]) / corr - 1) < 0.05, (P, Q, c, W[c] - k[0], corr)


@pytest.mark.parametrize("du,dphi,ha,hb", [(0.05, 2 * math.pi / 128, 1e-3, 2e-3),
                                           (math.log(25.0) / 256, 2 * math.pi / 512, 0.05, 0.005)])
def test_hat_weight_h_derivatives_match_central_differences(du, dphi, ha, hb):
    """d/dh_a and d/dh_b of the second-order weights (the kernel's h
    derivatives integrated with the same quadrature) against central
    differences of the weights themselves with Richardson extrapolation
    (steps 1e-3 h and 2e-3 h: the plain differences converge as step^2,
    1e-6 of the entry at 1e-3 h for the own cell); bar 1e-7 of the entry's
    larger component."""
    def cd(P, Q, which, e):
        hp = (ha + e, hb) if which == 1 else (ha, hb + e)
        hm = (ha - e, hb) if which == 1 else (ha, hb - e)
        wp = O.hat_weight(P, Q, du, dphi, *hp)
        wm = O.hat_weight(P, Q, du, dphi, *hm)
        return [(a - b) / (2 * e) for a, b in zip(wp, wm)]

    for P, Q in ((0, 0), (1, 0), (0, -1), (1, 1), (3, 2), (10, -7)):
        for which in (1, 2):
            e = 1e-3 * (ha if which == 1 else hb)
            d1, d2 = cd(P, Q, which, e), cd(P, Q, which, 2 * e)
            fd = [(4 * a - b) / 3 for a, b in zip(d1, d2)]
            got = O.hat_weight(P, Q, du, dphi, ha, hb, which)
            sc = max(abs(fd[0]), abs(fd[1]))
            for c in range(2):
                assert abs(got[c] - fd[c]) < 1e-7 * sc, (P, Q, which, c, got, fd)


def test_ring_hat_sum_equals_table_mode_for_constant_aspect_ratio():
    """The second-order sum with per-ring scale heights (ring-pair weights)
    reduces to the offset-table sum with hat weights when H = h r: every
    ring pair then has the same aspect ratios.  Two fluids, 5 x 8 (1e-13 of
    max|g|)."""
    nr, nphi, rmin, rmax = 5, 8, 0.5, 2.0
    rng = np.random.default_rng(0)
    sig = rng.uniform(0.5, 1.5, (2, nr, nphi))
    h = [0.05, 0.01]
    r = np.exp(np.log(rmin) + (np.arange(nr) + 0.5) * np.log(rmax / rmin) / nr)
    a = O.field_ring_hat(nr, nphi, rmin, rmax, np.stack([h[0] * r, h[1] * r]), sig)
    b = O.field_table(nr, nphi, rmin, rmax, h, sig, flags=O.SECOND_ORDER)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-13 * np.abs(y).max()


def _smooth_density(nr, nphi, urange, sig=0.7, kap=1.0):
    du = urange / nr
    u = (np.arange(nr) + 0.5) * du
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    return (np.exp(-(u - 0.5 * urange) ** 2 / (2 * sig ** 2))[:, None] *
            np.exp(kap * np.cos(phi - 1.0))[None, :])[None]


def test_hat_table_converges_at_second_order():
    """Self-convergence of the field of a smooth density (Gaussian in ln r,
    von Mises in phi, negligible at the radial edges) on a nearly razor-thin
    disc (h = 1e-4), under refinement by 3 in both directions, compared at
    the coarse cell centres (which are also centres of the finer grids).
    Point-sampled table: error ratio near 3 (first order); hat-weighted
    table: near 9 (second order), with a smaller error on each grid."""
    urange, h = 1.5 * math.pi, 1e-4
    res = {}
    for flags in (0, O.SECOND_ORDER):
        outs = []
        for f in (1, 3, 9):
            nr, nphi = 6 * f, 8 * f
            c = (f - 1) // 2
            I, J = np.meshgrid(np.arange(6) * f + c, np.arange(8) * f + c, indexing="ij")
            gr, gp = O.field_table(nr, nphi, 1.0, math.exp(urange), [h], _smooth_density(nr, nphi, urange),
                                   targets=(I * nphi + J).ravel(), flags=flags)
            outs.append(np.concatenate([gr[0], gp[0]]))
        e1 = np.linalg.norm(outs[0] - outs[1])
        e2 = np.linalg.norm(outs[1] - outs[2])
        res[flags] = (e1, e2)
    r0 = res[0][0] / res[0][1]
    r2 = res[O.SECOND_ORDER][0] / res[O.SECOND_ORDER][1]
    assert 2.4 < r0 < 3.6, res
    assert 7.5 < r2 < 11.0, res
    assert res[O.SECOND_ORDER][1] < 0.3 * res[0][1], res


def test_self_cell_h_derivatives_match_central_differences():
    du, dphi = 0.006, 0.006
    ha, hb, e = 0.05, 0.01, 1e-6
    for which, (da, db) in ((1, (e, 0)), (2, (0, e))):
        d = O.self_cell(ha, hb, du, dphi, which)
        fd = (O.self_cell(ha + da, hb + db, du, dphi) - O.self_cell(ha - da, hb - db, du, dphi)) / (2 * e)
        assert abs(d - fd) < 1e-6 * abs(fd)


# -------------------------------------------------------------- field sums
def _cart(nr, nphi, rmin, rmax, gr, gp):
    r, phi, du, dphi = O.grid(nr, nphi, rmin, rmax)
    P = np.broadcast_to(phi[None, :], (nr, nphi)).ravel()
    gx = gr * np.cos(P) - gp * np.sin(P)
    gy = gr * np.sin(P) + gp * np.cos(P)
    return gx, gy


def test_newton_third_law_general_H():
    """Pairwise symmetry of K (Sect. 2.2) gives zero net force on the whole
    disc when the self term is excluded, for any per-cell scale heights."""
    rng = np.random.default_rng(11)
    nr, nphi, rmin, rmax = 9, 14, 0.3, 2.0
    r, phi, du, dphi = O.grid(nr, nphi, rmin, rmax)
    sig = rng.uniform(0.2, 2.0, (2, nr, nphi))
    H = rng.uniform(0.01, 0.2, (2, nr, nphi))
    gr, gp = O.field_pairwise(nr, nphi, rmin, rmax, [0, 0], sig, H=H, flags=O.EXCLUDE_SELF)
    A = (r ** 2 * du * dphi)[:, None] * np.ones((nr, nphi))
    tot = np.zeros(2)
    scale = 0.0
    for b in range(2):
        gx, gy = _cart(nr, nphi, rmin, rmax, gr[b], gp[b])
        m = (sig[b] * A).ravel()
        tot += [np.sum(m * gx), np.sum(m * gy)]
        scale += np.sum(m * np.hypot(gx, gy))
    assert np.all(np.abs(tot) < 1e-13 * scale)


def test_axisymmetric_disc_has_no_azimuthal_field():
    nr, nphi, rmin, rmax = 12, 16, 0.2, 2.5
    r, phi, du, dphi = O.grid(nr, nphi, rmin, rmax)
    sig = np.stack([np.repeat((1 / r)[:, None], nphi, 1), np.repeat((0.01 * r)[:, None], nphi, 1)])
    for gr, gp in (O.field_pairwise(nr, nphi, rmin, rmax, [0.05, 0.01], sig),
                   O.field_table(nr, nphi, rmin, rmax, [0.05, 0.01], sig)):
        assert np.abs(gp).max() < 1e-13 * np.abs(gr).max()
        # and every ring is uniform
        g = gr.reshape(2, nr, nphi)
        assert np.abs(g - g[:, :, :1]).max() < 1e-13 * np.abs(g).max()


def test_phi_shift_equivariance_and_linearity():
    rng = np.random.default_rng(3)
    nr, nphi, rmin, rmax = 8, 12, 0.4, 3.0
    s1 = rng.uniform(0, 1, (2, nr, nphi))
    s2 = rng.uniform(0, 1, (2, nr, nphi))
    h = [0.08, 0.02]
    g1 = np.array(O.field_table(nr, nphi, rmin, rmax, h, s1))
    g2 = np.array(O.field_table(nr, nphi, rmin, rmax, h, s2))
    g12 = np.array(O.field_table(nr, nphi, rmin, rmax, h, 2 * s1 - 0.5 * s2))
    np.testing.assert_allclose(g12, 2 * g1 - 0.5 * g2, rtol=0, atol=1e-13 * np.abs(g1).max())
    gs = np.array(O.field_table(nr, nphi, rmin, rmax, h, np.roll(s1, 5, axis=2)))
    np.testing.assert_allclose(gs.reshape(2, 2, nr, nphi), np.roll(g1.reshape(2, 2, nr, nphi), 5, axis=3),
                               rtol=0, atol=1e-13 * np.abs(g1).max())


def test_table_mode_equals_pairwise_sum():
    """App. C convolution sum == plain pairwise Cartesian sum, bi-fluid,
    including the self term."""
    rng = np.random.default_rng(7)
    nr, nphi, rmin, rmax = 10, 16, 0.3, 2.0
    sig = rng.uniform(0.5, 1.5, (2, nr, nphi))
    h = [0.1, 0.03]
    gr, gp = O.field_pairwise(nr, nphi, rmin, rmax, h, sig)
    tr, tp = O.field_table(nr, nphi, rmin, rmax, h, sig)
    assert np.abs(gr - tr).max() < 1e-13 * np.abs(gr).max()
    assert np.abs(gp - tp).max() < 1e-13 * np.abs(gr).max()


def test_table_mode_equals_pairwise_sum_per_component_at_fp64_bar_size():
    """The 64 x 128 FP64 workload (Sigma = r^-1 (1 + 0.01 U), h = 0.05): the
    App. C offset-table sum and the Cartesian pairwise sum, two routes to the
    same discrete sum with different terms and rounding, agree per component
    far below the 1e-12 bar, g_phi (about 0.2 % of |g| here) included.  With
    double running sums, double cell centres and azimuth offsets taken in
    [0, 2 pi) the two sat 2.4e-12 apart on g_phi."""
    rng = np.random.default_rng(1)
    nr, nphi, rmin, rmax = 64, 128, 0.2, 2.5
    r, _, _, _ = O.grid(nr, nphi, rmin, rmax)
    sig = (1.0 / r)[None, :, None] * (1 + 0.01 * rng.uniform(-1, 1, (1, nr, nphi)))
    idx = np.sort(np.random.default_rng(2).choice(nr * nphi, 1024, replace=False))
    gr, gp = O.field_pairwise(nr, nphi, rmin, rmax, [0.05], sig, targets=idx)
    tr, tp = O.field_table(nr, nphi, rmin, rmax, [0.05], sig, targets=idx)
    e_r = np.linalg.norm(gr - tr) / np.linalg.norm(gr)
    e_p = np.linalg.norm(gp - tp) / np.linalg.norm(gp)
    assert e_r < 1e-13 and e_p < 1e-13, (e_r, e_p)  # seen 2.5e-16 and 3.4e-14


def test_pairwise_sum_equals_high_precision_sum():
    """The discrete sum at three seeded targets of a 16 x 32 disc of the FP64
    workload's recipe, evaluated term by term in 30-digit arithmetic (mpmath
    Bessel functions, exact cell centres): the oracle's pairwise and table
    sums agree with it per component to 1e-13 of the component itself
    (g_phi is about 1e-3 of |g| here, so this bounds the oracle's own
    rounding, not only its formulas)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 30
    rng = np.random.default_rng(1)
    nr, nphi, rmin, rmax, h = 16, 32, 0.2, 2.5, 0.05
    r, _, _, _ = O.grid(nr, nphi, rmin, rmax)
    sig = (1.0 / r)[None, :, None] * (1 + 0.01 * rng.uniform(-1, 1, (1, nr, nphi)))
    targets = np.array([37, 200, 411])
    pr, pp = O.field_pairwise(nr, nphi, rmin, rmax, [h], sig, targets=targets, flags=O.EXCLUDE_SELF)
    tr, tp = O.field_table(nr, nphi, rmin, rmax, [h], sig, targets=targets, flags=O.EXCLUDE_SELF)
    H = mp.mpf(h)
    lnr0 = mp.log(mp.mpf(rmin))
    DU = (mp.log(mp.mpf(rmax)) - lnr0) / nr
    DP = 2 * mp.pi / nphi
    rad = [mp.e ** (lnr0 + (i + mp.mpf(1) / 2) * DU) for i in range(nr)]
    ang = [(j + mp.mpf(1) / 2) * DP for j in range(nphi)]
    for t, i in enumerate(targets):
        ir, j = divmod(int(i), nphi)
        ri, pi_ = rad[ir], ang[j]
        xi, yi = ri * mp.cos(pi_), ri * mp.sin(pi_)
        Gx = Gy = mp.mpf(0)
        for kr in range(nr):
            rk = rad[kr]
            for kp in range(nphi):
                if kr == ir and kp == j:
                    continue
                dx, dy = xi - rk * mp.cos(ang[kp]), yi - rk * mp.sin(ang[kp])
                s = mp.sqrt(dx * dx + dy * dy)
                H2 = (H * H * rk * rk + H * H * ri * ri) / 2
                x = s * s / (8 * H2)
                K = mp.e ** x * (mp.besselk(1, x) - mp.besselk(0, x)) * (s / mp.sqrt(H2)) / 8 / (mp.sqrt(mp.pi) * H2)
                w = mp.mpf(float(sig[0, kr, kp])) * rk * rk * DU * DP * K / s
                Gx -= w * dx
                Gy -= w * dy
        gr = float(Gx * mp.cos(pi_) + Gy * mp.sin(pi_))
        gp = float(-Gx * mp.sin(pi_) + Gy * mp.cos(pi_))
        for got_r, got_p in ((pr[0, t], pp[0, t]), (tr[0, t], tp[0, t])):
            assert abs(got_r / gr - 1) < 1e-13, (i, got_r, gr)
            assert abs(got_p / gp - 1) < 1e-13, (i, got_p, gp)


def test_razor_thin_field_is_newtonian_sum():
    """h -> 0: the field is the point-mass Newtonian sum -sum m (x_i-x_k)/s^3."""
    rng = np.random.default_rng(2)
    nr, nphi, rmin, rmax = 6, 10, 0.5, 2.0
    r, phi, du, dphi = O.grid(nr, nphi, rmin, rmax)
    sig = rng.uniform(0.5, 1.5, (1, nr, nphi))
    gr, gp = O.field_pairwise(nr, nphi, rmin, rmax, [1e-7], sig, flags=O.EXCLUDE_SELF)
    R = np.repeat(r, nphi)
    P = np.tile(phi, nr)
    x, y = R * np.cos(P), R * np.sin(P)
    m = sig.ravel() * R ** 2 * du * dphi
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    s3 = np.hypot(dx, dy) ** 3
    np.fill_diagonal(s3, np.inf)
    Gx = -(m[None, :] * dx / s3).sum(1)
    Gy = -(m[None, :] * dy / s3).sum(1)
    ref_r = Gx * np.cos(P) + Gy * np.sin(P)
    ref_p = -Gx * np.sin(P) + Gy * np.cos(P)
    assert np.abs(gr[0] - ref_r).max() < 1e-9 * np.abs(ref_r).max()
    assert np.abs(gp[0] - ref_p).max() < 1e-9 * np.abs(ref_r).max()


def test_two_cell_system_by_hand():
    """Two cells on one ring (N_r = 1, N_phi = 2): the pull of cell 1 on cell 0
    points from 0 to 1 (attractive, radially inward for cell 0), magnitude
    Sigma A K(2r), K from 40-digit Bessel functions."""
    rmin, rmax = 1.0, 1.2
    r, phi, du, dphi = O.grid(1, 2, rmin, rmax)
    H = 0.3 * r[0]
    sig = np.array([[[0.0, 2.0]]])
    gr, gp = O.field_pairwise(1, 2, rmin, rmax, [0.3], sig, flags=O.EXCLUDE_SELF)
    s = 2 * r[0]
    d = s / H
    x = d * d / 8
    K = float(1 / mp.sqrt(mp.pi) / H ** 2 * d / 8 * _F_mp(x))
    A = r[0] ** 2 * du * dphi
    assert gr[0, 0] == pytest.approx(-2.0 * A * K, rel=1e-14)
    assert abs(gp[0, 0]) < 1e-15 * abs(gr[0, 0])
    assert gr[0, 1] == 0.0


def test_exponential_disc_continuum_normalisation():
    """Continuum check of the whole normalisation (G = 1, area element, 2D
    kernel) against the exponential-disc closed form of Sect. 4.2,
    g_r = -2 pi Sigma0 y [I0 K0 - I1 K1](y), y = r/(2 r0), at small h.
    Discretisation and finite thickness leave a few 1e-2 at this grid."""
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        e = json.load(fh)["exponential_disc_setup"]
    nr, nphi, h = 256, 512, 0.01
    rmin, rmax = e["r_in"] / e["r0"], e["r_out"] / e["r0"]   # lengths in units of r0
    r, phi, du, dphi = O.grid(nr, nphi, rmin, rmax)
    sig = np.exp(-r)[None, :, None] * np.ones((1, nr, nphi))
    sel = np.where((r > 0.25) & (r < 4.0))[0][::4]
    gr, _ = O.field_table(nr, nphi, rmin, rmax, [h], sig, targets=sel * nphi)
    y = r[sel] / 2
    ref = -2 * np.pi * y * (ss.i0(y) * ss.k0(y) - ss.i1(y) * ss.k1(y))
    assert np.all(np.abs(gr[0] / ref - 1) < 3e-2)


# ----------------------------------------------------------------- adjoint
def test_adjoint_sigma_equals_central_differences():
    """dL/dSigma for L = sum_b sum_c w (g - g*)^2: the oracle's transposed sum vs
    central differences of the oracle forward (exact, L is quadratic)."""
    rng = np.random.default_rng(4)
    nr, nphi, rmin, rmax = 6, 8, 0.3, 2.0
    h = [0.06, 0.012]
    sig = rng.uniform(0.5, 1.5, (2, nr, nphi))
    tgt = np.array(O.field_table(nr, nphi, rmin, rmax, h, rng.uniform(0.5, 1.5, (2, nr, nphi))))

    def loss(s):
        g = np.array(O.field_table(nr, nphi, rmin, rmax, h, s))
        return float(np.sum((g - tgt) ** 2))

    g = np.array(O.field_table(nr, nphi, rmin, rmax, h, sig))
    lam = 2 * (g - tgt)          # [c][b][N]
    ds = O.adjoint_sigma(nr, nphi, rmin, rmax, h, lam[0], lam[1])
    e = 1e-3
    for a, k in ((0, 0), (0, 17), (1, 5), (1, 47)):
        sp_ = sig.copy()
        sm_ = sig.copy()
        sp_.reshape(2, -1)[a, k] += e
        sm_.reshape(2, -1)[a, k] -= e
        fd = (loss(sp_) - loss(sm_)) / (2 * e)
        assert ds[a, k] == pytest.approx(fd, rel=1e-9, abs=1e-12)


def test_adjoint_h_equals_central_differences():
    rng = np.random.default_rng(6)
    nr, nphi, rmin, rmax = 6, 8, 0.3, 2.0
    h = np.array([0.06, 0.012])
    sig = rng.uniform(0.5, 1.5, (2, nr, nphi))
    tgt = np.array(O.field_table(nr, nphi, rmin, rmax, h * 1.1, sig))

    def loss(hh):
        g = np.array(O.field_table(nr, nphi, rmin, rmax, hh, sig))
        return float(np.sum((g - tgt) ** 2))

    g = np.array(O.field_table(nr, nphi, rmin, rmax, h, sig))
    lam = 2 * (g - tgt)
    dh = O.adjoint_h(nr, nphi, rmin, rmax, h, sig, lam[0], lam[1])
    for f in range(2):
        e = 1e-4 * h[f]
        hp, hm = h.copy(), h.copy()
        hp[f] += e
        hm[f] -= e
        fd = (loss(hp) - loss(hm)) / (2 * e)
        assert dh[f] == pytest.approx(fd, rel=1e-6)


# ------------------------------------------------------------ indirect term
def _grid_np(nr, nphi, rmin, rmax):
    du = math.log(rmax / rmin) / nr
    r = np.exp(math.log(rmin) + (np.arange(nr) + 0.5) * du)
    phi = (np.arange(nphi) + 0.5) * (2 * math.pi / nphi)
    return r, phi, du, 2 * math.pi / nphi


@pytest.mark.parametrize("r,H", [(1.0, 0.05), (0.3, 0.1), (2.0, 0.4), (1.0, 2.0)])
def test_indirect_kernel_equals_vertical_integral(r, H):
    """The star's pull by a vertically Gaussian column (first line of the
    indirect-term appendix): r' int e^{-z^2/2H^2}/(sqrt(2 pi) H) (r'^2+z^2)^{-3/2} dz,
    by brute-force quadrature, equals the oracle's sqrt(2) K_a for a one-cell disc."""
    nr, nphi, rmin = 1, 1, r / math.exp(0.5e-3)
    rmax = r * math.exp(0.5e-3)
    sig = np.ones((1, 1, 1))
    AB = O.indirect(nr, nphi, rmin, rmax, [H / r], sig)
    rc, phi, du, dphi = _grid_np(nr, nphi, rmin, rmax)
    mass = rc[0] ** 2 * du * dphi
    I, _ = si.quad(lambda z: math.exp(-0.5 * (z / H) ** 2) / (math.sqrt(2 * math.pi) * H)
                   * (rc[0] ** 2 + z * z) ** -1.5, -np.inf, np.inf, epsabs=0, epsrel=1e-13, limit=400)
    ref = mass * rc[0] * I
    got = math.hypot(AB[0, 0], AB[0, 1])
    assert abs(got / ref - 1) < 1e-11, (got, ref)
    assert abs(math.atan2(AB[0, 1], AB[0, 0]) - phi[0]) < 1e-12


def test_indirect_kernel_is_pair_kernel_with_point_target():
    """sqrt(2) K_a(d_a) equals the pair kernel K_ab(s = r'; H_a, H_b = 0) (the
    star has no thickness): one-cell disc at several radii and heights."""
    rng = np.random.default_rng(11)
    for _ in range(8):
        nr, nphi = 3, 5
        rmin, rmax = rng.uniform(0.2, 1.0), rng.uniform(2.0, 6.0)
        h = rng.uniform(0.01, 0.5)
        i, j = rng.integers(nr), rng.integers(nphi)
        sig = np.zeros((1, nr, nphi))
        sig[0, i, j] = 1.0
        AB = O.indirect(nr, nphi, rmin, rmax, [h], sig)
        r, phi, du, dphi = _grid_np(nr, nphi, rmin, rmax)
        ref = r[i] ** 2 * du * dphi * O.kernel(r[i], h * r[i], 0.0)[0]
        assert abs(AB[0, 0] - ref * math.cos(phi[j])) < 1e-13 * ref
        assert abs(AB[0, 1] - ref * math.sin(phi[j])) < 1e-13 * ref


def test_indirect_vanishes_for_axisymmetric_disc_and_rotates():
    nr, nphi = 16, 32
    r, phi, _, _ = _grid_np(nr, nphi, 0.2, 5.0)
    sig = np.broadcast_to((r ** -1.0)[:, None], (nr, nphi))[None].copy()
    AB = O.indirect(nr, nphi, 0.2, 5.0, [0.05], sig)
    scale = O.indirect(nr, nphi, 0.2, 5.0, [0.05], np.abs(sig) * (np.cos(phi) > 0))[0, 0]
    assert np.all(np.abs(AB) < 1e-13 * scale)
    # rotation by s cells multiplies A + iB by exp(i s dphi)
    rng = np.random.default_rng(3)
    sig = rng.uniform(0.5, 1.5, (2, nr, nphi))
    s = 5
    a = O.indirect(nr, nphi, 0.2, 5.0, [0.05, 0.01], sig)
    b = O.indirect(nr, nphi, 0.2, 5.0, [0.05, 0.01], np.roll(sig, s, axis=2))
    za = a[:, 0] + 1j * a[:, 1]
    zb = b[:, 0] + 1j * b[:, 1]
    np.testing.assert_allclose(zb, za * np.exp(1j * s * 2 * math.pi / nphi), rtol=1e-12)


@pytest.mark.parametrize("h", [0.02, 0.005])
def test_indirect_point_mass_limit_and_next_term(h):
    """Thin-disc limit: sqrt(2) K_a -> 1/r'^2 (Newtonian point masses), with the
    relative correction -3/8 / x + 45/128 / x^2 at x = 1/(4 h^2) (the printed
    large-x expansion of Sect. 5.3 applied to the star's kernel)."""
    nr, nphi = 12, 24
    rng = np.random.default_rng(5)
    sig = rng.uniform(0.0, 1.0, (1, nr, nphi))
    r, phi, du, dphi = _grid_np(nr, nphi, 0.3, 3.0)
    AB = O.indirect(nr, nphi, 0.3, 3.0, [h], sig)
    m = sig[0] * (r ** 2)[:, None] * du * dphi
    newton = np.array([(m * np.cos(phi) / (r ** 2)[:, None]).sum(), (m * np.sin(phi) / (r ** 2)[:, None]).sum()])
    x = 1 / (4 * h * h)
    corr = 1 - 3 / 8 / x + 45 / 128 / x ** 2
    np.testing.assert_allclose(AB[0], newton * corr, rtol=3 * (525 / 1024) / x ** 3 + 1e-13)


# ------------------------------------------------------ conservative potential
def test_G0_matches_arbitrary_precision_bessel():
    """e^y K0(y) (kernel of the conservative potential) vs 40-digit mpmath."""
    ys = np.logspace(-12, 4.6, 40)
    got = O.G0(ys)
    for y, v in zip(ys, got):
        ref = float(mp.e ** mp.mpf(y) * mp.besselk(0, mp.mpf(y)))
        assert abs(v - ref) <= 3e-15 * ref, (y, v, ref)


def test_potential_kernel_newtonian_limit():
    """s >> H: P_ab -> -1/s with the asymptotic correction of e^y K0(y),
    sqrt(pi/(2y)) (1 - 1/(8y) + 9/(128 y^2)), y = s^2/(8 H_ab^2)."""
    for s, Ha, Hb in [(1.0, 0.01, 0.02), (3.0, 0.05, 0.05), (0.5, 0.003, 0.001)]:
        Hab = math.sqrt(0.5 * (Ha * Ha + Hb * Hb))
        y = s * s / (8 * Hab * Hab)
        want = -1.0 / s * (1 - 1 / (8 * y) + 9 / (128 * y * y))
        got = O.potential_kernel([s], Ha, Hb)[0]
        assert abs(got / want - 1) < 2 * 225 / 3072 / y ** 3 + 1e-14, (s, got, want)


def test_potential_gradient_is_the_field_for_constant_H():
    """Constant H_a, H_b: -grad Phi_ab equals the pairwise field of the exact
    force kernel (the conservative case of Sect. 5.5), by central differences
    at points off the cell centres."""
    nr, nphi, rmin, rmax = 6, 12, 0.5, 2.0
    rng = np.random.default_rng(21)
    sig = rng.uniform(0.2, 1.0, (nr, nphi))
    for Ha, Hb in [(0.08, 0.08), (0.1, 0.03)]:
        ang = rng.uniform(0, 2 * math.pi, 6)
        rad = rng.uniform(0.6, 1.9, 6)
        px, py = rad * np.cos(ang), rad * np.sin(ang)
        _, gx, gy = O.point_fields(nr, nphi, rmin, rmax, Ha, Hb, sig, px, py)
        eps = 1e-5
        pxp, _, _ = O.point_fields(nr, nphi, rmin, rmax, Ha, Hb, sig, px + eps, py)
        pxm, _, _ = O.point_fields(nr, nphi, rmin, rmax, Ha, Hb, sig, px - eps, py)
        pyp, _, _ = O.point_fields(nr, nphi, rmin, rmax, Ha, Hb, sig, px, py + eps)
        pym, _, _ = O.point_fields(nr, nphi, rmin, rmax, Ha, Hb, sig, px, py - eps)
        fx = -(pxp - pxm) / (2 * eps)
        fy = -(pyp - pym) / (2 * eps)
        scale = np.hypot(gx, gy).max()
        assert np.abs(fx - gx).max() < 1e-7 * scale
        assert np.abs(fy - gy).max() < 1e-7 * scale


@pytest.mark.parametrize("r,Ha,Hb,du,dphi", [(1.0, 0.05, 0.05, 0.02, 0.05), (0.4, 0.02, 0.006, 0.05, 0.1),
                                             (2.0, 0.5, 0.3, 0.1, 0.2)])
def test_potential_self_term_independent_quadrature(r, Ha, Hb, du, dphi):
    """Own-cell integral of P_ab by scipy's adaptive quadrature in polar
    coordinates about the centre of the (X, phi) cell (an independent rule)."""
    def f(X, phi):
        s = r * math.sqrt(math.exp(X) * 4 * (math.sinh(0.5 * X) ** 2 + math.sin(0.5 * phi) ** 2))
        return O.potential_kernel([s], Ha, Hb)[0] * r * r * math.exp(2 * X)
    a, b = du / 2, dphi / 2
    total = 0.0
    for sx in (-1, 1):
        for sy in (-1, 1):
            # quadrant split at its diagonal; polar about the corner
            th_c = math.atan2(b, a)
            for th0, th1, edge in ((0, th_c, "a"), (th_c, math.pi / 2, "b")):
                def inner(th):
                    c, s_ = math.cos(th), math.sin(th)
                    rmax = a / c if edge == "a" else b / s_
                    v, _ = si.quad(lambda rho: rho * f(sx * rho * c, sy * rho * s_), 0, rmax,
                                   epsabs=0, epsrel=1e-12, limit=200, points=[rmax * 1e-3])
                    return v
                v, _ = si.quad(inner, th0, th1, epsabs=0, epsrel=1e-11, limit=200)
                total += v
    got = O.potential_self(r, Ha, Hb, du, dphi)
    assert abs(got / total - 1) < 1e-9, (got, total)


def test_potential_reciprocity_general_H():
    """sum_i m_b[i] Phi^{a->b}(i) = sum_k m_a[k] Phi^{b->a}(k) (the pair
    potential is symmetric in the two cells), self terms excluded."""
    nr, nphi, rmin, rmax = 5, 9, 0.4, 2.5
    rng = np.random.default_rng(8)
    sig = rng.uniform(0.1, 1.0, (2, nr, nphi))
    du = math.log(rmax / rmin) / nr
    r = np.exp(math.log(rmin) + (np.arange(nr) + 0.5) * du)
    H = rng.uniform(0.02, 0.2, (2, nr, nphi))
    area = (r ** 2 * du * 2 * math.pi / nphi)[:, None] * np.ones((1, nphi))

    def pot_from(a):
        s = np.zeros_like(sig)
        s[a] = sig[a]
        return O.potential_pairwise(nr, nphi, rmin, rmax, [0, 0], s, H=H, flags=O.EXCLUDE_SELF)
    pa = pot_from(0)  # field of fluid 0 at both fluids
    pb = pot_from(1)
    w01 = (sig[1] * area).ravel() @ pa[1]
    w10 = (sig[0] * area).ravel() @ pb[0]
    assert abs(w01 - w10) < 1e-13 * abs(w01)


# ------------------------------------------------- self-gravitating heights
def test_hsg_limits_and_defining_quadratic():
    """H^sg = sqrt(2/pi) H f(Qt) (Sect. 2.1): f -> sqrt(pi/2) without
    self-gravity (Q -> inf: H^sg -> H), f ~ x for strong self-gravity, and
    f is the positive root of (2x/pi) f^2 + f - x = 0."""
    H = np.array([[0.05, 0.05, 0.05], [0.01, 0.01, 0.01]])
    big = O.hsg(H, np.full((2, 3), 1e9))
    np.testing.assert_allclose(big, H, rtol=1e-8)
    Q = np.array([[1e-4, 2e-4, 5e-4], [1e-3, 1e-3, 1e-3]])
    x = 1 / (1 / Q[0] + 1 / Q[1])
    small = O.hsg(H, Q)
    np.testing.assert_allclose(small / (math.sqrt(2 / math.pi) * H), np.broadcast_to(x, (2, 3)), rtol=1e-6)
    rng = np.random.default_rng(4)
    Q = rng.uniform(0.1, 10, (2, 50))
    H = rng.uniform(0.01, 0.1, (2, 50))
    f = O.hsg(H, Q) / (math.sqrt(2 / math.pi) * H)
    x = 1 / (1 / Q[0] + 1 / Q[1])
    np.testing.assert_allclose(2 * x / math.pi * f[0] ** 2 + f[0] - x, 0, atol=1e-13)
    np.testing.assert_allclose(f[0], f[1], rtol=1e-15)


# ------------------------------------------------------- uniform radial grid
@pytest.mark.parametrize("ha,hb,du,dphi", [(0.05, 0.02, 0.01, 0.003), (0.1, 0.1, 0.2, 0.1),
                                           (0.01, 0.03, 0.05, 0.2)])
def test_self_cell_range_symmetric_equals_cell_average(ha, hb, du, dphi):
    """The one-sided quadrature of the own-cell integral over [-du/2, du/2]
    equals du dphi times the X-symmetrised average (two different rules)."""
    got = O.self_cell_range(ha, hb, -du / 2, du / 2, dphi)
    ref = du * dphi * O.self_cell(ha, hb, du, dphi)
    assert abs(got / ref - 1) < 1e-11


@pytest.mark.parametrize("ha,hb,delta,dphi", [(0.05, 0.05, 0.02, 0.01), (0.02, 0.1, 0.1, 0.05)])
def test_self_cell_range_asymmetric_strip(ha, hb, delta, dphi):
    """A uniform-grid cell spans X in [ln(1 - delta), ln(1 + delta)]: its own-cell
    integral is the symmetric part over |X| <= ln(1 + delta) plus the regular
    strip ln(1 - delta) <= X <= -ln(1 + delta), which scipy's adaptive dblquad
    integrates from the convolution kernels directly."""
    xlo, xhi = math.log1p(-delta), math.log1p(delta)
    sym = O.self_cell_range(ha, hb, -xhi, xhi, dphi)

    def f(phi, X):
        return O.conv_kernels(np.array([X]), np.array([phi]), ha, hb)[0][0]
    strip, _ = si.dblquad(f, xlo, -xhi, -dphi / 2, dphi / 2, epsabs=0, epsrel=1e-11)
    got = O.self_cell_range(ha, hb, xlo, xhi, dphi)
    assert abs(got - (sym + strip)) < 1e-10 * abs(got)


def test_potential_self_range_asymmetric_strip():
    """The same decomposition for the potential's own-cell integral."""
    r, Ha, Hb, delta, dphi = 1.5, 0.05, 0.08, 0.03, 0.02
    xlo, xhi = math.log1p(-delta), math.log1p(delta)
    sym = O.potential_self_range(r, Ha, Hb, -xhi, xhi, dphi)

    def f(phi, X):
        s = r * math.sqrt(math.exp(X) * 4 * (math.sinh(0.5 * X) ** 2 + math.sin(0.5 * phi) ** 2))
        return O.potential_kernel([s], Ha, Hb)[0] * r * r * math.exp(2 * X)
    strip, _ = si.dblquad(f, xlo, -xhi, -dphi / 2, dphi / 2, epsabs=0, epsrel=1e-11)
    got = O.potential_self_range(r, Ha, Hb, xlo, xhi, dphi)
    assert abs(got - (sym + strip)) < 1e-10 * abs(got)
    assert O.potential_self_range(r, Ha, Hb, -0.01, 0.01, dphi) == O.potential_self(r, Ha, Hb, 0.02, dphi)


def test_newton_third_law_uniform_radial_grid():
    """Zero net force on the whole disc on a uniform radial grid (cell areas
    r_i dr dphi), self term excluded, per-cell scale heights."""
    rng = np.random.default_rng(12)
    nr, nphi, rmin, rmax = 8, 13, 0.5, 2.5
    r, phi, dr, dphi = O.grid(nr, nphi, rmin, rmax, O.LINEAR_R)
    assert np.allclose(np.diff(r), dr)
    sig = rng.uniform(0.2, 2.0, (2, nr, nphi))
    H = rng.uniform(0.01, 0.2, (2, nr, nphi))
    gr, gp = O.field_pairwise(nr, nphi, rmin, rmax, [0, 0], sig, H=H, flags=O.EXCLUDE_SELF | O.LINEAR_R)
    A = (r * dr * dphi)[:, None] * np.ones((nr, nphi))
    tot = np.zeros(2)
    scale = 0.0
    P = np.broadcast_to(phi[None, :], (nr, nphi)).ravel()
    for b in range(2):
        gx = gr[b] * np.cos(P) - gp[b] * np.sin(P)
        gy = gr[b] * np.sin(P) + gp[b] * np.cos(P)
        m = (sig[b] * A).ravel()
        tot += [np.sum(m * gx), np.sum(m * gy)]
        scale += np.sum(m * np.hypot(gx, gy))
    assert np.all(np.abs(tot) < 1e-13 * scale)


def test_two_cell_system_uniform_grid_by_hand():
    """Two cells on one ring of a uniform radial grid: the pull is
    Sigma A K(2 r) with the sector area A = r dr dphi and r the arithmetic
    centre of the ring."""
    rmin, rmax = 1.0, 1.2
    r = 1.1
    H = 0.3 * r
    sig = np.array([[[0.0, 2.0]]])
    gr, gp = O.field_pairwise(1, 2, rmin, rmax, [0.3], sig, flags=O.EXCLUDE_SELF | O.LINEAR_R)
    d = 2 * r / H
    K = float(1 / mp.sqrt(mp.pi) / H ** 2 * d / 8 * _F_mp(d * d / 8))
    A = ((rmax ** 2 - rmin ** 2) / 2) * math.pi  # half the annulus
    assert gr[0, 0] == pytest.approx(-2.0 * A * K, rel=1e-14)
    assert gr[0, 1] == 0.0
