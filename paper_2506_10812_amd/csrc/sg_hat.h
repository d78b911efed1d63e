// sg_hat.h -- quadrature of the second-order (hat-weighted) kernel weights,
// shared by the FFT path's table build and the semi-spectral operator rows.
#pragma once
#include "sg_kfn.h"
#include "sg_table.h"

// SG_SECOND_ORDER: the sources are the piecewise-bilinear interpolant of the
// cell values on the (u, phi) grid (tensor-product hat functions Lambda
// centred on the cell centres, periodic in phi), integrated exactly against
// the kernel, so the table holds, in place of the point samples and the
// own-cell average,
//   W_c(P, Q) = int int Lambda(s) Lambda(t) K_c((P + s) du, (Q + t) dphi) ds dt
// over s, t in [-1, 1] (Lambda(x) = 1 - |x|).  The support splits into four
// unit squares on which the weight is bilinear.  A square whose corner is
// the kernel's singular point (s, t) = (-P, -Q) (|P|, |Q| <= 1) is done in
// polar coordinates about that corner (the Duffy split and geometric panels
// of the self-cell rule); at (P, Q) = (0, 0) the four squares are folded
// into one with K_r symmetrised in X (the 1/rho part of K_r is odd in X and
// cancels only between the halves; K_phi, odd in phi, gives 0).  Elsewhere
// tensor Gauss-Legendre rules of 6 x 6 points on sub-squares small against
// their distance to the singular point (at most a third of it).
static __device__ __constant__ double sg_gl6_x[6] = {0.0337652428984239860, 0.1693953067668677431,
                                                     0.3806904069584015457, 0.6193095930415984543,
                                                     0.8306046932331322569, 0.9662347571015760140};
static __device__ __constant__ double sg_gl6_w[6] = {0.0856622461895851725, 0.1803807865240693038,
                                                     0.2339569672863455237, 0.2339569672863455237,
                                                     0.1803807865240693038, 0.0856622461895851725};

__device__ inline double sg_hat(double x) { return fmax(0.0, 1.0 - fabs(x)); }

// Tensor Gauss-Legendre over pieces k in [k0, k1) (step dk) of the unit square
// [ds, ds + 1] x [dt, dt + 1] of entry (P, Q), cut into ms x mt sub-squares.
__device__ inline void sg_hat_square(int P, int Q, int ds, int dt, int ms, int mt, int k0, int k1, int dk,
                                     double du, double dphi, double ha, double hb, int which, const double *wq,
                                     double &wr, double &wp)
{
    for (int k = k0; k < k1; k += dk) {
        const int piece = k / 36, node = k % 36;
        const int is = piece % ms, it = piece / ms;
        const int a = node % 6, b = node / 6;
        const double s = ds + (is + sg_gl6_x[a]) / ms, t = dt + (it + sg_gl6_x[b]) / mt;
        const double w = sg_gl6_w[a] * sg_gl6_w[b] / (ms * mt) * sg_hat(s) * sg_hat(t);
        const double X = (P + s) * du, ph = (Q + t) * dphi;
        double kr, kp;
        sg_conv_kernel64(X, sin(0.5 * ph), sin(ph), ha, hb, which, wq, kr, kp);
        wr += w * kr;
        wp += w * kp;
    }
}

// Sub-square count per side: pieces at most a third of their distance to
// the singular point (physical units), at most 32.
__device__ inline void sg_hat_split(int P, int Q, int ds, int dt, double du, double dphi, int &ms, int &mt)
{
    const double x0 = (P + ds) * du, x1 = x0 + du, y0 = (Q + dt) * dphi, y1 = y0 + dphi;
    const double dx = x0 > 0.0 ? x0 : (x1 < 0.0 ? -x1 : 0.0);
    const double dy = y0 > 0.0 ? y0 : (y1 < 0.0 ? -y1 : 0.0);
    const double d = sqrt(dx * dx + dy * dy);
    ms = min(32, max(1, (int)ceil(3.0 * du / d)));
    mt = min(32, max(1, (int)ceil(3.0 * dphi / d)));
}

__device__ inline bool sg_hat_singular(int P, int Q, int ds, int dt)
{
    return (-P == ds || -P == ds + 1) && (-Q == dt || -Q == dt + 1);
}

// Polar rule on the unit square [ds, ds + 1] x [dt, dt + 1] whose corner is
// the singular point: (X, phi) = (sx du x, sy dphi y) with (x, y) in [0, 1]^2
// measured from the corner, cut along its diagonal, each triangle mapped to
// the unit square with the corner collapsed (x = xi, y = xi eta and
// x = xi eta, y = xi; Jacobian xi).  sym: K_r symmetrised in X (entry (0, 0)).
// Nodes k0, k0 + dk, ... of the rule (a block's threads, or one thread).
__device__ inline void sg_hat_corner(int P, int Q, int sx, int sy, bool sym, double du, double dphi, double ha,
                                     double hb, int which, const GLNodes &gl, const double *wq, int k0, int dk,
                                     double &wr, double &wp)
{
    constexpr int NX = SG_PANELS * SG_GLX_N;
    for (int idx = k0; idx < NX * SG_GL_N; idx += dk) {
        const int ix = idx / SG_GL_N, j = idx % SG_GL_N;
        const int pnl = ix / SG_GLX_N, i = ix % SG_GLX_N;
        const double hi = ldexp(1.0, -2 * (SG_PANELS - 1 - pnl));
        const double lo = pnl == 0 ? 0.0 : 0.25 * hi;
        const double xi = lo + (hi - lo) * gl.xr[i];
        const double eta = gl.x[j];
        const double wgt = (hi - lo) * gl.wr[i] * gl.w[j] * xi;
        for (int tri = 0; tri < 2; ++tri) {
            const double x = tri == 0 ? xi : xi * eta, y = tri == 0 ? xi * eta : xi;
            const double X = sx * x * du, ph = sy * y * dphi;
            // hats from the corner: 1 - x at a corner s = 0, x at s = +-1
            // (not 1 - |-1 + x|, which loses the digits of a small x)
            const double w = wgt * (P == 0 ? 1.0 - x : x) * (Q == 0 ? 1.0 - y : y);
            if (sym) {
                wr += w * sg_sym_kr64(X, ph, ha, hb, which, wq);
            } else {
                double kr, kp;
                sg_conv_kernel64(X, sin(0.5 * ph), sin(ph), ha, hb, which, wq, kr, kp);
                wr += w * kr;
                wp += w * kp;
            }
        }
    }
}

// Part of W_c(P, Q) (or an h derivative, which): the quadrature nodes
// k0, k0 + dk, ... of every piece (the polar rules at the singular corner for
// |P|, |Q| <= 1, split tensor squares elsewhere, as the table build's kernels
// apply them); the sum of the parts over k0 = 0 .. dk - 1 is the weight.
__device__ inline void sg_hat_weight_part(int P, int Q, double du, double dphi, double ha, double hb, int which,
                                          const GLNodes &gl, const double *wq, int k0, int dk, double &wr,
                                          double &wp)
{
    wr = 0.0;
    wp = 0.0;
    if (P == 0 && Q == 0) {
        double r = 0.0, t = 0.0;
        sg_hat_corner(0, 0, 1, 1, true, du, dphi, ha, hb, which, gl, wq, k0, dk, r, t);
        wr = 4.0 * r;
        return;
    }
    const bool near = abs(P) <= 1 && abs(Q) <= 1;
    for (int ds = -1; ds <= 0; ++ds)
        for (int dt = -1; dt <= 0; ++dt) {
            if (near && sg_hat_singular(P, Q, ds, dt)) {
                const int sx = (ds == -P) ? 1 : -1, sy = (dt == -Q) ? 1 : -1;
                sg_hat_corner(P, Q, sx, sy, false, du, dphi, ha, hb, which, gl, wq, k0, dk, wr, wp);
            } else {
                int ms, mt;
                sg_hat_split(P, Q, ds, dt, du, dphi, ms, mt);
                sg_hat_square(P, Q, ds, dt, ms, mt, k0, 36 * ms * mt, dk, du, dphi, ha, hb, which, wq, wr, wp);
            }
        }
}
