// sg_semispec.hip -- the semi-spectral solver: azimuthal FFT plus a direct
// radial sum per azimuthal mode (Sect. 5.2), for scale heights that are any
// function of radius (it lifts the H = h r condition of the full log-polar
// FFT, whose cost App. D quantifies).
//
// With H_a = H_a(r) the kernel between source ring i' and target ring i
// still depends on the azimuths only through phi = phi_target - phi_source,
// so for every ring pair the field is a circular convolution in phi:
//   g_c^{b}(i, j) = - du dphi sum_a sum_i' sum_j' Sigma_a(i', j')
//                   K_c(X_ii', (j - j') dphi; h_a = H_a(r_i')/r_i', h_b = H_b(r_i)/r_i)
// with X_ii' = u_i - u_i' and K_c the convolution-form kernels of App. C
// (there with constant h; the pair enters them only through
// h_ab^2 = (h_a^2 e^{-X} + h_b^2 e^X)/2 = H_ab^2 / (r r'), so the same
// formulas hold ring by ring).  In phi-Fourier space mode m decouples:
//   g^_c^{b}(m, i) = sum_a sum_i' T_c^{ab}(m, i, i') Sigma~_a(m, i'),
// an n_r x n_r operator per (m, pair).  K_r is even and K_phi odd in phi, so
// T_r is real and T_phi = i t_phi with t_phi real.
//
// Table (sg_ss_table, double precision, rounded to float at the end):
//   1. self-cell averages Kbar_r per (pair, ring) with h = H/r at the ring
//      (offset X = 0, phi = 0; zero with SG_SELF_CELL_EXCLUDE);
//   2. per row (b, a, i', i): samples K_r + i K_phi at phi = q dphi for
//      q <= n_phi/2, mirrored (K_r even, K_phi odd), one complex transform
//      (shared by two rows, whose transforms are real),
//      T_r(m) = (Z[m] + Z[-m])/2, t_phi(m) = (Z[-m] - Z[m])/2,
//      scaled by -du dphi / n_phi (the inverse transform of the last pass is
//      unnormalised); rows are written [row][m] to a chunk buffer;
//   3. a tiled transpose moves each chunk into the table: full modes keep
//      every (i', i) entry, banded modes the diagonals |i' - i| <= w (the
//      band rule is in sg_internal.h; dropped couplings are below about
//      2^-30 of the axisymmetric one, and SG_SS_FULL keeps every entry).
// SG_INDIRECT folds the indirect term (Sect. 5.4 and its appendix) into
// mode 1: in the same convolution form it is Sigma convolved with
//   r_i'^2 sqrt(2) K_a(d_i') (cos phi, -sin phi),  d_i' = r_i' / H_a(r_i'),
// whose transform at m = 1 adds r_i'^2 sqrt(2) K_a(d) n_phi / 2 to both T_r
// and t_phi before scaling.
//
// SG_POTENTIAL builds the operators of the potential instead (Sect. 5.5 and
// the appendix on the conservative force): Phi_b(i, j) = sum Sigma_a A_i'
// P_ab(s), P_ab = -e^y K0(y) / (2 sqrt(pi) H_ab), y = s^2 / (8 H_ab^2), with
// the own-cell integral of P at zero offset.  P is even in phi, so T_r carries
// its real spectrum and t_phi = 0: the solve writes Phi to g_r (and rounding
// noise of the inverse transform to g_phi).
//
// Solve (sg_field_fft with discs flagged SG_SEMI_SPECTRAL): pass 1 and pass 3
// of the FFT path (phi transforms), and k_ss_pass in place of pass 2.
#include "sg_kfn.h"
#include "sg_semispec.h"
#include "sg_adjoint.h"
#include "sg_table.h"
#include "sg_hat.h"

// ------------------------------------------------------------ table: rows
struct SsRowArgs {
    int nr, nrt, nf, excl, ind, pot, lin, second;
    double lnrmin, du, dphi, rmin, dr;  // du: log grid; rmin, dr: uniform radial grid
    GLNodes gl;                         // second: the polar rules' nodes
};

// SG_SECOND_ORDER rows: the sample at (P, q) = (i - i', q) becomes the
// hat-weighted weight W_c(P, q) of the FFT path's table with the row's
// aspect ratios h_a = H_a(r_i')/r_i', h_b = H_b(r_i)/r_i held across the hat
// (for H = h r this is the FFT path's table; otherwise the variation of h
// across the hat is odd in s and enters at second order only).  Within
// SG_SS_HAT_NEAR of the larger cell side from the singular point the weight
// is integrated (sg_hat_weight1); beyond, it is the point value plus the
// second moments of the hats, W = K + (D_X^2 K + D_phi^2 K)/12, with central
// second differences over one cell (D_phi from the neighbouring samples of
// the row, D_X from two extra samples at X +- du): the remainder is
// O((cell/distance)^4), below 3e-6 of the entry at 32 cells.  The integrated
// samples are computed by the whole group, one after the other (each
// thread takes every T-th quadrature node; the owner of the sample adds the
// parts in thread order), so that no single lane carries a polar rule.
#define SG_SS_HAT_NEAR 32.0

template <int N> struct SsRowShape {
    static constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
    static constexpr int WGS = T > 256 ? T : 256;
    static constexpr int G = WGS / T;
};

// A group of T threads takes RPG consecutive rows R = r0 + row of the
// (b, a, i', i) order (i fastest), out: [nrows][ncol] float2 (T_r, t_phi),
// m = 0 .. N/2.  Point-sampled rows go two to a group (RPG = 2): a row's
// samples z = K_r + i K_phi are Hermitian in phi, so its transform Z is real,
// and the group transforms z_A + i z_B once, reading Z_A from the real part
// and Z_B from the imaginary part.  The row count is even (n_rt is) and so
// is every chunk, so the two rows are always i and i + 1 of one (b, a, i').
// Second-order rows (SO) keep one row per group.
template <int N, bool SO>
__global__ void __launch_bounds__(SsRowShape<N>::WGS)
k_ss_rows(const double *H, const double *self, SsRowArgs A, size_t r0, int nrows, float2 *out)
{
    using S = SsRowShape<N>;
    constexpr int P = S::P, T = S::T, G = S::G, W = LdsPlane<double>::elems(N);
    constexpr int NC = N / 2 + 1;
    constexpr int RPG = SO ? 1 : 2;
    __shared__ __attribute__((aligned(16))) double2 lds[W * G];
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double2 qres[SO ? NC * G : 1];  // SO: the group's integrated samples
    __shared__ int qmax_wg;                    // SO: last integrated sample of any group
    sg_fill_weights<double>(wq);
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    const LdsPlane<double> pl{lds + W * g};
    const int row = (blockIdx.x * G + g) * RPG;  // the group's first row
    const bool valid = row < nrows;
    const size_t R = r0 + (size_t)(valid ? row : 0);
    const int i0 = (int)(R % A.nrt);
    size_t rest = R / A.nrt;
    const int ip = (int)(rest % A.nr);
    rest /= A.nr;
    const int a = (int)(rest % A.nf), b = (int)(rest / A.nf);
    const double rp = A.lin ? A.rmin + (ip + 0.5) * A.dr : exp(A.lnrmin + (ip + 0.5) * A.du);
    const double ha = H[a * A.nr + ip] / rp;
    // per row of the group: target ring (padding rows take the last ring and
    // stay zero), its radius, h_b and X
    bool live_[RPG];
    int ic_[RPG];
    double ri_[RPG], hb_[RPG], X_[RPG];
#pragma unroll
    for (int u = 0; u < RPG; ++u) {
        const int iu = i0 + u;
        live_[u] = valid && iu < A.nr;
        ic_[u] = iu < A.nr ? iu : A.nr - 1;
        ri_[u] = A.lin ? A.rmin + (ic_[u] + 0.5) * A.dr : exp(A.lnrmin + (ic_[u] + 0.5) * A.du);
        hb_[u] = H[b * A.nr + ic_[u]] / ri_[u];
        X_[u] = A.lin ? log(ri_[u] / rp) : (double)(ic_[u] - ip) * A.du;
    }
    const bool live = live_[0];
    const int ic = ic_[0];
    const double ri = ri_[0], hb = hb_[0], X = X_[0];
    __syncthreads();
    if constexpr (SO) {
        // 1'. hat-weighted samples (see SG_SS_HAT_NEAR): point values of K go
        // to the plane for the neighbours' second differences, the weights
        // stay in registers until every neighbour has been read
        constexpr int J = (N / 2 + 1 + T - 1) / T;
        double2 val[J];
        unsigned taylor = 0u;
        const int Pr = ic - ip;
        const double rn = SG_SS_HAT_NEAR * fmax(A.du, A.dphi), xq = Pr * A.du;
        // integrated samples: q <= qn (qn = -1: none); the predicate below is
        // the one the sample loop uses
        int qn = -1;
        if (live && xq * xq < rn * rn)
            while (qn < N / 2 && xq * xq + ((qn + 1) * A.dphi) * ((qn + 1) * A.dphi) < rn * rn) ++qn;
        if (threadIdx.x == 0) qmax_wg = -1;
        __syncthreads();
        if (t == 0 && qn >= 0) atomicMax(&qmax_wg, qn);
        __syncthreads();
        const int qm = qmax_wg;  // uniform over the workgroup: every group meets the same barriers
        for (int q = 0; q <= qm; ++q) {
            double wr = 0.0, wp = 0.0;
            if (q <= qn) sg_hat_weight_part(Pr, q, A.du, A.dphi, ha, hb, 0, A.gl, wq, t, T, wr, wp);
            pl.st(t, make_double2(wr, wp));
            __syncthreads();
            if (q <= qn && t == 0) {
                double sr = 0.0, sp = 0.0;
                for (int k = 0; k < T; ++k) {
                    const double2 v = pl.ld(k);
                    sr += v.x;
                    sp += v.y;
                }
                qres[g * NC + q] = make_double2(sr, sp);
            }
            __syncthreads();
        }
        // the row-only factors at X and at the D_X neighbours X +- du
        const ConvRow64 c0 = sg_conv_row64(X, ha, hb), c1 = sg_conv_row64(X + A.du, ha, hb),
                        c2 = sg_conv_row64(X - A.du, ha, hb);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int q = t + T * j;
            val[j] = make_double2(0.0, 0.0);
            if (q > N / 2) continue;
            double sh, ch;
            sincospi((double)q / N, &sh, &ch);
            const double s2 = 2.0 * sh * ch;
            double kr = 0.0, kp = 0.0;
            if (q <= qn) {
                val[j] = qres[g * NC + q];
                if (Pr != 0 || q != 0) sg_conv_kernel64_row(c0, sh, s2, wq, kr, kp);
            } else {
                double k1r, k1p, k2r, k2p;
                sg_conv_kernel64_row(c0, sh, s2, wq, kr, kp);
                sg_conv_kernel64_row(c1, sh, s2, wq, k1r, k1p);
                sg_conv_kernel64_row(c2, sh, s2, wq, k2r, k2p);
                val[j] = make_double2(kr + (k1r - 2.0 * kr + k2r) / 12.0, kp + (k1p - 2.0 * kp + k2p) / 12.0);
                taylor |= 1u << j;
            }
            pl.st(q, make_double2(kr, kp));
            if (q != 0 && q != N / 2) pl.st(N - q, make_double2(kr, -kp));
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int q = t + T * j;
            if (q > N / 2 || !((taylor >> j) & 1u)) continue;
            const double2 k0 = pl.ld(q), kl = pl.ld((q + N - 1) & (N - 1)), kh = pl.ld((q + 1) & (N - 1));
            val[j].x += (kl.x - 2.0 * k0.x + kh.x) / 12.0;
            val[j].y += (kl.y - 2.0 * k0.y + kh.y) / 12.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int q = t + T * j;
            if (q > N / 2) continue;
            pl.st(q, val[j]);
            if (q != 0 && q != N / 2) pl.st(N - q, make_double2(val[j].x, -val[j].y));
        }
    } else {
    // 1. samples q in [0, N/2] of both rows, packed as z_A + i z_B and
    // mirrored into the upper half (z(-q) = conj z(q) for each row); the
    // factors that depend on a row alone are formed once
    ConvRow64 cr[RPG];
    double sx[RPG], Hab2[RPG], pot_pref[RPG];
#pragma unroll
    for (int u = 0; u < RPG; ++u) {
        cr[u] = sg_conv_row64(X_[u], ha, hb_[u]);
        sx[u] = sinh(0.5 * X_[u]);
        Hab2[u] = 0.5 * (ha * rp * ha * rp + hb_[u] * ri_[u] * hb_[u] * ri_[u]);
        pot_pref[u] = rp * rp / (2.0 * SG_SQRT_PI * sqrt(Hab2[u]));
    }
#pragma unroll 1
    for (int q = t; q <= N / 2; q += T) {
        double sp, cp;
        sincospi((double)q / N, &sp, &cp);
        double kr[RPG], kp[RPG];
#pragma unroll
        for (int u = 0; u < RPG; ++u) {
            kr[u] = 0.0;
            kp[u] = 0.0;
            if (ic_[u] == ip && q == 0) {
                kr[u] = A.excl ? 0.0 : self[(size_t)(a * A.nf + b) * A.nr + ic_[u]];
            } else if (A.pot) {
                // -r'^2 P_ab(s), so that the common scale -du dphi / N gives A_i' P / N
                const double s2 = 4.0 * ri_[u] * rp * (sx[u] * sx[u] + sp * sp);
                kr[u] = pot_pref[u] * sg_G0_64(s2 / (8.0 * Hab2[u]), wq);
            } else {
                sg_conv_kernel64_row(cr[u], sp, 2.0 * sp * cp, wq, kr[u], kp[u]);
            }
        }
        // (kr0 + i kp0) + i (kr1 + i kp1), and at -q (kr0 - i kp0) + i (kr1 - i kp1)
        pl.st(q, make_double2(kr[0] - kp[1], kp[0] + kr[1]));
        if (q != 0 && q != N / 2) pl.st(N - q, make_double2(kr[0] + kp[1], kr[1] - kp[0]));
    }
    }
    __syncthreads();
    double2 z[P];
#pragma unroll
    for (int p = 0; p < P; ++p) z[p] = pl.ld(t + T * p);
    __syncthreads();
    // 2. transform; Z = T_r - t_phi at m and T_r + t_phi at -m
    fft<N, false>(z, t, pl, TwPow64<N>{t});
#pragma unroll
    for (int p = 0; p < P; ++p) pl.st(t + T * p, z[p]);
    __syncthreads();
    if (!valid) return;
    // the samples carry r'^2 (the log-grid measure per du dphi); the source
    // cell's measure is r'^2 wgt dphi with wgt = du, or dr / r' on a uniform grid
    const double scale = -(A.lin ? A.dr / rp : A.du) * A.dphi / N;
    double ind = 0.0;
    if (A.ind) {
        // r'^2 sqrt(2) K_a(d) n_phi / 2 (the convolution-form samples carry the
        // cell measure r'^2), K_a(d) = pi^{-1/2} H^{-2} (d/4) F(d^2/4)
        const double Ha = H[a * A.nr + ip], d = rp / Ha;
        ind = rp * rp * SG_SQRT2 * (1.0 / SG_SQRT_PI) / (Ha * Ha) * (0.25 * d) * sg_F64(0.25 * d * d, wq) *
              (0.5 * N);
    }
#pragma unroll
    for (int u = 0; u < RPG; ++u) {
        float2 *o = out + (size_t)(row + u) * NC;
        for (int m = t; m < NC; m += T) {
            float2 v = make_float2(0.f, 0.f);
            if (live_[u]) {
                const double2 wm = pl.ld(m), wn = pl.ld((N - m) & (N - 1));
                const double zm = u == 0 ? wm.x : wm.y, zn = u == 0 ? wn.x : wn.y;
                double tr = 0.5 * (zm + zn), tp = A.pot ? 0.0 : 0.5 * (zn - zm);
                if (m == 1) {
                    tr += ind;
                    tp += ind;
                }
                v = make_float2((float)(scale * tr), (float)(scale * tp));
            }
            gstore2(o, m, v);
        }
    }
}

// ------------------------------------------------------- table: transpose
// src [nrows][ncol] (rows r0 + row of the (b, a, i', i) order) into the
// modes' layouts, 32 x 32 tiles: for a fixed mode consecutive rows are
// consecutive target columns in both layouts.
__global__ void __launch_bounds__(256)
k_ss_scatter(const float2 *src, int nrows, int ncol, float2 *coef, const SsMode *modes, size_t r0, int nr,
             int nrt)
{
    __shared__ float2 tile[32][33];
    const int rb = blockIdx.x * 32, mb = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {
        const int r = rb + k, m = mb + tx;
        if (r < nrows && m < ncol) tile[k][tx] = gload2(src, (size_t)r * ncol + m);
    }
    __syncthreads();
    const int r = rb + tx;
    if (r >= nrows) return;
    const size_t R = r0 + r;
    const int i = (int)(R % nrt);
    const size_t rest = R / nrt;
    const int ip = (int)(rest % nr);
    const size_t pair = rest / nr;  // b * F + a
    for (int k = ty; k < 32; k += 8) {
        const int m = mb + k;
        if (m >= ncol) break;
        const SsMode md = modes[m];
        size_t dst;
        if (md.banded) {
            const int d = ip - i + md.w;
            if (d < 0 || d > 2 * md.w) continue;
            dst = md.off + (pair * (2 * md.w + 1) + d) * nrt + i;
        } else {
            dst = md.off + (pair * nr + ip) * nrt + i;
        }
        gstore2(coef, dst, tile[tx][k]);
    }
}

// Mode descriptors (one thread; the same band rule as the host layout, with
// the host's du).
__global__ void k_ss_modes(SsMode *modes, int ncol, int nr, int nrt, int nf, double du, int full)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t off = 0;
    for (int m = 0; m < ncol; ++m) {
        const int w = sg_ss_band(m, nr, du, full != 0);
        const bool b = sg_ss_is_banded(w, nr);
        SsMode md;
        md.off = off;
        md.w = w;
        md.banded = b ? 1 : 0;
        modes[m] = md;
        off += (uint64_t)nf * nf * (b ? 2 * w + 1 : nr) * nrt;
    }
}

// Own-cell terms on a uniform radial grid, one item per (pair, ring): the
// cell spans X = ln(r'/r) in [ln(1 - dr/(2r)), ln(1 + dr/(2r))], no longer
// symmetric, so each side of X = 0 is integrated on its own (the integrand
// is integrable: ~1/rho for the field, logarithmic for the potential) with
// the Duffy triangles and geometric panels of the log-cell quadrature, and
// doubled for phi < 0 (both kernels are even in phi).  Output: the table
// sample I / (wgt dphi) (field, I = int K_r dX dphi) or -I / (wgt dphi)
// (potential, I = int P dA'), wgt = dr / r; which = 1, 2: their derivatives
// with respect to h_a, h_b instead.  per: cells per ring of H
// and out (1: one value per ring; n_phi: per cell, for the direct sum with
// per-cell H), item = pair * n_r * per + cell.
__global__ void __launch_bounds__(256)
k_ss_self_lin(const double *H, int nf, int nr, int per, double rmin, double dr, double dphi, int pot, int which,
              double *out, GLNodes gl)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int64_t cells = (int64_t)nr * per;
    const int64_t item = blockIdx.x;
    if (item >= nf * nf * cells) return;
    const int pair = (int)(item / cells), fa = pair / nf, fb = pair % nf;
    const int64_t c = item % cells;
    const int ir = (int)(c / per);
    const double r = rmin + (ir + 0.5) * dr;
    const double Ha = H[fa * cells + c], Hb = H[fb * cells + c];
    const double ha = Ha / r, hb = Hb / r, Hab = sqrt(0.5 * (Ha * Ha + Hb * Hb));
    const double b = 0.5 * dphi;
    constexpr int NX = SG_PANELS * SG_GLX_N;
    double acc = 0.0;
    for (int sd = 0; sd < 2; ++sd) {
        const double sgn = sd == 0 ? 1.0 : -1.0;
        const double a = sd == 0 ? log1p(0.5 * dr / r) : -log1p(-0.5 * dr / r);
        for (int idx = threadIdx.x; idx < NX * SG_GL_N; idx += blockDim.x) {
            const int ix = idx / SG_GL_N, j = idx % SG_GL_N;
            const int pnl = ix / SG_GLX_N, i = ix % SG_GLX_N;
            const double hi = ldexp(1.0, -2 * (SG_PANELS - 1 - pnl));
            const double lo = pnl == 0 ? 0.0 : 0.25 * hi;
            const double xi = lo + (hi - lo) * gl.xr[i];
            const double eta = gl.x[j];
            const double wgt = (hi - lo) * gl.wr[i] * gl.w[j] * xi * a * b;
            double f = 0.0;
            for (int tri = 0; tri < 2; ++tri) {
                const double X = sgn * (tri == 0 ? a * xi : a * xi * eta);
                const double phi = tri == 0 ? b * xi * eta : b * xi;
                if (pot) {
                    const double sx = sinh(0.5 * X), sp = sin(0.5 * phi);
                    const double s2 = r * r * exp(X) * 4.0 * (sx * sx + sp * sp);
                    const double y = s2 / (8.0 * Hab * Hab);
                    if (which == 0) {
                        f += -sg_G0_64(y, wq) / (2.0 * SG_SQRT_PI * Hab) * r * r * exp(2.0 * X);
                    } else {
                        // dP/dH_ab = -(2 y F(y) - G0(y)) / (2 sqrt(pi) H_ab^2), times dH_ab/dh
                        const double ch = (which == 1 ? Ha : Hb) * r / (2.0 * Hab);
                        f += -(2.0 * y * sg_F64(y, wq) - sg_G0_64(y, wq)) / (2.0 * SG_SQRT_PI * Hab * Hab) * ch *
                             r * r * exp(2.0 * X);
                    }
                } else {
                    double kr, kp;
                    sg_conv_kernel64(X, sin(0.5 * phi), sin(phi), ha, hb, which, wq, kr, kp);
                    f += kr;
                }
            }
            acc += wgt * f;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double I = 2.0 * red[0], w = (dr / r) * dphi;
        out[item] = pot ? -I / w : I / w;
    }
}

__global__ void k_ss_scale(double *p, int n, double f)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] *= f;
}

__global__ void k_ss_zero(float2 *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        gstore2(p, i, make_float2(0.f, 0.f));
}

__global__ void k_ss_header(sg_ss_header *hd, sg_ss_header proto)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *hd = proto;
}

// ------------------------------------------------------------- table: host
#define SG_SS_CHUNK_BYTES ((size_t)128 << 20)
#define SG_SS_MAX_NR 2048

int sg_ss_max_nr() { return SG_SS_MAX_NR; }

static size_t ss_chunk_rows(const SsLayout &L)
{
    const size_t per = sizeof(float2) * (size_t)L.ncol;
    size_t rows = SG_SS_CHUNK_BYTES / per;
    rows = rows / 32 * 32;
    if (rows < 32) rows = 32;
    return rows < L.rows ? rows : L.rows;
}

size_t sg_ss_ws_bytes(int nr, int nphi, int nf)
{
    const SsLayout L = sg_ss_layout(nr, nphi, nf, 1.0, true);
    return sg_align256(sizeof(double) * (size_t)nf * nf * nr) +
           sg_align256(sizeof(float2) * L.ncol * ss_chunk_rows(L));
}

template <int N>
static void launch_ss_rows(const double *H, const double *self, const SsRowArgs &A, size_t r0, int nrows,
                           float2 *out, hipStream_t s)
{
    using S = SsRowShape<N>;
    if (A.second)  // its own instance: the quadrature's registers stay out of the point-sampled rows
        hipLaunchKernelGGL((k_ss_rows<N, true>), dim3((nrows + S::G - 1) / S::G), dim3(S::WGS), 0, s, H, self,
                           A, r0, nrows, out);
    else  // two rows per group (nrows is even: see k_ss_rows)
        hipLaunchKernelGGL((k_ss_rows<N, false>), dim3((nrows + 2 * S::G - 1) / (2 * S::G)), dim3(S::WGS), 0, s,
                           H, self, A, r0, nrows, out);
}

static bool dispatch_ss_rows(int nphi, const double *H, const double *self, const SsRowArgs &A, size_t r0,
                             int nrows, float2 *out, hipStream_t s)
{
    switch (nphi) {
    case 4: launch_ss_rows<4>(H, self, A, r0, nrows, out, s); return true;
    case 8: launch_ss_rows<8>(H, self, A, r0, nrows, out, s); return true;
    case 16: launch_ss_rows<16>(H, self, A, r0, nrows, out, s); return true;
    case 32: launch_ss_rows<32>(H, self, A, r0, nrows, out, s); return true;
    case 64: launch_ss_rows<64>(H, self, A, r0, nrows, out, s); return true;
    case 128: launch_ss_rows<128>(H, self, A, r0, nrows, out, s); return true;
    case 256: launch_ss_rows<256>(H, self, A, r0, nrows, out, s); return true;
    case 512: launch_ss_rows<512>(H, self, A, r0, nrows, out, s); return true;
    case 1024: launch_ss_rows<1024>(H, self, A, r0, nrows, out, s); return true;
    case 2048: launch_ss_rows<2048>(H, self, A, r0, nrows, out, s); return true;
    default: return false;
    }
}

sg_status sg_ss_table_build(const sg_grid *grid, int nf, const double *d_H, uint32_t flags, void *d_table,
                            void *d_ws, hipStream_t s)
{
    const int nr = grid->n_r, nphi = grid->n_phi;
    const double du = sg_ss_du(*grid, flags);  // band rule (and log-grid spacing)
    const bool full = (flags & SG_SS_FULL) != 0;
    const bool lin = (flags & SG_LINEAR_R) != 0;
    const double dr = (grid->r_max - grid->r_min) / nr;
    const SsLayout L = sg_ss_layout(nr, nphi, nf, du, full);
    const double dphi = 2.0 * SG_PI / nphi;
    char *tb = (char *)d_table;
    double *self = (double *)d_ws;
    float2 *chunk = (float2 *)((char *)d_ws + sg_align256(sizeof(double) * (size_t)nf * nf * nr));
    const bool excl = (flags & SG_SELF_CELL_EXCLUDE) != 0;
    const bool second = (flags & SG_SECOND_ORDER) != 0;  // log grid, force operators

    hipLaunchKernelGGL(k_twiddles, dim3((nphi + 255) / 256), dim3(256), 0, s, (float2 *)nullptr, 0,
                       (float2 *)(tb + L.off_tw_phi), nphi);
    SG_HIP(hipGetLastError());
    SsMode *modes = (SsMode *)(tb + L.off_modes);
    hipLaunchKernelGGL(k_ss_modes, dim3(1), dim3(64), 0, s, modes, L.ncol, nr, L.nrt, nf, du, full ? 1 : 0);
    SG_HIP(hipGetLastError());
    float2 *coef = (float2 *)(tb + L.off_coef);
    if (L.max_w >= 0) {  // banded modes: entries the scatter does not reach stay zero
        hipLaunchKernelGGL(k_ss_zero, dim3(2048), dim3(256), 0, s, coef, L.coef_elems);
        SG_HIP(hipGetLastError());
    }
    const bool pot = (flags & SG_POTENTIAL) != 0;
    if (!excl && !second) {  // second order: the own cell is a hat weight of the rows
        // one item per (pair, ring): the per-cell quadratures with one cell per ring
        GLNodes gl;
        sg_gl_nodes(gl);
        if (lin) {
            hipLaunchKernelGGL(k_ss_self_lin, dim3(nf * nf * nr), dim3(256), 0, s, d_H, nf, nr, 1, grid->r_min, dr,
                               dphi, pot ? 1 : 0, 0, self, gl);
        } else if (pot) {
            hipLaunchKernelGGL(k_pot_self<double>, dim3(nf * nf * nr), dim3(256), 0, s, d_H, (const double *)nullptr,
                               nf, nr, 1, log(grid->r_min), du, dphi, 0, self, gl, 0);
            SG_HIP(hipGetLastError());
            // own-cell integral I of P: the sample -I / (du dphi) scales to I / N
            hipLaunchKernelGGL(k_ss_scale, dim3((nf * nf * nr + 255) / 256), dim3(256), 0, s, self, nf * nf * nr,
                               -1.0 / (du * dphi));
        } else {
            hipLaunchKernelGGL(k_self_cell_percell<double>, dim3(nf * nf * nr), dim3(256), 0, s, d_H, nf, nr, 1,
                               log(grid->r_min), du, dphi, self, gl);
        }
        SG_HIP(hipGetLastError());
    }
    SsRowArgs A;
    A.nr = nr;
    A.nrt = L.nrt;
    A.nf = nf;
    A.excl = excl ? 1 : 0;
    A.ind = (flags & SG_INDIRECT) ? 1 : 0;
    A.pot = pot ? 1 : 0;
    A.lnrmin = log(grid->r_min);
    A.du = du;
    A.dphi = dphi;
    A.lin = lin ? 1 : 0;
    A.rmin = grid->r_min;
    A.dr = dr;
    A.second = second ? 1 : 0;
    sg_gl_nodes(A.gl);
    const size_t crows = ss_chunk_rows(L);
    for (size_t r0 = 0; r0 < L.rows; r0 += crows) {
        const int n = (int)std::min(crows, L.rows - r0);
        if (!dispatch_ss_rows(nphi, d_H, self, A, r0, n, chunk, s)) return SG_ERR_UNSUPPORTED;
        SG_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_ss_scatter, dim3((n + 31) / 32, (L.ncol + 31) / 32), dim3(256), 0, s, chunk, n,
                           L.ncol, coef, (const SsMode *)modes, r0, nr, L.nrt);
        SG_HIP(hipGetLastError());
    }
    sg_ss_header proto{};
    proto.magic = SG_SS_MAGIC;
    proto.version = 1;
    proto.n_r = nr;
    proto.n_phi = nphi;
    proto.n_fluids = nf;
    proto.flags = flags | SG_SEMI_SPECTRAL;
    proto.r_min = grid->r_min;
    proto.r_max = grid->r_max;
    proto.du = du;
    proto.total_bytes = L.total;
    hipLaunchKernelGGL(k_ss_header, dim3(1), dim3(1), 0, s, (sg_ss_header *)tb, proto);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// ------------------------------------------------------------ middle pass
// 16-byte load of two consecutive complex values at element offset i of a
// wave-uniform base (i even); NT: non-temporal (the operators are read once
// per solve, so they need not displace Sigma~ and g^ in the caches).
template <bool NT>
__device__ inline void ss_ld4(const float2 *p, uint32_t i, float2 &x, float2 &y)
{
    const sg_gcv4f *q = (const sg_gcv4f *)((const char *)p + (i << 3));
    sg_v4f v;
    if constexpr (NT) v = __builtin_nontemporal_load(q);
    else v = *q;
    x = make_float2(v.x, v.y);
    y = make_float2(v.z, v.w);
}

// Workgroup job (disc, m, b, target block): 256 threads in S row splits of
// LN = 256 / S lanes; lane l owns targets i0 .. i0 + V - 1, i0 = block TB +
// V l (TB = LN V), and split s sums the operator rows k = s (mod S) of every
// source fluid (source rows of a full mode, diagonals of a banded one); the
// splits are combined through LDS.  Sigma~_a(m, .) is staged in LDS first:
// the whole column for a full mode; for a banded mode the window of sources
// the block's targets reach, from blk TB - w (zero outside the grid), so
// that target i0 + v reads source i0 + v + d - w at window index V l + v + d.  The operator rows
// are streamed once with 16-byte loads, U rows in flight: this pass is bound
// by reading the table.
template <int NF, int V, int S, bool NT, int U>
__global__ void __launch_bounds__(256) k_ss_pass(const DiscDev *discs, const WJob *wj, int nj, const float2 *,
                                                 int kc)
{
    extern __shared__ __attribute__((aligned(16))) float2 ssh[];
    constexpr int LN = 256 / S, TB = LN * V;
    static_assert(V % 2 == 0, "targets per lane come in 16-byte pairs");
    const int w = sg_uniform(sg_xcd_remap(blockIdx.x, kc));
    if (w >= nj) return;
    if (sg_uniform(wj[w].n) == 0) return;  // cluster padding
    const int cd = sg_uniform(wj[w].disc), idx = sg_uniform(wj[w].base);
    const DiscDev *D = discs + cd;
    const int nr = D->nr, nrt = (nr + 1) & ~1, nb = (nr + TB - 1) / TB;
    const int blk = idx % nb, mb = idx / nb, b = mb % NF, m = mb / NF;
    const size_t fs = sg_blk_field_elems(D->nphi, nr);
    const SsMode md = D->modes[m];
    const bool banded = sg_uniform(md.banded) != 0;
    const int bw = banded ? sg_uniform(md.w) : 0;
    // staged sources: a full mode's whole column, a banded mode's window
    // [blk TB - w, blk TB + TB + w + 4) (zero outside the grid)
    const int cs = banded ? TB + 2 * bw + 4 : nr;
    const int nk = banded ? 2 * bw + 1 : nr;        // operator rows per (b, a)
    const int base = banded ? blk * TB - bw : 0;
    if (banded && bw > D->ss_wmax) return;  // table not built for this grid: never overrun the LDS
    for (int e = threadIdx.x; e < NF * cs; e += 256) {
        const int a = e / cs, ip = e - a * cs + base;
        ssh[e] = (ip >= 0 && ip < nr) ? gld2(D->st + a * fs, (uint32_t)sg_blk_index(m, ip, nr))
                                      : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int ln = threadIdx.x % LN, sp = threadIdx.x / LN;
    const int i0 = blk * TB + V * ln;
    // column of each target pair (pairs past the last row read column 0) and
    // each target's staged index (targets past the last row read index 0)
    uint32_t col[V / 2];
    int ie[V];
#pragma unroll
    for (int v = 0; v < V; v += 2) col[v / 2] = i0 + v < nr ? (uint32_t)(i0 + v) : 0u;
#pragma unroll
    for (int v = 0; v < V; ++v) ie[v] = i0 + v < nr ? V * ln + v : 0;
    float2 ar[V], ap[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ar[v] = ap[v] = make_float2(0.f, 0.f);
    const float2 *C = D->spec + md.off;
    for (int a = 0; a < NF; ++a) {
        const float2 *Tm = C + (size_t)(b * NF + a) * nk * nrt;
        const float2 *sa = ssh + a * cs;
        int k = sp;
        for (; k + S * (U - 1) < nk; k += S * U) {
            float2 t[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int v = 0; v < V; v += 2)
                    ss_ld4<NT>(Tm, (uint32_t)(k + S * u) * nrt + col[v / 2], t[u][v], t[u][v + 1]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    // full: source row k (all targets); banded: diagonal k
                    const float2 s = banded ? sa[ie[v] + k + S * u] : sa[k + S * u];
                    ar[v].x += t[u][v].x * s.x;
                    ar[v].y += t[u][v].x * s.y;
                    ap[v].x += t[u][v].y * s.x;
                    ap[v].y += t[u][v].y * s.y;
                }
            }
        }
        for (; k < nk; k += S) {
            float2 t[V];
#pragma unroll
            for (int v = 0; v < V; v += 2) ss_ld4<NT>(Tm, (uint32_t)k * nrt + col[v / 2], t[v], t[v + 1]);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float2 s = banded ? sa[ie[v] + k] : sa[k];
                ar[v].x += t[v].x * s.x;
                ar[v].y += t[v].x * s.y;
                ap[v].x += t[v].y * s.x;
                ap[v].y += t[v].y * s.y;
            }
        }
    }
    if constexpr (S > 1) {
        // combine the row splits: partials after the staged columns
        float2 *red = ssh + ((NF * cs + 1) & ~1);
        if (sp > 0) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                red[((sp - 1) * LN + ln) * 2 * V + 2 * v] = ar[v];
                red[((sp - 1) * LN + ln) * 2 * V + 2 * v + 1] = ap[v];
            }
        }
        __syncthreads();
        if (sp > 0) return;
#pragma unroll
        for (int q = 0; q < S - 1; ++q)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const float2 x = red[(q * LN + ln) * 2 * V + 2 * v], y = red[(q * LN + ln) * 2 * V + 2 * v + 1];
                ar[v].x += x.x;
                ar[v].y += x.y;
                ap[v].x += y.x;
                ap[v].y += y.y;
            }
    }
    float2 *gr = D->gh + (size_t)(b * 2) * fs, *gp = gr + fs;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int i = i0 + v;
        if (i < nr) {
            const uint32_t o = (uint32_t)sg_blk_index(m, i, nr);
            gst2(gr, o, ar[v]);
            gst2(gp, o, make_float2(-ap[v].y, ap[v].x));  // i t_phi Sigma~
        }
    }
}

template <int NF, int V, int S, bool NT = false, int U = 8> static SsPassInfo ss_info()
{
    constexpr int LN = 256 / S;
    SsPassInfo k;
    k.fn = k_ss_pass<NF, V, S, NT, U>;
    k.wgs = 256;
    k.tb = LN * V;
    k.lds_per_row = NF * (int)sizeof(float2);
    // column padded to an even count, then the split partials
    k.lds_fixed = (int)sizeof(float2) * (1 + (S > 1 ? (S - 1) * LN * 2 * V : 0));
    return k;
}

template <int NF> static bool ss_variant(int variant, SsPassInfo &out)
{
    switch (variant) {
    case 1: out = ss_info<NF, 2, 4, true>(); return true;
    case 2: out = ss_info<NF, 2, 1>(); return true;
    case 3: out = ss_info<NF, 4, 1>(); return true;
    case 4: out = ss_info<NF, 2, 4>(); return true;
    default: return false;
    }
}

bool sg_ss_pass_kernel(int nf, int variant, SsPassInfo &out)
{
    switch (nf) {
    case 1: return ss_variant<1>(variant, out);
    case 2: return ss_variant<2>(variant, out);
    case 3: return ss_variant<3>(variant, out);
    case 4: return ss_variant<4>(variant, out);
    default: return false;
    }
}

// Row splits with 128 targets per job and non-temporal operator loads
// measured fastest on every grid tried (256 x 512 to 1200 x 2048: many jobs
// per mode, short banded windows, Sigma~ and g^ kept in the caches); the
// autotuner tries the other shapes.
int sg_ss_default_variant(int) { return 1; }

// ------------------------------------------------ dL/dH (gradient in H(r))
// For L with dL/dg_r = lam_r, dL/dg_phi = lam_phi, the derivative with
// respect to the ring scale heights follows from differentiating every
// operator entry: T^{ab}(m, i, i') depends on h_a = H_a(r_i')/r_i' (source)
// and h_b = H_b(r_i)/r_i (target), the own-cell entry on both at its ring,
// and mode 1 on H_a(r_i') through the folded indirect term.  Since g is the
// inverse transform of the per-mode products,
//   dL/dtheta = sum_m w_m Re[conj(lam~_r) dT_r Sigma~ + conj(lam~_phi) i dt_phi Sigma~]
// (w_m = 1 for m = 0, n_phi/2 and 2 otherwise: the stored half of a
// Hermitian spectrum), accumulated per (b, a, i', i) row and added to
// dL/dh_a(i') and dL/dh_b(i) in double; finally dL/dH = (dL/dh) / r.  The
// derivative rows are sampled and transformed on the fly (the table's own
// construction with the kernels' h derivatives), never stored.

// Half spectra of lam rows (b, i) (r and phi parts) and of Sigma row pairs.
template <int N>
__global__ void __launch_bounds__(SsRowShape<N>::WGS)
k_ssg_phi(const float *lam_r, const float *lam_p, const float *sigma, const float2 *tw, float2 *lt, float2 *st,
          int nr, int nf)
{
    using S = SsRowShape<N>;
    constexpr int T = S::T, G = S::G, W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * G];
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    const int hp = (nr + 1) / 2, nl = nf * nr, count = nl + nf * hp;
    const int idx = blockIdx.x * G + g;
    const bool valid = idx < count;
    const int j = valid ? idx : 0;
    const size_t fs = sg_blk_field_elems(N, nr);
    const LdsPlane<float> pl{lds + W * g};
    const float *x1, *x2;
    float2 *d1, *d2;
    int i1, i2;
    if (j < nl) {
        const int b = j / nr, i = j % nr;
        x1 = lam_r + ((size_t)b * nr + i) * N;
        x2 = lam_p + ((size_t)b * nr + i) * N;
        d1 = lt + (size_t)(2 * b) * fs;
        d2 = d1 + fs;
        i1 = i2 = i;
    } else {
        const int q = j - nl, a = q / hp, jj = q % hp;
        i1 = 2 * jj;
        i2 = min(2 * jj + 1, nr - 1);
        x1 = sigma + ((size_t)a * nr + i1) * N;
        x2 = sigma + ((size_t)a * nr + i2) * N;
        d1 = d2 = st + (size_t)a * fs;
    }
    phi_fwd_pair<N>(x1, x2, d1, i1, d2, i2, nr, TwTable{tw}, t, pl, valid);
}

// One group of T threads per (b, a, i', i) row: for which = 1 (d/dh_a,
// source) and 2 (d/dh_b, target) the derivative samples are transformed as
// in k_ss_rows and contracted with lam~ and Sigma~ of the row's mode column.
// SO: the rows of second-order operators, whose samples are the h
// derivatives of the hat weights (k_ss_rows<N, true>: integrated near the
// singular point, point value plus second moments beyond; both are linear
// in the kernel, so they apply to its derivatives sample by sample).
template <int N, bool SO>
__global__ void __launch_bounds__(SsRowShape<N>::WGS)
k_ssg_rows(const double *H, const double *dself, SsRowArgs A, const float2 *lt, const float2 *st, size_t r0,
           int nrows, double *rowpart)
{
    using S = SsRowShape<N>;
    constexpr int P = S::P, T = S::T, G = S::G, W = LdsPlane<double>::elems(N);
    constexpr int NC = N / 2 + 1;
    __shared__ __attribute__((aligned(16))) double2 lds[W * G];
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[S::WGS];
    __shared__ double2 qres[SO ? 2 * NC * G : 1];  // SO: the group's integrated samples, both derivatives
    __shared__ int qmax_wg;
    sg_fill_weights<double>(wq);
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    const LdsPlane<double> pl{lds + W * g};
    const int row = blockIdx.x * G + g;
    const bool valid = row < nrows;
    const size_t R = r0 + (size_t)(valid ? row : 0);
    const int i = (int)(R % A.nrt);
    size_t rest = R / A.nrt;
    const int ip = (int)(rest % A.nr);
    rest /= A.nr;
    const int a = (int)(rest % A.nf), b = (int)(rest / A.nf);
    const bool live = valid && i < A.nr;
    const int ic = i < A.nr ? i : A.nr - 1;
    const double ri = A.lin ? A.rmin + (ic + 0.5) * A.dr : exp(A.lnrmin + (ic + 0.5) * A.du);
    const double rp = A.lin ? A.rmin + (ip + 0.5) * A.dr : exp(A.lnrmin + (ip + 0.5) * A.du);
    const double ha = H[a * A.nr + ip] / rp, hb = H[b * A.nr + ic] / ri;
    const double X = A.lin ? log(ri / rp) : (double)(ic - ip) * A.du;
    const double scale = -(A.lin ? A.dr / rp : A.du) * A.dphi / N;
    const uint32_t fs = (uint32_t)sg_blk_field_elems(N, A.nr);
    __syncthreads();
    // Both derivatives are sampled in one sweep (one F, F' evaluation per
    // azimuth) and transformed together.  Row d is z_d = K_r,d + i K_phi,d
    // with K_r even and K_phi odd in phi, so its transform Z_d is real; the
    // plane holds z = z_1 + i z_2, whose transform carries Z_1 (d/dh_a) in
    // its real part and Z_2 (d/dh_b) in its imaginary part.
    constexpr int Q = P / 2 + 1;
    if constexpr (SO) {
        // integrated samples, cooperatively (as in k_ss_rows<N, true>)
        const int Pr = ic - ip;
        const double rn = SG_SS_HAT_NEAR * fmax(A.du, A.dphi), xq = Pr * A.du;
        int qn = -1;
        if (live && xq * xq < rn * rn)
            while (qn < N / 2 && xq * xq + ((qn + 1) * A.dphi) * ((qn + 1) * A.dphi) < rn * rn) ++qn;
        if (threadIdx.x == 0) qmax_wg = -1;
        __syncthreads();
        if (t == 0 && qn >= 0) atomicMax(&qmax_wg, qn);
        __syncthreads();
        const int qm = qmax_wg;
        for (int q = 0; q <= qm; ++q) {
            for (int d = 1; d <= 2; ++d) {
                double wr = 0.0, wp = 0.0;
                if (q <= qn) sg_hat_weight_part(Pr, q, A.du, A.dphi, ha, hb, d, A.gl, wq, t, T, wr, wp);
                pl.st(t, make_double2(wr, wp));
                __syncthreads();
                if (q <= qn && t == 0) {
                    double sr = 0.0, sp = 0.0;
                    for (int k = 0; k < T; ++k) {
                        const double2 v = pl.ld(k);
                        sr += v.x;
                        sp += v.y;
                    }
                    qres[(g * 2 + (d - 1)) * NC + q] = make_double2(sr, sp);
                }
                __syncthreads();
            }
        }
        // point values of the packed derivative rows (for the neighbours),
        // and the second-order samples in registers: vq at q, vm at N - q
        double2 vq[Q], vm[Q];
        unsigned taylor = 0u;
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int q = t + T * u;
            vq[u] = make_double2(0.0, 0.0);
            vm[u] = make_double2(0.0, 0.0);
            if (q > N / 2) continue;
            const double sh = sinpi((double)q / N), s2 = sinpi(2.0 * q / N);
            double kr1 = 0.0, kp1 = 0.0, kr2 = 0.0, kp2 = 0.0;
            if (Pr != 0 || q != 0) sg_conv_kernel64_dh(X, sh, s2, ha, hb, wq, kr1, kp1, kr2, kp2);
            if (q <= qn) {
                const double2 w1 = qres[(g * 2 + 0) * NC + q], w2 = qres[(g * 2 + 1) * NC + q];
                vq[u] = make_double2(w1.x - w2.y, w1.y + w2.x);
                vm[u] = make_double2(w1.x + w2.y, w2.x - w1.y);
            } else {
                // D_X^2 of the packed rows: samples at X +- du
                double a1, b1, c1, e1, a2, b2, c2, e2;
                sg_conv_kernel64_dh(X + A.du, sh, s2, ha, hb, wq, a1, b1, c1, e1);
                sg_conv_kernel64_dh(X - A.du, sh, s2, ha, hb, wq, a2, b2, c2, e2);
                const double dr1 = a1 - 2.0 * kr1 + a2, dp1 = b1 - 2.0 * kp1 + b2;
                const double dr2 = c1 - 2.0 * kr2 + c2, dp2 = e1 - 2.0 * kp2 + e2;
                vq[u] = make_double2(kr1 - kp2 + (dr1 - dp2) / 12.0, kp1 + kr2 + (dp1 + dr2) / 12.0);
                vm[u] = make_double2(kr1 + kp2 + (dr1 + dp2) / 12.0, kr2 - kp1 + (dr2 - dp1) / 12.0);
                taylor |= 1u << u;
            }
            pl.st(q, make_double2(kr1 - kp2, kp1 + kr2));
            if (q != 0 && q != N / 2) pl.st(N - q, make_double2(kr1 + kp2, kr2 - kp1));
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int q = t + T * u;
            if (q > N / 2 || !((taylor >> u) & 1u)) continue;
            // D_phi^2 at q and at the mirror N - q (the plane holds the
            // packed rows on the whole circle)
            const double2 z0 = pl.ld(q), zl = pl.ld((q + N - 1) & (N - 1)), zh = pl.ld((q + 1) & (N - 1));
            vq[u].x += (zl.x - 2.0 * z0.x + zh.x) / 12.0;
            vq[u].y += (zl.y - 2.0 * z0.y + zh.y) / 12.0;
            if (q != 0 && q != N / 2) {
                const int qm2 = N - q;
                const double2 y0 = pl.ld(qm2), yl = pl.ld(qm2 - 1), yh = pl.ld((qm2 + 1) & (N - 1));
                vm[u].x += (yl.x - 2.0 * y0.x + yh.x) / 12.0;
                vm[u].y += (yl.y - 2.0 * y0.y + yh.y) / 12.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < Q; ++u) {
            const int q = t + T * u;
            if (q > N / 2) continue;
            pl.st(q, vq[u]);
            if (q != 0 && q != N / 2) pl.st(N - q, vm[u]);
        }
    } else {
#pragma unroll
    for (int u = 0; u < Q; ++u) {
        const int q = t + T * u;
        if (q > N / 2) break;
        double kr1 = 0.0, kp1 = 0.0, kr2 = 0.0, kp2 = 0.0;
        if (ic == ip && q == 0) {
            if (!A.excl) {
                const size_t o = (size_t)(a * A.nf + b) * A.nr + ic, wst = (size_t)A.nf * A.nf * A.nr;
                kr1 = dself[o];
                kr2 = dself[wst + o];
            }
        } else if (A.pot) {
            // d/dh of r'^2 G0(y) / (2 sqrt(pi) H_ab) (the forward's sample):
            // d(G0/H)/dH = (2 y F(y) - G0(y)) / H^2, dH_ab/dh_a = H_a r' / (2 H_ab),
            // dH_ab/dh_b = H_b r_i / (2 H_ab); even in phi (no K_phi part)
            const double sx = sinh(0.5 * X), sp = sinpi((double)q / N);
            const double s2 = 4.0 * ri * rp * (sx * sx + sp * sp);
            const double Ha = ha * rp, Hb = hb * ri, Hab2 = 0.5 * (Ha * Ha + Hb * Hb), Hab = sqrt(Hab2);
            const double y = s2 / (8.0 * Hab2);
            const double dq = rp * rp * (2.0 * y * sg_F64(y, wq) - sg_G0_64(y, wq)) / (2.0 * SG_SQRT_PI * Hab2);
            kr1 = dq * Ha * rp / (2.0 * Hab);
            kr2 = dq * Hb * ri / (2.0 * Hab);
        } else {
            sg_conv_kernel64_dh(X, sinpi((double)q / N), sinpi(2.0 * q / N), ha, hb, wq, kr1, kp1, kr2, kp2);
        }
        pl.st(q, make_double2(kr1 - kp2, kp1 + kr2));
        if (q != 0 && q != N / 2) pl.st(N - q, make_double2(kr1 + kp2, kr2 - kp1));
    }
    }
    __syncthreads();
    double2 z[P];
#pragma unroll
    for (int p = 0; p < P; ++p) z[p] = pl.ld(t + T * p);
    __syncthreads();
    fft<N, false>(z, t, pl, TwPow64<N>{t});
#pragma unroll
    for (int p = 0; p < P; ++p) pl.st(t + T * p, z[p]);
    __syncthreads();
    double dind = 0.0;
    if (A.ind) {
        // d/dh_a of r'^2 sqrt(2) K_a(r'/H_a) n_phi / 2, H_a = h_a r':
        // dK_a/dH = pi^{-1/2} r' / (4 H^4) (-3 F(x) - 2 x F'(x)), x = r'^2 / (4 H^2)
        const double Ha = ha * rp, x = rp * rp / (4.0 * Ha * Ha);
        double F, dF;
        sg_F64_dF(x, wq, F, dF);
        const double dK = (1.0 / SG_SQRT_PI) * rp / (4.0 * Ha * Ha * Ha * Ha) * (-3.0 * F - 2.0 * x * dF);
        dind = rp * rp * SG_SQRT2 * dK * rp * (0.5 * N);
    }
    double part[2] = {0.0, 0.0};
    if (live) {
        for (int m = t; m < NC; m += T) {
            const double2 zm = pl.ld(m), zn = pl.ld((N - m) & (N - 1));
            const uint32_t oi = (uint32_t)sg_blk_index(m, ic, A.nr), op = (uint32_t)sg_blk_index(m, ip, A.nr);
            const float2 lr = gld2(lt, (uint32_t)(2 * b) * fs + oi), lp = gld2(lt, (uint32_t)(2 * b + 1) * fs + oi);
            const float2 sv = gld2(st, (uint32_t)a * fs + op);
            // Re[conj(lr) T_r s] + Re[conj(lp) i t_phi s]
            const double cr = (double)lr.x * sv.x + (double)lr.y * sv.y;
            const double cp = -(double)lp.x * sv.y + (double)lp.y * sv.x;
            const double wm = ((m == 0 || m == N / 2) ? 1.0 : 2.0) * scale;
            double tr = 0.5 * (zm.x + zn.x), tp = A.pot ? 0.0 : 0.5 * (zn.x - zm.x);
            if (m == 1) {
                tr += dind;
                tp += dind;
            }
            part[0] += wm * (tr * cr + tp * cp);
            part[1] += wm * (0.5 * (zm.y + zn.y) * cr + (A.pot ? 0.0 : 0.5 * (zn.y - zm.y)) * cp);
        }
    }
    __syncthreads();
    // per-group sums, stored per row (part 0 belongs to dL/dh_a at the source
    // ring, part 1 to dL/dh_b at the target ring); k_ssg_finish adds them up
    for (int d = 0; d < 2; ++d) {
        red[threadIdx.x] = part[d];
        __syncthreads();
        for (int o = T / 2; o > 0; o >>= 1) {
            if (t < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (t == 0 && live) rowpart[2 * R + d] = red[threadIdx.x];
        __syncthreads();
    }
}

// dL/dH_f(r_k) = (1/r_k) dL/dh_f(r_k): the row partials that touch ring k of
// group f, in a fixed order (so the result is the same on every call).
// Row R = ((b nf + a) nr + i') nrt + i; ring k of group f is the source ring
// of rows (b, f, k, i) and the target ring of rows (f, a, i', k).
__global__ void __launch_bounds__(256) k_ssg_finish(const double *rowpart, SsRowArgs A, double *dH)
{
    __shared__ double red[256];
    const int f = blockIdx.x / A.nr, k = blockIdx.x % A.nr;
    const int n = A.nf * A.nr;
    double s = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const int o = j / A.nr, x = j % A.nr;
        s += rowpart[2 * ((((size_t)o * A.nf + f) * A.nr + k) * A.nrt + x)];
        s += rowpart[2 * ((((size_t)f * A.nf + o) * A.nr + x) * A.nrt + k) + 1];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double r = A.lin ? A.rmin + (k + 0.5) * A.dr : exp(A.lnrmin + (k + 0.5) * A.du);
        dH[blockIdx.x] = red[0] / r;
    }
}

struct SsGradWs {
    size_t lt, st, dself, rowpart, total;
};

static SsGradWs ssg_ws(int nr, int nphi, int nf)
{
    const size_t fs = sg_blk_field_elems(nphi, nr);
    const size_t rows = (size_t)nf * nf * nr * ((nr + 1) & ~1);
    SsGradWs w;
    w.lt = 0;
    w.st = sg_align256(sizeof(float2) * fs * 2 * nf);
    w.dself = w.st + sg_align256(sizeof(float2) * fs * nf);
    w.rowpart = w.dself + sg_align256(sizeof(double) * 2 * nf * nf * nr);
    w.total = w.rowpart + sg_align256(sizeof(double) * 2 * rows);
    return w;
}

size_t sg_ss_grad_ws_bytes(int nr, int nphi, int nf) { return ssg_ws(nr, nphi, nf).total; }

template <int N>
static void launch_ssg(const double *H, const double *dself, const SsRowArgs &A, const float *lam_r,
                       const float *lam_p, const float *sigma, const float2 *tw, float2 *lt, float2 *st,
                       double *rowpart, hipStream_t s)
{
    using S = SsRowShape<N>;
    const int nphi_jobs = A.nf * A.nr + A.nf * ((A.nr + 1) / 2);
    hipLaunchKernelGGL(k_ssg_phi<N>, dim3((nphi_jobs + S::G - 1) / S::G), dim3(S::WGS), 0, s, lam_r, lam_p,
                       sigma, tw, lt, st, A.nr, A.nf);
    const size_t rows = (size_t)A.nf * A.nf * A.nr * A.nrt;
    const size_t chunk = (size_t)1 << 22;
    for (size_t r0 = 0; r0 < rows; r0 += chunk) {
        const int n = (int)std::min(chunk, rows - r0);
        if (A.second)
            hipLaunchKernelGGL((k_ssg_rows<N, true>), dim3((n + S::G - 1) / S::G), dim3(S::WGS), 0, s, H, dself,
                               A, lt, st, r0, n, rowpart);
        else
            hipLaunchKernelGGL((k_ssg_rows<N, false>), dim3((n + S::G - 1) / S::G), dim3(S::WGS), 0, s, H, dself,
                               A, lt, st, r0, n, rowpart);
    }
}

sg_status sg_ss_grad_run(const sg_disc &d0, const double *d_H, const float *lam_r, const float *lam_p, double *dH,
                         void *d_ws, hipStream_t s)
{
    // species discs: the derivative of the group disc at the group sums
    // (placed after the gradient's own workspace)
    sg_disc d = d0;
    if (d0.n_species) {
        float *gsig = (float *)((char *)d_ws + sg_ss_grad_ws_bytes(d0.grid.n_r, d0.grid.n_phi, d0.fluids.n_fluids));
        const sg_status st = sg_species_group_sums(d0, gsig, s);
        if (st != SG_OK) return st;
        d.n_species = 0;
        d.sigma = gsig;
    }
    const sg_grid *grid = &d.grid;
    const int nr = grid->n_r, nphi = grid->n_phi, nf = d.fluids.n_fluids;
    const uint32_t flags = d.flags;
    const bool lin = (flags & SG_LINEAR_R) != 0;
    const SsLayout L = sg_ss_layout(nr, nphi, nf, sg_ss_du(*grid, flags), (flags & SG_SS_FULL) != 0);
    const float2 *tw = (const float2 *)((const char *)d.table + L.off_tw_phi);
    const SsGradWs W = ssg_ws(nr, nphi, nf);
    char *ws = (char *)d_ws;
    float2 *lt = (float2 *)(ws + W.lt), *st = (float2 *)(ws + W.st);
    double *dself = (double *)(ws + W.dself), *rowpart = (double *)(ws + W.rowpart);
    const double dphi = 2.0 * SG_PI / nphi;
    SsRowArgs A;
    A.nr = nr;
    A.nrt = L.nrt;
    A.nf = nf;
    A.excl = (flags & SG_SELF_CELL_EXCLUDE) ? 1 : 0;
    A.ind = (flags & SG_INDIRECT) ? 1 : 0;
    A.pot = (flags & SG_POTENTIAL) ? 1 : 0;
    A.lin = lin ? 1 : 0;
    A.lnrmin = log(grid->r_min);
    A.du = log(grid->r_max / grid->r_min) / nr;
    A.dphi = dphi;
    A.rmin = grid->r_min;
    A.dr = (grid->r_max - grid->r_min) / nr;
    A.second = (flags & SG_SECOND_ORDER) ? 1 : 0;
    sg_gl_nodes(A.gl);
    if (!A.excl && !A.second) {  // second order: the own cell is one of the integrated samples
        GLNodes gl;
        sg_gl_nodes(gl);
        for (int which = 1; which <= 2; ++which) {
            double *out = dself + (size_t)(which - 1) * nf * nf * nr;
            if (lin) {
                hipLaunchKernelGGL(k_ss_self_lin, dim3(nf * nf * nr), dim3(256), 0, s, d_H, nf, nr, 1, grid->r_min,
                                   A.dr, dphi, A.pot, which, out, gl);
            } else if (A.pot) {
                hipLaunchKernelGGL(k_pot_self<double>, dim3(nf * nf * nr), dim3(256), 0, s, d_H,
                                   (const double *)nullptr, nf, nr, 1, A.lnrmin, A.du, dphi, 0, out, gl, which);
                SG_HIP(hipGetLastError());
                // as the forward's own-cell sample: -I / (du dphi)
                hipLaunchKernelGGL(k_ss_scale, dim3((nf * nf * nr + 255) / 256), dim3(256), 0, s, out, nf * nf * nr,
                                   -1.0 / (A.du * dphi));
            } else {
                hipLaunchKernelGGL(k_self_cell_ring, dim3(nf * nf * nr), dim3(256), 0, s, d_H, nf, nr, A.lnrmin,
                                   A.du, dphi, which, out, gl);
            }
            SG_HIP(hipGetLastError());
        }
    }
    switch (nphi) {
    case 4: launch_ssg<4>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 8: launch_ssg<8>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 16: launch_ssg<16>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 32: launch_ssg<32>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 64: launch_ssg<64>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 128: launch_ssg<128>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 256: launch_ssg<256>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 512: launch_ssg<512>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 1024: launch_ssg<1024>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    case 2048: launch_ssg<2048>(d_H, dself, A, lam_r, lam_p, d.sigma, tw, lt, st, rowpart, s); break;
    default: return SG_ERR_UNSUPPORTED;
    }
    SG_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ssg_finish, dim3(nf * nr), dim3(256), 0, s, rowpart, A, dH);
    SG_HIP(hipGetLastError());
    return SG_OK;
}
