/*
 * sg_oracle.c -- CPU FP64 reference ("oracle") for the exact thin-disc
 * self-gravity kernel of Rendon Restrepo, Rometsch, Ziegler & Gressel,
 * "Self-gravity in thin protoplanetary discs 1" (arXiv 2506.10812).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header, table or constant
 * with the HIP library; both sides only receive the same seeded inputs.
 *
 * Every term is evaluated in plain double precision, written to be checked
 * by eye against the paper; the field, potential, adjoint and indirect sums
 * accumulate those terms in long double (x87 extended precision, 64-bit
 * significand) in the plain order of the definition, so that the order of
 * summation adds nothing measurable to the rounding of the terms themselves
 * (a double running sum over 10^4 - 10^6 terms of both signs sits about
 * 1e-12 from the exact sum of its terms, which is the size of the FP64
 * accuracy bar).  Speed is obtained only from OpenMP over target cells and
 * from a contiguous inner loop; no blocking or reordering of the sums.
 *
 * Discrete problem (readings of points the paper leaves open are marked
 * "reading"):
 *   grid      log-spaced radial cell edges r_min..r_max (reading: the range
 *             gives cell edges), centres u_i = ln r_min + (i+1/2) du,
 *             du = ln(r_max/r_min)/N_r; phi_j = (j+1/2) dphi, dphi = 2 pi/N_phi
 *             (the log-r x uniform-phi grid of Sect. 5.2 / App. C).
 *   area      A_i = r_i^2 du dphi (midpoint rule in u; reading).
 *   field     g^{a->b}(x_i) = - sum_{k != i} Sigma_a[k] A_k K_ab(s_ik) e_s
 *             (Eq. "volume force 2D" of Sect. 2.2 divided by Sigma_b; the
 *             target fluid b sits at x_i, the source fluid a at x_k) plus a
 *             self-cell term (reading: the principal-value cell average of
 *             the log-polar radial kernel over the own cell; the paper does
 *             not discuss the k = i term).
 *   kernel    K_ab = pi^{-1/2} H_ab^{-2} (d/8) e^x [K1(x) - K0(x)],
 *             x = d^2/8, d = s/H_ab, H_ab^2 = (H_a^2 + H_b^2)/2
 *             (Eq. "SG force kernel exact" and Eq. "mean root square height"
 *             of Sect. 2.2; the table of abbreviations drops the squares in
 *             H_ab, the equation is followed).
 *
 * Parity status of each exported function is stated at the function.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_SQRT_PI 1.77245385090551602730

/* ------------------------------------------------------------------------
 * F(x) = e^x [K1(x) - K0(x)]  and  F'(x).
 *
 * App. A reaches e^{x/4}[K1 - K0](x/4) through the integral F_1; here the
 * same function is evaluated from the textbook integral representation
 * K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (Abramowitz & Stegun
 * 9.6.24).  Subtracting nu = 0 from nu = 1 and multiplying by e^x gives the
 * cancellation-free form
 *     F(x) = int_0^inf exp(-x c(t)) c(t) dt,   c(t) = cosh t - 1 = 2 sinh^2(t/2),
 * and, differentiating under the integral,
 *     F'(x) = - int_0^inf exp(-x c(t)) c(t)^2 dt.
 * The integrand is even and entire in t and decays double-exponentially,
 * so the trapezoidal rule converges geometrically.  Step: h = min(1/5,
 * 2/(5 sqrt x)) keeps both aliasing terms (strip |Im t| < pi/2, and the
 * Gaussian width 1/sqrt(x) at large x) below e^-49.  Cut-off T solves
 * x c(T) = 60.  Parity pinned against mpmath Bessel values in the tests.
 * ------------------------------------------------------------------------ */
static void orc_F_dF(double x, double *F, double *dF)
{
    double h = 0.2;
    if (0.4 / sqrt(x) < h) h = 0.4 / sqrt(x);
    double T = 2.0 * asinh(sqrt(30.0 / x));
    long n = (long)ceil(T / h);
    double sF = 0.0, sD = 0.0;
    for (long k = 1; k <= n; ++k) {
        double sh = sinh(0.5 * (double)k * h);
        double c = 2.0 * sh * sh;
        double e = exp(-x * c);
        sF += e * c;
        sD += e * c * c;
    }
    *F = h * sF;          /* the t = 0 node carries weight h/2 and value 0 */
    if (dF) *dF = -h * sD;
}

/* D(x) = -x F'(x) - (3/2) F(x), the factor of the kernel's h derivative.
 * Its two terms cancel to O(x^{-5/2}) against O(x^{-3/2}) at large x, so it
 * is not formed from F and F'.  With c = cosh t - 1 the representation above
 * is F(x) = int_0^inf e^{-x c} sqrt(c/(c+2)) dc; integrating -x F' by parts
 * (x c e^{-xc} = -c d/dc e^{-xc}) gives
 *     D(x) = int_0^inf e^{-x c} (c g'(c) - g(c)/2) dc,  g = sqrt(c/(c+2)),
 * and c g' - g/2 = -(1/2) (c/(c+2))^{3/2} = -(1/2) tanh^3(t/2), so
 *     D(x) = -(1/2) int_0^inf exp(-x c(t)) tanh^3(t/2) sinh t dt,
 * an integrand of one sign, evaluated with F's trapezoidal rule (tanh(t/2)
 * is analytic in the same strip).  Parity pinned against -x F' - 3F/2 from
 * mpmath Bessel values at 40 digits (tests). */
static double orc_D(double x)
{
    double h = 0.2;
    if (0.4 / sqrt(x) < h) h = 0.4 / sqrt(x);
    double T = 2.0 * asinh(sqrt(30.0 / x));
    long n = (long)ceil(T / h);
    double s = 0.0;
    for (long k = 1; k <= n; ++k) {
        double th = tanh(0.5 * (double)k * h);
        double sh = sinh(0.5 * (double)k * h);
        s += exp(-x * 2.0 * sh * sh) * th * th * th * sinh((double)k * h);
    }
    return -0.5 * h * s;
}

double sg_oracle_D(double x) { return orc_D(x); }

double sg_oracle_F(double x)
{
    double F;
    orc_F_dF(x, &F, NULL);
    return F;
}

double sg_oracle_dF(double x)
{
    double F, dF;
    orc_F_dF(x, &F, &dF);
    return dF;
}

/* Exact kernel K_ab(s; H_a, H_b), Eq. "SG force kernel exact" (Sect. 2.2),
 * with H_ab from Eq. "mean root square height".  Parity pinned against the
 * vertical double integral of Eq. "SG force kernel general" (brute-force
 * quadrature in the tests), the small-d limit of Sect. 3.4, the razor-thin
 * limit of Sect. 4 and the planet special case of Sect. 4. */
double sg_oracle_kernel(double s, double Ha, double Hb)
{
    double Hab2 = 0.5 * (Ha * Ha + Hb * Hb);
    double d = s / sqrt(Hab2);
    double x = d * d / 8.0;
    return (1.0 / ORC_SQRT_PI) / Hab2 * (d / 8.0) * sg_oracle_F(x);
}

/* ------------------------------------------------------------------------
 * Convolution-form kernels of App. C (H_f = h_f r):
 *   h_ab^2   = (h_a^2 e^{-X} + h_b^2 e^{X}) / 2        (App. C; the printed
 *              "H_ab/(r r')" lacks a square, the right-hand side is used)
 *   d_ab^2   = 2 (cosh X - cos phi) / h_ab^2
 *   L_ab     = sqrt(pi) (d^2/8) F(d^2/8)
 *   K_r      = L/(pi d^2) [e^{-X}/h_ab^2]^{3/2} (e^X - cos phi)
 *   K_phi    = L/(pi d^2) [e^{-X}/h_ab^2]^{3/2} sin phi
 * X = u_target - u_source, phi = phi_target - phi_source.  With these, the
 * field is a pure convolution in (u, phi):
 *   g_r(u,phi) = - int Sigma_a(u',phi') K_r(u-u', phi-phi') du' dphi'.
 * cosh X - cos phi is evaluated as 2 sinh^2(X/2) + 2 sin^2(phi/2) and
 * e^X - cos phi as expm1(X) + 2 sin^2(phi/2) (identities; no cancellation).
 *
 * which = 0: (K_r, K_phi); 1: d/dh_a of both; 2: d/dh_b of both.
 * Derivative: with G = K h^3/F (independent of h), x = (cosh X - cos phi)
 * /(4 h^2), dK/d(h^2) = G (h^2)^{-5/2} D(x), D(x) = -x F'(x) - 3/2 F(x)
 * (orc_D, cancellation-free), and d(h^2)/dh_a = h_a e^{-X},
 * d(h^2)/dh_b = h_b e^{X}.
 * Parity pinned against the pairwise Cartesian sum (tests) and, for the
 * derivatives, against central differences of which = 0.
 * ------------------------------------------------------------------------ */
static void orc_conv(double X, double phi, double ha, double hb, int which,
                     double *Kr, double *Kphi)
{
    double h2 = 0.5 * (ha * ha * exp(-X) + hb * hb * exp(X));
    double sx = sinh(0.5 * X), sp = sin(0.5 * phi);
    double cosh_m_cos = 2.0 * sx * sx + 2.0 * sp * sp;
    double eX_m_cos = expm1(X) + 2.0 * sp * sp;
    double d2 = 2.0 * cosh_m_cos / h2;
    double x = d2 / 8.0;
    if (which == 0) {
        double F;
        orc_F_dF(x, &F, NULL);
        double L = ORC_SQRT_PI * x * F;
        double pref = L / (ORC_PI * d2) * pow(exp(-X) / h2, 1.5);
        *Kr = pref * eX_m_cos;
        *Kphi = pref * sin(phi);
        return;
    }
    /* G = e^{-3X/2} / (8 sqrt(pi)) times the angular factor */
    double G = exp(-1.5 * X) / (8.0 * ORC_SQRT_PI);
    double dK_dh2 = G * pow(h2, -2.5) * orc_D(x);
    double dh2 = (which == 1) ? ha * exp(-X) : hb * exp(X);
    *Kr = dK_dh2 * dh2 * eX_m_cos;
    *Kphi = dK_dh2 * dh2 * sin(phi);
}

void sg_oracle_conv_kernels(int64_t n, const double *X, const double *phi,
                            double ha, double hb, int which,
                            double *Kr, double *Kphi)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) orc_conv(X[i], phi[i], ha, hb, which, &Kr[i], &Kphi[i]);
}

/* ------------------------------------------------------------------------
 * Self-cell term (reading; the paper is silent on k = i).
 * Kbar = (1/(du dphi)) PV-int over the own cell [-du/2,du/2]x[-dphi/2,dphi/2]
 * of K_r(X, phi).  K_r is even in phi; its 1/rho singularity is odd in X,
 * so the X-symmetrised integrand S = (K_r(X,phi) + K_r(-X,phi))/2 is
 * bounded and Kbar = (1/(a b)) int_0^a int_0^b S, a = du/2, b = dphi/2.
 * The quarter cell is split along its diagonal into two triangles with a
 * vertex at the singular corner and integrated in polar coordinates about
 * that corner (the Jacobian rho removes the direction-dependent jump): 48
 * Gauss-Legendre nodes in the angle and, in rho, 20 nodes on each of seven
 * geometrically shrinking panels [0, R 4^-6], [R 4^-(j+1), R 4^-j] (so the
 * transition of F at rho ~ H inside cells much larger than H is resolved;
 * the integrand is rho S0(theta) + O(rho^3 ln rho) near the corner).
 * Parity pinned by brute-force midpoint sums with Richardson extrapolation
 * and by the closed-form small-cell limit (tests).  which: as orc_conv.
 * ------------------------------------------------------------------------ */
#define ORC_GL_N 48
#define ORC_GLR_N 20
#define ORC_PANELS 7
static double orc_gl_x[ORC_GL_N], orc_gl_w[ORC_GL_N];
static double orc_glr_x[ORC_GLR_N], orc_glr_w[ORC_GLR_N];
static int orc_gl_ready = 0;

/* Gauss-Legendre nodes on [0,1] by Newton iteration on P_n (textbook). */
static void orc_legendre(int n, double z, double *p, double *dp)
{
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *p = p1;
    *dp = n * (z * p1 - p0) / (z * z - 1.0);
}

static void orc_gl_nodes(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), p, dp;
        for (int it = 0; it < 100; ++it) {
            orc_legendre(n, z, &p, &dp);
            double dz = p / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        orc_legendre(n, z, &p, &dp);
        /* map [-1,1] -> [0,1]: node (1-z)/2, weight w/2 with w = 2/((1-z^2) P_n'^2) */
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

static void orc_gl_init(void)
{
    if (orc_gl_ready) return;
    orc_gl_nodes(ORC_GL_N, orc_gl_x, orc_gl_w);
    orc_gl_nodes(ORC_GLR_N, orc_glr_x, orc_glr_w);
    orc_gl_ready = 1;
}

static double orc_sym_Kr(double X, double phi, double ha, double hb, int which)
{
    double k1, k2, t;
    orc_conv(X, phi, ha, hb, which, &k1, &t);
    orc_conv(-X, phi, ha, hb, which, &k2, &t);
    return 0.5 * (k1 + k2);
}

double sg_oracle_self_cell(double ha, double hb, double du, double dphi, int which)
{
    orc_gl_init();
    const double a = 0.5 * du, b = 0.5 * dphi;
    const double thc = atan2(b, a);
    double total = 0.0;
    for (int tri = 0; tri < 2; ++tri) {
        double th0 = tri == 0 ? 0.0 : thc;
        double th1 = tri == 0 ? thc : 0.5 * ORC_PI;
        double acc = 0.0;
        for (int i = 0; i < ORC_GL_N; ++i) {
            double th = th0 + (th1 - th0) * orc_gl_x[i];
            double c = cos(th), s = sin(th);
            double rmax = tri == 0 ? a / c : b / s;
            double inner = 0.0;
            for (int pnl = 0; pnl < ORC_PANELS; ++pnl) {
                /* panel [lo, hi] in units of rmax: [0, 4^-6], then [4^-(j+1), 4^-j] */
                double hi = pow(4.0, -(double)(ORC_PANELS - 1 - pnl));
                double lo = pnl == 0 ? 0.0 : hi / 4.0;
                double part = 0.0;
                for (int j = 0; j < ORC_GLR_N; ++j) {
                    double rho = rmax * (lo + (hi - lo) * orc_glr_x[j]);
                    part += orc_glr_w[j] * rho * orc_sym_Kr(rho * c, rho * s, ha, hb, which);
                }
                inner += part * (hi - lo) * rmax;
            }
            acc += orc_gl_w[i] * inner;
        }
        total += acc * (th1 - th0);
    }
    return total / (a * b);
}

/* ------------------------------------------------------------------------
 * Own-cell integral over an X range that need not be symmetric (the cells of
 * a uniform radial grid, reading "linear radial grids"):
 *   I = int_{xlo}^{xhi} int_{-dphi/2}^{dphi/2} K_r(X, phi) dX dphi
 * (K_r of orc_conv, which carries the measure r'^2; the field's own-cell
 * term is -Sigma I).  K_r behaves like 1/rho at the origin, which is
 * integrable, so each side X > 0 and X < 0 is integrated on its own: polar
 * coordinates about the origin over [0, a] x [0, b] (two triangles split at
 * the diagonal, geometric radial panels as above), doubled for phi < 0
 * (K_r is even in phi).  For xlo = -xhi it equals du dphi times
 * sg_oracle_self_cell (test).
 * ------------------------------------------------------------------------ */
static double orc_quadrant(double a, double b, double ha, double hb, int sgn, int which)
{
    const double thc = atan2(b, a);
    double total = 0.0;
    for (int tri = 0; tri < 2; ++tri) {
        double th0 = tri == 0 ? 0.0 : thc;
        double th1 = tri == 0 ? thc : 0.5 * ORC_PI;
        double acc = 0.0;
        for (int i = 0; i < ORC_GL_N; ++i) {
            double th = th0 + (th1 - th0) * orc_gl_x[i];
            double c = cos(th), sn = sin(th);
            double rmax = tri == 0 ? a / c : b / sn;
            double inner = 0.0;
            for (int pnl = 0; pnl < ORC_PANELS; ++pnl) {
                double hi = pow(4.0, -(double)(ORC_PANELS - 1 - pnl));
                double lo = pnl == 0 ? 0.0 : hi / 4.0;
                double part = 0.0;
                for (int j = 0; j < ORC_GLR_N; ++j) {
                    double rho = rmax * (lo + (hi - lo) * orc_glr_x[j]);
                    double kr, kp;
                    orc_conv(sgn * rho * c, rho * sn, ha, hb, which, &kr, &kp);
                    part += orc_glr_w[j] * rho * kr;
                }
                inner += part * (hi - lo) * rmax;
            }
            acc += orc_gl_w[i] * inner;
        }
        total += acc * (th1 - th0);
    }
    return total;
}

double sg_oracle_self_cell_range(double ha, double hb, double xlo, double xhi, double dphi)
{
    orc_gl_init();
    const double b = 0.5 * dphi;
    double I = 0.0;
    if (xhi > 0.0) I += orc_quadrant(xhi, b, ha, hb, 1, 0);
    if (xlo < 0.0) I += orc_quadrant(-xlo, b, ha, hb, -1, 0);
    return 2.0 * I;
}

/* ------------------------------------------------------------------------
 * Grid helpers: log r (the default) or uniform r (ORC_FLAG_LINEAR_R; the
 * semi-spectral method allows linear radial grids, Sect. 5.2, and NIRVANA's
 * tests use one, Sect. 4.1) x uniform phi.  Uniform r: edges r_min + k dr,
 * centres r_min + (i + 1/2) dr, cell measure r_i dr dphi (the exact area
 * of the annular sector); its own cell spans X = ln(r/r_i) in
 * [ln(1 - dr/(2 r_i)), ln(1 + dr/(2 r_i))].
 * ------------------------------------------------------------------------ */
typedef struct {
    int nr, nphi, linear;
    double du, dphi, lnrmin, rmin, dr, rmax;
} orc_grid;

#define ORC_FLAG_EXCLUDE_SELF 1u
#define ORC_FLAG_LINEAR_R 2u
#define ORC_FLAG_SECOND_ORDER 4u

static orc_grid orc_make_grid_f(int nr, int nphi, double rmin, double rmax, unsigned flags)
{
    orc_grid g;
    g.nr = nr;
    g.nphi = nphi;
    g.linear = (flags & ORC_FLAG_LINEAR_R) != 0;
    g.lnrmin = log(rmin);
    g.du = log(rmax / rmin) / nr;
    g.rmin = rmin;
    g.rmax = rmax;
    g.dr = (rmax - rmin) / nr;
    g.dphi = 2.0 * ORC_PI / nphi;
    return g;
}
static orc_grid orc_make_grid(int nr, int nphi, double rmin, double rmax)
{
    return orc_make_grid_f(nr, nphi, rmin, rmax, 0u);
}
static double orc_r(const orc_grid *g, int i)
{
    return g->linear ? g->rmin + (i + 0.5) * g->dr : exp(g->lnrmin + (i + 0.5) * g->du);
}
static double orc_phi(const orc_grid *g, int j) { return (j + 0.5) * g->dphi; }
/* Cell centre in extended precision (pairwise sums): the separation of two
 * neighbouring cells is a small difference of coordinates of order r, so the
 * coordinates' own rounding must sit well below a double ulp of the
 * separation (a double phi_j near 2 pi carries an absolute error of ~4e-16,
 * a relative error of ~1e-14 in the separation of adjacent cells there). */
static void orc_centre_l(const orc_grid *g, int i, int j, long double *x, long double *y)
{
    const long double pi_l = 3.141592653589793238462643383279502884L;
    long double r;
    if (g->linear)
        r = (long double)g->rmin + (i + 0.5L) * (((long double)g->rmax - g->rmin) / g->nr);
    else
        r = expl(logl((long double)g->rmin) +
                 (i + 0.5L) * (logl((long double)g->rmax / g->rmin) / g->nr));
    const long double p = (j + 0.5L) * (2.0L * pi_l / g->nphi);
    *x = r * cosl(p);
    *y = r * sinl(p);
}
static double orc_area(const orc_grid *g, int i)
{
    const double r = orc_r(g, i);
    return g->linear ? r * g->dr * g->dphi : r * r * g->du * g->dphi;
}
/* X range of the own cell of ring i */
static void orc_cell_x(const orc_grid *g, int i, double *xlo, double *xhi)
{
    if (!g->linear) {
        *xlo = -0.5 * g->du;
        *xhi = 0.5 * g->du;
        return;
    }
    const double r = orc_r(g, i);
    *xlo = log1p(-0.5 * g->dr / r);
    *xhi = log1p(0.5 * g->dr / r);
}

/* small direct-mapped memo of self-cell values keyed on (ha, hb) bits */
typedef struct {
    double ha, hb, xlo, v;
    int used;
} orc_memo;

/* Own-cell integral I (see sg_oracle_self_cell_range) of a cell with the
 * given X range, memoised on (ha, hb, xlo); log cells (xlo = -du/2) use the
 * symmetric average, I = du dphi Kbar. */
static double orc_self_memo(orc_memo *m, int nm, double ha, double hb, double xlo, double xhi,
                            double dphi, int linear)
{
    uint64_t ka, kb, kx;
    memcpy(&ka, &ha, 8);
    memcpy(&kb, &hb, 8);
    memcpy(&kx, &xlo, 8);
    uint64_t key = (ka * 0x9E3779B97F4A7C15ull) ^ (kb + (ka >> 7)) ^ (kx * 0xC2B2AE3D27D4EB4Full);
    orc_memo *e = &m[key % (uint64_t)nm];
    if (e->used && e->ha == ha && e->hb == hb && e->xlo == xlo) return e->v;
    double v = linear ? sg_oracle_self_cell_range(ha, hb, xlo, xhi, dphi)
                      : (xhi - xlo) * dphi * sg_oracle_self_cell(ha, hb, xhi - xlo, dphi, 0);
    e->ha = ha;
    e->hb = hb;
    e->xlo = xlo;
    e->v = v;
    e->used = 1;
    return v;
}

/* ------------------------------------------------------------------------
 * Conservative potential (Sect. 5.5 and the appendix "Conservative force"):
 * for spatially constant H_a, H_b the field of fluid a on fluid b is
 * -grad Phi_ab with
 *   Phi_ab(x) = sum over the disc of Sigma_a A P_ab(|x - x'|),
 *   P_ab(s)   = - e^y K0(y) / (2 sqrt(pi) H_ab),  y = d^2/8,  d = s/H_ab.
 * e^y K0(y) is evaluated like F: from K_0(y) = int_0^inf exp(-y cosh t) dt
 * (Abramowitz & Stegun 9.6.24), G0(y) = int_0^inf exp(-y c(t)) dt with the
 * same trapezoidal rule (the t = 0 node has value 1 and weight h/2).
 * Parity pinned against mpmath Bessel values, the Newtonian limit -1/s and
 * the gradient: -grad Phi equals the pairwise field (tests).
 * ------------------------------------------------------------------------ */
double sg_oracle_G0(double y)
{
    double h = 0.2;
    if (0.4 / sqrt(y) < h) h = 0.4 / sqrt(y);
    double T = 2.0 * asinh(sqrt(30.0 / y));
    long n = (long)ceil(T / h);
    double sum = 0.5;
    for (long k = 1; k <= n; ++k) {
        double sh = sinh(0.5 * (double)k * h);
        sum += exp(-y * 2.0 * sh * sh);
    }
    return h * sum;
}

double sg_oracle_potential_kernel(double s, double Ha, double Hb)
{
    double Hab = sqrt(0.5 * (Ha * Ha + Hb * Hb));
    double d = s / Hab;
    return -sg_oracle_G0(d * d / 8.0) / (2.0 * ORC_SQRT_PI * Hab);
}

/* Self term of the potential (reading: the paper does not treat k = i): the
 * integral of P_ab(|x_i - x'|) over the own cell, x' = r e^X (cos phi,
 * sin phi) relative to the centre direction, |x_i - x'|^2 =
 * r^2 e^X (4 sinh^2(X/2) + 4 sin^2(phi/2)), dA' = r^2 e^{2X} dX dphi,
 * |X| <= du/2, |phi| <= dphi/2, with the cell's own H_a, H_b.  The log
 * singularity at the centre is integrated in polar coordinates about it
 * (four quadrants, two triangles each, as the force self term). */
static double orc_pot_integrand(double X, double phi, double r, double Ha, double Hb)
{
    double sx = sinh(0.5 * X), sp = sin(0.5 * phi);
    double s = r * sqrt(exp(X) * 4.0 * (sx * sx + sp * sp));
    return sg_oracle_potential_kernel(s, Ha, Hb) * r * r * exp(2.0 * X);
}

/* Own-cell integral over X in [xlo, xhi] (the two sides of X = 0 separately;
 * xlo = -du/2, xhi = du/2 for a log cell). */
double sg_oracle_potential_self_range(double r, double Ha, double Hb, double xlo, double xhi, double dphi)
{
    orc_gl_init();
    const double b = 0.5 * dphi;
    double total = 0.0;
    for (int sgn = -1; sgn <= 1; sgn += 2) {  /* X < 0 and X > 0; phi: even, doubled */
        const double a = sgn > 0 ? xhi : -xlo;
        if (!(a > 0.0)) continue;
        const double thc = atan2(b, a);
        for (int tri = 0; tri < 2; ++tri) {
            double th0 = tri == 0 ? 0.0 : thc;
            double th1 = tri == 0 ? thc : 0.5 * ORC_PI;
            double acc = 0.0;
            for (int i = 0; i < ORC_GL_N; ++i) {
                double th = th0 + (th1 - th0) * orc_gl_x[i];
                double c = cos(th), sn = sin(th);
                double rmax = tri == 0 ? a / c : b / sn;
                double inner = 0.0;
                for (int pnl = 0; pnl < ORC_PANELS; ++pnl) {
                    double hi = pow(4.0, -(double)(ORC_PANELS - 1 - pnl));
                    double lo = pnl == 0 ? 0.0 : hi / 4.0;
                    double part = 0.0;
                    for (int j = 0; j < ORC_GLR_N; ++j) {
                        double rho = rmax * (lo + (hi - lo) * orc_glr_x[j]);
                        part += orc_glr_w[j] * rho * orc_pot_integrand(sgn * rho * c, rho * sn, r, Ha, Hb);
                    }
                    inner += part * (hi - lo) * rmax;
                }
                acc += orc_gl_w[i] * inner;
            }
            total += 2.0 * acc * (th1 - th0);
        }
    }
    return total;
}

double sg_oracle_potential_self(double r, double Ha, double Hb, double du, double dphi)
{
    return sg_oracle_potential_self_range(r, Ha, Hb, -0.5 * du, 0.5 * du, dphi);
}

/* Potential at cell centres, per target fluid b:
 *   Phi_b(i) = sum_a sum_{k != i} Sigma_a[k] A_k P_ab(s_ik; H_a[k], H_b[i])
 *            + sum_a Sigma_a[i] (self integral with H_a[i], H_b[i]),
 * the self part unless excluded (flag bit 0).  H == NULL: H_f = h[f] r
 * (for which -grad Phi is not the field; the gradient identity needs
 * constant H).  Output pot: [n_fluids][n_targets]. */
int sg_oracle_potential_pairwise(int nr, int nphi, double rmin, double rmax, int nf,
                                 const double *h, const double *H, const double *sigma,
                                 int64_t nt, const int64_t *targets, unsigned flags, double *pot)
{
    if (nr < 1 || nphi < 1 || nf < 1 || nf > 4 || !(rmax > rmin) || !(rmin > 0)) return 1;
    orc_grid g = orc_make_grid_f(nr, nphi, rmin, rmax, flags);
    const int64_t N = (int64_t)nr * nphi;
    for (int64_t ti = 0; ti < nt; ++ti)
        if (targets && (targets[ti] < 0 || targets[ti] >= N)) return 2;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ti = 0; ti < nt; ++ti) {
        const int64_t i = targets ? targets[ti] : ti;
        const int ir = (int)(i / nphi), jr = (int)(i % nphi);
        const double ri = orc_r(&g, ir), pi_ = orc_phi(&g, jr);
        const double xi = ri * cos(pi_), yi = ri * sin(pi_);
        for (int b = 0; b < nf; ++b) {
            const double Hb = H ? H[(int64_t)b * N + i] : h[b] * ri;
            long double acc = 0.0L;
            for (int a = 0; a < nf; ++a) {
                for (int kr = 0; kr < nr; ++kr) {
                    const double rk = orc_r(&g, kr);
                    const double area = orc_area(&g, kr);
                    for (int kp = 0; kp < nphi; ++kp) {
                        const int64_t k = (int64_t)kr * nphi + kp;
                        if (k == i) continue;
                        const double pk = orc_phi(&g, kp);
                        const double dx = xi - rk * cos(pk), dy = yi - rk * sin(pk);
                        const double Ha = H ? H[(int64_t)a * N + k] : h[a] * rk;
                        acc += sigma[(int64_t)a * N + k] * area *
                               sg_oracle_potential_kernel(sqrt(dx * dx + dy * dy), Ha, Hb);
                    }
                }
                if (!(flags & ORC_FLAG_EXCLUDE_SELF)) {
                    const double Ha = H ? H[(int64_t)a * N + i] : h[a] * ri;
                    double xlo, xhi;
                    orc_cell_x(&g, ir, &xlo, &xhi);
                    acc += sigma[(int64_t)a * N + i] * sg_oracle_potential_self_range(ri, Ha, Hb, xlo, xhi, g.dphi);
                }
            }
            pot[(int64_t)b * nt + ti] = (double)acc;
        }
    }
    return 0;
}

/* Potential and Cartesian field of one source fluid at arbitrary points
 * (px, py), constant H_a (source) and H_b (target), summed over all source
 * cells (points must not coincide with a cell centre):
 *   Phi(p) = sum_k Sigma[k] A_k P_ab(|p - x_k|),
 *   g(p)   = - sum_k Sigma[k] A_k K_ab(|p - x_k|) (p - x_k)/|p - x_k|.
 * For the gradient identity -grad Phi = g of the conservative case. */
int sg_oracle_point_fields(int nr, int nphi, double rmin, double rmax, double Ha, double Hb,
                           const double *sigma, int64_t np, const double *px, const double *py,
                           double *pot, double *gx, double *gy)
{
    if (nr < 1 || nphi < 1 || !(rmax > rmin) || !(rmin > 0)) return 1;
    orc_grid g = orc_make_grid(nr, nphi, rmin, rmax);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < np; ++q) {
        double P = 0.0, X = 0.0, Y = 0.0;
        for (int kr = 0; kr < nr; ++kr) {
            const double rk = orc_r(&g, kr);
            const double area = rk * rk * g.du * g.dphi;
            for (int kp = 0; kp < nphi; ++kp) {
                const double pk = orc_phi(&g, kp);
                const double dx = px[q] - rk * cos(pk), dy = py[q] - rk * sin(pk);
                const double s = sqrt(dx * dx + dy * dy);
                const double m = sigma[(int64_t)kr * nphi + kp] * area;
                P += m * sg_oracle_potential_kernel(s, Ha, Hb);
                const double K = sg_oracle_kernel(s, Ha, Hb);
                X -= m * K * dx / s;
                Y -= m * K * dy / s;
            }
        }
        pot[q] = P;
        gx[q] = X;
        gy[q] = Y;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Self-gravitating scale heights (Sect. 2.1, stratification parameters):
 *   H_f^sg = sqrt(2/pi) H_f f(Qt),  Qt = (sum_f 1/Q_f)^-1,
 *   f(x) = pi/(4x) [sqrt(1 + 8 x^2/pi) - 1],
 * written out as printed (no rearrangement).  Arrays [F][n].  Parity pinned
 * by the limits f -> sqrt(pi/2) (no self-gravity: H^sg -> H) and f ~ x
 * (strong self-gravity), and by f being the positive root of
 * (2x/pi) f^2 + f - x = 0 (tests).
 * ------------------------------------------------------------------------ */
void sg_oracle_hsg(int64_t n, int nf, const double *H, const double *Q, double *Hsg)
{
    for (int64_t i = 0; i < n; ++i) {
        double inv = 0.0;
        for (int f = 0; f < nf; ++f) inv += 1.0 / Q[(int64_t)f * n + i];
        double x = 1.0 / inv;
        double fx = ORC_PI / (4.0 * x) * (sqrt(1.0 + 8.0 * x * x / ORC_PI) - 1.0);
        for (int f = 0; f < nf; ++f) Hsg[(int64_t)f * n + i] = sqrt(2.0 / ORC_PI) * H[(int64_t)f * n + i] * fx;
    }
}

/* ------------------------------------------------------------------------
 * Indirect term (Sect. 5.4 "Indirect term" and the appendix of the same
 * name): the pull of fluid a on the star, in the form derived there,
 *   A_a = sqrt(2) sum_k Sigma_a[k] A_k K_a(d_k) cos(phi_k),
 *   B_a = sqrt(2) sum_k Sigma_a[k] A_k K_a(d_k) sin(phi_k),
 *   K_a(d) = pi^{-1/2} H_a^{-2} (d/4) e^{d^2/4} [K1 - K0](d^2/4),
 *   d_k = r_k / H_a(x_k)  (H_a = h_a r unless per-cell H is given),
 * i.e. the disc integral of the appendix with the cell masses Sigma A_k of
 * the area reading.  The gradient of the indirect potential is then
 *   grad Phi_a = (A_a cos phi + B_a sin phi) e_r + (-A_a sin phi + B_a cos phi) e_phi.
 * Output AB[2a] = A_a, AB[2a+1] = B_a.  Parity pinned by the vertical
 * integral of the appendix's first line (brute-force quadrature), the
 * equality sqrt(2) K_a = K_ab with H_b = 0, a one-cell disc, axisymmetry,
 * rotation equivariance and the point-mass limit with its next term (tests).
 * ------------------------------------------------------------------------ */
int sg_oracle_indirect(int nr, int nphi, double rmin, double rmax, int nf, const double *h,
                       const double *H, const double *sigma, unsigned flags, double *AB)
{
    if (nr < 1 || nphi < 1 || nf < 1 || nf > 4 || !(rmax > rmin) || !(rmin > 0)) return 1;
    orc_grid g = orc_make_grid_f(nr, nphi, rmin, rmax, flags);
    const int64_t N = (int64_t)nr * nphi;
    for (int a = 0; a < nf; ++a) {
        long double sa = 0.0L, sb = 0.0L;
        for (int i = 0; i < nr; ++i) {
            const double r = orc_r(&g, i);
            const double area = orc_area(&g, i);
            for (int j = 0; j < nphi; ++j) {
                const int64_t k = (int64_t)a * N + (int64_t)i * nphi + j;
                const double Hk = H ? H[k] : h[a] * r;
                const double d = r / Hk;
                const double Ka = (1.0 / ORC_SQRT_PI) / (Hk * Hk) * (d / 4.0) * sg_oracle_F(d * d / 4.0);
                const double w = sqrt(2.0) * sigma[k] * area * Ka;
                const double ph = orc_phi(&g, j);
                sa += w * cos(ph);
                sb += w * sin(ph);
            }
        }
        AB[2 * a] = (double)sa;
        AB[2 * a + 1] = (double)sb;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Pairwise (plain definition) field.
 * For each requested target cell i and target fluid b:
 *   G = - sum_a sum_{k != i} Sigma_a[k] A_k K_ab(|x_i - x_k|; H_a[k], H_b[i])
 *         (x_i - x_k)/|x_i - x_k|          (Cartesian vectors)
 *   g_r = G . e_r(phi_i),  g_phi = G . e_phi(phi_i)
 *   plus, unless excluded, the self term
 *   g_r += - du dphi sum_a Sigma_a[i] Kbar_r^{ab}(h_a = H_a[i]/r_i, h_b = H_b[i]/r_i)
 *   (on a uniform radial grid, ORC_FLAG_LINEAR_R: - sum_a Sigma_a[i] I^{ab}
 *   with I the own-cell integral of sg_oracle_self_cell_range).
 * H == NULL means H_f = h[f] r.  Layout: arrays [fluid][i_r][j_phi].
 * Outputs gr, gphi: [n_fluids][n_targets].
 * Parity pinned by Newton's third law, axisymmetry, the razor-thin
 * Newtonian sum, hand-computed two/three-cell systems (tests).
 * ------------------------------------------------------------------------ */
int sg_oracle_field_pairwise(int nr, int nphi, double rmin, double rmax, int nf,
                             const double *h, const double *H, const double *sigma,
                             int64_t nt, const int64_t *targets, unsigned flags,
                             double *gr, double *gphi)
{
    if (nr < 1 || nphi < 1 || nf < 1 || nf > 4 || !(rmax > rmin) || !(rmin > 0)) return 1;
    orc_gl_init();
    orc_grid g = orc_make_grid_f(nr, nphi, rmin, rmax, flags);
    const int64_t N = (int64_t)nr * nphi;
    long double *xs = malloc(sizeof(long double) * N), *ys = malloc(sizeof(long double) * N);
    double *A = malloc(sizeof(double) * N), *Hc = malloc(sizeof(double) * nf * N);
    double *rr = malloc(sizeof(double) * N);
    if (!xs || !ys || !A || !Hc || !rr) return 2;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nphi; ++j) {
            int64_t k = (int64_t)i * nphi + j;
            double r = orc_r(&g, i);
            rr[k] = r;
            orc_centre_l(&g, i, j, &xs[k], &ys[k]);
            A[k] = orc_area(&g, i);
            for (int f = 0; f < nf; ++f) Hc[f * N + k] = H ? H[f * N + k] : h[f] * r;
        }
    const int want_self = !(flags & ORC_FLAG_EXCLUDE_SELF);
#pragma omp parallel
    {
        orc_memo memo[64];
        memset(memo, 0, sizeof(memo));
#pragma omp for schedule(dynamic, 4)
        for (int64_t t = 0; t < nt; ++t) {
            int64_t i = targets ? targets[t] : t;
            /* e_r, e_phi of the target from its extended-precision centre
             * (g_phi, a small projection of the Cartesian sum, keeps the
             * digits that a double cos, sin would round away) */
            long double cx, cy;
            orc_centre_l(&g, (int)(i / nphi), (int)(i % nphi), &cx, &cy);
            const long double rl = sqrtl(cx * cx + cy * cy);
            const long double cp = cx / rl, sp = cy / rl;
            for (int b = 0; b < nf; ++b) {
                long double Gx = 0.0L, Gy = 0.0L, gself = 0.0L;
                for (int a = 0; a < nf; ++a) {
                    const double *Sa = sigma + a * N;
                    const double *Ha = Hc + a * N;
                    double Hb = Hc[b * N + i];
                    for (int64_t k = 0; k < N; ++k) {
                        if (k == i) continue;
                        double dx = (double)(xs[i] - xs[k]), dy = (double)(ys[i] - ys[k]);
                        double s = sqrt(dx * dx + dy * dy);
                        double K = sg_oracle_kernel(s, Ha[k], Hb);
                        double w = Sa[k] * A[k] * K / s;
                        Gx -= w * dx;
                        Gy -= w * dy;
                    }
                    if (want_self) {
                        double ha = Ha[i] / rr[i], hb = Hb / rr[i];
                        if (!H) {
                            ha = h[a];
                            hb = h[b];
                        }
                        double xlo, xhi;
                        orc_cell_x(&g, (int)(i / nphi), &xlo, &xhi);
                        gself -= Sa[i] * orc_self_memo(memo, 64, ha, hb, xlo, xhi, g.dphi, g.linear);
                    }
                }
                gr[b * nt + t] = (double)(Gx * cp + Gy * sp + gself);
                gphi[b * nt + t] = (double)(-Gx * sp + Gy * cp);
            }
        }
    }
    free(xs);
    free(ys);
    free(A);
    free(Hc);
    free(rr);
    return 0;
}

/* ------------------------------------------------------------------------
 * Offset-table (log-polar) field, H_f = h_f r (App. C convolution form):
 *   out^{a->b}_c[i] = - du dphi sum_{i'} Sigma_a[i'] T_c^{ab}(i_r - i'_r, j - j')
 * with T_c^{ab}(p, q) = K_c(p du, q dphi) from orc_conv (which = deriv) and
 * T_r(0,0) = self-cell term (0 when excluded), T_phi(0,0) = 0.
 * Output out: [a][b][c][n_targets], c = 0 (r), 1 (phi), NOT summed over a,
 * so that derivatives can be attached to the right pair by the caller.
 * Parity: equals the pairwise sum (tests, 1e-12) and is the same discrete
 * problem.
 * ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------
 * Second-order weights (ORC_FLAG_SECOND_ORDER; reading, an option beyond the
 * paper).  The convolution of App. C is applied to the piecewise-bilinear
 * interpolant of the cell values: in cell units (s, t) = ((u' - u_k)/du,
 * (phi' - phi_k)/dphi) every source cell carries the tensor hat
 * Lambda(s) Lambda(t), Lambda(x) = max(0, 1 - |x|) (periodic in phi), and the
 * offset table holds, for all offsets including (0, 0),
 *   W_c(P, Q) = int_{-1}^{1} int_{-1}^{1} Lambda(s) Lambda(t)
 *               K_c((P + s) du, (Q + t) dphi) ds dt,   c = r, phi,
 * in place of the point value K_c(P du, Q dphi) and the own-cell average;
 * which = 1, 2 integrates the kernel's h_a, h_b derivatives (orc_conv) the
 * same way, giving the derivatives of W.
 * Integrated square by square (Lambda(s) Lambda(t) is bilinear on each of
 * the four unit squares of the support).  A square that has the kernel's
 * singular point (s, t) = (-P, -Q) as a corner is integrated in polar
 * coordinates (rho, theta) about that corner, which makes the integrand
 * rho K bounded; every other square as an iterated integral in (s, t).
 * Each one-dimensional integral: adaptive bisection with the 10-point
 * Gauss-Legendre rule (an interval is accepted when the rule on its two
 * halves agrees with the rule on the whole to the tolerance, which halves
 * at each level, or to 64 ulps of the integral of |f| over the interval,
 * below which the difference is rounding), relative tolerance 1e-13 inside,
 * 1e-12 outside.
 * Parity pinned against an independent scipy quadrature of the same
 * definition, the far-field expansion W = K + (du^2 K_XX + dphi^2 K_phiphi)/12
 * + ..., and the second-order convergence of the resulting field (tests).
 * ------------------------------------------------------------------------ */
#define ORC_AGL_N 10
static double orc_agl_x[ORC_AGL_N], orc_agl_w[ORC_AGL_N];
static int orc_agl_ready = 0;

typedef void (*orc_vfn)(double x, void *ctx, double y[2]);

/* 10-point rule on [a, b] for both components and for their magnitudes */
static void orc_vrule(orc_vfn f, void *ctx, double a, double b, double v[2], double m[2])
{
    v[0] = v[1] = m[0] = m[1] = 0.0;
    for (int i = 0; i < ORC_AGL_N; ++i) {
        double y[2];
        f(a + (b - a) * orc_agl_x[i], ctx, y);
        v[0] += orc_agl_w[i] * y[0];
        v[1] += orc_agl_w[i] * y[1];
        m[0] += orc_agl_w[i] * fabs(y[0]);
        m[1] += orc_agl_w[i] * fabs(y[1]);
    }
    for (int c = 0; c < 2; ++c) {
        v[c] *= b - a;
        m[c] *= b - a;
    }
}

static void orc_vadapt_rec(orc_vfn f, void *ctx, double a, double b, const double whole[2],
                           const double tol[2], int depth, double out[2])
{
    const double mid = 0.5 * (a + b);
    double l[2], r[2], ml[2], mr[2];
    orc_vrule(f, ctx, a, mid, l, ml);
    orc_vrule(f, ctx, mid, b, r, mr);
    /* accepted at the tolerance, or where the difference is rounding (a few
     * dozen ulps of the integral of |f| over the interval) */
    const double fl0 = 64.0 * DBL_EPSILON * (ml[0] + mr[0]), fl1 = 64.0 * DBL_EPSILON * (ml[1] + mr[1]);
    if (depth == 0 || (fabs(l[0] + r[0] - whole[0]) <= fmax(tol[0], fl0) &&
                       fabs(l[1] + r[1] - whole[1]) <= fmax(tol[1], fl1))) {
        out[0] = l[0] + r[0];
        out[1] = l[1] + r[1];
        return;
    }
    const double half[2] = {0.5 * tol[0], 0.5 * tol[1]};
    double o1[2], o2[2];
    orc_vadapt_rec(f, ctx, a, mid, l, half, depth - 1, o1);
    orc_vadapt_rec(f, ctx, mid, b, r, half, depth - 1, o2);
    out[0] = o1[0] + o2[0];
    out[1] = o1[1] + o2[1];
}

static void orc_vadapt(orc_vfn f, void *ctx, double a, double b, double rel, double out[2])
{
    double whole[2], mag[2];
    orc_vrule(f, ctx, a, b, whole, mag);
    const double tol[2] = {rel * mag[0] + 1e-300, rel * mag[1] + 1e-300};
    orc_vadapt_rec(f, ctx, a, b, whole, tol, 48, out);
}

static double orc_hat(double x) { return fabs(x) < 1.0 ? 1.0 - fabs(x) : 0.0; }

typedef struct {
    double du, dphi, ha, hb;
    int P, Q, which;
    int sx, sy;     /* singular square: directions of the square seen from the corner */
    double s_lo, t_lo; /* regular square: lower corner */
    double outer;   /* the outer variable (theta, or s) fixed for the inner integral */
} orc_hatctx;

/* integrand at cell-unit source offset (s, t): Lambda(s) Lambda(t) K(X, phi) */
static void orc_hat_point(const orc_hatctx *c, double s, double t, double y[2])
{
    const double w = orc_hat(s) * orc_hat(t);
    if (w == 0.0) {
        y[0] = y[1] = 0.0;
        return;
    }
    double kr, kp;
    orc_conv((c->P + s) * c->du, (c->Q + t) * c->dphi, c->ha, c->hb, c->which, &kr, &kp);
    y[0] = w * kr;
    y[1] = w * kp;
}

/* polar about the corner (-P, -Q): inner integrand in rho at fixed theta.
 * With (x, y) = rho (cos theta, sin theta) measured from the corner into the
 * square, the offsets are (sx x du, sy y dphi) and the hats are 1 - x for a
 * corner at s = 0 and x for a corner at s = +-1 (likewise in t); written so,
 * neither loses digits near the corner (1 - |-1 + x| would). */
static void orc_hat_rho(double rho, void *vc, double y[2])
{
    const orc_hatctx *c = vc;
    const double px = rho * cos(c->outer), py = rho * sin(c->outer);
    const double w = (c->P == 0 ? 1.0 - px : px) * (c->Q == 0 ? 1.0 - py : py);
    double kr, kp;
    orc_conv(c->sx * px * c->du, c->sy * py * c->dphi, c->ha, c->hb, c->which, &kr, &kp);
    y[0] = rho * w * kr;
    y[1] = rho * w * kp;
}

static void orc_hat_theta(double th, void *vc, double y[2])
{
    orc_hatctx c = *(const orc_hatctx *)vc;
    c.outer = th;
    const double rmax = 1.0 / fmax(cos(th), sin(th));
    orc_vadapt(orc_hat_rho, &c, 0.0, rmax, 1e-13, y);
}

static void orc_hat_t(double t, void *vc, double y[2])
{
    const orc_hatctx *c = vc;
    orc_hat_point(c, c->outer, t, y);
}

static void orc_hat_s(double s, void *vc, double y[2])
{
    orc_hatctx c = *(const orc_hatctx *)vc;
    c.outer = s;
    orc_vadapt(orc_hat_t, &c, c.t_lo, c.t_lo + 1.0, 1e-13, y);
}

static void orc_agl_init(void)
{
    if (orc_agl_ready) return;
    orc_gl_nodes(ORC_AGL_N, orc_agl_x, orc_agl_w);
    orc_agl_ready = 1;
}

/* W_r, W_phi of offset (P, Q) for cell sizes du, dphi, or their h
 * derivatives (which; nodes initialised) */
static void orc_hat_weight(int P, int Q, double du, double dphi, double ha, double hb, int which, double *W)
{
    orc_hatctx c = {du, dphi, ha, hb, P, Q, which, 1, 1, 0.0, 0.0, 0.0};
    W[0] = W[1] = 0.0;
    for (int s0 = -1; s0 <= 0; ++s0)
        for (int t0 = -1; t0 <= 0; ++t0) {
            double y[2];
            const int corner_s = (-P == s0 || -P == s0 + 1), corner_t = (-Q == t0 || -Q == t0 + 1);
            if (corner_s && corner_t) {
                c.sx = (-P == s0) ? 1 : -1;
                c.sy = (-Q == t0) ? 1 : -1;
                double y1[2];
                orc_vadapt(orc_hat_theta, &c, 0.0, 0.25 * ORC_PI, 1e-12, y);
                orc_vadapt(orc_hat_theta, &c, 0.25 * ORC_PI, 0.5 * ORC_PI, 1e-12, y1);
                y[0] += y1[0];
                y[1] += y1[1];
            } else {
                c.s_lo = s0;
                c.t_lo = t0;
                orc_vadapt(orc_hat_s, &c, (double)s0, (double)s0 + 1.0, 1e-12, y);
            }
            W[0] += y[0];
            W[1] += y[1];
        }
}

void sg_oracle_hat_weight(int P, int Q, double du, double dphi, double ha, double hb, int which, double *W)
{
    orc_agl_init();
    orc_hat_weight(P, Q, du, dphi, ha, hb, which, W);
}

typedef struct {
    int nr, nphi;
    double *Tr, *Tp; /* [(2nr-1)][2 nphi], reversed-and-doubled in phi */
} orc_table;

/* Build T for one pair.  Storage R[p][m] = T(p - (nr-1), (N - (m mod N)) mod N)
 * for m in [0, 2N), so that T(i_r - i', j - j') = R[i_r - i' + nr - 1][j' - j + N]
 * and the inner sum over j' reads R contiguously. */
static int orc_build_table(const orc_grid *g, double ha, double hb, int which, int want_self,
                           int second, orc_table *t)
{
    const int nr = g->nr, np = g->nphi;
    const int P = 2 * nr - 1;
    t->nr = nr;
    t->nphi = np;
    t->Tr = malloc(sizeof(double) * (size_t)P * 2 * np);
    t->Tp = malloc(sizeof(double) * (size_t)P * 2 * np);
    if (!t->Tr || !t->Tp) return 2;
    double self = want_self && !second ? sg_oracle_self_cell(ha, hb, g->du, g->dphi, which) : 0.0;
    if (second) orc_agl_init();
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t e = 0; e < (int64_t)P * np; ++e) {
        const int p = (int)(e / np), q = (int)(e % np);
        double X = (double)(p - (nr - 1)) * g->du;
        {
            double kr, kp;
            if (second) {
                double W[2];
                orc_hat_weight(p - (nr - 1), 2 * q <= np ? q : q - np, g->du, g->dphi, ha, hb, which, W);
                kr = W[0];
                kp = W[1];
            } else if (p == nr - 1 && q == 0) {
                kr = self;
                kp = 0.0;
            } else {
                /* offset q and q - N are the same azimuth; the one in
                 * (-pi, pi] keeps sin(phi) and sin(phi/2) at full relative
                 * accuracy for the near neighbours across phi = 0 */
                const int qs = 2 * q <= np ? q : q - np;
                orc_conv(X, (double)qs * g->dphi, ha, hb, which, &kr, &kp);
            }
            /* T(p, q) goes to every m with (N - m) mod N == q */
            int m0 = (np - q) % np;
            t->Tr[(size_t)p * 2 * np + m0] = kr;
            t->Tr[(size_t)p * 2 * np + m0 + np] = kr;
            t->Tp[(size_t)p * 2 * np + m0] = kp;
            t->Tp[(size_t)p * 2 * np + m0 + np] = kp;
        }
    }
    return 0;
}

static void orc_free_table(orc_table *t)
{
    free(t->Tr);
    free(t->Tp);
}

int sg_oracle_field_table(int nr, int nphi, double rmin, double rmax, int nf, const double *h,
                          const double *sigma, int64_t nt, const int64_t *targets,
                          unsigned flags, int which, double *out)
{
    if (nr < 1 || nphi < 1 || nf < 1 || nf > 4 || !(rmax > rmin) || !(rmin > 0)) return 1;
    if (which < 0 || which > 2) return 1;
    const int second = (flags & ORC_FLAG_SECOND_ORDER) != 0;
    if (second && (nphi < 4 || (flags & ORC_FLAG_EXCLUDE_SELF))) return 1;
    orc_grid g = orc_make_grid(nr, nphi, rmin, rmax);
    const int64_t N = (int64_t)nr * nphi;
    const double scale = -g.du * g.dphi;
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
            orc_table T;
            if (orc_build_table(&g, h[a], h[b], which, !(flags & ORC_FLAG_EXCLUDE_SELF), second, &T))
                return 2;
            const double *Sa = sigma + a * N;
            double *o_r = out + ((size_t)(a * nf + b) * 2 + 0) * nt;
            double *o_p = out + ((size_t)(a * nf + b) * 2 + 1) * nt;
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t t = 0; t < nt; ++t) {
                int64_t i = targets ? targets[t] : t;
                int ir = (int)(i / nphi), j = (int)(i % nphi);
                long double sr = 0.0L, sp = 0.0L;
                for (int ip = 0; ip < nr; ++ip) {
                    const double *row = Sa + (size_t)ip * nphi;
                    const double *Rr = T.Tr + (size_t)(ir - ip + nr - 1) * 2 * nphi + (nphi - j);
                    const double *Rp = T.Tp + (size_t)(ir - ip + nr - 1) * 2 * nphi + (nphi - j);
                    long double ar = 0.0L, ap = 0.0L;
                    for (int jp = 0; jp < nphi; ++jp) {
                        ar += (long double)row[jp] * Rr[jp];
                        ap += (long double)row[jp] * Rp[jp];
                    }
                    sr += ar;
                    sp += ap;
                }
                o_r[t] = (double)(scale * sr);
                o_p[t] = (double)(scale * sp);
            }
            orc_free_table(&T);
        }
    return 0;
}

/* ------------------------------------------------------------------------
 * Second-order field with scale heights that depend on radius (the
 * semi-spectral path's model, Sect. 5.2, with the weights of
 * ORC_FLAG_SECOND_ORDER; reading): for target ring i and source ring i' the
 * weights are W_c(i - i', q) of sg_oracle_hat_weight with the rings' aspect
 * ratios h_a = H_a(r_i')/r_i', h_b = H_b(r_i)/r_i held across the hats, and
 *   g_b(i, j) = - du dphi sum_a sum_i' sum_j' Sigma_a[i'][j'] W(i - i', j - j').
 * H: [nf][nr] at the ring centres.  out: [b][c][nt] summed over sources.
 * For H = h r it is the offset-table sum with ORC_FLAG_SECOND_ORDER (tests).
 * ------------------------------------------------------------------------ */
int sg_oracle_field_ring_hat(int nr, int nphi, double rmin, double rmax, int nf, const double *H,
                             const double *sigma, int64_t nt, const int64_t *targets, double *out)
{
    if (nr < 1 || nphi < 4 || nf < 1 || nf > 4 || !(rmax > rmin) || !(rmin > 0)) return 1;
    orc_grid g = orc_make_grid(nr, nphi, rmin, rmax);
    orc_agl_init();
    const int64_t npr = (int64_t)nf * nf * nr * nr;  /* (a, b, i, i') */
    double *Wr = malloc(sizeof(double) * (size_t)npr * nphi);
    double *Wp = malloc(sizeof(double) * (size_t)npr * nphi);
    if (!Wr || !Wp) {
        free(Wr);
        free(Wp);
        return 2;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t e = 0; e < npr * nphi; ++e) {
        const int q = (int)(e % nphi);
        int64_t r = e / nphi;
        const int ip = (int)(r % nr);
        r /= nr;
        const int i = (int)(r % nr);
        r /= nr;
        const int b = (int)(r % nf), a = (int)(r / nf);
        const double ha = H[a * nr + ip] / orc_r(&g, ip), hb = H[b * nr + i] / orc_r(&g, i);
        double W[2];
        orc_hat_weight(i - ip, 2 * q <= nphi ? q : q - nphi, g.du, g.dphi, ha, hb, 0, W);
        Wr[e] = W[0];
        Wp[e] = W[1];
    }
    const int64_t N = (int64_t)nr * nphi;
    const double scale = -g.du * g.dphi;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t k = targets ? targets[t] : t;
        const int i = (int)(k / nphi), j = (int)(k % nphi);
        for (int b = 0; b < nf; ++b) {
            long double sr = 0.0L, sp = 0.0L;
            for (int a = 0; a < nf; ++a)
                for (int ip = 0; ip < nr; ++ip) {
                    const int64_t e0 = ((((int64_t)a * nf + b) * nr + i) * nr + ip) * nphi;
                    const double *row = sigma + a * N + (int64_t)ip * nphi;
                    for (int jp = 0; jp < nphi; ++jp) {
                        const int q = ((j - jp) % nphi + nphi) % nphi;
                        sr += (long double)row[jp] * Wr[e0 + q];
                        sp += (long double)row[jp] * Wp[e0 + q];
                    }
                }
            out[((size_t)b * 2 + 0) * nt + t] = (double)(scale * sr);
            out[((size_t)b * 2 + 1) * nt + t] = (double)(scale * sp);
        }
    }
    free(Wr);
    free(Wp);
    return 0;
}

/* ------------------------------------------------------------------------
 * Adjoint with respect to Sigma (transposed offset-table sum):
 *   dL/dSigma_a[k] = - du dphi sum_b sum_c sum_i lam_{b,c}[i] T_c^{ab}(i - k)
 * lam: [b][c][N] (c = 0: dL/dg_r, 1: dL/dg_phi).  Output: [a][n_k].
 * Parity pinned by central differences of sg_oracle_field_table (exact for
 * a loss that is quadratic in Sigma) in the tests.
 * ------------------------------------------------------------------------ */
int sg_oracle_adjoint_sigma(int nr, int nphi, double rmin, double rmax, int nf, const double *h,
                            const double *lam, int64_t nk, const int64_t *kidx, unsigned flags,
                            double *dsigma)
{
    if (nr < 1 || nphi < 1 || nf < 1 || nf > 4 || !(rmax > rmin) || !(rmin > 0)) return 1;
    const int second = (flags & ORC_FLAG_SECOND_ORDER) != 0;
    if (second && (nphi < 4 || (flags & ORC_FLAG_EXCLUDE_SELF))) return 1;
    orc_grid g = orc_make_grid(nr, nphi, rmin, rmax);
    const int64_t N = (int64_t)nr * nphi;
    const double scale = -g.du * g.dphi;
    for (int64_t t = 0; t < (int64_t)nf * nk; ++t) dsigma[t] = 0.0;
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
            orc_table T;
            if (orc_build_table(&g, h[a], h[b], 0, !(flags & ORC_FLAG_EXCLUDE_SELF), second, &T)) return 2;
            const double *lr = lam + ((size_t)b * 2 + 0) * N;
            const double *lp = lam + ((size_t)b * 2 + 1) * N;
#pragma omp parallel for schedule(dynamic, 4)
            for (int64_t t = 0; t < nk; ++t) {
                int64_t k = kidx ? kidx[t] : t;
                int kr = (int)(k / nphi), kj = (int)(k % nphi);
                long double acc = 0.0L;
                for (int ir = 0; ir < nr; ++ir) {
                    /* T(ir - kr, j - kj) = R[ir - kr + nr - 1][kj - j + N];  as j
                     * increases the index decreases, so walk it backwards. */
                    const double *Rr = T.Tr + (size_t)(ir - kr + nr - 1) * 2 * nphi;
                    const double *Rp = T.Tp + (size_t)(ir - kr + nr - 1) * 2 * nphi;
                    const double *l1 = lr + (size_t)ir * nphi, *l2 = lp + (size_t)ir * nphi;
                    long double s = 0.0L;
                    for (int j = 0; j < nphi; ++j) {
                        int m = kj - j + nphi;
                        s += (long double)l1[j] * Rr[m] + (long double)l2[j] * Rp[m];
                    }
                    acc += s;
                }
                dsigma[(size_t)a * nk + t] += (double)(scale * acc);
            }
            orc_free_table(&T);
        }
    return 0;
}

int sg_oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
