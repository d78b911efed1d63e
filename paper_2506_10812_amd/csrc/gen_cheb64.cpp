// gen_cheb64.cpp -- host build step: writes sg_cheb64.h, the Chebyshev
// coefficients of the double-precision mid-range branch of
//     F(x) = e^x [K1(x) - K0(x)],  F'(x) = dF/dx   and   G0(x) = e^x K0(x)
// (the force kernel's function of Sect. 2.2 and App. A, and the potential
// kernel's of Sect. 5.5) on the dyadic intervals
// [2^(k-1), 2^k), k = 0 .. SG_CHEB_NI - 1, i.e. 1/2 <= x < 32.
//
// Values come from the integral representation of the Macdonald functions,
// K_nu(x) = int_0^inf e^{-x cosh t} cosh(nu t) dt, which gives
//     F(x)  =  int_0^inf e^{-x (cosh t - 1)} (cosh t - 1) dt,
//     F'(x) = -int_0^inf e^{-x (cosh t - 1)} (cosh t - 1)^2 dt,
//     G0(x) =  int_0^inf e^{-x (cosh t - 1)} dt,
// evaluated in long double with the trapezoid rule: the integrands are even,
// entire and decay doubly exponentially, so the rule converges geometrically
// in 1/step (step 1/64 here, far below what 64-bit mantissas need).
//
// On each interval x = a (3 + t) / 2, t in [-1, 1], a = 2^(k-1), and
//     f(x) = sum_{j < M} c_j T_j(t)
// with c_j from the discrete cosine transform of f at the NN Chebyshev points
// of the first kind (c_0 already halved).  M = 27 terms leave a truncation
// below 1e-17 of the interval's largest value (the nearest singularity, at
// x = 0, lies one interval length below every interval, so all intervals
// converge alike); the program checks that the last kept coefficients are
// that small and fails otherwise.
#include <cmath>
#include <cstdio>
#include <cstdlib>

static const int NI = 6;   // intervals [1/2,1), [1,2), [2,4), ..., [16,32)
static const int M = 27;   // terms kept
static const int NN = 48;  // Chebyshev points per interval

static void fdf(long double x, long double &F, long double &dF, long double &G)
{
    const long double h = 1.0L / 64.0L;
    long double s = 0.0L, sd = 0.0L, sg = 0.0L;
    for (int k = 0;; ++k) {
        const long double t = k * h;
        const long double sh = sinhl(0.5L * t);
        const long double c = 2.0L * sh * sh;  // cosh t - 1 without the cancellation
        const long double e = expl(-x * c);
        const long double wgt = k == 0 ? 0.5L : 1.0L;
        s += wgt * e * c;
        sd += wgt * e * c * c;
        sg += wgt * e;
        if (x * c > 60.0L) break;  // e^{-60} ~ 1e-26
    }
    F = s * h;
    dF = -sd * h;
    G = sg * h;
}

int main()
{
    static double cf[NI][M], cd[NI][M], cg[NI][M];
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < NI; ++k) {
        const long double a = ldexpl(1.0L, k - 1);
        long double fv[NN], dv[NN], gv[NN];
        long double fmax = 0.0L, dmax = 0.0L, gmax = 0.0L;
        for (int j = 0; j < NN; ++j) {
            const long double t = cosl(pi * (j + 0.5L) / NN);
            fdf(a * (3.0L + t) / 2.0L, fv[j], dv[j], gv[j]);
            fmax = fmaxl(fmax, fabsl(fv[j]));
            dmax = fmaxl(dmax, fabsl(dv[j]));
            gmax = fmaxl(gmax, fabsl(gv[j]));
        }
        for (int m = 0; m < M; ++m) {
            long double sf = 0.0L, sd = 0.0L, sg = 0.0L;
            for (int j = 0; j < NN; ++j) {
                const long double c = cosl(pi * m * (j + 0.5L) / NN);
                sf += fv[j] * c;
                sd += dv[j] * c;
                sg += gv[j] * c;
            }
            const long double sc = (m == 0 ? 1.0L : 2.0L) / NN;
            cf[k][m] = (double)(sf * sc);
            cd[k][m] = (double)(sd * sc);
            cg[k][m] = (double)(sg * sc);
        }
        // the dropped tail: the last kept terms bound it (geometric decay)
        if (fabsl((long double)cf[k][M - 1]) > 1e-17L * fmax || fabsl((long double)cd[k][M - 1]) > 1e-17L * dmax ||
            fabsl((long double)cg[k][M - 1]) > 1e-17L * gmax) {
            fprintf(stderr, "gen_cheb64: interval %d: last coefficients %g %g %g too large\n", k, cf[k][M - 1],
                    cd[k][M - 1], cg[k][M - 1]);
            return 1;
        }
    }
    printf("// sg_cheb64.h -- written by gen_cheb64.cpp at build time; do not edit.\n");
    printf("#pragma once\n#define SG_CHEB_NI %d\n#define SG_CHEB_M %d\n", NI, M);
    const char *names[3] = {"sg_cheb_f", "sg_cheb_df", "sg_cheb_g0"};
    double(*tabs[3])[M] = {cf, cd, cg};
    for (int q = 0; q < 3; ++q) {
        printf("static constexpr double %s[SG_CHEB_NI * SG_CHEB_M] = {\n", names[q]);
        for (int k = 0; k < NI; ++k)
            for (int m = 0; m < M; ++m) printf("    %.17e,\n", tabs[q][k][m]);
        printf("};\n");
    }
    return 0;
}
