// sg_kfn.h -- device evaluation of F(x) = e^x [K1(x) - K0(x)] and of the
// exact kernel in its Cartesian and log-polar (App. C) forms.
//
// F(x) is the function of App. A (there at argument x/4) that carries the
// whole distance dependence of the exact kernel (Sect. 2.2):
//     K_ab(s) = pi^{-1/2} H_ab^{-2} (d/8) F(d^2/8),  d = s/H_ab.
// Evaluation never forms e^x K1(x) and e^x K0(x) separately at large x (their
// difference cancels and e^x overflows, the NaN problem noted in Sect. 5.3):
//   x < 1/2 (float: x < 1)  power series of I0, I1, K0, K1 (Abramowitz &
//           Stegun 9.6.10, 9.6.11), F = e^x (K1 - K0), where the two
//           cancellations inside K0 and K1 - K0 cost at most a few ulps (in
//           double they grow to 3e-14 just below x = 2, hence the Chebyshev
//           branch above 1/2);
//   1 <= x < 32 (float)  F = sqrt(2) x^{-3/2} J(x),  J(x) = int_0^inf v^2 e^{-v^2}
//           (1 + v^2/(2x))^{-1/2} dv, obtained from the integral
//           representation K_nu(x) = int_0^inf e^{-x cosh t} cosh(nu t) dt by
//           the substitution sinh(t/2) = v / sqrt(2x).  The integrand is even
//           and analytic for |Im v| < sqrt(2x), so the trapezoidal rule on a
//           fixed grid converges geometrically, its error ~ exp(-2 pi
//           sqrt(2x) / step): step 1/2 and 9 nodes (2e-8 at x = 1, below a
//           float ulp; the tail beyond v = 4.5 is e^{-20});
//   1/2 <= x < 32 (double) Chebyshev series of F and F' on the dyadic
//           intervals [1/2, 1), [1, 2), ..., [16, 32), 27 terms each, their
//           coefficients computed at build time in long double from the same
//           integral representation (gen_cheb64.cpp; sg_cheb64.h): within
//           7e-16 of F and F' over the range, with no square roots (a
//           26-node trapezoid in double, used before, took a double
//           reciprocal square root per node and ten times the instructions);
//   x >= 32 the asymptotic series J = (sqrt(pi)/4)
//           sum_n c_n x^-n, c_0 = 1, c_n = -c_{n-1} (4 n^2 - 1)/(8 n)
//           (term-by-term integration of the binomial series; its first three
//           terms are the expansion printed in Sect. 5.3), truncated after c_5
//           (float) or c_16 (double).  (1 + t)^{-1/2} is completely monotone, so
//           the binomial remainder alternates and is bounded by the first
//           omitted term, and so is J's: |c_17| 32^-17 = 1.3e-18 for F, and for F'
//           (series differentiated term by term, two such pieces of one sign)
//           |c_17| (17 + 3/2) / (3/2) 32^-17 = 1.7e-17 of its leading term.
// The float trapezoidal weights e^{-v_k^2}, and for double the asymptotic
// coefficients (for the rolled series) and the Chebyshev coefficients, are
// copied once per workgroup into LDS by sg_fill_weights().
#pragma once
#include "sg_internal.h"
#include "sg_cheb64.h"

#define SG_EULER_GAMMA 0.57721566490153286061

// Table of TABLE entries.  Float: w[k-1] = exp(-(k STEP)^2), k = 1..NODES.
// Double: c_n (n = 0..ASYM), -(n + 3/2) c_n, the G0 coefficients a_n, and the
// Chebyshev coefficients of F, F' and G0 (SG_CHEB_NI intervals of SG_CHEB_M).
template <typename R> struct FQuad;
template <> struct FQuad<double> {
    static constexpr int ASYM = 16;
    static constexpr int C = 0, D = C + ASYM + 1, A = D + ASYM + 1;
    static constexpr int CH = A + ASYM + 1, CHD = CH + SG_CHEB_NI * SG_CHEB_M;
    static constexpr int CHG = CHD + SG_CHEB_NI * SG_CHEB_M;
    static constexpr int TABLE = CHG + SG_CHEB_NI * SG_CHEB_M;
};
template <> struct FQuad<float> {
    static constexpr int NODES = 9;
    static constexpr float STEP = 0.5f;
    static constexpr int TABLE = NODES;
};

// Reciprocal and reciprocal square root of the working type.  Float takes the
// hardware v_rcp_f32 / v_rsq_f32 (about 1 ulp; arguments here are normal and
// positive): rsqrt() has only a double overload, so a float argument would be
// promoted to the double sequence, and '/' costs the full IEEE division.
__device__ inline float sg_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double sg_rcp(double x) { return 1.0 / x; }
__device__ inline float sg_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double sg_rsqrt(double x) { return rsqrt(x); }

// Double asymptotic coefficients, generated at compile time from their
// recurrences: c_n (F), d_n = -(n + 3/2) c_n (F'), a_n (G0); see the branch
// comments below.
struct AsymCoef64 {
    static constexpr int N = FQuad<double>::ASYM;
    double c[N + 1], d[N + 1], a[N + 1];
    constexpr AsymCoef64() : c{}, d{}, a{}
    {
        double v = 1.0, g = 1.0;
        for (int n = 0; n <= N; ++n) {
            if (n) {
                v = -v * (4.0 * n * n - 1.0) / (8.0 * n);
                g = -g * (2.0 * n - 1.0) * (2.0 * n - 1.0) / (8.0 * n);
            }
            c[n] = v;
            d[n] = -v * (n + 1.5);
            a[n] = g;
        }
    }
};

template <typename R> __device__ inline R sg_weight_entry(int k)
{
    if constexpr (sizeof(R) == 4) {
        const double v = (k + 1) * (double)FQuad<float>::STEP;
        return (R)exp(-v * v);
    } else {
        using Q = FQuad<double>;
        if (k >= Q::CHG) return sg_cheb_g0[k - Q::CHG];
        if (k >= Q::CHD) return sg_cheb_df[k - Q::CHD];
        if (k >= Q::CH) return sg_cheb_f[k - Q::CH];
        constexpr AsymCoef64 C;
        return k >= Q::A ? C.a[k - Q::A] : k >= Q::D ? C.d[k - Q::D] : C.c[k - Q::C];
    }
}

// Call from every thread, then sync.
template <typename R> __device__ inline void sg_fill_weights(R *w)
{
    for (int k = threadIdx.x; k < FQuad<R>::TABLE; k += blockDim.x) w[k] = sg_weight_entry<R>(k);
}

// Series branch, x < 2.  NT terms.
template <typename R, int NT>
__device__ inline void sg_F_series(R x, R &F, R *dF)
{
    const R y = x * x * R(0.25);
    const R Lg = log(x * R(0.5)) + R(SG_EULER_GAMMA);
    R tk = R(1), sk = R(1), Hk = R(0);
    R I0 = R(0), I1s = R(0), K0s = R(0), K1s = R(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const R Hk1 = Hk + R(1) / R(k + 1);
        I0 += tk;
        I1s += sk;
        K0s += Hk * tk;
        K1s += (Hk + Hk1) * sk;
        tk *= y * (R(1) / R((k + 1) * (k + 1)));  // constant reciprocals, folded
        sk *= y * (R(1) / R((k + 1) * (k + 2)));
        Hk = Hk1;
    }
    const R ix = sg_rcp(x);
    const R I1 = x * R(0.5) * I1s;
    const R K0 = -Lg * I0 + K0s;
    const R K1 = ix + Lg * I1 - x * R(0.25) * K1s;
    const R ex = exp(x);
    F = ex * (K1 - K0);
    if (dF) *dF = ex * (R(2) * (K1 - K0) - K1 * ix);
}

// Trapezoidal branch, x >= 2: F = sqrt(2) x^-3/2 J, F' from J' =
// int v^2 e^{-v^2} v^2/(4x^2) (1 + v^2/(2x))^{-3/2} dv.
template <typename R>
__device__ inline void sg_F_quad(R x, const R *w, R &F, R *dF)
{
    const R ix = sg_rcp(x);
    const R i2x = R(0.5) * ix;
    R J = R(0), Jd = R(0);
#pragma unroll
    for (int k = 1; k <= FQuad<R>::NODES; ++k) {
        const R v2 = R(k * k) * (FQuad<R>::STEP * FQuad<R>::STEP);
        const R rho = sg_rsqrt(R(1) + v2 * i2x);
        const R base = w[k - 1] * v2 * rho;
        J += base;
        if (dF) Jd += base * rho * rho * v2;
    }
    J *= FQuad<R>::STEP;
    const R x32 = sg_rsqrt(x) * ix;  // x^-3/2
    F = R(SG_SQRT2) * x32 * J;
    if (dF) {
        const R Jp = Jd * FQuad<R>::STEP * R(0.25) * (ix * ix);
        *dF = R(SG_SQRT2) * x32 * (Jp - R(1.5) * J * ix);
    }
}

// Asymptotic branch (float), x >= 32.
struct AsymCoef {
    float c[6];
    constexpr AsymCoef() : c{}
    {
        double v = 1.0;
        c[0] = 1.0f;
        for (int n = 1; n < 6; ++n) {
            v = -v * (4.0 * n * n - 1.0) / (8.0 * n);
            c[n] = (float)v;
        }
    }
};

// Asymptotic branch (double), x >= 32: F and F' = (sqrt(2 pi)/4) sum_n c_n
// (-n - 3/2) x^{-n-5/2}.  ROLLED: a rolled Horner loop over the LDS copy of
// the coefficients.  Unrolled with literal coefficients, the compiler keeps
// them in registers across the caller's loop, which drops the direct sums
// from 3 to 1 waves per SIMD; the table and gradient kernels, whose occupancy
// is set by other state, run fastest that way.
template <bool ROLLED>
__device__ inline void sg_F_asym64(double x, const double *w, double &F, double *dF)
{
    using Q = FQuad<double>;
    const double u = 1.0 / x;
    double s, sd = 0.0;
    if constexpr (ROLLED) {
        s = w[Q::C + Q::ASYM];
        sd = w[Q::D + Q::ASYM];
#pragma unroll 1
        for (int n = Q::ASYM - 1; n >= 0; --n) {
            s = s * u + w[Q::C + n];
            if (dF) sd = sd * u + w[Q::D + n];
        }
    } else {
        constexpr AsymCoef64 C;
        s = C.c[Q::ASYM];
        sd = C.d[Q::ASYM];
#pragma unroll
        for (int n = Q::ASYM - 1; n >= 0; --n) {
            s = s * u + C.c[n];
            if (dF) sd = sd * u + C.d[n];
        }
    }
    const double pre = (SG_SQRT2 * SG_SQRT_PI * 0.25) * rsqrt(x) * u;
    F = pre * s;
    if (dF) *dF = pre * u * sd;
}

__device__ inline float sg_F_asym(float x)
{
    constexpr AsymCoef C;
    const float u = sg_rcp(x);
    float s = C.c[5];
#pragma unroll
    for (int n = 4; n >= 0; --n) s = s * u + C.c[n];
    const float J = float(SG_SQRT_PI * 0.25) * s;
    const float rx = sg_rsqrt(x);
    return float(SG_SQRT2) * rx * u * J;
}

// Mid-range branch (double), 1/2 <= x < 32: x = m 2^e with m in [1/2, 1) lies
// in interval k = e at t = 4 m - 3 in [-1, 1); the series of F (and F')
// are summed by Clenshaw's recurrence from the LDS copy of the coefficients.
// Lanes outside the range (whose result is discarded) are clamped to an
// interval so that every address stays in the table.
__device__ inline void sg_F_cheb64(double x, const double *w, double &F, double *dF)
{
    using Q = FQuad<double>;
    int e;
    const double m = frexp(x, &e);
    const int k = min(max(e, 0), SG_CHEB_NI - 1);
    const double t = 4.0 * m - 3.0, t2 = 2.0 * t;
    const double *cf = w + Q::CH + k * SG_CHEB_M;
    const double *cd = w + Q::CHD + k * SG_CHEB_M;
    double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll 3
    for (int j = SG_CHEB_M - 1; j > 0; --j) {
        const double b0 = fma(t2, b1, cf[j] - b2);
        b2 = b1;
        b1 = b0;
        if (dF) {
            const double d0 = fma(t2, d1, cd[j] - d2);
            d2 = d1;
            d1 = d0;
        }
    }
    F = fma(t, b1, cf[0] - b2);
    if (dF) *dF = fma(t, d1, cd[0] - d2);
}

// Full-range evaluators.  The double asymptotic branch alone runs when every
// active lane of the wave has x >= 32.  Otherwise the series (x < 1/2), the
// double Chebyshev branch (1/2 <= x < 32) or the float trapezoid (x >= 1), and
// the double asymptotic branch (x >= 32) each run only when some lane of the
// wave needs them, every lane keeping its own branch's value.
// SG_NO_SPECULATE, an empty asm statement that emits no instruction, keeps
// the compiler from if-converting such wave-uniform branches into
// straight-line code that evaluates every branch for every lane.
#define SG_NO_SPECULATE() asm volatile("")

template <bool ROLLED>
__device__ inline void sg_F64_any(double x, const double *w, double &F, double *dF)
{
    if (__all(x >= 32.0)) {
        sg_F_asym64<ROLLED>(x, w, F, dF);
        return;
    }
    const bool ser = x < 0.5, asy = x >= 32.0, mid = !ser && !asy;
    double t, td = 0.0;
    F = 0.0;
    if (dF) *dF = 0.0;
    if (__any(ser)) {
        SG_NO_SPECULATE();
        sg_F_series<double, 10>(x, t, dF ? &td : nullptr);  // y = x^2/4 < 1/16: y^10/(10!)^2 < 1e-25
        if (ser) {
            F = t;
            if (dF) *dF = td;
        }
    }
    if (__any(mid)) {
        SG_NO_SPECULATE();
        sg_F_cheb64(x, w, t, dF ? &td : nullptr);
        if (mid) {
            F = t;
            if (dF) *dF = td;
        }
    }
    if (__any(asy)) {
        SG_NO_SPECULATE();
        sg_F_asym64<ROLLED>(x, w, t, dF ? &td : nullptr);
        if (asy) {
            F = t;
            if (dF) *dF = td;
        }
    }
}

template <bool ROLLED = false> __device__ inline double sg_F64(double x, const double *w)
{
    double F;
    sg_F64_any<ROLLED>(x, w, F, nullptr);
    return F;
}

template <bool ROLLED = false> __device__ inline void sg_F64_dF(double x, const double *w, double &F, double &dF)
{
    sg_F64_any<ROLLED>(x, w, F, &dF);
}

// Float: each branch runs only when some lane of the wave needs it, and each
// lane keeps its own branch's value (a wave whose lanes all fall in one range
// pays for one branch).
__device__ inline float sg_F32(float x, const float *w)
{
    const bool ser = x < 1.0f, asy = x >= 32.0f, quad = !ser && !asy;
    float F = 0.0f, t;
    if (__any(ser)) {
        SG_NO_SPECULATE();
        sg_F_series<float, 8>(x, t, nullptr);
        F = ser ? t : F;
    }
    if (__any(quad)) {
        SG_NO_SPECULATE();
        sg_F_quad<float>(x, w, t, nullptr);
        F = quad ? t : F;
    }
    if (__any(asy)) {
        SG_NO_SPECULATE();
        t = sg_F_asym(x);
        F = asy ? t : F;
    }
    return F;
}

// ------------------------------------------------------------------------
// G0(x) = e^x K0(x), the kernel of the conservative potential (Sect. 5.5,
// appendix "Conservative force"): P_ab(s) = -G0(d^2/8) / (2 sqrt(pi) H_ab).
//   x < 1/2 (float: x < 1)  A&S series of I0 and K0, G0 = e^x K0;
//   1 <= x < 32 (float)  G0 = sqrt(2/x) int_0^inf e^{-v^2}
//        (1 + v^2/(2x))^{-1/2} dv (the same substitution as for F; the
//        trapezoid's v = 0 node has value 1 and weight STEP/2);
//   1/2 <= x < 32 (double)  Chebyshev series on the same dyadic intervals as
//        F (gen_cheb64.cpp, from G0 = int_0^inf e^{-x (cosh t - 1)} dt);
//   x >= 32  sqrt(pi/(2x)) sum_n a_n x^-n, a_0 = 1,
//        a_n = -a_{n-1} (2n - 1)^2 / (8 n), through a_5 (float) or a_16
//        (double: remainder 1.2e-16 at x = 32).
// ------------------------------------------------------------------------
template <typename R, int NT> __device__ inline R sg_G0_series(R x)
{
    const R y = x * x * R(0.25);
    const R Lg = log(x * R(0.5)) + R(SG_EULER_GAMMA);
    R tk = R(1), Hk = R(0), I0 = R(0), K0s = R(0);
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        I0 += tk;
        K0s += Hk * tk;
        tk *= y * (R(1) / R((k + 1) * (k + 1)));
        Hk += R(1) / R(k + 1);
    }
    return exp(x) * (-Lg * I0 + K0s);
}

template <typename R> __device__ inline R sg_G0_quad(R x, const R *w)
{
    const R i2x = R(0.5) * sg_rcp(x);
    R acc = R(0.5);
#pragma unroll
    for (int k = 1; k <= FQuad<R>::NODES; ++k) {
        const R v2 = R(k * k) * (FQuad<R>::STEP * FQuad<R>::STEP);
        acc += w[k - 1] * sg_rsqrt(R(1) + v2 * i2x);
    }
    return acc * FQuad<R>::STEP * R(SG_SQRT2) * sg_rsqrt(x);
}

struct AsymCoefG0 {
    float c[6];
    constexpr AsymCoefG0() : c{}
    {
        double v = 1.0;
        c[0] = 1.0f;
        for (int n = 1; n < 6; ++n) {
            v = -v * (2.0 * n - 1.0) * (2.0 * n - 1.0) / (8.0 * n);
            c[n] = (float)v;
        }
    }
};

// double, x >= 32: through a_16 (LDS table); K0's asymptotic remainder for
// real x is bounded by the first omitted term.
template <bool ROLLED> __device__ inline double sg_G0_asym64(double x, const double *w)
{
    using Q = FQuad<double>;
    const double u = 1.0 / x;
    double s;
    if constexpr (ROLLED) {
        s = w[Q::A + Q::ASYM];
#pragma unroll 1
        for (int n = Q::ASYM - 1; n >= 0; --n) s = s * u + w[Q::A + n];
    } else {
        constexpr AsymCoef64 C;
        s = C.a[Q::ASYM];
#pragma unroll
        for (int n = Q::ASYM - 1; n >= 0; --n) s = s * u + C.a[n];
    }
    return sqrt(SG_PI * 0.5 * u) * s;
}

// double, 1/2 <= x < 32: Clenshaw's recurrence over the G0 coefficients, with
// the interval mapping of sg_F_cheb64.
__device__ inline double sg_G0_cheb64(double x, const double *w)
{
    using Q = FQuad<double>;
    int e;
    const double m = frexp(x, &e);
    const int k = min(max(e, 0), SG_CHEB_NI - 1);
    const double t = 4.0 * m - 3.0, t2 = 2.0 * t;
    const double *cg = w + Q::CHG + k * SG_CHEB_M;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll 3
    for (int j = SG_CHEB_M - 1; j > 0; --j) {
        const double b0 = fma(t2, b1, cg[j] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(t, b1, cg[0] - b2);
}

// Branches as in sg_F64_any: the asymptotic series alone when the whole wave
// has x >= 32, else each of series, Chebyshev and asymptotic series runs when
// some lane needs it.
template <bool ROLLED = false> __device__ inline double sg_G0_64(double x, const double *w)
{
    if (__all(x >= 32.0)) return sg_G0_asym64<ROLLED>(x, w);
    const bool ser = x < 0.5, asy = x >= 32.0, mid = !ser && !asy;
    double G = 0.0;
    if (__any(ser)) {
        SG_NO_SPECULATE();
        const double t = sg_G0_series<double, 10>(x);  // y = x^2/4 < 1/16
        G = ser ? t : G;
    }
    if (__any(mid)) {
        SG_NO_SPECULATE();
        const double t = sg_G0_cheb64(x, w);
        G = mid ? t : G;
    }
    if (__any(asy)) {
        SG_NO_SPECULATE();
        const double t = sg_G0_asym64<ROLLED>(x, w);
        G = asy ? t : G;
    }
    return G;
}

// Branches as in sg_F32: run only when some lane of the wave needs them.
__device__ inline float sg_G0_32(float x, const float *w)
{
    const bool ser = x < 1.0f, asy = x >= 32.0f, quad = !ser && !asy;
    float G = 0.0f;
    if (__any(ser)) {
        SG_NO_SPECULATE();
        const float t = sg_G0_series<float, 8>(x);
        G = ser ? t : G;
    }
    if (__any(quad)) {
        SG_NO_SPECULATE();
        const float t = sg_G0_quad<float>(x, w);
        G = quad ? t : G;
    }
    if (__any(asy)) {
        SG_NO_SPECULATE();
        constexpr AsymCoefG0 C;
        const float u = sg_rcp(x);
        float s = C.c[5];
#pragma unroll
        for (int n = 4; n >= 0; --n) s = s * u + C.c[n];
        const float t = float(SG_SQRT_PI / SG_SQRT2) * sg_rsqrt(x) * s;
        G = asy ? t : G;
    }
    return G;
}

// ------------------------------------------------------------------------
// Log-polar (App. C) kernels for H_f = h_f r, double precision:
//   h^2(X) = (h_a^2 e^{-X} + h_b^2 e^{X}) / 2,  x = (cosh X - cos phi)/(4 h^2),
//   K_r   = F(x) e^{-3X/2} h^{-3} (e^X - cos phi) / (8 sqrt(pi)),
//   K_phi = F(x) e^{-3X/2} h^{-3} sin phi / (8 sqrt(pi)),
// (App. C's L/(pi d^2) [e^{-X}/h^2]^{3/2} with L = sqrt(pi) x F(x), x = d^2/8).
// cosh X - cos phi = 2 sinh^2(X/2) + 2 sin^2(phi/2) and e^X - cos phi =
// expm1(X) + 2 sin^2(phi/2) avoid cancellation near the origin.
// which = 1, 2: derivatives with respect to h_a, h_b:
//   dK/d(h^2) = K-prefactor (h^2)^{-5/2} [-x F'(x) - 3/2 F(x)],
//   d(h^2)/dh_a = h_a e^{-X},  d(h^2)/dh_b = h_b e^{X}.
// sin(phi/2), sin(phi) are passed in so callers can use exact arguments.
// ------------------------------------------------------------------------
// The factors of sg_conv_kernel64 (which = 0) that depend on the row alone
// (X, h_a, h_b): a semi-spectral operator row samples the kernel at N/2 + 1
// azimuths with these fixed, so they are formed once per row.
struct ConvRow64 {
    double two_sxh2;  // 2 sinh^2(X/2) = cosh X - 1
    double em1;       // e^X - 1
    double inv4h2;    // 1 / (4 h_ab^2(X))
    double pref;      // e^{-3X/2} / (8 sqrt(pi) h_ab^3)
};

__device__ inline ConvRow64 sg_conv_row64(double X, double ha, double hb)
{
    const double eX = exp(X);
    const double h2 = 0.5 * (ha * ha / eX + hb * hb * eX);
    const double sxh = sinh(0.5 * X);
    ConvRow64 c;
    c.two_sxh2 = 2.0 * sxh * sxh;
    c.em1 = expm1(X);
    c.inv4h2 = 1.0 / (4.0 * h2);
    c.pref = exp(-1.5 * X) * (1.0 / (8.0 * SG_SQRT_PI)) / (h2 * sqrt(h2));
    return c;
}

// sg_conv_kernel64 (which = 0) at one azimuth of a row.
__device__ inline void sg_conv_kernel64_row(const ConvRow64 &c, double sphi_half, double sphi, const double *w,
                                            double &Kr, double &Kp)
{
    const double two_s2 = 2.0 * sphi_half * sphi_half;
    const double p = sg_F64((c.two_sxh2 + two_s2) * c.inv4h2, w) * c.pref;
    Kr = p * (c.em1 + two_s2);
    Kp = p * sphi;
}

__device__ inline void sg_conv_kernel64(double X, double sphi_half, double sphi, double ha,
                                        double hb, int which, const double *w, double &Kr,
                                        double &Kp)
{
    const double eX = exp(X);
    const double h2 = 0.5 * (ha * ha / eX + hb * hb * eX);
    const double sxh = sinh(0.5 * X);
    const double two_s2 = 2.0 * sphi_half * sphi_half;
    const double cmc = 2.0 * sxh * sxh + two_s2;   // cosh X - cos phi
    const double emc = expm1(X) + two_s2;          // e^X - cos phi
    const double x = cmc / (4.0 * h2);
    const double G = exp(-1.5 * X) * (1.0 / (8.0 * SG_SQRT_PI));
    if (which == 0) {
        const double F = sg_F64(x, w);
        const double pref = F * G / (h2 * sqrt(h2));
        Kr = pref * emc;
        Kp = pref * sphi;
        return;
    }
    double F, dF;
    sg_F64_dF(x, w, F, dF);
    const double dK = G / (h2 * h2 * sqrt(h2)) * (-x * dF - 1.5 * F);
    const double dh2 = which == 1 ? ha / eX : hb * eX;
    Kr = dK * dh2 * emc;
    Kp = dK * dh2 * sphi;
}

// Both h derivatives at once (one F, F' evaluation): (Kr1, Kp1) = d/dh_a,
// (Kr2, Kp2) = d/dh_b, as sg_conv_kernel64 with which = 1 and 2.
__device__ inline void sg_conv_kernel64_dh(double X, double sphi_half, double sphi, double ha, double hb,
                                           const double *w, double &Kr1, double &Kp1, double &Kr2, double &Kp2)
{
    const double eX = exp(X);
    const double h2 = 0.5 * (ha * ha / eX + hb * hb * eX);
    const double sxh = sinh(0.5 * X);
    const double two_s2 = 2.0 * sphi_half * sphi_half;
    const double cmc = 2.0 * sxh * sxh + two_s2;
    const double emc = expm1(X) + two_s2;
    const double x = cmc / (4.0 * h2);
    const double G = exp(-1.5 * X) * (1.0 / (8.0 * SG_SQRT_PI));
    double F, dF;
    sg_F64_dF(x, w, F, dF);
    const double dK = G / (h2 * h2 * sqrt(h2)) * (-x * dF - 1.5 * F);
    const double d1 = dK * (ha / eX), d2 = dK * (hb * eX);
    Kr1 = d1 * emc;
    Kp1 = d1 * sphi;
    Kr2 = d2 * emc;
    Kp2 = d2 * sphi;
}

// X-symmetrised radial kernel used by the self-cell average.
__device__ inline double sg_sym_kr64(double X, double phi, double ha, double hb, int which,
                                     const double *w)
{
    const double sh = sin(0.5 * phi), s = sin(phi);
    double k1, k2, t;
    sg_conv_kernel64(X, sh, s, ha, hb, which, w, k1, t);
    sg_conv_kernel64(-X, sh, s, ha, hb, which, w, k2, t);
    return 0.5 * (k1 + k2);
}
