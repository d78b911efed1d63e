// sg_fft.h -- register/LDS radix-8/4/2 Stockham FFT building blocks (gfx950).
//
// A transform of length N is carried by T = N/P threads ("a group"), each
// holding P = min(8, N) points in registers in the thread-interleaved
// distribution v[p] = x[t + T p].  Every Stockham stage reads its radix-R
// butterfly inputs at stride N/R, which in this distribution are registers of
// the same thread, and writes its outputs to LDS positions that the next
// stage reads back in the same distribution.  The last stage writes to
// positions t + T p again, so the natural-order result stays in registers
// (no exchange): a forward transform leaves X[t + T p] in v[p], which is
// exactly the input distribution of the next inverse transform.  Between the
// two, spectral multiplies are register-local.
//
// Radices: 8 while N/L >= 8, then 4 or 2 for the last stage.  Twiddles come
// from a provider: FP32 reads a precomputed table (double-computed, rounded),
// FP64 computes them with sincospi.
//
// All threads of the workgroup must call the same sequence of transforms
// (stages contain __syncthreads()).
#pragma once
#include "sg_internal.h"

// ------------------------------------------------------------ small DFTs
template <bool INV, typename V> __device__ inline void dft2(V &a, V &b)
{
    V t = a;
    a = c_add(t, b);
    b = c_sub(t, b);
}

template <bool INV, typename V> __device__ inline void dft4(V &v0, V &v1, V &v2, V &v3)
{
    V a = c_add(v0, v2), b = c_sub(v0, v2), c = c_add(v1, v3);
    V d = c_mul_mi<INV>(c_sub(v1, v3));
    v0 = c_add(a, c);
    v2 = c_sub(a, c);
    v1 = c_add(b, d);
    v3 = c_sub(b, d);
}

// multiply by w8^1 = e^{-+ i pi/4}
template <bool INV, typename V> __device__ inline V mul_w8(V a)
{
    using R = decltype(a.x);
    const R s = R(0.70710678118654752440);
    V r;
    if (INV) { r.x = (a.x - a.y) * s; r.y = (a.x + a.y) * s; }
    else     { r.x = (a.x + a.y) * s; r.y = (a.y - a.x) * s; }
    return r;
}
// multiply by w8^3 = e^{-+ 3 i pi/4}
template <bool INV, typename V> __device__ inline V mul_w83(V a)
{
    using R = decltype(a.x);
    const R s = R(0.70710678118654752440);
    V r;
    if (INV) { r.x = (-a.x - a.y) * s; r.y = (a.x - a.y) * s; }
    else     { r.x = (a.y - a.x) * s; r.y = (-a.x - a.y) * s; }
    return r;
}

template <bool INV, typename V> __device__ inline void dft8(V (&u)[8])
{
    dft4<INV>(u[0], u[2], u[4], u[6]);  // E0..E3 in u0,u2,u4,u6
    dft4<INV>(u[1], u[3], u[5], u[7]);  // O0..O3 in u1,u3,u5,u7
    V o1 = mul_w8<INV>(u[3]);
    V o2 = c_mul_mi<INV>(u[5]);
    V o3 = mul_w83<INV>(u[7]);
    V e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6], o0 = u[1];
    u[0] = c_add(e0, o0);
    u[4] = c_sub(e0, o0);
    u[1] = c_add(e1, o1);
    u[5] = c_sub(e1, o1);
    u[2] = c_add(e2, o2);
    u[6] = c_sub(e2, o2);
    u[3] = c_add(e3, o3);
    u[7] = c_sub(e3, o3);
}

template <int R, bool INV, typename V> __device__ inline void dftR(V (&u)[R]);
template <> __device__ inline void dftR<2, false, float2>(float2 (&u)[2]) { dft2<false>(u[0], u[1]); }
template <> __device__ inline void dftR<2, true, float2>(float2 (&u)[2]) { dft2<true>(u[0], u[1]); }
template <> __device__ inline void dftR<2, false, double2>(double2 (&u)[2]) { dft2<false>(u[0], u[1]); }
template <> __device__ inline void dftR<2, true, double2>(double2 (&u)[2]) { dft2<true>(u[0], u[1]); }
template <> __device__ inline void dftR<4, false, float2>(float2 (&u)[4]) { dft4<false>(u[0], u[1], u[2], u[3]); }
template <> __device__ inline void dftR<4, true, float2>(float2 (&u)[4]) { dft4<true>(u[0], u[1], u[2], u[3]); }
template <> __device__ inline void dftR<4, false, double2>(double2 (&u)[4]) { dft4<false>(u[0], u[1], u[2], u[3]); }
template <> __device__ inline void dftR<4, true, double2>(double2 (&u)[4]) { dft4<true>(u[0], u[1], u[2], u[3]); }
template <> __device__ inline void dftR<8, false, float2>(float2 (&u)[8]) { dft8<false>(u); }
template <> __device__ inline void dftR<8, true, float2>(float2 (&u)[8]) { dft8<true>(u); }
template <> __device__ inline void dftR<8, false, double2>(double2 (&u)[8]) { dft8<false>(u); }
template <> __device__ inline void dftR<8, true, double2>(double2 (&u)[8]) { dft8<true>(u); }

// ------------------------------------------------------------ twiddles
// A provider returns e^{-2 pi i n / N} for the flat index n = j k N/(L R) of
// stage S, butterfly beta, leg j (the transforms conjugate for INV).
struct TwTable {
    const float2 *tab;
    template <int S> __device__ inline float2 get(int n, int, int) const { return gload2(tab, n); }
};


// ------------------------------------------------------------ LDS exchange
// One plane of N complex values per transform (plus one pad element per 16),
// accessed with 64-bit (float2) or 128-bit (double2) LDS instructions at
// pad(i) = i + (i >> 4).  For every Stockham stage of this radix plan the
// butterfly's R outputs go to pad(base) + (jL + (jL >> 4)) -- a compile-time
// offset from one address -- and the reads to pad(t) + (Tp + (Tp >> 4)), so
// no per-element address arithmetic is needed; the residual bank conflicts
// average ~1.17x for 16-lane 64-bit access groups (checked exhaustively for
// N = 512..4096 when the layout was chosen).
template <typename R> struct LdsPlane {
    using V = cplx_t<R>;
    V *c;
    __device__ static inline int pad(int i) { return i + (i >> 4); }
    static constexpr int off(int d) { return d + (d >> 4); }
    __device__ inline void st(int i, V v) const { c[pad(i)] = v; }
    __device__ inline V ld(int i) const { return c[pad(i)]; }
    static constexpr int elems(int n) { return n + n / 16 + 1; }
};

template <int N> struct FftShape {
    static constexpr int P = N >= 8 ? 8 : N;
    static constexpr int T = N / P;
};

// Compile-time stage plan: stage s has sub-length L(s), radix RAD(s) and
// NB(s) butterflies per thread; TWOFF(s) is the offset of its twiddles in a
// per-thread register table (stage 0 needs none).  When N is not a power of
// P, one stage has the smaller radix N / P^k: the last one by default, the
// first one (which needs no twiddles) when SF is set.
template <int N, bool SF = false> struct FftPlan {
    static constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
    static constexpr int SMALL() { int r = N; while (r >= P) r /= P; return r; }  // 1 if none
    static constexpr int L(int s) { int l = 1; for (int i = 0; i < s; ++i) l *= RAD(i); return l; }
    static constexpr int RAD(int s)
    {
        if (SF && SMALL() > 1) return s == 0 ? SMALL() : P;
        int l = 1;
        for (int i = 0; i < s; ++i) l *= (N / l) >= P ? P : (N / l);
        return (N / l) >= P ? P : (N / l);
    }
    static constexpr int NB(int s) { return P / RAD(s); }
    static constexpr int NST() { int s = 0; while (L(s) < N) ++s; return s; }
    static constexpr int TWOFF(int s) { int o = 0; for (int i = 1; i < s; ++i) o += NB(i) * (RAD(i) - 1); return o; }
    static constexpr int NTW() { return TWOFF(NST()) > 0 ? TWOFF(NST()) : 1; }
};

// Twiddles of one thread for every stage, loaded once from the table and
// kept in registers (all indices compile-time after unrolling).
template <int N> struct TwReg {
    float2 w[FftPlan<N>::NTW()];
    __device__ inline void load(const float2 *tab, int t) { load_stage<1>(tab, t); }
    template <int S> __device__ inline void load_stage(const float2 *g, int t)
    {
        using PL = FftPlan<N>;
        if constexpr (S < PL::NST()) {
            constexpr int Ls = PL::L(S), R = PL::RAD(S), NB = PL::NB(S), O = PL::TWOFF(S);
#pragma unroll
            for (int beta = 0; beta < NB; ++beta) {
                const int k = (t + PL::T * beta) & (Ls - 1);
#pragma unroll
                for (int j = 1; j < R; ++j) w[O + beta * (R - 1) + j - 1] = gload2(g, j * k * (N / (Ls * R)));
            }
            load_stage<S + 1>(g, t);
        }
    }
    template <int S> __device__ inline float2 get(int, int beta, int j) const
    {
        using PL = FftPlan<N>;
        return w[PL::TWOFF(S) + beta * (PL::RAD(S) - 1) + j - 1];
    }
};

// Compact variant: one twiddle w^k per (stage, butterfly) in registers; the
// powers w^{jk} are formed by complex products (depth <= 3, a few ulps),
// once per stage and shared by all transforms of the stage.
template <int N, bool SF = false> struct FftPlanC {
    using PL = FftPlan<N, SF>;
    static constexpr int OFF(int s) { int o = 0; for (int i = 1; i < s; ++i) o += PL::NB(i); return o; }
    static constexpr int NTW() { return OFF(PL::NST()) > 0 ? OFF(PL::NST()) : 1; }
};

template <int N, bool SF = false> struct TwRegC {
    using Plan = FftPlan<N, SF>;
    float2 w[FftPlanC<N, SF>::NTW()];
    static constexpr bool POWERS = true;
    __device__ inline void load(const float2 *tab, int t) { load_stage<1>(tab, t); }
    template <int S> __device__ inline void load_stage(const float2 *g, int t)
    {
        using PL = Plan;
        if constexpr (S < PL::NST()) {
            constexpr int Ls = PL::L(S), R = PL::RAD(S), NB = PL::NB(S);
#pragma unroll
            for (int beta = 0; beta < NB; ++beta) {
                const int k = (t + PL::T * beta) & (Ls - 1);
                w[FftPlanC<N, SF>::OFF(S) + beta] = gload2(g, k * (N / (Ls * R)));
            }
            load_stage<S + 1>(g, t);
        }
    }
    template <int S> __device__ inline float2 base(int beta) const { return w[FftPlanC<N, SF>::OFF(S) + beta]; }
};

// Stage plan of a twiddle provider: its own Plan type, else the default.
// Double twiddles for the FP64 row transforms of the table builds: one exact
// base e^{-2 pi i k/(L R)} per butterfly (sincospi), legs j = 2..R-1 as its
// powers by complex products (a few ulps in double; every caller rounds the
// result to float or accumulates a derivative checked at 1e-6), so a
// length-2048 transform evaluates 3 sincospi per thread instead of 17.
template <int N> struct TwPow64 {
    using Plan = FftPlan<N>;
    static constexpr bool POWERS = true;
    int t;  // thread index within the transform
    template <int S> __device__ inline double2 base(int beta) const
    {
        constexpr int L = Plan::L(S), LR = Plan::L(S) * Plan::RAD(S);
        const int k = (t + Plan::T * beta) & (L - 1);
        double s, c;
        sincospi(-2.0 * (double)k / (double)LR, &s, &c);
        return make_double2(c, s);
    }
};

template <typename TW, int N, typename = void> struct plan_of { using type = FftPlan<N>; };
template <typename TW, int N> struct plan_of<TW, N, decltype((void)sizeof(typename TW::Plan), void())> {
    using type = typename TW::Plan;
};

template <typename TW, typename = void> struct tw_has_powers { static constexpr bool value = false; };
template <typename TW> struct tw_has_powers<TW, decltype((void)TW::POWERS, void())> {
    static constexpr bool value = TW::POWERS;
};

// One Stockham stage on M independent transforms sharing the barriers.
// v[m]: this thread's P points of transform m; t: thread index in the group.
template <int N, int S, bool INV, int M, typename V, typename TW, typename R>
__device__ inline void fft_stage_m(V (&v)[M][FftShape<N>::P], int t, const LdsPlane<R> (&lds)[M],
                                   const TW &tw)
{
    using PL = typename plan_of<TW, N>::type;
    constexpr int P = PL::P;
    constexpr int T = PL::T;
    constexpr int L = PL::L(S);
    constexpr int RAD = PL::RAD(S);
    constexpr int NB = PL::NB(S);
    constexpr bool LAST = (L * RAD == N);
    V w[NB][RAD];
    if (L > 1) {
#pragma unroll
        for (int beta = 0; beta < NB; ++beta) {
            if constexpr (tw_has_powers<TW>::value) {
                V x = tw.template base<S>(beta);
                if (INV) x.y = -x.y;
                w[beta][1] = x;
                if constexpr (RAD > 2) w[beta][2] = c_mul(x, x);
                if constexpr (RAD > 3) w[beta][3] = c_mul(w[beta][2], x);
                if constexpr (RAD > 4) {
                    w[beta][4] = c_mul(w[beta][2], w[beta][2]);
                    w[beta][5] = c_mul(w[beta][4], x);
                    w[beta][6] = c_mul(w[beta][4], w[beta][2]);
                    w[beta][7] = c_mul(w[beta][4], w[beta][3]);
                }
            } else {
                const int k = (t + T * beta) & (L - 1);
#pragma unroll
                for (int j = 1; j < RAD; ++j) {
                    V x = tw.template get<S>(j * k * (N / (L * RAD)), beta, j);
                    if (INV) x.y = -x.y;
                    w[beta][j] = x;
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        V y[P];
#pragma unroll
        for (int beta = 0; beta < NB; ++beta) {
            const int b = t + T * beta;
            const int k = b & (L - 1);
            V u[RAD];
#pragma unroll
            for (int j = 0; j < RAD; ++j) u[j] = v[m][beta + NB * j];
            if (L > 1) {
#pragma unroll
                for (int j = 1; j < RAD; ++j) u[j] = c_mul(u[j], w[beta][j]);
            }
            dftR<RAD, INV>(u);
            if (LAST) {
#pragma unroll
                for (int j = 0; j < RAD; ++j) y[beta + NB * j] = u[j];
            } else {
                const int pb = LdsPlane<R>::pad((b / L) * L * RAD + k);
#pragma unroll
                for (int j = 0; j < RAD; ++j) lds[m].c[pb + LdsPlane<R>::off(j * L)] = u[j];
            }
        }
        if (LAST) {
#pragma unroll
            for (int p = 0; p < P; ++p) v[m][p] = y[p];
        }
    }
    if (!LAST) {
        __syncthreads();
        const int pt = LdsPlane<R>::pad(t);
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int p = 0; p < P; ++p) v[m][p] = lds[m].c[pt + LdsPlane<R>::off(T * p)];
        __syncthreads();
    }
}

template <int N, int S, bool INV, int M, typename V, typename TW, typename R>
__device__ inline void fft_rec_m(V (&v)[M][FftShape<N>::P], int t, const LdsPlane<R> (&lds)[M],
                                 const TW &tw)
{
    if constexpr (S < plan_of<TW, N>::type::NST()) {
        fft_stage_m<N, S, INV, M>(v, t, lds, tw);
        fft_rec_m<N, S + 1, INV, M>(v, t, lds, tw);
    }
}

// M independent transforms (unnormalised): forward X_k = sum x_n e^{-2 pi i nk/N},
// inverse with e^{+...}.
template <int N, bool INV, int M, typename V, typename TW, typename R>
__device__ inline void fft_m(V (&v)[M][FftShape<N>::P], int t, const LdsPlane<R> (&lds)[M],
                             const TW &tw)
{
    fft_rec_m<N, 0, INV, M>(v, t, lds, tw);
}

// Single transform.
template <int N, bool INV, typename V, typename TW, typename R>
__device__ inline void fft(V (&v)[FftShape<N>::P], int t, LdsPlane<R> lds, const TW &tw)
{
    constexpr int P = FftShape<N>::P;
    V vv[1][P];
#pragma unroll
    for (int p = 0; p < P; ++p) vv[0][p] = v[p];
    const LdsPlane<R> l1[1] = {lds};
    fft_m<N, INV, 1>(vv, t, l1, tw);
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = vv[0][p];
}
