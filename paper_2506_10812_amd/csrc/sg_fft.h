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
// get(n) = e^{-2 pi i n / N} (forward); the transforms conjugate for INV.
struct TwTable {
    const float2 *tab;
    __device__ inline float2 get(int n) const { return tab[n]; }
};

template <int N> struct TwExact64 {
    __device__ inline double2 get(int n) const
    {
        double s, c;
        sincospi(-2.0 * (double)n / (double)N, &s, &c);
        return make_double2(c, s);
    }
};

// ------------------------------------------------------------ LDS exchange
// Separate real / imaginary planes, padded one word per 32 to spread banks.
template <typename R> struct LdsPlane {
    R *re, *im;
    __device__ static inline int pad(int i) { return i + (i >> 5); }
    static constexpr int words(int n) { return n + (n >> 5) + 1; }
};

template <int N> struct FftShape {
    static constexpr int P = N >= 8 ? 8 : N;
    static constexpr int T = N / P;
};

// One Stockham stage.  v: this thread's P points; t: thread index in group.
template <int N, int L, bool INV, typename V, typename TW, typename R>
__device__ inline void fft_stage(V (&v)[FftShape<N>::P], int t, LdsPlane<R> lds, const TW &tw)
{
    constexpr int P = FftShape<N>::P;
    constexpr int T = FftShape<N>::T;
    constexpr int RAD = (N / L) >= P ? P : (N / L);
    constexpr int NB = P / RAD;
    constexpr bool LAST = (L * RAD == N);
    V y[P];
#pragma unroll
    for (int beta = 0; beta < NB; ++beta) {
        const int b = t + T * beta;
        const int k = b & (L - 1);
        V u[RAD];
#pragma unroll
        for (int j = 0; j < RAD; ++j) u[j] = v[beta + NB * j];
        if (L > 1) {
#pragma unroll
            for (int j = 1; j < RAD; ++j) {
                V w = tw.get(j * k * (N / (L * RAD)));
                if (INV) w.y = -w.y;
                u[j] = c_mul(u[j], w);
            }
        }
        dftR<RAD, INV>(u);
        if (LAST) {
#pragma unroll
            for (int j = 0; j < RAD; ++j) y[beta + NB * j] = u[j];
        } else {
            const int base = (b / L) * L * RAD + k;
#pragma unroll
            for (int j = 0; j < RAD; ++j) {
                const int pos = LdsPlane<R>::pad(base + j * L);
                lds.re[pos] = u[j].x;
                lds.im[pos] = u[j].y;
            }
        }
    }
    if (LAST) {
#pragma unroll
        for (int p = 0; p < P; ++p) v[p] = y[p];
    } else {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int pos = LdsPlane<R>::pad(t + T * p);
            v[p].x = lds.re[pos];
            v[p].y = lds.im[pos];
        }
        __syncthreads();
    }
}

template <int N, int L, bool INV, typename V, typename TW, typename R>
__device__ inline void fft_rec(V (&v)[FftShape<N>::P], int t, LdsPlane<R> lds, const TW &tw)
{
    if constexpr (L < N) {
        constexpr int P = FftShape<N>::P;
        constexpr int RAD = (N / L) >= P ? P : (N / L);
        fft_stage<N, L, INV>(v, t, lds, tw);
        fft_rec<N, L * RAD, INV>(v, t, lds, tw);
    }
}

// Full transform (unnormalised): forward X_k = sum x_n e^{-2 pi i nk/N},
// inverse with e^{+...}.
template <int N, bool INV, typename V, typename TW, typename R>
__device__ inline void fft(V (&v)[FftShape<N>::P], int t, LdsPlane<R> lds, const TW &tw)
{
    fft_rec<N, 1, INV>(v, t, lds, tw);
}
