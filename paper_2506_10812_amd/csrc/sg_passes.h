// sg_passes.h -- the three device passes of the log-polar FFT convolution
// (App. C convolution form with the radial zero padding of Sect. 5.2) and the
// pieces the adjoint reuses.  Float arithmetic throughout.
//
// Data flow for one disc (F fluids, n_r x n_phi, NU = 2 n_r):
//   pass 1  rows:    Sigma (real) --phi FFT--> Sigma~[a][m][i], m <= n_phi/2
//                    (two real rows per complex transform, Hermitian split)
//   pass 2  columns: Sigma~[.][m][:] --zero-padded u FFT (length NU)-->
//                    multiply by the kernel spectra of every ordered pair and
//                    both components (gg, dg, gd, dd fused) --inverse u FFT,
//                    first n_r outputs--> g^[b][c][m][i]
//   pass 3  rows:    g^[b][r][.][i] + i g^[b][phi][.][i] --inverse phi FFT-->
//                    g_r[b][i][:] + i g_phi[b][i][:]  (two real outputs per
//                    complex transform)
// The kernel spectra already carry the factor -du dphi/(2 n_r n_phi), so no
// pass scales.  Intermediates use the tiled layout of sg_blk_index.
#pragma once
#include "sg_fft.h"

struct DiscDev {
    const float *sigma;
    float *gr, *gp;
    const float2 *spec;     // [m][pair][c][kk]
    const float2 *dspec;    // [m][pair][d][c][kk] or null
    const float2 *tw_u, *tw_phi;
    float2 *st;             // [F][blk]
    float2 *gh;             // [F][2][blk]
    const double *ind;      // table header: indirect-term coefficients [F]
    int nr, nphi, nf;
    uint32_t flags;
    const SsMode *modes;    // semi-spectral table: mode descriptors
    int ss_wmax;            // widest band of the grid's banded modes (-1: none)
    int ns;                 // species summed into groups (0: one density per fluid)
    int gcount[4];          // species of each group
    uint8_t gsp[4][8];      // their indices
};

// A job is (disc index, job index inside the disc); disc < 0 marks padding.
struct Job {
    int disc, idx;
};

// Workgroup job of the passes: groups g < n of the workgroup take
// jobs base + g of disc `disc`; groups g >= n (and all groups when n = 0)
// repeat job `base` without storing, so every load address stays valid.
struct WJob {
    int disc, base, n, pad_;
};

// Launch shape of pass 3, shared by host and device: G transforms (rows) per
// workgroup, a multiple of 4 and at least 256 threads, times the tile-shape
// factor GM (a tuning parameter); K: default XCD cluster size.
template <int N, int GM = 1> struct PassShape {
    static constexpr int P = FftShape<N>::P;
    static constexpr int T = FftShape<N>::T;
    static constexpr int G = GM * (256 / T > 4 ? 256 / T : 4);
    static constexpr int WGS = G * T;
    static constexpr int K = 1;
};

// ------------------------------------------------------------------ pass 1
// Forward phi transform of two real rows x1 + i x2 (length N) followed by the
// Hermitian split
//   X1[m] = (Z[m] + conj Z[-m]) / 2,  X2[m] = (Z[m] - conj Z[-m]) / (2i),
// written for m in [0, N/2] to block-layout fields d1 (row i1) and d2 (row i2).
//
// Loads are unconditional (padding groups pass valid addresses) so that they
// are all in flight at once; only the stores depend on `valid`.
template <int N>
__device__ inline void p1_load(const float *x1, const float *x2, float2 (&z)[FftShape<N>::P], int t)
{
    constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
#pragma unroll
    for (int p = 0; p < P; ++p) z[p] = make_float2(gload1(x1, t + T * p), gload1(x2, t + T * p));
}

template <int N, typename TW>
__device__ inline void p1_finish(float2 (&z)[FftShape<N>::P], float2 *d1, int i1, float2 *d2,
                                 int i2, int nr, const TW &tw, int t, LdsPlane<float> pl,
                                 bool valid)
{
    constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
    fft<N, false>(z, t, pl, tw);
#pragma unroll
    for (int p = 0; p < P; ++p) pl.st(t + T * p, z[p]);
    __syncthreads();
    if (valid) {
#pragma unroll
        for (int p = 0; p <= P / 2; ++p) {
            const int m = t + T * p;
            if (p == P / 2 && t != 0) break;
            const float2 Z = pl.ld(m);
            const float2 C = pl.ld((N - m) & (N - 1));
            // conj(C) = (C.x, -C.y)
            const float2 v1 = make_float2(0.5f * (Z.x + C.x), 0.5f * (Z.y - C.y));
            const float2 v2 = make_float2(0.5f * (Z.y + C.y), -0.5f * (Z.x - C.x));
            gst2(d1, (uint32_t)sg_blk_index(m, i1, nr), v1);
            gst2(d2, (uint32_t)sg_blk_index(m, i2, nr), v2);
        }
    }
    __syncthreads();
}

template <int N, typename TW>
__device__ inline void phi_fwd_pair(const float *x1, const float *x2, float2 *d1, int i1,
                                    float2 *d2, int i2, int nr, const TW &tw, int t,
                                    LdsPlane<float> pl, bool valid)
{
    float2 z[FftShape<N>::P];
    p1_load<N>(x1, x2, z, t);
    p1_finish<N>(z, d1, i1, d2, i2, nr, tw, t, pl, valid);
}

// ------------------------------------------------------------------ pass 3
// Inverse phi transform of A + i B, where A (row iA) and B (row iB) are half
// spectra of real rows extended by G[N - m] = conj G[m]; the real and
// imaginary parts of the result are the two real rows o1, o2.  Loads, their
// combination and the transform are separate steps for the same reason as
// in pass 1.
template <int N>
__device__ inline void p3_load(const float2 *A, int iA, const float2 *B, int iB, int nr,
                               float2 (&a)[FftShape<N>::P], float2 (&b)[FftShape<N>::P], int t)
{
    constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int m = t + T * p;
        const int mm = m > N / 2 ? N - m : m;
        a[p] = gld2(A, (uint32_t)sg_blk_index(mm, iA, nr));
        b[p] = gld2(B, (uint32_t)sg_blk_index(mm, iB, nr));
    }
}

template <int N>
__device__ inline void p3_combine(const float2 (&a)[FftShape<N>::P], const float2 (&b)[FftShape<N>::P],
                                  float2 (&z)[FftShape<N>::P], int t)
{
    constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int m = t + T * p;
        float2 x = a[p], y = b[p];
        const float s = m > N / 2 ? -1.f : 1.f;  // upper half: conjugate of the mirror
        x.y *= s;
        y.y *= s;
        z[p] = make_float2(x.x - y.y, x.y + y.x);  // x + i y
    }
}

template <int N, typename TW>
__device__ inline void p3_finish(float2 (&z)[FftShape<N>::P], const TW &tw, float *o1, float *o2,
                                 int t, LdsPlane<float> pl, bool valid)
{
    constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
    fft<N, true>(z, t, pl, tw);
    if (valid) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            gst1(o1, t + T * p, z[p].x);
            gst1(o2, t + T * p, z[p].y);
        }
    }
}

template <int N, typename TW>
__device__ inline void phi_inv_pair(const float2 *A, int iA, const float2 *B, int iB, int nr,
                                    const TW &tw, float *o1, float *o2, int t,
                                    LdsPlane<float> pl, bool valid)
{
    constexpr int P = FftShape<N>::P;
    float2 a[P], b[P], z[P];
    p3_load<N>(A, iA, B, iB, nr, a, b, t);
    p3_combine<N>(a, b, z, t);
    p3_finish<N>(z, tw, o1, o2, t, pl, valid);
}

// Kernel-spectrum lookup at u-frequency k (0 <= k < NU) for component c:
// stored for k <= NU/2; K_r is Hermitian and K_phi anti-Hermitian in k.
template <int NU>
__device__ inline float2 kspec(const float2 *col, int k, int c)
{
    constexpr int H = NU / 2;
    if (k <= H) return col[k];
    const float2 v = col[NU - k];
    return c == 0 ? make_float2(v.x, -v.y) : make_float2(-v.x, v.y);
}

// Load of the kernel spectrum at k = t + T p in the thread-interleaved
// distribution: for p < P/2 the stored half is read directly; for p >= P/2
// the mirror NU - k is read and conjugated (negated too for K_phi).  The
// Nyquist point k = NU/2 (t = 0, p = P/2) reads itself, whose value is real
// (K_r) or imaginary (K_phi), so the same rule holds for it.
template <int NU, int P, int C>
__device__ inline float2 kspec_p(const float2 *col, int t, int p)
{
    constexpr int T = NU / P;
    const int k = t + T * p;
    if (p < P / 2) return gload2(col, k);
    const float2 v = gload2(col, NU - k);
    return C == 0 ? make_float2(v.x, -v.y) : make_float2(-v.x, v.y);
}

// Branch-free form on a global pointer: mirror index and sign by select.
template <int NU>
__device__ inline float2 kspec_g(const float2 *col, int k, int c)
{
    constexpr int H = NU / 2;
    const bool up = k > H;
    const float2 v = gload2(col, up ? NU - k : k);
    const float sy = up ? -1.f : 1.f;           // conjugate in the upper half
    const float sx = (up && c == 1) ? -1.f : 1.f;  // K_phi: minus conjugate
    return make_float2(sx * v.x, sx * sy * v.y);
}
