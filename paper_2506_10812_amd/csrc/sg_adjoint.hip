// sg_adjoint.hip -- reverse mode of sg_field_fft for one disc.
//
// The forward map is linear in Sigma: g_{b,c} = sum_a C F^H diag(K'_c^{ab}) F P
// Sigma_a, with P the radial zero padding, C the crop to the first n_r rows,
// F the unnormalised 2D DFT and K' the scaled kernel spectra (App. C
// convolution form; -du dphi/(2 n_r n_phi) folded in).  Its transpose gives
//   dL/dSigma_a = sum_{b,c} P^T F^H diag(conj K'_c^{ab}) F C^T lam_{b,c},
// i.e. the same three passes on lam with conjugated spectra (a correlation
// with the kernel instead of a convolution).  For the aspect ratios,
//   dL/dh = sum_{a,b,c} lam_{b,c}^T C F^H diag(D') F P Sigma_a
//         = sum_k conj(lam^_{b,c}(k)) D'(k) Sigma^_a(k)        (Parseval),
// with D' the scaled spectra of dK/dh_a (attributed to the source fluid a) and
// dK/dh_b (to the target fluid b), self term included.  The sum over the full
// 2D spectrum is taken over the stored half (m <= n_phi/2) with weight 2 for
// 0 < m < n_phi/2 (the three spectra are Hermitian), accumulated in double.
//
// Semi-spectral discs: the middle step is per azimuthal mode, g^(m) =
// M(m) Sigma~(m) with M = T_r (real) for g_r and i t_phi for g_phi, so its
// transpose is dSigma~_a(m, i') = sum_{b,i} [T_r lam~_r^b(m, i) - i t_phi
// lam~_phi^b(m, i)] (T at (m, b, a, i, i')): the same operators read once,
// summed over targets instead of sources (k_ss_adj_full, k_ss_adj_band);
// the phi transforms are those of the FFT-path adjoint.
#include "sg_adjoint.h"
#include "sg_fftpath.h"
#include "sg_kfn.h"
#include "sg_passes.h"

struct AdjDev {
    DiscDev D;
    const float *lam_r, *lam_p;
    float *dsig;
    float2 *lt;     // lam~ [F][2][blk]
    float2 *st;     // Sigma~ [F][blk]  (for dh)
    float2 *dt;     // dSigma~ [F][blk]
    double *part;   // [ncol][F] dh partials
    int count;      // jobs of the launch
};

// Launch shape of the adjoint kernels: one transform per T threads, at least
// 256 threads per workgroup, XCD clusters of K workgroups sharing the 32-byte
// tile columns of the intermediates.
template <int N> struct AdjShape {
    static constexpr int P = FftShape<N>::P;
    static constexpr int T = FftShape<N>::T;
    static constexpr int WGS = T > 256 ? T : 256;
    static constexpr int G = WGS / T;
    static constexpr int K = G >= 4 ? 1 : 4 / G;
};

__device__ inline int adj_job(int G, int K, int g, bool &whole_invalid, int count, bool &valid)
{
    const int wl = sg_xcd_remap(blockIdx.x, K);
    whole_invalid = wl * G >= count;
    const int idx = wl * G + g;
    valid = idx < count;
    return idx;
}

// pass 1 on lam: job (b, i): z = lam_r[b][i] + i lam_phi[b][i]
template <int N>
__global__ void __launch_bounds__(AdjShape<N>::WGS) k_adj_lam(AdjDev A)
{
    using S = AdjShape<N>;
    constexpr int W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t = threadIdx.x % S::T;
    bool none, valid;
    const int idx = adj_job(S::G, S::K, g, none, A.count, valid);
    if (none) return;
    LdsPlane<float> pl{lds + W * g};
    const int nr = A.D.nr;
    const int b = valid ? idx / nr : 0, i = valid ? idx % nr : 0;
    const size_t fs = sg_blk_field_elems(N, nr);
    const size_t row = (size_t)b * nr * N + (size_t)i * N;
    phi_fwd_pair<N>(A.lam_r + row, A.lam_p + row, A.lt + (b * 2 + 0) * fs, i,
                    A.lt + (b * 2 + 1) * fs, i, nr, TwTable{A.D.tw_phi}, t, pl, valid);
}

// Row pairs of the phi transforms of Sigma (adjoint pass 1) and dSigma (pass
// 3): fluid pairs (2p, 2p + 1) row by row, then, for an odd fluid count, the
// last fluid's rows 2q, 2q + 1 (an odd last row pairs with itself).
template <int NF> __host__ __device__ inline int adj_pairs(int nr)
{
    return (NF / 2) * nr + (NF % 2 ? (nr + 1) / 2 : 0);
}

template <int NF> __device__ inline void adj_pair(int j, int nr, int &f1, int &f2, int &i1, int &i2)
{
    const int paired = (NF / 2) * nr;
    if (j < paired) {
        f1 = 2 * (j / nr);
        f2 = f1 + 1;
        i1 = i2 = j % nr;
    } else {
        const int q = j - paired;
        f1 = f2 = NF - 1;
        i1 = 2 * q;
        i2 = min(2 * q + 1, nr - 1);
    }
}

// pass 1 on Sigma (only when dh is requested)
template <int N, int NF>
__global__ void __launch_bounds__(AdjShape<N>::WGS) k_adj_sig(AdjDev A)
{
    using S = AdjShape<N>;
    constexpr int W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t = threadIdx.x % S::T;
    bool none, valid;
    const int idx = adj_job(S::G, S::K, g, none, A.count, valid);
    if (none) return;
    LdsPlane<float> pl{lds + W * g};
    const int nr = A.D.nr;
    const size_t fs = sg_blk_field_elems(N, nr);
    const size_t plane = (size_t)nr * N;
    const int j = valid ? idx : 0;
    int f1, f2, i1, i2;
    adj_pair<NF>(j, nr, f1, f2, i1, i2);
    phi_fwd_pair<N>(A.D.sigma + f1 * plane + (size_t)i1 * N, A.D.sigma + f2 * plane + (size_t)i2 * N,
                    A.st + f1 * fs, i1, A.st + f2 * fs, i2, nr, TwTable{A.D.tw_phi}, t, pl, valid);
}

// pass 2: column m.  dSigma^_a = sum_{b,c} conj(K'_c^{ab}) lam^_{b,c}; with DH,
// also the Parseval partials of lam^ against D' Sigma^ for this column.
template <int NU, int NF, bool DH>
__global__ void __launch_bounds__(AdjShape<NU>::WGS) k_adj_col(AdjDev A)
{
    using S = AdjShape<NU>;
    constexpr int P = S::P, T = S::T, G = S::G;
    constexpr int W = LdsPlane<float>::elems(NU);
    constexpr int NR = NU / 2;
    __shared__ __attribute__((aligned(16))) float2 lds[W * G];
    __shared__ double red[DH ? S::WGS * NF : 1];
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    bool none, valid;
    const int m = adj_job(G, S::K, g, none, A.count, valid);
    if (none) return;
    LdsPlane<float> pl{lds + W * g};
    const TwTable tw{A.D.tw_u};
    const size_t fs = sg_blk_field_elems(A.D.nphi, NR);
    const int mm = valid ? m : 0;

    float2 lh[NF][2][P];
#pragma unroll
    for (int b = 0; b < NF; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                lh[b][c][p] = make_float2(0.f, 0.f);
                if (valid && p < P / 2)
                    lh[b][c][p] = A.lt[(b * 2 + c) * fs + sg_blk_index(mm, t + T * p, NR)];
            }
            fft<NU, false>(lh[b][c], t, pl, tw);
        }
    const size_t kk = NR + 1;
    const float2 *col = A.D.spec + (size_t)mm * (NF * NF) * 2 * kk;
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        float2 acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) {
            acc[p] = make_float2(0.f, 0.f);
            const int k = t + T * p;
#pragma unroll
            for (int b = 0; b < NF; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    // conj(K) * lam^
                    const float2 K = kspec<NU>(col + ((a * NF + b) * 2 + c) * kk, k, c);
                    acc[p].x += K.x * lh[b][c][p].x + K.y * lh[b][c][p].y;
                    acc[p].y += K.x * lh[b][c][p].y - K.y * lh[b][c][p].x;
                }
        }
        fft<NU, true>(acc, t, pl, tw);
        if (valid) {
#pragma unroll
            for (int p = 0; p < P / 2; ++p)
                A.dt[a * fs + sg_blk_index(mm, t + T * p, NR)] = acc[p];
        }
    }
    if constexpr (DH) {
        double dh[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) dh[f] = 0.0;
        const float2 *dcol = A.D.dspec + (size_t)mm * (NF * NF) * 4 * kk;
#pragma unroll
        for (int a = 0; a < NF; ++a) {
            float2 sh[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                sh[p] = make_float2(0.f, 0.f);
                if (valid && p < P / 2) sh[p] = A.st[a * fs + sg_blk_index(mm, t + T * p, NR)];
            }
            fft<NU, false>(sh, t, pl, tw);
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int k = t + T * p;
#pragma unroll
                for (int b = 0; b < NF; ++b)
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        // q = D' Sigma^ ; Re(conj(lam^) q)
                        const double lr = lh[b][c][p].x, li = lh[b][c][p].y;
                        const double sr = sh[p].x, si = sh[p].y;
#pragma unroll
                        for (int d = 0; d < 2; ++d) {
                            const float2 Dk =
                                kspec<NU>(dcol + (((a * NF + b) * 2 + d) * 2 + c) * kk, k, c);
                            const double qr = Dk.x * sr - Dk.y * si, qi = Dk.x * si + Dk.y * sr;
                            const double v = lr * qr + li * qi;
                            dh[d == 0 ? a : b] += v;
                        }
                    }
            }
        }
        const double wm = (mm == 0 || mm == A.D.nphi / 2) ? 1.0 : 2.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) red[f * S::WGS + threadIdx.x] = valid ? wm * dh[f] : 0.0;
        __syncthreads();
        if (t == 0 && valid) {
            for (int f = 0; f < NF; ++f) {
                double s = 0.0;
                for (int u = 0; u < T; ++u) s += red[f * S::WGS + g * T + u];
                A.part[(size_t)m * NF + f] = s;
            }
        }
    }
}

// pass 2 with three or four groups: the same sums taken target by target, so
// that only one lam^ (and, with DH, one Sigma^) transform is held at a time
// next to the NF accumulators: for each (b, c) the transform of lam_{b,c}
// is added to every dSigma^_a with conj(K'_c^{ab}); with DH the Parseval
// partials of lam^_{b,c} against D' Sigma^_a are formed with Sigma^_a
// transformed again for each (b, c) (arithmetic traded for registers).
template <int NU, int NF, bool DH>
__global__ void __launch_bounds__(AdjShape<NU>::WGS) k_adj_col_many(AdjDev A)
{
    using S = AdjShape<NU>;
    constexpr int P = S::P, T = S::T, G = S::G;
    constexpr int W = LdsPlane<float>::elems(NU);
    constexpr int NR = NU / 2;
    __shared__ __attribute__((aligned(16))) float2 lds[W * G];
    __shared__ double red[DH ? S::WGS * NF : 1];
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    bool none, valid;
    const int m = adj_job(G, S::K, g, none, A.count, valid);
    if (none) return;
    LdsPlane<float> pl{lds + W * g};
    const TwTable tw{A.D.tw_u};
    const size_t fs = sg_blk_field_elems(A.D.nphi, NR);
    const int mm = valid ? m : 0;
    const size_t kk = NR + 1;
    const float2 *col = A.D.spec + (size_t)mm * (NF * NF) * 2 * kk;
    const float2 *dcol = DH ? A.D.dspec + (size_t)mm * (NF * NF) * 4 * kk : nullptr;
    float2 acc[NF][P];
    double dh[NF];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        dh[a] = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) acc[a][p] = make_float2(0.f, 0.f);
    }
    for (int b = 0; b < NF; ++b)
        for (int c = 0; c < 2; ++c) {
            float2 lh[P];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                lh[p] = make_float2(0.f, 0.f);
                if (valid && p < P / 2) lh[p] = A.lt[(b * 2 + c) * fs + sg_blk_index(mm, t + T * p, NR)];
            }
            fft<NU, false>(lh, t, pl, tw);
#pragma unroll
            for (int a = 0; a < NF; ++a)
#pragma unroll
                for (int p = 0; p < P; ++p) {
                    // conj(K) * lam^
                    const float2 K = kspec<NU>(col + ((a * NF + b) * 2 + c) * kk, t + T * p, c);
                    acc[a][p].x += K.x * lh[p].x + K.y * lh[p].y;
                    acc[a][p].y += K.x * lh[p].y - K.y * lh[p].x;
                }
            if constexpr (DH) {
                for (int a = 0; a < NF; ++a) {
                    float2 sh[P];
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        sh[p] = make_float2(0.f, 0.f);
                        if (valid && p < P / 2) sh[p] = A.st[a * fs + sg_blk_index(mm, t + T * p, NR)];
                    }
                    fft<NU, false>(sh, t, pl, tw);
#pragma unroll
                    for (int p = 0; p < P; ++p) {
                        const int k = t + T * p;
                        // q = D' Sigma^ ; Re(conj(lam^) q)
                        const double lr = lh[p].x, li = lh[p].y;
                        const double sr = sh[p].x, si = sh[p].y;
#pragma unroll
                        for (int d = 0; d < 2; ++d) {
                            const float2 Dk = kspec<NU>(dcol + (((a * NF + b) * 2 + d) * 2 + c) * kk, k, c);
                            const double qr = Dk.x * sr - Dk.y * si, qi = Dk.x * si + Dk.y * sr;
                            const double v = lr * qr + li * qi;
                            if (d == 0) dh[a] += v;
                            else dh[b] += v;
                        }
                    }
                }
            }
        }
    for (int a = 0; a < NF; ++a) {
        fft<NU, true>(acc[a], t, pl, tw);
        if (valid) {
#pragma unroll
            for (int p = 0; p < P / 2; ++p) A.dt[a * fs + sg_blk_index(mm, t + T * p, NR)] = acc[a][p];
        }
    }
    if constexpr (DH) {
        const double wm = (mm == 0 || mm == A.D.nphi / 2) ? 1.0 : 2.0;
#pragma unroll
        for (int f = 0; f < NF; ++f) red[f * S::WGS + threadIdx.x] = valid ? wm * dh[f] : 0.0;
        __syncthreads();
        if (t == 0 && valid) {
            for (int f = 0; f < NF; ++f) {
                double sm = 0.0;
                for (int u = 0; u < T; ++u) sm += red[f * S::WGS + g * T + u];
                A.part[(size_t)m * NF + f] = sm;
            }
        }
    }
}

// ------------------------------------------------- semi-spectral middle step
// Full modes m < m0: job (m, a, block of 16 source rows i'), four rows per
// wave; lanes run over the targets i (two per lane, 16-byte operator loads
// along the stored row i'), lam~^b(m, .) of both components staged in LDS
// (zero beyond n_r), one wave reduction per row at the end.
__device__ inline float sg_wave_sum(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NF>
__global__ void __launch_bounds__(256) k_ss_adj_full(AdjDev A, int m0)
{
    constexpr int RB = 16, RW = 4;
    __shared__ __attribute__((aligned(16))) float2 lam[2][2048 + 128];
    const int nr = A.D.nr, nrt = (nr + 1) & ~1, nb = (nr + RB - 1) / RB;
    const int job = blockIdx.x;
    if (job >= m0 * NF * nb) return;
    const int blk = job % nb, a = (job / nb) % NF, m = job / (nb * NF);
    const size_t fs = sg_blk_field_elems(A.D.nphi, nr);
    const SsMode md = A.D.modes[m];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int span = (nrt + 127) / 128 * 128;  // staged targets, zero beyond n_r
    float2 acc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) acc[q] = make_float2(0.f, 0.f);
    for (int b = 0; b < NF; ++b) {
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * span; e += 256) {
            const int c = e / span, i = e - c * span;
            lam[c][i] = i < nr ? A.lt[(b * 2 + c) * fs + sg_blk_index(m, i, nr)] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const float2 *C = A.D.spec + md.off + (size_t)(b * NF + a) * nr * nrt;
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int ip = min(blk * RB + wv * RW + q, nr - 1);
            const float2 *row = C + (size_t)ip * nrt;
            for (int i = 2 * lane; i < span; i += 128) {
                const int ic = i < nrt ? i : 0;
                float2 t0, t1;  // (T_r, t_phi) of targets i, i + 1
                gld2x2(row + ic, t0, t1);
                const float2 r0 = lam[0][i], r1 = lam[0][i + 1], p0 = lam[1][i], p1 = lam[1][i + 1];
                acc[q].x += t0.x * r0.x + t0.y * p0.y + t1.x * r1.x + t1.y * p1.y;
                acc[q].y += t0.x * r0.y - t0.y * p0.x + t1.x * r1.y - t1.y * p1.x;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const float x = sg_wave_sum(acc[q].x), y = sg_wave_sum(acc[q].y);
        const int ip = blk * RB + wv * RW + q;
        if (lane == 0 && ip < nr) A.dt[a * fs + sg_blk_index(m, ip, nr)] = make_float2(x, y);
    }
}

// Banded modes m >= m0: job (m, a, block of 256 source rows), one row i' per
// thread: dSigma~(i') = sum_d T[d][i' + w - d] lam~(i' + w - d), the
// diagonal d read lane-consecutively, lam~ from a zero-padded LDS window.
template <int NF>
__global__ void __launch_bounds__(256) k_ss_adj_band(AdjDev A, int m0, int ncol)
{
    __shared__ __attribute__((aligned(16))) float2 lam[2][256 + 2 * 512 + 2];
    const int nr = A.D.nr, nrt = (nr + 1) & ~1, nb = (nr + 255) / 256;
    const int job = blockIdx.x;
    if (job >= (ncol - m0) * NF * nb) return;
    const int blk = job % nb, a = (job / nb) % NF, m = m0 + job / (nb * NF);
    const size_t fs = sg_blk_field_elems(A.D.nphi, nr);
    const SsMode md = A.D.modes[m];
    const int w = md.w, nd = 2 * w + 1, win = 256 + 2 * w;
    if (w > 512) return;  // not a banded mode of a supported grid
    const int ip = blk * 256 + threadIdx.x, base = blk * 256 - w;
    float2 acc = make_float2(0.f, 0.f);
    for (int b = 0; b < NF; ++b) {
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * win; e += 256) {
            const int c = e / win, i = base + (e - c * win);
            lam[c][e - c * win] = (i >= 0 && i < nr) ? A.lt[(b * 2 + c) * fs + sg_blk_index(m, i, nr)]
                                                     : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const float2 *C = A.D.spec + md.off + (size_t)(b * NF + a) * nd * nrt;
        for (int d = 0; d < nd; ++d) {
            const int i = ip + w - d;                     // target of diagonal d
            const int ic = (i >= 0 && i < nrt) ? i : 0;   // lam~ is zero there
            const float2 t = gload2(C, (size_t)d * nrt + ic);
            const int k = threadIdx.x + 2 * w - d;        // window index of i
            const float2 r = lam[0][k], p = lam[1][k];
            acc.x += t.x * r.x + t.y * p.y;
            acc.y += t.x * r.y - t.y * p.x;
        }
    }
    if (ip < nr) A.dt[a * fs + sg_blk_index(m, ip, nr)] = acc;
}

// pass 3: inverse phi transform of dSigma~ pairs (as the forward pass 1 pairing)
template <int N, int NF>
__global__ void __launch_bounds__(AdjShape<N>::WGS) k_adj_out(AdjDev A)
{
    using S = AdjShape<N>;
    constexpr int W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t = threadIdx.x % S::T;
    bool none, valid;
    const int idx = adj_job(S::G, S::K, g, none, A.count, valid);
    if (none) return;
    LdsPlane<float> pl{lds + W * g};
    const int nr = A.D.nr;
    const size_t fs = sg_blk_field_elems(N, nr);
    const size_t plane = (size_t)nr * N;
    const int j = valid ? idx : 0;
    int f1, f2, i1, i2;
    adj_pair<NF>(j, nr, f1, f2, i1, i2);
    phi_inv_pair<N>(A.dt + f1 * fs, i1, A.dt + f2 * fs, i2, nr, TwTable{A.D.tw_phi},
                    A.dsig + f1 * plane + (size_t)i1 * N, A.dsig + f2 * plane + (size_t)i2 * N, t, pl, valid);
}

__global__ void k_adj_dh_reduce(const double *part, int ncol, int nf, double *dh)
{
    __shared__ double red[256];
    for (int f = 0; f < nf; ++f) {
        double s = 0.0;
        for (int m = threadIdx.x; m < ncol; m += blockDim.x) s += part[(size_t)m * nf + f];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = blockDim.x / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) dh[f] = red[0];
        __syncthreads();
    }
}

// ------------------------------------------------------------------- host
#define SG_ADJ_IND_BLOCKS 256

// Indirect-term buffers of the FFT-path adjoint: block partials of (L_A, L_B)
// and their sum, then block partials of the dL/dh sums per fluid.
static size_t adj_ind_bytes()
{
    return sg_align256(sizeof(double2) * (SG_ADJ_IND_BLOCKS + 1)) + sg_align256(sizeof(double) * SG_ADJ_IND_BLOCKS * 4);
}

static size_t adj_base_bytes(const sg_disc &d)
{
    const int nf = d.fluids.n_fluids;
    const size_t fs = sg_blk_field_elems(d.grid.n_phi, d.grid.n_r);
    return sg_align256(sizeof(float2) * fs * 2 * nf) + sg_align256(sizeof(float2) * fs * nf) * 2 +
           sg_align256(sizeof(double) * (d.grid.n_phi / 2 + 1) * nf) + adj_ind_bytes();
}

// ------------------------------------------------ indirect term, FFT path
// The forward adds to every target fluid the field of A + i B = sum_a c_a
// sum_k Sigma_a[k] e^{i phi_k} (c_a in the table header: with H = h r the
// r_k^2 of the cell measure cancels that of K_a), g_r = -(A cos phi + B sin
// phi), g_phi = -(-A sin phi + B cos phi).  Its transpose: with
//   L_A = -sum_{b,i} (lam_r cos phi_i - lam_phi sin phi_i),
//   L_B = -sum_{b,i} (lam_r sin phi_i + lam_phi cos phi_i),
// dL/dSigma_a[k] += c_a (L_A cos phi_k + L_B sin phi_k), and dL/dh_a +=
// c_a' sum_k Sigma_a[k] (L_A cos phi_k + L_B sin phi_k), c_a' the h_a
// derivative of c_a = sqrt(2) pi^{-1/2} F(x) / (4 h_a^3) du dphi,
// x = 1/(4 h_a^2): c_a' = sqrt(2) pi^{-1/2} du dphi (-3 F - 2 x F') / (4 h_a^4).
// Block partials in double are added in a fixed order (deterministic).
__device__ inline void adj_block_sum2(double &a, double &b, double *ra, double *rb)
{
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            ra[threadIdx.x] += ra[threadIdx.x + o];
            rb[threadIdx.x] += rb[threadIdx.x + o];
        }
        __syncthreads();
    }
    a = ra[0];
    b = rb[0];
}

__global__ void __launch_bounds__(256) k_adj_ind_lam(const float *lr, const float *lp, int64_t n, int nphi,
                                                     double2 *part)
{
    __shared__ double ra[256], rb[256];
    const double dphi = 2.0 * SG_PI / nphi;
    double la = 0.0, lb = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) {
        double sp, cp;
        sincos(((double)(k % nphi) + 0.5) * dphi, &sp, &cp);
        const double r = lr[k], p = lp[k];
        la -= r * cp - p * sp;
        lb -= r * sp + p * cp;
    }
    adj_block_sum2(la, lb, ra, rb);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(la, lb);
}

__global__ void k_adj_ind_fin(const double2 *part, int nb, double2 *out)
{
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nb; ++i) {
        a += part[i].x;
        b += part[i].y;
    }
    *out = make_double2(a, b);
}

// dsig[a][k] += c_a (L_A cos phi_k + L_B sin phi_k); with want_dh the block
// partials of sum_k Sigma_a[k] (L_A cos phi_k + L_B sin phi_k) per fluid.
__global__ void __launch_bounds__(256) k_adj_ind_sig(const sg_table_header *hd, const double2 *LAB,
                                                     const float *sig, float *dsig, int nf, int64_t N, int nphi,
                                                     int want_dh, double *spart)
{
    __shared__ double ra[256], rb[256];
    const double dphi = 2.0 * SG_PI / nphi;
    const double2 L = *LAB;
    double sa[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x; k < nf * N; k += (int64_t)gridDim.x * 256) {
        const int a = (int)(k / N);
        double sp, cp;
        sincos(((double)((k % N) % nphi) + 0.5) * dphi, &sp, &cp);
        const double cs = L.x * cp + L.y * sp;
        dsig[k] += (float)(hd->ind_coef[a] * cs);
        if (want_dh) {
#pragma unroll
            for (int f = 0; f < 4; ++f)
                if (a == f) sa[f] += (double)sig[k] * cs;
        }
    }
    if (!want_dh) return;  // uniform across the launch
    for (int f = 0; f < nf; f += 2) {
        __syncthreads();  // ra, rb free again
        adj_block_sum2(sa[f], sa[f + 1], ra, rb);
        if (threadIdx.x == 0) {
            spart[4 * blockIdx.x + f] = sa[f];
            spart[4 * blockIdx.x + f + 1] = sa[f + 1];
        }
    }
}

__global__ void k_adj_ind_dh(const sg_table_header *hd, const double *spart, int nb, int nf, double *dh)
{
    // the wave fills the coefficient table; lane 0 sums
    __shared__ double w[FQuad<double>::TABLE];
    sg_fill_weights<double>(w);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double du = log(hd->r_max / hd->r_min) / hd->n_r, dphi = 2.0 * SG_PI / hd->n_phi;
    for (int a = 0; a < nf; ++a) {
        double S = 0.0;
        for (int b = 0; b < nb; ++b) S += spart[4 * b + a];
        const double h = hd->h[a], x = 0.25 / (h * h);
        double F, dF;
        sg_F64_dF(x, w, F, dF);
        const double cp = SG_SQRT2 / SG_SQRT_PI * du * dphi * (-3.0 * F - 2.0 * x * dF) / (4.0 * h * h * h * h);
        dh[a] += cp * S;
    }
}

static sg_status adjoint_indirect(const sg_disc &d, const float *lam_r, const float *lam_p, float *dsig,
                                  double *dh, char *buf, hipStream_t s)
{
    const int nf = d.fluids.n_fluids;
    const int64_t N = (int64_t)d.grid.n_r * d.grid.n_phi;
    double2 *part = (double2 *)buf;
    double2 *lab = part + SG_ADJ_IND_BLOCKS;
    double *spart = (double *)(buf + sg_align256(sizeof(double2) * (SG_ADJ_IND_BLOCKS + 1)));
    const sg_table_header *hd = (const sg_table_header *)d.table;
    int64_t nb = (nf * N + 255) / 256;
    if (nb > SG_ADJ_IND_BLOCKS) nb = SG_ADJ_IND_BLOCKS;
    hipLaunchKernelGGL(k_adj_ind_lam, dim3((unsigned)nb), dim3(256), 0, s, lam_r, lam_p, nf * N, d.grid.n_phi, part);
    hipLaunchKernelGGL(k_adj_ind_fin, dim3(1), dim3(64), 0, s, (const double2 *)part, (int)nb, lab);
    hipLaunchKernelGGL(k_adj_ind_sig, dim3((unsigned)nb), dim3(256), 0, s, hd, (const double2 *)lab, d.sigma, dsig,
                       nf, N, d.grid.n_phi, dh ? 1 : 0, spart);
    if (dh) hipLaunchKernelGGL(k_adj_ind_dh, dim3(1), dim3(64), 0, s, hd, (const double *)spart, (int)nb, nf, dh);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// Species discs add the group densities and the group dL/dSigma after the
// group run's workspace.
size_t sg_adjoint_ws_bytes(const sg_disc &d)
{
    size_t b = adj_base_bytes(d);
    if (d.n_species) b += 2 * sg_align256(sizeof(float) * d.fluids.n_fluids * (size_t)d.grid.n_r * d.grid.n_phi);
    return b;
}

// ------------------------------------------------------------- species
// The forward sums each group's species rows (in species order, from zero)
// before the transform, so every species of a group has that group's
// dL/dSigma, and dL/dh sees the group sums, formed here in the same order
// so that they equal the forward's bit for bit.
struct SpeciesMap {
    int ns, nf;
    int gcount[4];
    uint8_t gsp[4][8];
    uint8_t group[8];
};

__global__ void k_species_sum(const float *sig, SpeciesMap M, size_t cells, float *gsig)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)M.nf * cells) return;
    const int f = (int)(k / cells);
    const size_t c = k % cells;
    float acc = 0.f;
    for (int j = 0; j < M.gcount[f]; ++j) acc += sig[(size_t)M.gsp[f][j] * cells + c];
    gsig[k] = acc;
}

__global__ void k_species_bcast(const float *gds, SpeciesMap M, size_t cells, float *dsig)
{
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (size_t)M.ns * cells) return;
    const int s = (int)(k / cells);
    dsig[k] = gds[(size_t)M.group[s] * cells + k % cells];
}

static SpeciesMap species_map(const sg_disc &d)
{
    SpeciesMap M{};
    M.ns = d.n_species;
    M.nf = d.fluids.n_fluids;
    for (int sp = 0; sp < d.n_species; ++sp) {
        const int g = d.species_group[sp];
        M.group[sp] = (uint8_t)g;
        M.gsp[g][M.gcount[g]++] = (uint8_t)sp;
    }
    return M;
}

sg_status sg_species_group_sums(const sg_disc &d, float *gsig, hipStream_t s)
{
    const size_t cells = (size_t)d.grid.n_r * d.grid.n_phi, n = (size_t)d.fluids.n_fluids * cells;
    hipLaunchKernelGGL(k_species_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d.sigma, species_map(d),
                       cells, gsig);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

static sg_status adjoint_species(const sg_disc &d, const float *lam_r, const float *lam_p, float *dsig,
                                 double *dh, void *ws, hipStream_t s)
{
    const int nf = d.fluids.n_fluids;
    const size_t cells = (size_t)d.grid.n_r * d.grid.n_phi;
    char *extra = (char *)ws + adj_base_bytes(d);
    float *gsig = (float *)extra;
    float *gds = (float *)(extra + sg_align256(sizeof(float) * nf * cells));
    const SpeciesMap M = species_map(d);
    sg_disc g = d;
    g.n_species = 0;
    g.sigma = gsig;
    if (dh) {
        const size_t n = (size_t)nf * cells;
        hipLaunchKernelGGL(k_species_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d.sigma, M, cells,
                           gsig);
        SG_HIP(hipGetLastError());
    }
    const sg_status st = sg_adjoint_run(g, lam_r, lam_p, gds, dh, ws, s);
    if (st != SG_OK) return st;
    const size_t n = (size_t)d.n_species * cells;
    hipLaunchKernelGGL(k_species_bcast, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gds, M, cells, dsig);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

template <int N> static int nwg_for(int count)
{
    using S = AdjShape<N>;
    int nwg = (count + S::G - 1) / S::G;
    const int q = 8 * S::K;
    return (nwg + q - 1) / q * q;
}

template <int NPHI, int NU, int NF>
static sg_status adj_launch(AdjDev A, bool dh, double *d_dh, int ncol, hipStream_t s)
{
    const int nr = A.D.nr;
    A.count = NF * nr;
    hipLaunchKernelGGL(k_adj_lam<NPHI>, dim3(nwg_for<NPHI>(A.count)), dim3(AdjShape<NPHI>::WGS), 0,
                       s, A);
    SG_HIP(hipGetLastError());
    const int pairs = adj_pairs<NF>(nr);
    if (dh) {
        A.count = pairs;
        hipLaunchKernelGGL((k_adj_sig<NPHI, NF>), dim3(nwg_for<NPHI>(pairs)),
                           dim3(AdjShape<NPHI>::WGS), 0, s, A);
        SG_HIP(hipGetLastError());
    }
    A.count = ncol;
    if constexpr (NF <= 2) {
        if (dh)
            hipLaunchKernelGGL((k_adj_col<NU, NF, true>), dim3(nwg_for<NU>(ncol)),
                               dim3(AdjShape<NU>::WGS), 0, s, A);
        else
            hipLaunchKernelGGL((k_adj_col<NU, NF, false>), dim3(nwg_for<NU>(ncol)),
                               dim3(AdjShape<NU>::WGS), 0, s, A);
    } else {
        if (dh)
            hipLaunchKernelGGL((k_adj_col_many<NU, NF, true>), dim3(nwg_for<NU>(ncol)),
                               dim3(AdjShape<NU>::WGS), 0, s, A);
        else
            hipLaunchKernelGGL((k_adj_col_many<NU, NF, false>), dim3(nwg_for<NU>(ncol)),
                               dim3(AdjShape<NU>::WGS), 0, s, A);
    }
    SG_HIP(hipGetLastError());
    A.count = pairs;
    hipLaunchKernelGGL((k_adj_out<NPHI, NF>), dim3(nwg_for<NPHI>(pairs)),
                       dim3(AdjShape<NPHI>::WGS), 0, s, A);
    SG_HIP(hipGetLastError());
    if (dh) {
        hipLaunchKernelGGL(k_adj_dh_reduce, dim3(1), dim3(256), 0, s, A.part, ncol, NF, d_dh);
        SG_HIP(hipGetLastError());
    }
    return SG_OK;
}

template <int NPHI, int NF>
static sg_status adj_nu(int nu, AdjDev A, bool dh, double *d_dh, int ncol, hipStream_t s)
{
    switch (nu) {
    case 4: return adj_launch<NPHI, 4, NF>(A, dh, d_dh, ncol, s);
    case 8: return adj_launch<NPHI, 8, NF>(A, dh, d_dh, ncol, s);
    case 16: return adj_launch<NPHI, 16, NF>(A, dh, d_dh, ncol, s);
    case 32: return adj_launch<NPHI, 32, NF>(A, dh, d_dh, ncol, s);
    case 64: return adj_launch<NPHI, 64, NF>(A, dh, d_dh, ncol, s);
    case 128: return adj_launch<NPHI, 128, NF>(A, dh, d_dh, ncol, s);
    case 256: return adj_launch<NPHI, 256, NF>(A, dh, d_dh, ncol, s);
    case 512: return adj_launch<NPHI, 512, NF>(A, dh, d_dh, ncol, s);
    case 1024: return adj_launch<NPHI, 1024, NF>(A, dh, d_dh, ncol, s);
    case 2048: return adj_launch<NPHI, 2048, NF>(A, dh, d_dh, ncol, s);
    case 4096:
        if constexpr (NF <= 2) return adj_launch<NPHI, 4096, NF>(A, dh, d_dh, ncol, s);
        else return SG_ERR_UNSUPPORTED;  // beyond two groups n_r <= 1024
    }
    return SG_ERR_UNSUPPORTED;
}

// Semi-spectral disc: lam transform, the two middle kernels, inverse transform.
template <int NPHI, int NF>
static sg_status adj_ss_launch(AdjDev A, int m0, int ncol, hipStream_t s)
{
    const int nr = A.D.nr;
    A.count = NF * nr;
    hipLaunchKernelGGL(k_adj_lam<NPHI>, dim3(nwg_for<NPHI>(A.count)), dim3(AdjShape<NPHI>::WGS), 0, s, A);
    SG_HIP(hipGetLastError());
    if (m0 > 0) {
        hipLaunchKernelGGL(k_ss_adj_full<NF>, dim3(m0 * NF * ((nr + 15) / 16)), dim3(256), 0, s, A, m0);
        SG_HIP(hipGetLastError());
    }
    if (m0 < ncol) {
        hipLaunchKernelGGL(k_ss_adj_band<NF>, dim3((ncol - m0) * NF * ((nr + 255) / 256)), dim3(256), 0, s, A, m0,
                           ncol);
        SG_HIP(hipGetLastError());
    }
    const int pairs = adj_pairs<NF>(nr);
    A.count = pairs;
    hipLaunchKernelGGL((k_adj_out<NPHI, NF>), dim3(nwg_for<NPHI>(pairs)), dim3(AdjShape<NPHI>::WGS), 0, s, A);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

template <int NF>
static sg_status adj_ss_phi(int nphi, AdjDev A, int m0, int ncol, hipStream_t s)
{
    switch (nphi) {
    case 4: return adj_ss_launch<4, NF>(A, m0, ncol, s);
    case 8: return adj_ss_launch<8, NF>(A, m0, ncol, s);
    case 16: return adj_ss_launch<16, NF>(A, m0, ncol, s);
    case 32: return adj_ss_launch<32, NF>(A, m0, ncol, s);
    case 64: return adj_ss_launch<64, NF>(A, m0, ncol, s);
    case 128: return adj_ss_launch<128, NF>(A, m0, ncol, s);
    case 256: return adj_ss_launch<256, NF>(A, m0, ncol, s);
    case 512: return adj_ss_launch<512, NF>(A, m0, ncol, s);
    case 1024: return adj_ss_launch<1024, NF>(A, m0, ncol, s);
    case 2048: return adj_ss_launch<2048, NF>(A, m0, ncol, s);
    }
    return SG_ERR_UNSUPPORTED;
}

template <int NF>
static sg_status adj_phi(int nphi, int nu, AdjDev A, bool dh, double *d_dh, int ncol, hipStream_t s)
{
    switch (nphi) {
    case 4: return adj_nu<4, NF>(nu, A, dh, d_dh, ncol, s);
    case 8: return adj_nu<8, NF>(nu, A, dh, d_dh, ncol, s);
    case 16: return adj_nu<16, NF>(nu, A, dh, d_dh, ncol, s);
    case 32: return adj_nu<32, NF>(nu, A, dh, d_dh, ncol, s);
    case 64: return adj_nu<64, NF>(nu, A, dh, d_dh, ncol, s);
    case 128: return adj_nu<128, NF>(nu, A, dh, d_dh, ncol, s);
    case 256: return adj_nu<256, NF>(nu, A, dh, d_dh, ncol, s);
    case 512: return adj_nu<512, NF>(nu, A, dh, d_dh, ncol, s);
    case 1024: return adj_nu<1024, NF>(nu, A, dh, d_dh, ncol, s);
    case 2048: return adj_nu<2048, NF>(nu, A, dh, d_dh, ncol, s);
    }
    return SG_ERR_UNSUPPORTED;
}

sg_status sg_adjoint_run(const sg_disc &d, const float *lam_r, const float *lam_p, float *dsig,
                         double *dh, void *ws, hipStream_t s)
{
    const int nr = d.grid.n_r, nphi = d.grid.n_phi, nf = d.fluids.n_fluids;
    if (d.n_species) return adjoint_species(d, lam_r, lam_p, dsig, dh, ws, s);
    if (d.flags & SG_SEMI_SPECTRAL) {
        const bool full = (d.flags & SG_SS_FULL) != 0;
        const SsLayout L = sg_ss_layout(nr, nphi, nf, sg_ss_du(d.grid, d.flags), full);
        const char *tb = (const char *)d.table;
        AdjDev A{};
        A.D.spec = (const float2 *)(tb + L.off_coef);
        A.D.modes = (const SsMode *)(tb + L.off_modes);
        A.D.tw_phi = (const float2 *)(tb + L.off_tw_phi);
        A.D.nr = nr;
        A.D.nphi = nphi;
        A.D.nf = nf;
        A.lam_r = lam_r;
        A.lam_p = lam_p;
        A.dsig = dsig;
        const size_t fs = sg_blk_field_elems(nphi, nr);
        A.lt = (float2 *)ws;
        A.dt = (float2 *)((char *)ws + sg_align256(sizeof(float2) * fs * 2 * nf));
        // full modes first (the band shrinks with m), then the banded ones
        int m0 = 0;
        while (m0 < L.ncol && !sg_ss_is_banded(sg_ss_band(m0, nr, L.du, full), nr)) ++m0;
        switch (nf) {
        case 1: return adj_ss_phi<1>(nphi, A, m0, L.ncol, s);
        case 2: return adj_ss_phi<2>(nphi, A, m0, L.ncol, s);
        case 3: return adj_ss_phi<3>(nphi, A, m0, L.ncol, s);
        case 4: return adj_ss_phi<4>(nphi, A, m0, L.ncol, s);
        }
        return SG_ERR_UNSUPPORTED;
    }
    const TableLayout L = sg_table_layout(nr, nphi, nf, d.flags);
    const char *tb = (const char *)d.table;
    AdjDev A{};
    A.D.sigma = d.sigma;
    A.D.spec = (const float2 *)(tb + L.off_spec);
    A.D.dspec = (d.flags & SG_WITH_DH) ? (const float2 *)(tb + L.off_dspec) : nullptr;
    A.D.tw_u = (const float2 *)(tb + L.off_tw_u);
    A.D.tw_phi = (const float2 *)(tb + L.off_tw_phi);
    A.D.nr = nr;
    A.D.nphi = nphi;
    A.D.nf = nf;
    A.lam_r = lam_r;
    A.lam_p = lam_p;
    A.dsig = dsig;
    const size_t fs = sg_blk_field_elems(nphi, nr);
    char *o = (char *)ws;
    A.lt = (float2 *)o;
    o += sg_align256(sizeof(float2) * fs * 2 * nf);
    A.st = (float2 *)o;
    o += sg_align256(sizeof(float2) * fs * nf);
    A.dt = (float2 *)o;
    o += sg_align256(sizeof(float2) * fs * nf);
    A.part = (double *)o;
    const int ncol = nphi / 2 + 1;
    o += sg_align256(sizeof(double) * ncol * nf);
    const bool want_dh = dh != nullptr;
    sg_status st = SG_ERR_UNSUPPORTED;
    switch (nf) {
    case 1: st = adj_phi<1>(nphi, 2 * nr, A, want_dh, dh, ncol, s); break;
    case 2: st = adj_phi<2>(nphi, 2 * nr, A, want_dh, dh, ncol, s); break;
    case 3: st = adj_phi<3>(nphi, 2 * nr, A, want_dh, dh, ncol, s); break;
    case 4: st = adj_phi<4>(nphi, 2 * nr, A, want_dh, dh, ncol, s); break;
    }
    if (st != SG_OK || !(d.flags & SG_INDIRECT)) return st;
    return adjoint_indirect(d, lam_r, lam_p, dsig, dh, o, s);
}
