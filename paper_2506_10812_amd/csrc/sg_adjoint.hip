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
#include "sg_adjoint.h"
#include "sg_fftpath.h"
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

// pass 1 on Sigma (only when dh is requested): same pairing as the forward
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
    const int i1 = NF == 2 ? j : 2 * j, i2 = NF == 2 ? j : 2 * j + 1;
    const int f2 = NF == 2 ? 1 : 0;
    phi_fwd_pair<N>(A.D.sigma + (size_t)i1 * N, A.D.sigma + f2 * plane + (size_t)i2 * N, A.st, i1,
                    A.st + f2 * fs, i2, nr, TwTable{A.D.tw_phi}, t, pl, valid);
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
    const int i1 = NF == 2 ? j : 2 * j, i2 = NF == 2 ? j : 2 * j + 1;
    const int f2 = NF == 2 ? 1 : 0;
    phi_inv_pair<N>(A.dt, i1, A.dt + f2 * fs, i2, nr, TwTable{A.D.tw_phi}, A.dsig + (size_t)i1 * N,
                    A.dsig + f2 * plane + (size_t)i2 * N, t, pl, valid);
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
size_t sg_adjoint_ws_bytes(const sg_disc &d)
{
    const int nf = d.fluids.n_fluids;
    const size_t fs = sg_blk_field_elems(d.grid.n_phi, d.grid.n_r);
    return sg_align256(sizeof(float2) * fs * 2 * nf) + sg_align256(sizeof(float2) * fs * nf) * 2 +
           sg_align256(sizeof(double) * (d.grid.n_phi / 2 + 1) * nf);
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
    const int pairs = NF == 2 ? nr : nr / 2;
    if (dh) {
        A.count = pairs;
        hipLaunchKernelGGL((k_adj_sig<NPHI, NF>), dim3(nwg_for<NPHI>(pairs)),
                           dim3(AdjShape<NPHI>::WGS), 0, s, A);
        SG_HIP(hipGetLastError());
    }
    A.count = ncol;
    if (dh)
        hipLaunchKernelGGL((k_adj_col<NU, NF, true>), dim3(nwg_for<NU>(ncol)),
                           dim3(AdjShape<NU>::WGS), 0, s, A);
    else
        hipLaunchKernelGGL((k_adj_col<NU, NF, false>), dim3(nwg_for<NU>(ncol)),
                           dim3(AdjShape<NU>::WGS), 0, s, A);
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
    case 4096: return adj_launch<NPHI, 4096, NF>(A, dh, d_dh, ncol, s);
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
    const bool want_dh = dh != nullptr;
    if (nf == 1) return adj_phi<1>(nphi, 2 * nr, A, want_dh, dh, ncol, s);
    return adj_phi<2>(nphi, 2 * nr, A, want_dh, dh, ncol, s);
}
