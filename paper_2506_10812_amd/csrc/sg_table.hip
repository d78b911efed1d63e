// sg_table.hip -- one-off, double-precision construction of the kernel
// spectra for the log-polar FFT path (sg_kernel_table), the self-cell
// quadrature, and device evaluation of F for tests.
//
// App. C: with H_f = h_f r the radial and azimuthal fields are convolutions
// in (u = ln r, phi) with offset-only kernels K_r(X, phi), K_phi(X, phi);
// Sect. 5.2: zero padding of the radial axis to 2 n_r makes the periodic
// convolution equal the aperiodic one, and the kernel is computed once.
// Steps (all double precision):
//   1. sample K_r + i K_phi on the wrapped offset grid X = p du
//      (p in (-n_r, n_r), stored at p mod 2 n_r; row n_r is zero), phi = q dphi;
//      offset (0,0) holds the self-cell average (SG_SECOND_ORDER: every entry,
//      (0,0) included, is the hat-weighted integral of the kernel instead);
//   2. phi transform of each row, split into the spectra of K_r and K_phi
//      (two real rows in one complex transform);
//   3. u transform (length 2 n_r) of each column m <= n_phi/2, keep
//      k_u <= n_r (K_r is Hermitian and K_phi anti-Hermitian in k_u because
//      K_r is even and K_phi odd in phi), scale by -du dphi/(2 n_r n_phi),
//      round to float.
#include "sg_fft.h"
#include "sg_kfn.h"
#include "sg_table.h"
#include "sg_hat.h"

// ------------------------------------------------------------------ twiddles
__global__ void k_twiddles(float2 *tw_u, int nu, float2 *tw_phi, int nphi)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nu) {
        double s, c;
        sincospi(-2.0 * i / nu, &s, &c);
        tw_u[i] = make_float2((float)c, (float)s);
    }
    if (i < nphi) {
        double s, c;
        sincospi(-2.0 * i / nphi, &s, &c);
        tw_phi[i] = make_float2((float)c, (float)s);
    }
}

// --------------------------------------------------------------- self cell
// Kbar = (1/(du dphi)) PV-int over the own cell of K_r.  By symmetry
// (K_r even in phi; its 1/rho singularity odd in X) it is (1/(a b)) times the
// integral of S = (K_r(X,phi) + K_r(-X,phi))/2 over [0,a]x[0,b], a = du/2,
// b = dphi/2.  The quarter cell is cut along its diagonal; each triangle is
// mapped to the unit square with the singular corner collapsed
// (X = a xi, phi = b xi eta and X = a xi eta, phi = b xi; Jacobian a b xi),
// which turns the direction-dependent limit at the corner into a smooth
// integrand.  eta: one Gauss-Legendre rule; xi: Gauss-Legendre on geometric
// panels [0, 4^-6], [4^-(j+1), 4^-j] so that the transition of F at distances
// ~H inside cells much larger than H is resolved.  Nodes come from the host.
__device__ inline double self_cell_partial(double ha, double hb, int which, double a, double b,
                                           const GLNodes &gl, const double *wq)
{
    constexpr int NX = SG_PANELS * SG_GLX_N;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < NX * SG_GL_N; idx += blockDim.x) {
        const int ix = idx / SG_GL_N, j = idx % SG_GL_N;
        const int pnl = ix / SG_GLX_N, i = ix % SG_GLX_N;
        const double hi = ldexp(1.0, -2 * (SG_PANELS - 1 - pnl));
        const double lo = pnl == 0 ? 0.0 : 0.25 * hi;
        const double xi = lo + (hi - lo) * gl.xr[i];
        const double eta = gl.x[j];
        const double wgt = (hi - lo) * gl.wr[i] * gl.w[j] * xi;
        acc += wgt * (sg_sym_kr64(a * xi, b * xi * eta, ha, hb, which, wq) +
                      sg_sym_kr64(a * xi * eta, b * xi, ha, hb, which, wq));
    }
    return acc;
}

__device__ inline double block_sum256(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

__global__ void k_self_cell(SelfItems items, double *out, double du, double dphi, GLNodes gl)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int it = blockIdx.x;
    const double acc = self_cell_partial(items.ha[it], items.hb[it], items.which[it], 0.5 * du,
                                         0.5 * dphi, gl, wq);
    const double tot = block_sum256(acc, red);
    if (threadIdx.x == 0) out[it] = tot;
}

// Per-cell variant for the direct path with general H: item = (pair, cell);
// h_a = H_a[i]/r_i, h_b = H_b[i]/r_i computed from the caller's arrays.
template <typename T>
__global__ void k_self_cell_percell(const T *H, int nf, int nr, int nphi, double lnrmin, double du,
                                    double dphi, double *out, GLNodes gl)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int64_t N = (int64_t)nr * nphi;
    const int64_t item = blockIdx.x;  // pair * N + cell
    if (item >= (int64_t)nf * nf * N) return;
    const int pair = (int)(item / N);
    const int64_t cell = item % N;
    const int fa = pair / nf, fb = pair % nf;
    const int ir = (int)(cell / nphi);
    const double r = exp(lnrmin + (ir + 0.5) * du);
    const double ha = (double)H[fa * N + cell] / r, hb = (double)H[fb * N + cell] / r;
    const double acc = self_cell_partial(ha, hb, 0, 0.5 * du, 0.5 * dphi, gl, wq);
    const double tot = block_sum256(acc, red);
    if (threadIdx.x == 0) out[item] = tot;
}
// Per-ring variant with a derivative selector for the semi-spectral
// gradient: item = (pair, ring), h = H[f][ring] / r; which = 0: Kbar,
// 1: dKbar/dh_a, 2: dKbar/dh_b.
__global__ void k_self_cell_ring(const double *H, int nf, int nr, double lnrmin, double du, double dphi, int which,
                                 double *out, GLNodes gl)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int item = blockIdx.x;
    if (item >= nf * nf * nr) return;
    const int pair = item / nr, ir = item % nr;
    const int fa = pair / nf, fb = pair % nf;
    const double r = exp(lnrmin + (ir + 0.5) * du);
    const double acc = self_cell_partial(H[fa * nr + ir] / r, H[fb * nr + ir] / r, which, 0.5 * du, 0.5 * dphi, gl, wq);
    const double tot = block_sum256(acc, red);
    if (threadIdx.x == 0) out[item] = tot;
}

template __global__ void k_self_cell_percell<float>(const float *, int, int, int, double, double,
                                                    double, double *, GLNodes);
template __global__ void k_self_cell_percell<double>(const double *, int, int, int, double, double,
                                                     double, double *, GLNodes);

// Own-cell integral of the potential kernel (reading: the paper does not
// treat k = i): int P_ab(|x_i - x'|) dA' over the cell, x' = r e^X (cos phi,
// sin phi) relative to the centre direction, |x_i - x'|^2 = r^2 e^X
// (4 sinh^2(X/2) + 4 sin^2(phi/2)), dA' = r^2 e^{2X} dX dphi; even in phi,
// so 2 x (X >= 0 and X <= 0 halves) over [0,a]x[0,b] with the same Duffy
// rule as the force self term (the singularity is logarithmic).
// which = 0: P; which = 1: dP/dH_ab (H_ab the r.m.s. height: with
// G0 = e^y K0(y), dG0/dy = -F(y), so dP/dH = -(2 y F(y) - G0(y)) /
// (2 sqrt(pi) H^2); like P, logarithmic at s -> 0).
__device__ inline double pot_integrand(double X, double phi, double r, double Hab, const double *wq, int which = 0)
{
    const double sx = sinh(0.5 * X), sp = sin(0.5 * phi);
    const double s2 = r * r * exp(X) * 4.0 * (sx * sx + sp * sp);
    const double y = s2 / (8.0 * Hab * Hab);
    if (which) return -(2.0 * y * sg_F64(y, wq) - sg_G0_64(y, wq)) / (2.0 * SG_SQRT_PI * Hab * Hab) * r * r * exp(2.0 * X);
    return -sg_G0_64(y, wq) / (2.0 * SG_SQRT_PI * Hab) * r * r * exp(2.0 * X);
}

__device__ inline double pot_self_partial(double r, double Hab, double a, double b, const GLNodes &gl,
                                          const double *wq, int which = 0)
{
    constexpr int NX = SG_PANELS * SG_GLX_N;
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < NX * SG_GL_N; idx += blockDim.x) {
        const int ix = idx / SG_GL_N, j = idx % SG_GL_N;
        const int pnl = ix / SG_GLX_N, i = ix % SG_GLX_N;
        const double hi = ldexp(1.0, -2 * (SG_PANELS - 1 - pnl));
        const double lo = pnl == 0 ? 0.0 : 0.25 * hi;
        const double xi = lo + (hi - lo) * gl.xr[i];
        const double eta = gl.x[j];
        const double wgt = (hi - lo) * gl.wr[i] * gl.w[j] * xi * a * b;
        double f = 0.0;
        for (int sg = -1; sg <= 1; sg += 2)
            f += pot_integrand(sg * a * xi, b * xi * eta, r, Hab, wq, which) +
                 pot_integrand(sg * a * xi * eta, b * xi, r, Hab, wq, which);
        acc += 2.0 * wgt * f;
    }
    return acc;
}

// Item = (pair, row) when per_row (H_f = h_f r: depends on the row only),
// else (pair, cell) with the caller's H at that cell.  which = 1, 2: the
// integral's derivative with respect to h_a = H_a / r, h_b = H_b / r
// (dH_ab/dh_a = H_a r / (2 H_ab), likewise for b) instead.
template <typename T>
__global__ void k_pot_self(const T *H, const double *h, int nf, int nr, int nphi, double lnrmin,
                           double du, double dphi, int per_row, double *out, GLNodes gl, int which)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int64_t N = (int64_t)nr * nphi, per = per_row ? nr : N;
    const int64_t item = blockIdx.x;
    if (item >= (int64_t)nf * nf * per) return;
    const int pair = (int)(item / per);
    const int64_t c = item % per;
    const int fa = pair / nf, fb = pair % nf;
    const int ir = per_row ? (int)c : (int)(c / nphi);
    const double r = exp(lnrmin + (ir + 0.5) * du);
    double Ha, Hb;
    if (per_row) {
        Ha = h[fa] * r;
        Hb = h[fb] * r;
    } else {
        Ha = (double)H[fa * N + c];
        Hb = (double)H[fb * N + c];
    }
    const double Hab = sqrt(0.5 * (Ha * Ha + Hb * Hb));
    const double chain = which == 0 ? 1.0 : (which == 1 ? Ha : Hb) * r / (2.0 * Hab);
    const double acc = pot_self_partial(r, Hab, 0.5 * du, 0.5 * dphi, gl, wq, which != 0);
    const double tot = block_sum256(acc, red);
    if (threadIdx.x == 0) out[item] = chain * tot;
}
template __global__ void k_pot_self<float>(const float *, const double *, int, int, int, double, double,
                                           double, int, double *, GLNodes, int);
template __global__ void k_pot_self<double>(const double *, const double *, int, int, int, double, double,
                                            double, int, double *, GLNodes, int);

__global__ void k_fill_f64(double *p, int64_t n, double v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------- second-order (hat) weights
// (the rules themselves are in sg_hat.h)
// One thread per entry of the wrapped offset grid (as k_sample): entries with
// |P| >= 2 or |Q| >= 2 (no singular square); row n_r (offset +-n_r) is zero.
// which: 0 the weights, 1 and 2 their derivatives in h_a and h_b (the
// kernel's derivatives integrated with the same rules).
__global__ void k_sample_hat_far(double2 *A, int nr, int nphi, double du, double ha, double hb, int which)
{
    __shared__ double wq[FQuad<double>::TABLE];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int p = blockIdx.y;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nphi) return;
    const int P = p < nr ? p : p - 2 * nr, Q = 2 * q <= nphi ? q : q - nphi;
    if (p == nr) {
        A[(size_t)p * nphi + q] = make_double2(0.0, 0.0);
        return;
    }
    if (abs(P) <= 1 && abs(Q) <= 1) return;  // k_sample_hat_near
    const double dphi = 2.0 * SG_PI / nphi;
    double wr = 0.0, wp = 0.0;
    for (int ds = -1; ds <= 0; ++ds)
        for (int dt = -1; dt <= 0; ++dt) {
            int ms, mt;
            sg_hat_split(P, Q, ds, dt, du, dphi, ms, mt);
            sg_hat_square(P, Q, ds, dt, ms, mt, 0, 36 * ms * mt, 1, du, dphi, ha, hb, which, wq, wr, wp);
        }
    A[(size_t)p * nphi + q] = make_double2(wr, wp);
}

// One 256-thread block per entry with |P|, |Q| <= 1 (nine entries).
__global__ void __launch_bounds__(256) k_sample_hat_near(double2 *A, int nr, int nphi, double du, double ha,
                                                          double hb, int which, GLNodes gl)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double red[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int P = (int)(blockIdx.x % 3) - 1, Q = (int)(blockIdx.x / 3) - 1;
    const double dphi = 2.0 * SG_PI / nphi;
    double wr = 0.0, wp = 0.0;
    if (P == 0 && Q == 0) {
        // four squares with the singular corner; folded: 2 x 2 x [0,1]^2 with
        // K_r symmetrised in X and even in phi (K_phi contributes 0)
        double r = 0.0, t = 0.0;
        sg_hat_corner(0, 0, 1, 1, true, du, dphi, ha, hb, which, gl, wq, threadIdx.x, blockDim.x, r, t);
        wr = 4.0 * r;
    } else {
        for (int ds = -1; ds <= 0; ++ds)
            for (int dt = -1; dt <= 0; ++dt) {
                if (sg_hat_singular(P, Q, ds, dt)) {
                    // orientation of the square seen from the corner (-P, -Q)
                    const int sx = (ds == -P) ? 1 : -1, sy = (dt == -Q) ? 1 : -1;
                    sg_hat_corner(P, Q, sx, sy, false, du, dphi, ha, hb, which, gl, wq, threadIdx.x, blockDim.x,
                                  wr, wp);
                } else {
                    int ms, mt;
                    sg_hat_split(P, Q, ds, dt, du, dphi, ms, mt);
                    sg_hat_square(P, Q, ds, dt, ms, mt, threadIdx.x, 36 * ms * mt, blockDim.x, du, dphi, ha, hb,
                                  which, wq, wr, wp);
                }
            }
    }
    const double tr = block_sum256(wr, red);
    __syncthreads();
    const double tp = block_sum256(wp, red);
    if (threadIdx.x == 0) {
        const int p = P < 0 ? P + 2 * nr : P, q = Q < 0 ? Q + nphi : Q;
        A[(size_t)p * nphi + q] = make_double2(tr, tp);
    }
}

__global__ void k_copy_w00(const double2 *A, double *out) { *out = A[0].x; }

// ------------------------------------------------------------------ sample
__global__ void k_sample(double2 *A, int nr, int nphi, double du, double ha, double hb, int which,
                         const double *self_val)
{
    __shared__ double wq[FQuad<double>::TABLE];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int p = blockIdx.y;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nphi) return;
    double kr = 0.0, kp = 0.0;
    if (p == 0 && q == 0) {
        kr = *self_val;
    } else if (p != nr) {
        const double X = (double)(p < nr ? p : p - 2 * nr) * du;
        const double sh = sinpi((double)q / nphi);        // sin(phi/2)
        const double s = sinpi(2.0 * (double)q / nphi);   // sin(phi)
        sg_conv_kernel64(X, sh, s, ha, hb, which, wq, kr, kp);
    }
    A[(size_t)p * nphi + q] = make_double2(kr, kp);
}

// ------------------------------------------------------- phi transform rows
// One group of T threads per row of A (length N = n_phi, complex K_r + i K_phi).
// Output B[c][m][p] (c = 0: K_r, 1: K_phi) for m in [0, N/2].
template <int N>
__global__ void k_tab_phi(const double2 *A, double2 *B, int rows)
{
    using Sh = FftShape<N>;
    constexpr int P = Sh::P, T = Sh::T;
    constexpr int WGS = T > 256 ? T : 256;
    constexpr int G = WGS / T;
    constexpr int W = LdsPlane<double>::elems(N);
    __shared__ __attribute__((aligned(16))) double2 lds[W * G];
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    LdsPlane<double> pl{lds + W * g};
    const int row = blockIdx.x * G + g;
    const bool valid = row < rows;
    double2 v[P];
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = valid ? A[(size_t)row * N + t + T * p] : make_double2(0, 0);
    fft<N, false>(v, t, pl, TwPow64<N>{t});
#pragma unroll
    for (int p = 0; p < P; ++p) pl.st(t + T * p, v[p]);
    __syncthreads();
    if (!valid) return;
    const int ncol = N / 2 + 1;
    for (int m = t; m <= N / 2; m += T) {
        const double2 Zm = pl.ld(m), Zn = pl.ld((N - m) & (N - 1));
        const double zr = Zm.x, zi = Zm.y;
        const double cr = Zn.x, ci = -Zn.y;  // conj Z[-m]
        // K_r~ = (Z + conj Z[-m]) / 2,  K_phi~ = (Z - conj Z[-m]) / (2i)
        B[(size_t)m * rows + row] = make_double2(0.5 * (zr + cr), 0.5 * (zi + ci));
        B[((size_t)ncol + m) * rows + row] = make_double2(0.5 * (zi - ci), -0.5 * (zr - cr));
    }
}

// ---------------------------------------------------------- u transform cols
// One group per column (c, m) of B (length NU = 2 n_r).  Writes k in [0, n_r]
// scaled and rounded into dst[m * col_stride + comp_off[c] + k].
template <int NU>
__global__ void k_tab_u(const double2 *B, float2 *dst, int ncol, size_t col_stride,
                        size_t comp_off0, size_t comp_off1, double scale)
{
    using Sh = FftShape<NU>;
    constexpr int P = Sh::P, T = Sh::T;
    constexpr int WGS = T > 256 ? T : 256;
    constexpr int G = WGS / T;
    constexpr int W = LdsPlane<double>::elems(NU);
    __shared__ __attribute__((aligned(16))) double2 lds[W * G];
    const int g = threadIdx.x / T, t = threadIdx.x % T;
    LdsPlane<double> pl{lds + W * g};
    const int col = blockIdx.x * G + g;  // c * ncol + m
    const bool valid = col < 2 * ncol;
    double2 v[P];
#pragma unroll
    for (int p = 0; p < P; ++p) v[p] = valid ? B[(size_t)col * NU + t + T * p] : make_double2(0, 0);
    fft<NU, false>(v, t, pl, TwPow64<NU>{t});
    if (!valid) return;
    const int c = col / ncol, m = col % ncol;
    float2 *out = dst + (size_t)m * col_stride + (c ? comp_off1 : comp_off0);
    constexpr int H = NU / 2;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const int k = t + T * p;
        if (k <= H) out[k] = make_float2((float)(v[p].x * scale), (float)(v[p].y * scale));
    }
}

// The pair column after the last one: for the FFT pass that transforms the
// two real columns m = 0 and n_phi/2 as one complex column, A = (K0 + KN)/2
// in the K_r place and B = (K0 - KN)/2 in the K_phi place, from K_r of
// column 0 (K0) and of column n_phi/2 (KN), for every pair and k.
__global__ void k_pair_col(float2 *spec, int ncol, int npair, int kk)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npair * kk) return;
    const int pair = e / kk, k = e % kk;
    const size_t cs = (size_t)npair * 2 * kk;
    const float2 k0 = spec[(size_t)pair * 2 * kk + k];
    const float2 kn = spec[(size_t)(ncol - 1) * cs + (size_t)pair * 2 * kk + k];
    float2 *o = spec + (size_t)ncol * cs + (size_t)pair * 2 * kk;
    o[k] = make_float2(0.5f * (k0.x + kn.x), 0.5f * (k0.y + kn.y));
    o[kk + k] = make_float2(0.5f * (k0.x - kn.x), 0.5f * (k0.y - kn.y));
}

// Header, including the indirect-term coefficient of each source fluid: with
// H_a = h_a r the star's kernel has d = 1/h_a at every cell, so
//   sqrt(2) K_a A_k = sqrt(2) pi^{-1/2} h_a^{-3} / 4 F(1 / (4 h_a^2)) du dphi
// (times Sigma_a[k] e^{i phi_k} in the sum), the same for all cells.
__global__ void k_header(sg_table_header *hd, sg_table_header proto, const double *selfbuf,
                         int npair, int with_dh)
{
    // one wave fills the coefficient table; lane 0 writes the header
    __shared__ double w[FQuad<double>::TABLE];
    sg_fill_weights<double>(w);
    __syncthreads();
    if (threadIdx.x != 0) return;
    sg_table_header h = proto;
    const double du = log(proto.r_max / proto.r_min) / proto.n_r;
    const double dphi = 2.0 * SG_PI / proto.n_phi;
    for (int a = 0; a < 4; ++a) {
        h.ind_coef[a] = 0.0;
        if (a < proto.n_fluids) {
            const double ha = proto.h[a];
            h.ind_coef[a] = SG_SQRT2 / SG_SQRT_PI / (4.0 * ha * ha * ha) * sg_F64(0.25 / (ha * ha), w) * du * dphi;
        }
    }
    for (int p = 0; p < npair; ++p) {
        h.self_r[p] = selfbuf[p];
        if (with_dh) {
            h.dself_r[p][0] = selfbuf[npair + 2 * p];
            h.dself_r[p][1] = selfbuf[npair + 2 * p + 1];
        }
    }
    *hd = h;
}

// ------------------------------------------------------------- F for tests
template <typename T>
__global__ void k_eval_F(const T *x, T *F, T *dF, int64_t n)
{
    __shared__ T wq[FQuad<T>::TABLE];
    sg_fill_weights<T>(wq);
    __syncthreads();
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if constexpr (sizeof(T) == 8) {
        double f, d;
        sg_F64_dF(x[i], wq, f, d);
        F[i] = f;
        if (dF) dF[i] = d;
    } else {
        F[i] = sg_F32(x[i], wq);
        if (dF) dF[i] = 0.0f;
    }
}

template <typename T>
__global__ void k_eval_G0(const T *x, T *G, int64_t n)
{
    __shared__ T wq[FQuad<T>::TABLE];
    sg_fill_weights<T>(wq);
    __syncthreads();
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if constexpr (sizeof(T) == 8) G[i] = sg_G0_64(x[i], wq);
    else G[i] = sg_G0_32(x[i], wq);
}

// ------------------------------------------------------------------- host
// Gauss-Legendre nodes and weights on [0,1] (Newton iteration on the
// Legendre three-term recurrence).
static void gl_rule(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        double z = cos(SG_PI * (i + 0.75) / (n + 0.5)), p1 = 0, dp = 1;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0;
            p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

void sg_gl_nodes(GLNodes &gl)
{
    static GLNodes cache;
    static bool ready = false;
    if (!ready) {
        gl_rule(SG_GL_N, cache.x, cache.w);
        gl_rule(SG_GLX_N, cache.xr, cache.wr);
        ready = true;
    }
    gl = cache;
}

template <int NPHI>
static void launch_tab_phi(const double2 *A, double2 *B, int rows, hipStream_t s)
{
    using Sh = FftShape<NPHI>;
    constexpr int WGS = Sh::T > 256 ? Sh::T : 256;
    constexpr int G = WGS / Sh::T;
    hipLaunchKernelGGL(k_tab_phi<NPHI>, dim3((rows + G - 1) / G), dim3(WGS), 0, s, A, B, rows);
}

template <int NU>
static void launch_tab_u(const double2 *B, float2 *dst, int ncol, size_t col_stride, size_t o0,
                         size_t o1, double scale, hipStream_t s)
{
    using Sh = FftShape<NU>;
    constexpr int WGS = Sh::T > 256 ? Sh::T : 256;
    constexpr int G = WGS / Sh::T;
    hipLaunchKernelGGL(k_tab_u<NU>, dim3((2 * ncol + G - 1) / G), dim3(WGS), 0, s, B, dst, ncol,
                       col_stride, o0, o1, scale);
}

static bool dispatch_tab_phi(int nphi, const double2 *A, double2 *B, int rows, hipStream_t s)
{
    switch (nphi) {
    case 4: launch_tab_phi<4>(A, B, rows, s); return true;
    case 8: launch_tab_phi<8>(A, B, rows, s); return true;
    case 16: launch_tab_phi<16>(A, B, rows, s); return true;
    case 32: launch_tab_phi<32>(A, B, rows, s); return true;
    case 64: launch_tab_phi<64>(A, B, rows, s); return true;
    case 128: launch_tab_phi<128>(A, B, rows, s); return true;
    case 256: launch_tab_phi<256>(A, B, rows, s); return true;
    case 512: launch_tab_phi<512>(A, B, rows, s); return true;
    case 1024: launch_tab_phi<1024>(A, B, rows, s); return true;
    case 2048: launch_tab_phi<2048>(A, B, rows, s); return true;
    default: return false;
    }
}

static bool dispatch_tab_u(int nu, const double2 *B, float2 *dst, int ncol, size_t cs, size_t o0,
                           size_t o1, double scale, hipStream_t s)
{
    switch (nu) {
    case 4: launch_tab_u<4>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 8: launch_tab_u<8>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 16: launch_tab_u<16>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 32: launch_tab_u<32>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 64: launch_tab_u<64>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 128: launch_tab_u<128>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 256: launch_tab_u<256>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 512: launch_tab_u<512>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 1024: launch_tab_u<1024>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 2048: launch_tab_u<2048>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    case 4096: launch_tab_u<4096>(B, dst, ncol, cs, o0, o1, scale, s); return true;
    default: return false;
    }
}

size_t sg_table_ws_bytes(int nr, int nphi)
{
    const size_t A = sizeof(double2) * 2 * (size_t)nr * nphi;
    const size_t B = sizeof(double2) * 2 * (size_t)(nphi / 2 + 1) * 2 * nr;
    return sg_align256(A) + sg_align256(B) + 256;
}

sg_status sg_table_build(const sg_grid *grid, const sg_fluids *fl, uint32_t flags, void *d_table,
                         void *d_ws, hipStream_t s)
{
    const int nr = grid->n_r, nphi = grid->n_phi, nf = fl->n_fluids;
    const TableLayout L = sg_table_layout(nr, nphi, nf, flags);
    const double du = log(grid->r_max / grid->r_min) / nr;
    const double dphi = 2.0 * SG_PI / nphi;
    char *tb = (char *)d_table;
    char *ws = (char *)d_ws;
    double2 *A = (double2 *)ws;
    double2 *B = (double2 *)(ws + sg_align256(sizeof(double2) * 2 * (size_t)nr * nphi));
    double *selfbuf = (double *)((char *)B + sg_align256(sizeof(double2) * 2 * (size_t)L.ncol * 2 * nr));
    const bool with_dh = (flags & SG_WITH_DH) != 0;
    const bool excl = (flags & SG_SELF_CELL_EXCLUDE) != 0;
    const bool second = (flags & SG_SECOND_ORDER) != 0;  // no own-cell switch

    // twiddle tables
    {
        const int n = 2 * nr > nphi ? 2 * nr : nphi;
        hipLaunchKernelGGL(k_twiddles, dim3((n + 255) / 256), dim3(256), 0, s,
                           (float2 *)(tb + L.off_tw_u), 2 * nr, (float2 *)(tb + L.off_tw_phi), nphi);
        SG_HIP(hipGetLastError());
    }
    // self-cell items: [pair] for which = 0, then [pair][d] for the derivatives
    SelfItems items{};
    int nit = 0;
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
            items.ha[nit] = fl->h[a];
            items.hb[nit] = fl->h[b];
            items.which[nit] = 0;
            ++nit;
        }
    if (with_dh)
        for (int a = 0; a < nf; ++a)
            for (int b = 0; b < nf; ++b)
                for (int d = 0; d < 2; ++d) {
                    items.ha[nit] = fl->h[a];
                    items.hb[nit] = fl->h[b];
                    items.which[nit] = 1 + d;
                    ++nit;
                }
    if (excl) {
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, selfbuf, (int64_t)nit, 0.0);
        SG_HIP(hipGetLastError());
    } else if (!second) {  // second order: W_r(0, 0) is copied in per pair below
        GLNodes gl;
        sg_gl_nodes(gl);
        hipLaunchKernelGGL(k_self_cell, dim3(nit), dim3(256), 0, s, items, selfbuf, du, dphi, gl);
        SG_HIP(hipGetLastError());
    }

    const double scale = -du * dphi / (2.0 * nr * (double)nphi);
    const size_t col_stride = (size_t)L.npair * 2 * L.kk;        // spec: [m][pair][c][k]
    const size_t dcol_stride = (size_t)L.npair * 4 * L.kk;       // dspec: [m][pair][d][c][k]
    float2 *spec = (float2 *)(tb + L.off_spec);
    float2 *dspec = (float2 *)(tb + L.off_dspec);
    const int nwhich = with_dh ? 3 : 1;
    for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
            const int pair = a * nf + b;
            for (int w = 0; w < nwhich; ++w) {
                const double *sv = w == 0 ? selfbuf + pair : selfbuf + L.npair + 2 * pair + (w - 1);
                if (second) {
                    GLNodes gl;
                    sg_gl_nodes(gl);
                    hipLaunchKernelGGL(k_sample_hat_far, dim3((nphi + 255) / 256, 2 * nr), dim3(256), 0, s, A, nr,
                                       nphi, du, fl->h[a], fl->h[b], w);
                    hipLaunchKernelGGL(k_sample_hat_near, dim3(9), dim3(256), 0, s, A, nr, nphi, du, fl->h[a],
                                       fl->h[b], w, gl);
                    // the header's own-cell value of this pair (or its derivative): W_r(0, 0)
                    hipLaunchKernelGGL(k_copy_w00, dim3(1), dim3(1), 0, s, (const double2 *)A, (double *)sv);
                } else {
                    hipLaunchKernelGGL(k_sample, dim3((nphi + 255) / 256, 2 * nr), dim3(256), 0, s, A,
                                       nr, nphi, du, fl->h[a], fl->h[b], w, sv);
                }
                SG_HIP(hipGetLastError());
                if (!dispatch_tab_phi(nphi, A, B, 2 * nr, s)) return SG_ERR_UNSUPPORTED;
                SG_HIP(hipGetLastError());
                float2 *dst;
                size_t cs, o0, o1;
                if (w == 0) {
                    dst = spec;
                    cs = col_stride;
                    o0 = ((size_t)pair * 2 + 0) * L.kk;
                    o1 = ((size_t)pair * 2 + 1) * L.kk;
                } else {
                    dst = dspec;
                    cs = dcol_stride;
                    o0 = (((size_t)pair * 2 + (w - 1)) * 2 + 0) * L.kk;
                    o1 = (((size_t)pair * 2 + (w - 1)) * 2 + 1) * L.kk;
                }
                if (!dispatch_tab_u(2 * nr, B, dst, L.ncol, cs, o0, o1, scale, s))
                    return SG_ERR_UNSUPPORTED;
                SG_HIP(hipGetLastError());
            }
        }
    hipLaunchKernelGGL(k_pair_col, dim3((L.npair * L.kk + 255) / 256), dim3(256), 0, s, spec, L.ncol, L.npair,
                       L.kk);
    SG_HIP(hipGetLastError());
    sg_table_header proto{};
    proto.magic = SG_TABLE_MAGIC;
    proto.version = 1;
    proto.n_r = nr;
    proto.n_phi = nphi;
    proto.n_fluids = nf;
    proto.flags = flags;
    for (int a = 0; a < 4; ++a) proto.h[a] = a < nf ? fl->h[a] : 0.0;
    proto.r_min = grid->r_min;
    proto.r_max = grid->r_max;
    proto.total_bytes = L.total;
    hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, (sg_table_header *)tb, proto, selfbuf,
                       L.npair, with_dh ? 1 : 0);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

sg_status sg_self_cell_launch(const sg_grid *grid, const double *ha, const double *hb, int n,
                              int which, double *d_out, hipStream_t s)
{
    if (n < 1 || n > SG_SELF_MAX || which < 0 || which > 2) return SG_ERR_ARG;
    SelfItems items{};
    for (int i = 0; i < n; ++i) {
        items.ha[i] = ha[i];
        items.hb[i] = hb[i];
        items.which[i] = which;
    }
    GLNodes gl;
    sg_gl_nodes(gl);
    const double du = log(grid->r_max / grid->r_min) / grid->n_r;
    const double dphi = 2.0 * SG_PI / grid->n_phi;
    hipLaunchKernelGGL(k_self_cell, dim3(n), dim3(256), 0, s, items, d_out, du, dphi, gl);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

sg_status sg_eval_G0_launch(const void *x, void *G, int64_t n, sg_dtype dt, hipStream_t s)
{
    const int64_t nb = (n + 255) / 256;
    if (dt == SG_F64)
        hipLaunchKernelGGL(k_eval_G0<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double *)x,
                           (double *)G, n);
    else
        hipLaunchKernelGGL(k_eval_G0<float>, dim3((unsigned)nb), dim3(256), 0, s, (const float *)x,
                           (float *)G, n);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

sg_status sg_eval_F_launch(const void *x, void *F, void *dF, int64_t n, sg_dtype dt, hipStream_t s)
{
    const int64_t nb = (n + 255) / 256;
    if (dt == SG_F64)
        hipLaunchKernelGGL(k_eval_F<double>, dim3((unsigned)nb), dim3(256), 0, s, (const double *)x,
                           (double *)F, (double *)dF, n);
    else
        hipLaunchKernelGGL(k_eval_F<float>, dim3((unsigned)nb), dim3(256), 0, s, (const float *)x,
                           (float *)F, (float *)dF, n);
    SG_HIP(hipGetLastError());
    return SG_OK;
}
