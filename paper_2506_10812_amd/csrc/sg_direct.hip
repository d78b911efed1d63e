// sg_direct.hip -- O(N^2) direct summation of the exact kernel (Sect. 2.2,
// the 2D force through the kernel, divided by Sigma_b) for general per-cell
// scale heights, in float or double.
//
// For target cell i (fluid b) and source cell k != i (fluid a) on the log-r x
// uniform-phi grid, with X = u_i - u_k and phi = phi_i - phi_k:
//   s^2        = r_i r_k (4 sinh^2(X/2) + 4 sin^2(phi/2))    (cancellation-free)
//   H_ab^2     = (H_a[k]^2 + H_b[i]^2) / 2,  x = s^2 / (8 H_ab^2)
//   K_ab / s   = F(x) / (8 sqrt(pi) H_ab^3)
//   e_s . e_r  = (r_i - r_k cos phi)/s = r_k (e^X - cos phi)/s,
//   e_s . e_phi = r_k sin phi / s,
//   g_r  -= Sigma_a[k] A_k (K/s) r_k (expm1(X) + 2 sin^2(phi/2)),
//   g_phi -= Sigma_a[k] A_k (K/s) r_k sin phi.
// The offset factors depend only on (i_r - k_r) and (j - l) and are tabulated
// once per call in double (rounded for the float path).  On a uniform radial
// grid (SG_LINEAR_R: centres r_min + (i + 1/2) dr, sector areas r dr dphi)
// the radial factors 4 sinh^2(X/2) = (r_i - r_k)^2 / (r_i r_k) and
// expm1(X) = (r_i - r_k) / r_k are formed per source row instead.
//
// Layout: one thread per target cell (256 per workgroup), all target fluids
// in registers; the source loop runs over whole radial rows so every
// per-source quantity is wave-uniform (scalar loads); the source rows are
// split over blockIdx.y when there are too few targets to fill 256 CUs, and
// the per-split partial sums are reduced in a fixed order by a second kernel
// that also adds the self term and, with SG_INDIRECT, the indirect term
// (deterministic; no atomics).
//
// Accumulation (both precisions): the sources of a row are taken in chunks of
// SG_DCHUNK azimuths, each chunk summed into a fresh partial, and the chunk
// partials are added to the running total with an error-free transformation
// (Knuth's TwoSum), whose rounding errors are carried in a second
// accumulator.  A single running sum over all 2^21 sources of a 1024 x 2048
// disc would lose about three digits to the cancellation between the pull of
// the inner and of the outer disc; chunking bounds the plain-sum part to 64
// terms and the compensated outer sum is exact to first order, so the result
// sits at the rounding floor of the individual terms.  Each split hands
// (sum, carried error) to the reduction, which adds them in double.
#include "sg_direct.h"
#include "sg_kfn.h"
#include "sg_table.h"

template <typename T> struct DirectArgs {
    int nr, nphi, rps;   // rows per split
    int lin;             // uniform radial grid
    int64_t N;
    const T *rrow, *sx, *ex, *sph, *snp, *mass, *H2;
    T *partial;          // [split][fluid][component][hi, lo][N]
};

#define SG_DCHUNK 64

// s + v = (s', e') exactly (Knuth's TwoSum); the error goes into c.  No
// products, so contraction into FMAs cannot change it.
template <typename T> __device__ inline void sg_two_sum_acc(T &s, T &c, T v)
{
    const T t = s + v;
    const T bp = t - s;
    c += (s - (t - bp)) + (v - bp);
    s = t;
}

// Ring radius: log grid (lin = 0) or uniform grid (a = r_min, b = dr).
__device__ inline double dir_radius(int lin, double lnrmin, double du, double rmin, double dr, int i)
{
    return lin ? rmin + (i + 0.5) * dr : exp(lnrmin + (i + 0.5) * du);
}

template <typename T>
__global__ void k_direct_prep(int nr, int nphi, int nf, double lnrmin, double du, double dphi,
                              const double *h, const T *sigma, const T *H, T *rrow, T *sx, T *ex,
                              T *sph, T *snp, T *mass, T *H2, int lin, double rmin, double dr, double *Hd)
{
    const int64_t N = (int64_t)nr * nphi;
    const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < nr; i += stride) rrow[i] = (T)dir_radius(lin, lnrmin, du, rmin, dr, (int)i);
    for (int64_t p = tid; p < 2 * nr - 1; p += stride) {
        const double X = (double)(p - (nr - 1)) * du;
        const double s = sinh(0.5 * X);
        sx[p] = (T)(4.0 * s * s);
        ex[p] = (T)expm1(X);
    }
    for (int64_t q = tid; q < nphi; q += stride) {
        const double s = sinpi((double)q / nphi);
        sph[q] = (T)(4.0 * s * s);
        snp[q] = (T)sinpi(2.0 * (double)q / nphi);
    }
    for (int64_t k = tid; k < nf * N; k += stride) {
        const int64_t cell = k % N;
        const int ir = (int)(cell / nphi);
        const double r = dir_radius(lin, lnrmin, du, rmin, dr, ir);
        mass[k] = (T)((double)sigma[k] * (lin ? r * dr : r * r * du) * dphi);
        double Hk;
        if (H) Hk = (double)H[k];
        else Hk = h[k / N] * r;
        H2[k] = (T)(Hk * Hk);
        if (lin && H) Hd[k] = Hk;  // double H per cell for the own-cell integrals
    }
    if (lin && !H)  // double H per ring
        for (int64_t k = tid; k < (int64_t)nf * nr; k += stride)
            Hd[k] = h[k / nr] * dir_radius(1, 0.0, 0.0, rmin, dr, (int)(k % nr));
}

template <typename T> __device__ inline T sg_F_any(T x, const T *w);
template <> __device__ inline double sg_F_any<double>(double x, const double *w) { return sg_F64<true>(x, w); }
template <> __device__ inline float sg_F_any<float>(float x, const float *w) { return sg_F32(x, w); }

template <typename T, int NF>
__global__ void __launch_bounds__(256) k_direct(DirectArgs<T> A)
{
    __shared__ T wq[FQuad<T>::TABLE];
    sg_fill_weights<T>(wq);
    __syncthreads();
    const int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (t >= A.N) return;
    const int nphi = A.nphi, nr = A.nr;
    const int ir = (int)(t / nphi), j = (int)(t % nphi);
    const T ri = A.rrow[ir];
    T hb2[NF], accr[NF], accp[NF], errr[NF], errp[NF];
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        hb2[b] = A.H2[b * A.N + t];
        accr[b] = T(0);
        accp[b] = T(0);
        errr[b] = T(0);
        errp[b] = T(0);
    }
    const T c8 = T(1.0 / (8.0 * SG_SQRT_PI));
    const int r0 = blockIdx.y * A.rps;
    const int r1 = min(nr, r0 + A.rps);
    for (int kr = r0; kr < r1; ++kr) {
        const T rk = A.rrow[kr];
        T SX, EX;
        if (A.lin) {
            const T d = ri - rk;
            SX = d * d / (ri * rk);
            EX = d / rk;
        } else {
            const int p = ir - kr + nr - 1;
            SX = A.sx[p];
            EX = A.ex[p];
        }
        const T rr8 = ri * rk * T(0.125);
        const int64_t kbase = (int64_t)kr * nphi;
        const int lself = kr == ir ? j : -1;  // the own cell: l == j on the own ring
        for (int l0 = 0; l0 < nphi; l0 += SG_DCHUNK) {
            const int l1 = min(nphi, l0 + SG_DCHUNK);
            T pr[NF], pp[NF];  // this chunk's partial sums
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                pr[b] = T(0);
                pp[b] = T(0);
            }
            for (int l = l0; l < l1; ++l) {
                const int64_t k = kbase + l;
                int q = j - l;
                q += q < 0 ? nphi : 0;
                const T sp = A.sph[q];
                const T s2_8 = rr8 * (SX + sp);  // s^2 / 8
                const T emc = EX + T(0.5) * sp;
                const T sn = A.snp[q];
                const bool self = l == lself;
#pragma unroll
                for (int a = 0; a < NF; ++a) {
                    const T m = A.mass[a * A.N + k] * rk * c8;
                    const T ha2 = A.H2[a * A.N + k];
#pragma unroll
                    for (int b = 0; b < NF; ++b) {
                        const T H2ab = T(0.5) * (ha2 + hb2[b]);
                        const T rH = sg_rsqrt(H2ab), rH2 = rH * rH;
                        const T x = s2_8 * rH2;
                        const T F = self ? T(0) : sg_F_any<T>(self ? T(1) : x, wq);
                        const T c = m * F * (rH2 * rH);
                        pr[b] -= c * emc;
                        pp[b] -= c * sn;
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < NF; ++b) {
                sg_two_sum_acc(accr[b], errr[b], pr[b]);
                sg_two_sum_acc(accp[b], errp[b], pp[b]);
            }
        }
    }
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        T *o = A.partial + (int64_t)(blockIdx.y * NF + b) * 4 * A.N + t;
        o[0] = accr[b];
        o[A.N] = errr[b];
        o[2 * A.N] = accp[b];
        o[3 * A.N] = errp[b];
    }
}

// Indirect term (SG_INDIRECT; Sect. 5.4 and the appendix "Indirect term"):
//   A + i B = sum_a sqrt(2) sum_k Sigma_a[k] A_k K_a(d_k) e^{i phi_k},
//   K_a(d) = pi^{-1/2} H_a^{-2} (d/4) F(d^2/4),  d_k = r_k / H_a[k],
// in double for both precisions (a reduction over the cells, like the self
// term).  Block b sums a fixed strided set of cells and the blocks' sums are
// added in order by one thread, so the result is deterministic.
#define SG_IND_BLOCKS 1024
template <typename T>
__global__ void __launch_bounds__(256) k_indirect_part(int nr, int nphi, int nf, double lnrmin, double du,
                                                       double dphi, const double *h, const T *sigma,
                                                       const T *H, double2 *part, int lin, double rmin,
                                                       double dr)
{
    __shared__ double wq[FQuad<double>::TABLE];
    __shared__ double ra[256], rb[256];
    sg_fill_weights<double>(wq);
    __syncthreads();
    const int64_t N = (int64_t)nr * nphi, total = nf * N;
    double sa = 0.0, sb = 0.0;
    for (int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x; k < total; k += (int64_t)gridDim.x * 256) {
        const int a = (int)(k / N);
        const int64_t cell = k % N;
        const int ir = (int)(cell / nphi), j = (int)(cell % nphi);
        const double r = dir_radius(lin, lnrmin, du, rmin, dr, ir);
        const double Hk = H ? (double)H[k] : h[a] * r;
        const double d = r / Hk;
        const double Ka = 1.0 / (SG_SQRT_PI * Hk * Hk) * (0.25 * d) * sg_F64(0.25 * d * d, wq);
        const double w = SG_SQRT2 * (double)sigma[k] * (lin ? r * dr : r * r * du) * dphi * Ka;
        double sp, cp;
        sincos((j + 0.5) * dphi, &sp, &cp);
        sa += w * cp;
        sb += w * sp;
    }
    ra[threadIdx.x] = sa;
    rb[threadIdx.x] = sb;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            ra[threadIdx.x] += ra[threadIdx.x + o];
            rb[threadIdx.x] += rb[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(ra[0], rb[0]);
}

__global__ void k_indirect_fin(const double2 *part, int n, double2 *AB)
{
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < n; ++i) {
        a += part[i].x;
        b += part[i].y;
    }
    *AB = make_double2(a, b);
}

// self: per pair (log grid, H = h r), per cell (percell = 1) or, on a
// uniform grid without per-cell H, per ring (percell = 2); the own-cell
// values are cell averages per (du dphi), or per (dr / r_i) dphi on a
// uniform grid (lin; rmin, dr give r_i).
template <typename T, int NF>
__global__ void k_direct_reduce(const T *partial, int S, int64_t N, const double *self,
                                int percell, int with_self, const T *sigma, double dudphi,
                                const double2 *ind, int nphi, T *gr, T *gp, int lin, double rmin, double dr)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N) return;
    double ir = 0.0, ip = 0.0;  // indirect acceleration at this cell (all targets)
    if (ind) {
        const double2 AB = *ind;
        double sp, cp;
        sincos(((double)(t % nphi) + 0.5) * (2.0 * SG_PI / nphi), &sp, &cp);
        ir = -(AB.x * cp + AB.y * sp);
        ip = -(-AB.x * sp + AB.y * cp);
    }
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        // the splits' (sum, carried error) pairs, added in double in a fixed
        // order (compensated, so the double pass adds no error of its own
        // that matters for either precision)
        double sr = 0.0, er = 0.0, sp = 0.0, ep = 0.0;
        for (int s = 0; s < S; ++s) {
            const T *pp = partial + (int64_t)(s * NF + b) * 4 * N + t;
            sg_two_sum_acc(sr, er, (double)pp[0]);
            sg_two_sum_acc(sr, er, (double)pp[N]);
            sg_two_sum_acc(sp, ep, (double)pp[2 * N]);
            sg_two_sum_acc(sp, ep, (double)pp[3 * N]);
        }
        sr += er;
        sp += ep;
        if (with_self) {
            const int ir = (int)(t / nphi);
            const double w = lin ? dr / (rmin + (ir + 0.5) * dr) * (2.0 * SG_PI / nphi) : dudphi;
            const int64_t nring = N / nphi;
            double st = 0.0;
#pragma unroll
            for (int a = 0; a < NF; ++a) {
                const int pair = a * NF + b;
                const double kb = percell == 1   ? self[(int64_t)pair * N + t]
                                  : percell == 2 ? self[(int64_t)pair * nring + ir]
                                                 : self[pair];
                st -= w * (double)sigma[a * N + t] * kb;
            }
            sr += st;
        }
        if (ind) {
            sr += ir;
            sp += ip;
        }
        gr[b * N + t] = (T)sr;
        gp[b * N + t] = (T)sp;
    }
}

// --------------------------------------------------------------- potential
// Conservative potential (Sect. 5.5, appendix "Conservative force"):
//   Phi_b(i) = sum_a sum_{k != i} Sigma_a[k] A_k P_ab(s_ik),
//   P_ab(s) = -e^y K0(y) / (2 sqrt(pi) H_ab),  y = s^2/(8 H_ab^2),
// H_ab from the source cell's H_a and the target cell's H_b; the own cell
// adds Sigma_a[i] times the cell integral of P_ab (k_pot_self).  Same
// layout and splitting as the field sum; one accumulator per target fluid.
template <typename T> __device__ inline T sg_G0_any(T x, const T *w);
template <> __device__ inline double sg_G0_any<double>(double x, const double *w) { return sg_G0_64<true>(x, w); }
template <> __device__ inline float sg_G0_any<float>(float x, const float *w) { return sg_G0_32(x, w); }

template <typename T, int NF>
__global__ void __launch_bounds__(256) k_potential(DirectArgs<T> A)
{
    __shared__ T wq[FQuad<T>::TABLE];
    sg_fill_weights<T>(wq);
    __syncthreads();
    const int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (t >= A.N) return;
    const int nphi = A.nphi, nr = A.nr;
    const int ir = (int)(t / nphi), j = (int)(t % nphi);
    const T ri = A.rrow[ir];
    T hb2[NF], acc[NF], err[NF];
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        hb2[b] = A.H2[b * A.N + t];
        acc[b] = T(0);
        err[b] = T(0);
    }
    const T c2 = T(-0.5 / SG_SQRT_PI);
    const int r0 = blockIdx.y * A.rps;
    const int r1 = min(nr, r0 + A.rps);
    for (int kr = r0; kr < r1; ++kr) {
        const int p = ir - kr + nr - 1;
        const T SX = A.sx[p];
        const T rr = ri * A.rrow[kr];
        const int64_t kbase = (int64_t)kr * nphi;
        for (int l0 = 0; l0 < nphi; l0 += SG_DCHUNK) {
            const int l1 = min(nphi, l0 + SG_DCHUNK);
            T pc[NF];  // this chunk's partial sums
#pragma unroll
            for (int b = 0; b < NF; ++b) pc[b] = T(0);
            for (int l = l0; l < l1; ++l) {
                const int64_t k = kbase + l;
                int q = j - l;
                q += q < 0 ? nphi : 0;
                const T s2 = rr * (SX + A.sph[q]);
                const bool self = (k == t);
#pragma unroll
                for (int a = 0; a < NF; ++a) {
                    const T m = A.mass[a * A.N + k] * c2;
                    const T ha2 = A.H2[a * A.N + k];
#pragma unroll
                    for (int b = 0; b < NF; ++b) {
                        const T H2ab = T(0.5) * (ha2 + hb2[b]);
                        const T rH = sg_rsqrt(H2ab);
                        const T y = s2 * T(0.125) * (rH * rH);
                        const T G = self ? T(0) : sg_G0_any<T>(self ? T(1) : y, wq);
                        pc[b] += m * G * rH;
                    }
                }
            }
#pragma unroll
            for (int b = 0; b < NF; ++b) sg_two_sum_acc(acc[b], err[b], pc[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        T *o = A.partial + (int64_t)(blockIdx.y * NF + b) * 2 * A.N + t;
        o[0] = acc[b];
        o[A.N] = err[b];
    }
}

template <typename T, int NF>
__global__ void k_potential_reduce(const T *partial, int S, int64_t N, int nphi, const double *self,
                                   int per_row, int with_self, const T *sigma, T *pot)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N) return;
    const int64_t si = per_row ? t / nphi : t;
    const int64_t per = per_row ? N / nphi : N;
#pragma unroll
    for (int b = 0; b < NF; ++b) {
        double sum = 0.0, e = 0.0;
        for (int s = 0; s < S; ++s) {
            const T *pp = partial + (int64_t)(s * NF + b) * 2 * N + t;
            sg_two_sum_acc(sum, e, (double)pp[0]);
            sg_two_sum_acc(sum, e, (double)pp[N]);
        }
        sum += e;
        if (with_self) {
            double st = 0.0;
#pragma unroll
            for (int a = 0; a < NF; ++a) st += (double)sigma[a * N + t] * self[(int64_t)(a * NF + b) * per + si];
            sum += st;
        }
        pot[b * N + t] = (T)sum;
    }
}

// -------------------------------------------- self-gravitating scale heights
// H_f^sg = sqrt(2/pi) H_f f(Qt), Qt = (sum_f 1/Q_f)^-1 (Sect. 2.1), with
// f(x) = pi/(4x) [sqrt(1 + 8x^2/pi) - 1] evaluated as the equal
// 2x / (sqrt(1 + 8x^2/pi) + 1), which does not cancel at small x.
__global__ void k_hsg(int64_t n, int nf, const double *H, const double *Q, double *Hsg)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double inv = 0.0;
        for (int f = 0; f < nf; ++f) inv += 1.0 / Q[f * n + i];
        const double x = 1.0 / inv;
        const double fx = 2.0 * x / (sqrt(1.0 + 8.0 * x * x / SG_PI) + 1.0);
        for (int f = 0; f < nf; ++f) Hsg[f * n + i] = sqrt(2.0 / SG_PI) * H[f * n + i] * fx;
    }
}

sg_status sg_hsg_launch(int64_t n, int nf, const double *H, const double *Q, double *Hsg, hipStream_t s)
{
    int64_t nb = (n + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(k_hsg, dim3((unsigned)nb), dim3(256), 0, s, n, nf, H, Q, Hsg);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// ------------------------------------------------------------------- host
static int direct_splits(int nr, int64_t N)
{
    const int64_t gx = (N + 255) / 256;
    int64_t S = (2048 + gx - 1) / gx;
    if (S < 1) S = 1;
    if (S > nr) S = nr;
    const int rps = (int)((nr + S - 1) / S);
    return (nr + rps - 1) / rps;
}

size_t sg_direct_ws_bytes(int nr, int nphi, int nf, sg_dtype dt, int percell)
{
    const size_t es = dt == SG_F64 ? 8 : 4;
    const int64_t N = (int64_t)nr * nphi;
    const int S = direct_splits(nr, N);
    size_t o = 0;
    o += sg_align256(es * nr);
    o += 2 * sg_align256(es * (2 * (size_t)nr - 1));
    o += 2 * sg_align256(es * nphi);
    o += 2 * sg_align256(es * nf * N);
    o += sg_align256(sizeof(double) * nf * nf * (percell ? N : nr));
    o += sg_align256(es * (size_t)S * nf * 4 * N);
    o += sg_align256(sizeof(double) * 4);
    o += sg_align256(sizeof(double2) * (SG_IND_BLOCKS + 1));
    return o;
}

template <typename T>
static sg_status direct_run(const sg_grid *g, int nf, const double *h, const T *sigma, const T *H,
                            T *gr, T *gp, uint32_t flags, void *ws, hipStream_t s)
{
    const int nr = g->n_r, nphi = g->n_phi;
    const int64_t N = (int64_t)nr * nphi;
    const double du = log(g->r_max / g->r_min) / nr;
    const double dphi = 2.0 * SG_PI / nphi;
    const double lnrmin = log(g->r_min);
    const int lin = (flags & SG_LINEAR_R) ? 1 : 0;
    const double dr = (g->r_max - g->r_min) / nr;
    const int S = direct_splits(nr, N);
    const int rps = (nr + S - 1) / S;
    char *o = (char *)ws;
    auto take = [&](size_t bytes) {
        char *p = o;
        o += sg_align256(bytes);
        return p;
    };
    T *rrow = (T *)take(sizeof(T) * nr);
    T *sx = (T *)take(sizeof(T) * (2 * (size_t)nr - 1));
    T *ex = (T *)take(sizeof(T) * (2 * (size_t)nr - 1));
    T *sph = (T *)take(sizeof(T) * nphi);
    T *snp = (T *)take(sizeof(T) * nphi);
    T *mass = (T *)take(sizeof(T) * nf * N);
    T *H2 = (T *)take(sizeof(T) * nf * N);
    const int percell = H != nullptr;
    double *self = (double *)take(sizeof(double) * nf * nf * (percell ? N : nr));
    T *partial = (T *)take(sizeof(T) * (size_t)S * nf * 4 * N);
    // uniform grid: double H for the own-cell integrals, per cell or per ring,
    // in the partial-sum buffer (at least nf N doubles; written before the sum)
    double *Hd = (double *)partial;
    double *dh = (double *)take(sizeof(double) * 4);
    double2 *ipart = (double2 *)take(sizeof(double2) * (SG_IND_BLOCKS + 1));
    double2 *iab = ipart + SG_IND_BLOCKS;

    // h lives on the host: pass through a kernel argument copy in device memory
    // is avoided by writing it with a fill kernel.
    for (int f = 0; f < nf; ++f) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, dh + f, (int64_t)1, h[f]);
    SG_HIP(hipGetLastError());
    {
        int64_t work = nf * N > 2 * nr ? nf * N : 2 * nr;
        if (work < nphi) work = nphi;
        int64_t nb = (work + 255) / 256;
        if (nb > 65536) nb = 65536;
        hipLaunchKernelGGL(k_direct_prep<T>, dim3((unsigned)nb), dim3(256), 0, s, nr, nphi, nf,
                           lnrmin, du, dphi, (const double *)dh, sigma, H, rrow, sx, ex, sph, snp,
                           mass, H2, lin, g->r_min, dr, Hd);
        SG_HIP(hipGetLastError());
    }
    const int with_self = !(flags & SG_SELF_CELL_EXCLUDE);
    if (with_self) {
        GLNodes gl;
        sg_gl_nodes(gl);
        if (lin) {
            const int per = percell ? nphi : 1;
            const int64_t items = (int64_t)nf * nf * nr * per;
            hipLaunchKernelGGL(k_ss_self_lin, dim3((unsigned)items), dim3(256), 0, s, (const double *)Hd, nf, nr,
                               per, g->r_min, dr, dphi, 0, 0, self, gl);
        } else if (percell) {
            const int64_t items = (int64_t)nf * nf * N;
            hipLaunchKernelGGL(k_self_cell_percell<T>, dim3((unsigned)items), dim3(256), 0, s, H, nf,
                               nr, nphi, lnrmin, du, dphi, self, gl);
        } else {
            SelfItems it{};
            for (int a = 0; a < nf; ++a)
                for (int b = 0; b < nf; ++b) {
                    it.ha[a * nf + b] = h[a];
                    it.hb[a * nf + b] = h[b];
                    it.which[a * nf + b] = 0;
                }
            hipLaunchKernelGGL(k_self_cell, dim3(nf * nf), dim3(256), 0, s, it, self, du, dphi, gl);
        }
        SG_HIP(hipGetLastError());
    }
    const bool ind = (flags & SG_INDIRECT) != 0;
    if (ind) {
        int64_t nb = (nf * N + 255) / 256;
        if (nb > SG_IND_BLOCKS) nb = SG_IND_BLOCKS;
        hipLaunchKernelGGL(k_indirect_part<T>, dim3((unsigned)nb), dim3(256), 0, s, nr, nphi, nf, lnrmin,
                           du, dphi, (const double *)dh, sigma, H, ipart, lin, g->r_min, dr);
        hipLaunchKernelGGL(k_indirect_fin, dim3(1), dim3(64), 0, s, (const double2 *)ipart, (int)nb, iab);
        SG_HIP(hipGetLastError());
    }
    DirectArgs<T> A;
    A.nr = nr;
    A.nphi = nphi;
    A.rps = rps;
    A.lin = lin;
    A.N = N;
    A.rrow = rrow;
    A.sx = sx;
    A.ex = ex;
    A.sph = sph;
    A.snp = snp;
    A.mass = mass;
    A.H2 = H2;
    A.partial = partial;
    dim3 grid((unsigned)((N + 255) / 256), (unsigned)S);
    switch (nf) {
    case 1: hipLaunchKernelGGL((k_direct<T, 1>), grid, dim3(256), 0, s, A); break;
    case 2: hipLaunchKernelGGL((k_direct<T, 2>), grid, dim3(256), 0, s, A); break;
    case 3: hipLaunchKernelGGL((k_direct<T, 3>), grid, dim3(256), 0, s, A); break;
    default: hipLaunchKernelGGL((k_direct<T, 4>), grid, dim3(256), 0, s, A); break;
    }
    SG_HIP(hipGetLastError());
    const unsigned nb = (unsigned)((N + 255) / 256);
    const double2 *indp = ind ? (const double2 *)iab : nullptr;
    const int smode = percell ? 1 : (lin ? 2 : 0);
#define SG_RED(NF)                                                                                      \
    hipLaunchKernelGGL((k_direct_reduce<T, NF>), dim3(nb), dim3(256), 0, s, partial, S, N, self, smode,    \
                       with_self, sigma, du * dphi, indp, nphi, gr, gp, lin, g->r_min, dr)
    switch (nf) {
    case 1: SG_RED(1); break;
    case 2: SG_RED(2); break;
    case 3: SG_RED(3); break;
    default: SG_RED(4); break;
    }
#undef SG_RED
    SG_HIP(hipGetLastError());
    return SG_OK;
}

size_t sg_potential_ws_bytes(int nr, int nphi, int nf, sg_dtype dt, int percell)
{
    const size_t es = dt == SG_F64 ? 8 : 4;
    const int64_t N = (int64_t)nr * nphi;
    const int S = direct_splits(nr, N);
    size_t o = 0;
    o += sg_align256(es * nr);
    o += 2 * sg_align256(es * (2 * (size_t)nr - 1));
    o += 2 * sg_align256(es * nphi);
    o += 2 * sg_align256(es * nf * N);
    o += sg_align256(sizeof(double) * nf * nf * (percell ? N : nr));
    o += sg_align256(es * (size_t)S * nf * 2 * N);
    o += sg_align256(sizeof(double) * 4);
    return o;
}

template <typename T>
static sg_status potential_run(const sg_grid *g, int nf, const double *h, const T *sigma, const T *H,
                               T *pot, uint32_t flags, void *ws, hipStream_t s)
{
    const int nr = g->n_r, nphi = g->n_phi;
    const int64_t N = (int64_t)nr * nphi;
    const double du = log(g->r_max / g->r_min) / nr;
    const double dphi = 2.0 * SG_PI / nphi;
    const double lnrmin = log(g->r_min);
    const int S = direct_splits(nr, N);
    const int rps = (nr + S - 1) / S;
    char *o = (char *)ws;
    auto take = [&](size_t bytes) {
        char *p = o;
        o += sg_align256(bytes);
        return p;
    };
    T *rrow = (T *)take(sizeof(T) * nr);
    T *sx = (T *)take(sizeof(T) * (2 * (size_t)nr - 1));
    T *ex = (T *)take(sizeof(T) * (2 * (size_t)nr - 1));
    T *sph = (T *)take(sizeof(T) * nphi);
    T *snp = (T *)take(sizeof(T) * nphi);
    T *mass = (T *)take(sizeof(T) * nf * N);
    T *H2 = (T *)take(sizeof(T) * nf * N);
    const int percell = H != nullptr;
    double *self = (double *)take(sizeof(double) * nf * nf * (percell ? N : nr));
    T *partial = (T *)take(sizeof(T) * (size_t)S * nf * 2 * N);
    double *dh = (double *)take(sizeof(double) * 4);
    for (int f = 0; f < nf; ++f)
        hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, dh + f, (int64_t)1, h ? h[f] : 0.0);
    SG_HIP(hipGetLastError());
    {
        int64_t work = nf * N > 2 * nr ? nf * N : 2 * nr;
        if (work < nphi) work = nphi;
        int64_t nb = (work + 255) / 256;
        if (nb > 65536) nb = 65536;
        hipLaunchKernelGGL(k_direct_prep<T>, dim3((unsigned)nb), dim3(256), 0, s, nr, nphi, nf,
                           lnrmin, du, dphi, (const double *)dh, sigma, H, rrow, sx, ex, sph, snp,
                           mass, H2, 0, 0.0, 0.0, nullptr);
        SG_HIP(hipGetLastError());
    }
    const int with_self = !(flags & SG_SELF_CELL_EXCLUDE);
    if (with_self) {
        GLNodes gl;
        sg_gl_nodes(gl);
        const int64_t items = (int64_t)nf * nf * (percell ? N : nr);
        hipLaunchKernelGGL(k_pot_self<T>, dim3((unsigned)items), dim3(256), 0, s, H, (const double *)dh, nf,
                           nr, nphi, lnrmin, du, dphi, percell ? 0 : 1, self, gl, 0);
        SG_HIP(hipGetLastError());
    }
    DirectArgs<T> A;
    A.lin = 0;
    A.nr = nr;
    A.nphi = nphi;
    A.rps = rps;
    A.N = N;
    A.rrow = rrow;
    A.sx = sx;
    A.ex = ex;
    A.sph = sph;
    A.snp = snp;
    A.mass = mass;
    A.H2 = H2;
    A.partial = partial;
    dim3 grid((unsigned)((N + 255) / 256), (unsigned)S);
    switch (nf) {
    case 1: hipLaunchKernelGGL((k_potential<T, 1>), grid, dim3(256), 0, s, A); break;
    case 2: hipLaunchKernelGGL((k_potential<T, 2>), grid, dim3(256), 0, s, A); break;
    case 3: hipLaunchKernelGGL((k_potential<T, 3>), grid, dim3(256), 0, s, A); break;
    default: hipLaunchKernelGGL((k_potential<T, 4>), grid, dim3(256), 0, s, A); break;
    }
    SG_HIP(hipGetLastError());
    const unsigned nb = (unsigned)((N + 255) / 256);
#define SG_PRED(NF)                                                                                      \
    hipLaunchKernelGGL((k_potential_reduce<T, NF>), dim3(nb), dim3(256), 0, s, partial, S, N, nphi, self, \
                       percell ? 0 : 1, with_self, sigma, pot)
    switch (nf) {
    case 1: SG_PRED(1); break;
    case 2: SG_PRED(2); break;
    case 3: SG_PRED(3); break;
    default: SG_PRED(4); break;
    }
#undef SG_PRED
    SG_HIP(hipGetLastError());
    return SG_OK;
}

sg_status sg_potential_launch(const sg_grid *g, int nf, const double *h, const void *sigma,
                              const void *H, void *pot, sg_dtype dt, uint32_t flags, void *ws,
                              hipStream_t s)
{
    if (dt == SG_F64)
        return potential_run<double>(g, nf, h, (const double *)sigma, (const double *)H, (double *)pot,
                                     flags, ws, s);
    return potential_run<float>(g, nf, h, (const float *)sigma, (const float *)H, (float *)pot, flags,
                                ws, s);
}

sg_status sg_direct_launch(const sg_grid *g, int nf, const double *h, const void *sigma,
                           const void *H, void *gr, void *gp, sg_dtype dt, uint32_t flags,
                           void *ws, hipStream_t s)
{
    if (dt == SG_F64)
        return direct_run<double>(g, nf, h, (const double *)sigma, (const double *)H, (double *)gr,
                                  (double *)gp, flags, ws, s);
    return direct_run<float>(g, nf, h, (const float *)sigma, (const float *)H, (float *)gr,
                             (float *)gp, flags, ws, s);
}
