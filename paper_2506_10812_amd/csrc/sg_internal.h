// sg_internal.h -- shared internals of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/sg.h"

#define SG_PI 3.14159265358979323846
#define SG_SQRT_PI 1.77245385090551602730
#define SG_SQRT2 1.41421356237309504880

// ---------------------------------------------------------------- complex
__host__ __device__ inline float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 c_mul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 c_conj(float2 a) { return make_float2(a.x, -a.y); }
__host__ __device__ inline float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 c_mul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 c_conj(double2 a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

template <typename R> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename R> using cplx_t = typename cplx_of<R>::type;

template <typename V> __host__ __device__ inline V c_make(double re, double im);
template <> __host__ __device__ inline float2 c_make<float2>(double re, double im)
{
    return make_float2((float)re, (float)im);
}
template <> __host__ __device__ inline double2 c_make<double2>(double re, double im)
{
    return make_double2(re, im);
}

// multiply by -i (forward) or +i (inverse)
template <bool INV, typename V> __host__ __device__ inline V c_mul_mi(V a)
{
    V r;
    if (INV) { r.x = -a.y; r.y = a.x; }
    else     { r.x = a.y;  r.y = -a.x; }
    return r;
}

// --------------------------------------------------- global-memory access
// Loads and stores through address-space-1 pointers compile to global_load /
// global_store instead of flat accesses (flat accesses also count against the
// LDS wait counter, so every LDS barrier would wait for them).
typedef float sg_v2f __attribute__((ext_vector_type(2)));
typedef const sg_v2f __attribute__((address_space(1))) sg_gcv2f;
typedef sg_v2f __attribute__((address_space(1))) sg_gv2f;
typedef const float __attribute__((address_space(1))) sg_gcf;
typedef float __attribute__((address_space(1))) sg_gf;

__device__ inline float2 gload2(const float2 *p, size_t i)
{
    const sg_v2f v = ((sg_gcv2f *)p)[i];
    return make_float2(v.x, v.y);
}
__device__ inline void gstore2(float2 *p, size_t i, float2 v)
{
    sg_v2f w;
    w.x = v.x;
    w.y = v.y;
    ((sg_gv2f *)p)[i] = w;
}
__device__ inline float gload1(const float *p, size_t i) { return ((sg_gcf *)p)[i]; }
__device__ inline void gstore1(float *p, size_t i, float v) { ((sg_gf *)p)[i] = v; }

// The same with a 32-bit element offset from a (usually wave-uniform) base:
// the byte offset is formed in 32 bits, so the access can use the scalar
// base + vector offset addressing form.  Callers keep every buffer addressed
// this way below 4 GiB (the FFT path's largest buffer is a few hundred MB).
__device__ inline float2 gld2(const float2 *p, uint32_t i)
{
    const sg_v2f v = *(sg_gcv2f *)((const char *)p + (i << 3));
    return make_float2(v.x, v.y);
}
__device__ inline void gst2(float2 *p, uint32_t i, float2 v)
{
    sg_v2f w;
    w.x = v.x;
    w.y = v.y;
    *(sg_gv2f *)((char *)p + (i << 3)) = w;
}
__device__ inline float gld1(const float *p, uint32_t i) { return *(sg_gcf *)((const char *)p + (i << 2)); }
// Non-temporal store: for outputs written once and not read back by the
// library (they need not displace the intermediates in the caches).
__device__ inline void gst1nt(float *p, uint32_t i, float v)
{
    __builtin_nontemporal_store(v, (sg_gf *)((char *)p + (i << 2)));
}
__device__ inline void gst1(float *p, uint32_t i, float v) { *(sg_gf *)((char *)p + (i << 2)) = v; }

// 16-byte access of two consecutive complex values (16-byte aligned).
typedef float sg_v4f __attribute__((ext_vector_type(4)));
typedef const sg_v4f __attribute__((address_space(1))) sg_gcv4f;
typedef sg_v4f __attribute__((address_space(1))) sg_gv4f;
__device__ inline void gld2x2(const float2 *p, float2 &a, float2 &b)
{
    const sg_v4f v = *(sg_gcv4f *)p;
    a = make_float2(v.x, v.y);
    b = make_float2(v.z, v.w);
}
__device__ inline void gst2x2(float2 *p, float2 a, float2 b)
{
    sg_v4f v;
    v.x = a.x;
    v.y = a.y;
    v.z = b.x;
    v.w = b.y;
    *(sg_gv4f *)p = v;
}

// Forces a value that is equal in all lanes into a scalar register.
__device__ inline int sg_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------ table layout
// Device kernel-table layout (all offsets 256-byte aligned, computable on the
// host from the arguments alone):
//   header   sg_table_header
//   tw_u     float2[2 n_r]       e^{-2 pi i n / (2 n_r)}
//   tw_phi   float2[n_phi]       e^{-2 pi i n / n_phi}
//   spec     float2[ncol][npair][2][kk]   scaled half spectra of K_r, K_phi
//   dspec    float2[ncol][npair][2][2][kk] d/dh_a, d/dh_b spectra (SG_WITH_DH)
// with ncol = n_phi/2 + 1, kk = n_r + 1, pair = a * n_fluids + b (a source,
// b target), component 0 = r, 1 = phi.
#define SG_TABLE_MAGIC 0x31544753u  // "SGT1"

struct sg_table_header {
    uint32_t magic, version;
    int32_t n_r, n_phi, n_fluids;
    uint32_t flags;
    double h[4];
    double r_min, r_max;
    double self_r[16];      // self-cell average per pair (double)
    double dself_r[16][2];  // its d/dh_a, d/dh_b
    double ind_coef[4];     // indirect term: sqrt(2) K_a A_k / r_k^2 per source fluid
    uint64_t total_bytes;
};

struct TableLayout {
    int nr, nphi, nf, npair, ncol, kk;
    uint32_t flags;
    size_t off_tw_u, off_tw_phi, off_spec, off_dspec, total;
};

inline size_t sg_align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline TableLayout sg_table_layout(int nr, int nphi, int nf, uint32_t flags)
{
    TableLayout L;
    L.nr = nr;
    L.nphi = nphi;
    L.nf = nf;
    L.npair = nf * nf;
    L.ncol = nphi / 2 + 1;
    L.kk = nr + 1;
    L.flags = flags;
    size_t o = sg_align256(sizeof(sg_table_header));
    L.off_tw_u = o;
    o = sg_align256(o + sizeof(float2) * 2 * (size_t)nr);
    L.off_tw_phi = o;
    o = sg_align256(o + sizeof(float2) * (size_t)nphi);
    L.off_spec = o;
    // columns m = 0 .. n_phi/2, then the pair column (K0 + KN)/2, (K0 - KN)/2
    o = sg_align256(o + sizeof(float2) * (size_t)(L.ncol + 1) * L.npair * 2 * L.kk);
    L.off_dspec = o;
    if (flags & SG_WITH_DH) o = sg_align256(o + sizeof(float2) * (size_t)L.ncol * L.npair * 4 * L.kk);
    L.total = o;
    return L;
}

// Semi-spectral table layout (sg_ss_table; H_f any function of r):
//   header   sg_ss_header
//   tw_phi   float2[n_phi]       e^{-2 pi i n / n_phi}
//   modes    SsMode[ncol]        where each mode's operators start, its band
//   coef     the operators of m = 0, 1, ..., n_phi/2 in order, each
//              full:   float2[F][F][n_r][nrt]      [b][a][i'][i]
//              banded: float2[F][F][2w+1][nrt]     [b][a][d][i], i' = i + d - w
// (b target fluid, a source fluid, i' source row, i target row).  Element
// (t_r, t_phi) is the radial operator of mode m: g^_r gets t_r Sigma~ and
// g^_phi gets i t_phi Sigma~.  nrt = n_r rounded up to even (the padding
// target column is zero), so target pairs are 16-byte aligned.  Banded
// entries whose source row falls outside the grid are zero.
//
// Band of mode m: the kernels are analytic in phi within |Im phi| < |X|
// (X = u_i - u_i'; their only singularity, s = 0, sits at phi = +-i X), so
// the mode-m coupling of two rings falls off like e^{-m |X|}; entries with
// m |X| > SG_SS_BAND_L (about 2^-30 of the axisymmetric coupling) are
// dropped.  w = ceil(L / (m du)); a mode is stored banded when
// 4 w + 2 <= n_r, full otherwise (and always with SG_SS_FULL, and for m = 0).
#define SG_SS_MAGIC 0x31535347u  // "GSS1"
#define SG_SS_BAND_L 20.794415416798359  // 30 ln 2

struct sg_ss_header {
    uint32_t magic, version;
    int32_t n_r, n_phi, n_fluids;
    uint32_t flags;
    double r_min, r_max, du;
    uint64_t total_bytes;
};

struct SsMode {
    uint64_t off;     // first float2 of the mode in coef
    int32_t w;        // band half-width (banded modes)
    int32_t banded;
};

__host__ __device__ inline int sg_ss_band(int m, int nr, double du, bool full)
{
    if (full || m == 0 || nr < 2) return nr - 1;
    const double w = ceil(SG_SS_BAND_L / ((double)m * du));
    return w >= (double)(nr - 1) ? nr - 1 : (int)w;
}
__host__ __device__ inline bool sg_ss_is_banded(int w, int nr) { return 4 * w + 2 <= nr; }

struct SsLayout {
    int nr, nphi, nf, ncol, nrt;
    bool full;
    double du;
    size_t rows;        // F * F * n_r * nrt: (b, a, i', i) rows of one full mode
    size_t coef_elems;  // float2 elements of all modes
    int max_w;          // widest band of a banded mode (-1: none banded)
    size_t off_tw_phi, off_modes, off_coef, total;
};

// Host-side: sizes and offsets (du = ln(r_max/r_min)/n_r as the build uses it).
inline SsLayout sg_ss_layout(int nr, int nphi, int nf, double du, bool full)
{
    SsLayout L;
    L.nr = nr;
    L.nphi = nphi;
    L.nf = nf;
    L.ncol = nphi / 2 + 1;
    L.nrt = (nr + 1) & ~1;
    L.full = full;
    L.du = du;
    L.rows = (size_t)nf * nf * nr * L.nrt;
    L.coef_elems = 0;
    L.max_w = -1;
    for (int m = 0; m < L.ncol; ++m) {
        const int w = sg_ss_band(m, nr, du, full);
        const bool b = sg_ss_is_banded(w, nr);
        L.coef_elems += (size_t)nf * nf * (b ? 2 * w + 1 : nr) * L.nrt;
        if (b && w > L.max_w) L.max_w = w;
    }
    size_t o = sg_align256(sizeof(sg_ss_header));
    L.off_tw_phi = o;
    o = sg_align256(o + sizeof(float2) * (size_t)nphi);
    L.off_modes = o;
    o = sg_align256(o + sizeof(SsMode) * (size_t)L.ncol);
    L.off_coef = o;
    o = sg_align256(o + sizeof(float2) * L.coef_elems);
    L.total = o;
    return L;
}

// Log spacing of the band rule: du of a log grid; on a uniform radial grid
// (SG_LINEAR_R) the smallest log spacing of adjacent centres (outer edge).
inline double sg_ss_du(const sg_grid &g, uint32_t flags)
{
    if (!(flags & SG_LINEAR_R)) return log(g.r_max / g.r_min) / g.n_r;
    if (g.n_r < 2) return 1.0;
    const double dr = (g.r_max - g.r_min) / g.n_r;
    return log((g.r_max - 0.5 * dr) / (g.r_max - 1.5 * dr));
}

// Tiled layout of the half-spectrum intermediates between the passes: tiles
// of 4 columns x 4 rows (128 bytes), each column's 4 rows contiguous inside
// the tile, and the tiles of one 4-column group following each other down
// the rows.  A column job of pass 2 then reads and writes 32 contiguous bytes
// per 4 rows, and a workgroup of 4 consecutive rows in passes 1 and 3 moves
// whole tiles.  Row counts are padded to a multiple of 4 (the padding rows
// are written by pass 1 and never read as data).
__host__ __device__ inline int sg_blk_rows(int nr) { return (nr + 3) & ~3; }
__host__ __device__ inline size_t sg_blk_index(int m, int i, int nr)
{
    return ((size_t)(m >> 2) * sg_blk_rows(nr) + (i & ~3)) * 4 + (m & 3) * 4 + (i & 3);
}
// first element of tile (column group q, rows i0 .. i0 + 3), i0 % 4 == 0
__host__ __device__ inline size_t sg_blk_tile(int q, int i0, int nr)
{
    return ((size_t)q * sg_blk_rows(nr) + i0) * 4;
}
__host__ __device__ inline size_t sg_blk_field_elems(int nphi, int nr)
{
    return (size_t)((nphi / 2 + 1 + 3) >> 2) * sg_blk_rows(nr) * 4;
}

// XCD-aware remap of workgroup ids: MI355X dispatches consecutive workgroups
// round-robin over its 8 XCDs.  The remap gives the K workgroups that share
// cache lines consecutive logical ids on one XCD.  n_wg must be a multiple of
// 8 K; the result is a bijection on [0, n_wg).
__device__ inline int sg_xcd_remap(int w, int K)
{
    int x = w & 7, s = w >> 3;
    return (s / K) * 8 * K + x * K + (s % K);
}

inline int sg_ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}
inline bool sg_is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// status helper: returns SG_ERR_HIP from the enclosing function on failure
#define SG_HIP(call)                                \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return SG_ERR_HIP;    \
    } while (0)
