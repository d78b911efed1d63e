// sg_fftpath.hip -- sg_field_fft: batched three-pass log-polar FFT
// convolution, one HIP graph per batch signature.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "sg_fftpath.h"
#include "sg_passes.h"

// ---------------------------------------------------------------- kernels
// Passes 1 and 3 are persistent: workgroup b takes workgroup jobs
// w = sg_xcd_remap(b, K), w + gridDim.x, ... < nj, and issues the loads of its
// next job before it transforms the current one, so that the memory traffic
// of one job overlaps the arithmetic of the previous one.  gridDim.x is a
// multiple of 8 K (a whole number of XCD clusters).  Twiddles depend only on
// the transform length, so one table serves every disc of a launch.

// Pass 1: job = one row pair (two fluids: row idx of each; one fluid: rows
// 2 idx and 2 idx + 1).  Job state is kept as wave-uniform scalars (disc,
// first job, valid count) and addresses are rebuilt from them where needed.
template <int N, int NF>
__device__ inline void p1_rows(int idx, int &i1, int &i2)
{
    i1 = NF == 2 ? idx : 2 * idx;
    i2 = NF == 2 ? idx : 2 * idx + 1;
}

template <int N, int NF>
__device__ inline void p1_issue(const DiscDev *D, int idx, int t, float2 (&z)[FftShape<N>::P])
{
    constexpr int P = FftShape<N>::P, T = FftShape<N>::T;
    int i1, i2;
    p1_rows<N, NF>(idx, i1, i2);
    const uint32_t o1 = (uint32_t)i1 * N + t;
    const uint32_t o2 = (NF == 2 ? (uint32_t)D->nr * N : 0u) + (uint32_t)i2 * N + t;
    const float *x = D->sigma;
#pragma unroll
    for (int p = 0; p < P; ++p) z[p] = make_float2(gld1(x, o1 + T * p), gld1(x, o2 + T * p));
}

template <int N, int NF>
__global__ void __launch_bounds__(PassShape<N>::WGS)
k_pass1(const DiscDev *discs, const WJob *wj, int nj, const float2 *twp)
{
    using S = PassShape<N>;
    constexpr int P = S::P, W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t0 = threadIdx.x % S::T;
    int w = sg_uniform(sg_xcd_remap(blockIdx.x, S::K));
    if (w >= nj) return;
    const LdsPlane<float> pl{lds + W * g};
    TwRegC<N> tw;
    tw.load(twp, t0);
    int cd = sg_uniform(wj[w].disc), cb = sg_uniform(wj[w].base), cn = sg_uniform(wj[w].n);
    float2 nx[P];
    p1_issue<N, NF>(discs + cd, g < cn ? cb + g : cb, t0, nx);
    for (;;) {
        const int t = sg_opaque(t0);
        float2 z[P];
#pragma unroll
        for (int p = 0; p < P; ++p) z[p] = nx[p];
        const int wn = w + gridDim.x;
        const bool more = wn < nj;
        int nd = cd, nb = cb, nn = cn;
        if (more) {
            nd = sg_uniform(wj[wn].disc);
            nb = sg_uniform(wj[wn].base);
            nn = sg_uniform(wj[wn].n);
            p1_issue<N, NF>(discs + nd, g < nn ? nb + g : nb, t, nx);
        }
        {
            const DiscDev *D = discs + cd;
            int i1, i2;
            p1_rows<N, NF>(g < cn ? cb + g : cb, i1, i2);
            const size_t fs = sg_blk_field_elems(N, D->nr);
            p1_finish<N>(z, D->st, i1, D->st + (NF == 2 ? fs : 0), i2, D->nr, tw, t, pl, g < cn);
        }
        if (!more) break;
        w = wn;
        cd = nd;
        cb = nb;
        cn = nn;
    }
}

// Pass 2 launch shape: a column is carried by NF * T threads; for two fluids
// the two halves each own one fluid (forward transform of that source fluid,
// then spectral multiply and inverse transforms for that target fluid), so
// no thread holds more than one fluid's accumulators.
template <int NU, int NF> struct P2Shape {
    static constexpr int P = FftShape<NU>::P, T = FftShape<NU>::T;
    static constexpr int CT = NF * T;
    static constexpr int WGS = CT > 256 ? CT : 256;
    static constexpr int G = WGS / CT;
    static constexpr int K = G >= 4 ? 1 : 4 / G;
};

// Loads of pass-2 column job m for half h: Sigma~_h at rows t + T p (p < P/2;
// the upper half of the padded column is zero) and the unique kernel-spectrum
// values K(k_lo), k_lo = t + T j (j < P/2), and K(NU/2) of every source a.
template <int NU, int NF>
__device__ inline void p2_issue(const DiscDev *D, int m, int h, int t, float2 (&sh)[FftShape<NU>::P / 2],
                                float2 (&K)[NF][2][FftShape<NU>::P / 2], float2 (&KN)[NF][2])
{
    constexpr int P = FftShape<NU>::P, T = FftShape<NU>::T, H = P / 2, NR = NU / 2;
    constexpr uint32_t kk = NR + 1;
    const uint32_t fs = (uint32_t)sg_blk_field_elems(D->nphi, NR);
    const float2 *st = D->st;
    const float2 *spec = D->spec;
#pragma unroll
    for (int p = 0; p < H; ++p) sh[p] = gld2(st, h * fs + (uint32_t)sg_blk_index(m, t + T * p, NR));
#pragma unroll
    for (int a = 0; a < NF; ++a)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const uint32_t o = (((uint32_t)m * (NF * NF) + a * NF + h) * 2 + cc) * kk;
#pragma unroll
            for (int j = 0; j < H; ++j) K[a][cc][j] = gld2(spec, o + t + T * j);
            KN[a][cc] = gld2(spec, o + NR);
        }
}

// Pass 2, one column job m in [0, n_phi/2] per group of NF * T threads (half
// h owns fluid h; NF = 1 has one half); one workgroup job per workgroup (the
// spectra of a column are too many registers to load one job ahead):
//   1. issue all loads: Sigma~_h and the kernel spectra; the spectra arrive
//      while the zero-padded forward u transform of Sigma~_h runs;
//   2. both halves put their natural-order spectra in LDS; thread t reads
//      Sigma^_a at k_lo and at the mirrors k_hi = NU - k_lo (k_hi = NU/2 for
//      t = 0, j = 0) for every a.  K(k_hi) is K(k_lo) conjugated (negated
//      too for K_phi), so every stored spectrum value is loaded exactly once;
//   3. multiply-accumulate g^_{h,c}(k) = sum_a K_c^{a h}(k) Sigma^_a(k) at the
//      2 (P/2) frequencies;
//   4. the products go to LDS in natural order and come back in the
//      transform distribution; inverse u transforms of the (r, phi) pair; the
//      first n_r outputs are stored.
template <int NU, int NF>
__global__ void __launch_bounds__((P2Shape<NU, NF>::WGS)) __attribute__((amdgpu_waves_per_eu(4)))
k_pass2(const DiscDev *discs, const WJob *wj, int nj, const float2 *twu)
{
    using S = P2Shape<NU, NF>;
    constexpr int P = S::P, T = S::T, H = P / 2;
    constexpr int NR = NU / 2;
    constexpr int W = LdsPlane<float>::elems(NU);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G * 2 * NF];
    const int g = threadIdx.x / S::CT;
    const int h = (threadIdx.x % S::CT) / T;
    const int t = threadIdx.x % T;
    const int w = sg_uniform(sg_xcd_remap(blockIdx.x, S::K));
    if (w >= nj) return;
    float2 *base = lds + W * g * 2 * NF;
    // planes: F_h (forward / output r) and X_h (spectrum / output phi)
    const LdsPlane<float> pl[2] = {LdsPlane<float>{base + W * (2 * h)},
                                   LdsPlane<float>{base + W * (2 * h + 1)}};
    const int cd = sg_uniform(wj[w].disc), cb = sg_uniform(wj[w].base), cn = sg_uniform(wj[w].n);
    const DiscDev *D = discs + cd;
    const int m = g < cn ? cb + g : cb;
    // 1. loads
    float2 sh[H], K[NF][2][H], KN[NF][2];
    p2_issue<NU, NF>(D, m, h, t, sh, K, KN);
    TwRegC<NU> tw;
    tw.load(twu, t);
    // forward transform of the own fluid
    {
        float2 v[1][P];
#pragma unroll
        for (int p = 0; p < P; ++p) v[0][p] = p < H ? sh[p] : make_float2(0.f, 0.f);
        const LdsPlane<float> p1[1] = {pl[0]};
        fft_m<NU, false, 1>(v, t, p1, tw);
        // 2. spectra of all fluids at k_lo and k_hi
#pragma unroll
        for (int p = 0; p < P; ++p) pl[1].st(t + T * p, v[0][p]);
    }
    __syncthreads();
    float2 slo[NF][H], shi[NF][H];
#pragma unroll
    for (int a = 0; a < NF; ++a) {
        const LdsPlane<float> X{base + W * (2 * a + 1)};
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int klo = t + T * j;
            const int khi = (j == 0 && t == 0) ? NR : NU - klo;
            slo[a][j] = X.ld(klo);
            shi[a][j] = X.ld(khi);
        }
    }
    __syncthreads();
    // 3. multiply-accumulate at k_lo and k_hi
    float2 olo[2][H], ohi[2][H];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float2 a1 = make_float2(0.f, 0.f), a2 = make_float2(0.f, 0.f);
#pragma unroll
            for (int a = 0; a < NF; ++a) {
                const float2 k1 = K[a][cc][j];
                // mirror: conj (K_r) or minus conj (K_phi); Nyquist reads K(NU/2)
                float2 k2 = (j == 0 && t == 0) ? KN[a][cc] : k1;
                k2 = cc == 0 ? make_float2(k2.x, -k2.y) : make_float2(-k2.x, k2.y);
                const float2 lo = slo[a][j], hi = shi[a][j];
                a1.x += k1.x * lo.x - k1.y * lo.y;
                a1.y += k1.x * lo.y + k1.y * lo.x;
                a2.x += k2.x * hi.x - k2.y * hi.y;
                a2.y += k2.x * hi.y + k2.y * hi.x;
            }
            olo[cc][j] = a1;
            ohi[cc][j] = a2;
        }
    // 4. back to the transform distribution, inverse pair, first n_r outputs
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int klo = t + T * j;
            const int khi = (j == 0 && t == 0) ? NR : NU - klo;
            pl[cc].st(klo, olo[cc][j]);
            pl[cc].st(khi, ohi[cc][j]);
        }
    __syncthreads();
    float2 acc[2][P];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int p = 0; p < P; ++p) acc[cc][p] = pl[cc].ld(t + T * p);
    __syncthreads();
    fft_m<NU, true, 2>(acc, t, pl, tw);
    if (g < cn) {
        const uint32_t fs = (uint32_t)sg_blk_field_elems(D->nphi, NR);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
            for (int p = 0; p < H; ++p)
                gst2(D->gh, (h * 2 + cc) * fs + (uint32_t)sg_blk_index(m, t + T * p, NR), acc[cc][p]);
    }
}

// Pass 3: job = (target fluid b, row i): inverse phi transform of
// g^_r + i g^_phi, whose real and imaginary parts are g_r and g_phi.
template <int N>
__device__ inline void p3_issue(const DiscDev *D, int idx, int t, float2 (&a)[FftShape<N>::P],
                                float2 (&b)[FftShape<N>::P])
{
    const int nr = D->nr;
    const int bf = idx / nr, i = idx % nr;
    const size_t fs = sg_blk_field_elems(N, nr);
    const float2 *A = D->gh + (size_t)(bf * 2) * fs;
    p3_load<N>(A, i, A + fs, i, nr, a, b, t);
}

template <int N, int NF>
__global__ void __launch_bounds__(PassShape<N>::WGS)
k_pass3(const DiscDev *discs, const WJob *wj, int nj, const float2 *twp)
{
    using S = PassShape<N>;
    constexpr int P = S::P, W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t0 = threadIdx.x % S::T;
    int w = sg_uniform(sg_xcd_remap(blockIdx.x, S::K));
    if (w >= nj) return;
    const LdsPlane<float> pl{lds + W * g};
    TwRegC<N> tw;
    tw.load(twp, t0);
    int cd = sg_uniform(wj[w].disc), cb = sg_uniform(wj[w].base), cn = sg_uniform(wj[w].n);
    float2 a[P], b[P];
    p3_issue<N>(discs + cd, g < cn ? cb + g : cb, t0, a, b);
    for (;;) {
        const int t = sg_opaque(t0);
        float2 z[P];
        p3_combine<N>(a, b, z, t);
        const int wn = w + gridDim.x;
        const bool more = wn < nj;
        int nd = cd, nb = cb, nn = cn;
        if (more) {
            nd = sg_uniform(wj[wn].disc);
            nb = sg_uniform(wj[wn].base);
            nn = sg_uniform(wj[wn].n);
            p3_issue<N>(discs + nd, g < nn ? nb + g : nb, t, a, b);
        }
        {
            const DiscDev *D = discs + cd;
            const int idx = g < cn ? cb + g : cb;
            const int nr = D->nr;
            const size_t plane = (size_t)nr * N;
            const size_t o = (size_t)(idx / nr) * plane + (size_t)(idx % nr) * N;
            p3_finish<N>(z, tw, D->gr + o, D->gp + o, t, pl, g < cn);
        }
        if (!more) break;
        w = wn;
        cd = nd;
        cb = nb;
        cn = nn;
    }
}

// ------------------------------------------------------------- launching

using KernelFn = void (*)(const DiscDev *, const WJob *, int, const float2 *);

struct PassKernel {
    KernelFn fn;
    int wgs, G, K;
    bool persistent;  // loops over workgroup jobs (else one per workgroup)
};

template <int N, int NF> static PassKernel pk1()
{
    using S = PassShape<N>;
    return {k_pass1<N, NF>, S::WGS, S::G, S::K, true};
}
template <int N, int NF> static PassKernel pk2()
{
    using S = P2Shape<N, NF>;
    return {k_pass2<N, NF>, S::WGS, S::G, S::K, false};
}
template <int N, int NF> static PassKernel pk3()
{
    using S = PassShape<N>;
    return {k_pass3<N, NF>, S::WGS, S::G, S::K, true};
}

#define SG_SIZE_CASES(F, NF)                                                                      \
    case 4: return F<4, NF>();                                                                     \
    case 8: return F<8, NF>();                                                                     \
    case 16: return F<16, NF>();                                                                   \
    case 32: return F<32, NF>();                                                                   \
    case 64: return F<64, NF>();                                                                   \
    case 128: return F<128, NF>();                                                                 \
    case 256: return F<256, NF>();                                                                 \
    case 512: return F<512, NF>();                                                                 \
    case 1024: return F<1024, NF>();                                                               \
    case 2048: return F<2048, NF>();

static bool pass_kernel(int pass, int n, int nf, PassKernel &out)
{
    auto pick = [&]() -> PassKernel {
        if (pass == 1) {
            if (nf == 1) switch (n) { SG_SIZE_CASES(pk1, 1) }
            else switch (n) { SG_SIZE_CASES(pk1, 2) }
        } else if (pass == 2) {
            if (nf == 1) switch (n) { SG_SIZE_CASES(pk2, 1) case 4096: return pk2<4096, 1>(); }
            else switch (n) { SG_SIZE_CASES(pk2, 2) case 4096: return pk2<4096, 2>(); }
        } else {
            if (nf == 1) switch (n) { SG_SIZE_CASES(pk3, 1) }
            else switch (n) { SG_SIZE_CASES(pk3, 2) }
        }
        return PassKernel{nullptr, 0, 0, 0, false};
    };
    out = pick();
    return out.fn != nullptr;
}

// ------------------------------------------------------------- batch plan
struct Launch {
    PassKernel k;
    size_t wj_off;    // offset (in WJob units) into the workgroup-job table
    int nj;           // workgroup jobs of this launch
    int grid;         // workgroups (a multiple of 8 K)
    const float2 *tw; // twiddles of this launch's transform length
    int pass;
};

struct Plan {
    std::vector<DiscDev> discs;
    std::vector<WJob> wjobs;
    std::vector<Launch> launches;
};

size_t sg_fft_disc_ws_bytes(const sg_disc &d)
{
    const size_t fs = sg_blk_field_elems(d.grid.n_phi, d.grid.n_r);
    return sg_align256(sizeof(float2) * fs * d.fluids.n_fluids) +
           sg_align256(sizeof(float2) * fs * 2 * d.fluids.n_fluids);
}

// Jobs of one disc in a pass: pass 1 row pairs, pass 2 columns m <= n_phi/2,
// pass 3 (target fluid, row) pairs.
static int pass_jobs(const sg_disc &d, int pass)
{
    const int nf = d.fluids.n_fluids;
    if (pass == 1) return nf == 2 ? d.grid.n_r : d.grid.n_r / 2;
    if (pass == 2) return d.grid.n_phi / 2 + 1;
    return nf * d.grid.n_r;
}

// Grid of a launch: whole XCD clusters of 8 K workgroups.  A persistent
// kernel gets its resident workgroups per CU times the CU count (at least one
// cluster, at most the work available); the others one workgroup per job.
static int launch_grid(const PassKernel &k, int nj)
{
    const int cluster = 8 * k.K;
    const int need = (nj + cluster - 1) / cluster * cluster;
    if (!k.persistent) return need;
    int dev = 0, ncu = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k.fn, k.wgs, 0) != hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    int grid = per_cu * ncu / cluster * cluster;
    if (grid < cluster) grid = cluster;
    return grid < need ? grid : need;
}

static void build_plan(const sg_disc *discs, int n, char *ws, Plan &P)
{
    P.discs.resize(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const sg_disc &d = discs[i];
        const TableLayout L = sg_table_layout(d.grid.n_r, d.grid.n_phi, d.fluids.n_fluids, d.flags);
        const char *tb = (const char *)d.table;
        DiscDev &D = P.discs[i];
        D.sigma = d.sigma;
        D.gr = d.g_r;
        D.gp = d.g_phi;
        D.spec = (const float2 *)(tb + L.off_spec);
        D.dspec = (d.flags & SG_WITH_DH) ? (const float2 *)(tb + L.off_dspec) : nullptr;
        D.tw_u = (const float2 *)(tb + L.off_tw_u);
        D.tw_phi = (const float2 *)(tb + L.off_tw_phi);
        const size_t fs = sg_blk_field_elems(d.grid.n_phi, d.grid.n_r);
        D.st = (float2 *)(ws + off);
        D.gh = (float2 *)(ws + off + sg_align256(sizeof(float2) * fs * d.fluids.n_fluids));
        off += sg_fft_disc_ws_bytes(d);
        D.nr = d.grid.n_r;
        D.nphi = d.grid.n_phi;
        D.nf = d.fluids.n_fluids;
        D.pad_ = 0;
    }
    // one launch per (pass, transform length, fluid count); jobs in disc order
    for (int pass = 1; pass <= 3; ++pass) {
        std::map<std::pair<int, int>, std::vector<int>> classes;
        for (int i = 0; i < n; ++i) {
            const int len = pass == 2 ? 2 * discs[i].grid.n_r : discs[i].grid.n_phi;
            classes[{len, discs[i].fluids.n_fluids}].push_back(i);
        }
        for (auto &kv : classes) {
            PassKernel k;
            pass_kernel(pass, kv.first.first, kv.first.second, k);
            std::vector<WJob> list;
            for (int di : kv.second) {
                const int cnt = pass_jobs(discs[di], pass);
                for (int b = 0; b < cnt; b += k.G) list.push_back({di, b, std::min(k.G, cnt - b), 0});
                // keep each disc's workgroup jobs aligned to whole clusters of
                // K so that cache-line sharing stays inside one disc
                while (list.size() % k.K) list.push_back({di, 0, 0, 0});
            }
            Launch La;
            La.k = k;
            La.wj_off = P.wjobs.size();
            La.nj = (int)list.size();
            La.grid = launch_grid(k, La.nj);
            const DiscDev &D0 = P.discs[kv.second[0]];
            La.tw = pass == 2 ? D0.tw_u : D0.tw_phi;
            La.pass = pass;
            P.wjobs.insert(P.wjobs.end(), list.begin(), list.end());
            P.launches.push_back(La);
        }
    }
}

struct Cached {
    void *dmem = nullptr;      // descriptors + jobs on the device
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    Plan plan;
};

static std::mutex g_mu;
static std::map<std::vector<uint64_t>, Cached *> g_cache;

static std::vector<uint64_t> signature(const sg_disc *discs, int n, void *ws)
{
    std::vector<uint64_t> k;
    k.reserve(n * 8 + 2);
    int dev = 0;
    (void)hipGetDevice(&dev);
    k.push_back((uint64_t)dev);
    k.push_back((uint64_t)(uintptr_t)ws);
    for (int i = 0; i < n; ++i) {
        const sg_disc &d = discs[i];
        k.push_back(((uint64_t)d.grid.n_r << 32) | (uint32_t)d.grid.n_phi);
        k.push_back(((uint64_t)d.fluids.n_fluids << 32) | d.flags);
        k.push_back((uint64_t)(uintptr_t)d.sigma);
        k.push_back((uint64_t)(uintptr_t)d.g_r);
        k.push_back((uint64_t)(uintptr_t)d.g_phi);
        k.push_back((uint64_t)(uintptr_t)d.table);
    }
    return k;
}

static sg_status launch(const Cached &C, const Launch &L, hipStream_t s)
{
    const DiscDev *dd = (const DiscDev *)C.dmem;
    const WJob *wj = (const WJob *)((const char *)C.dmem + sg_align256(sizeof(DiscDev) * C.plan.discs.size()));
    hipLaunchKernelGGL(L.k.fn, dim3(L.grid), dim3(L.k.wgs), 0, s, dd, wj + L.wj_off, L.nj, L.tw);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

static sg_status enqueue(const Cached &C, hipStream_t s)
{
    for (const Launch &L : C.plan.launches) {
        const sg_status st = launch(C, L, s);
        if (st != SG_OK) return st;
    }
    return SG_OK;
}

static bool use_graph()
{
    const char *e = getenv("SG_NO_GRAPH");
    return !(e && e[0] == '1');
}

sg_status sg_fft_run(const sg_disc *discs, int n, void *ws, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = signature(discs, n, ws);
    Cached *C;
    auto it = g_cache.find(key);
    if (it == g_cache.end()) {
        C = new Cached;
        build_plan(discs, n, (char *)ws, C->plan);
        const size_t bd = sg_align256(sizeof(DiscDev) * n);
        const size_t bytes = bd + sizeof(WJob) * C->plan.wjobs.size();
        if (hipMalloc(&C->dmem, bytes) != hipSuccess) {
            delete C;
            return SG_ERR_HIP;
        }
        if (hipMemcpy(C->dmem, C->plan.discs.data(), sizeof(DiscDev) * n, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy((char *)C->dmem + bd, C->plan.wjobs.data(), sizeof(WJob) * C->plan.wjobs.size(),
                      hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(C->dmem);
            delete C;
            return SG_ERR_HIP;
        }
        if (use_graph()) {
            hipStream_t cs;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return SG_ERR_HIP;
            bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
            sg_status st = ok ? enqueue(*C, cs) : SG_ERR_HIP;
            hipGraph_t gph = nullptr;
            ok = hipStreamEndCapture(cs, &gph) == hipSuccess && ok && st == SG_OK;
            if (ok) ok = hipGraphInstantiate(&C->exec, gph, nullptr, nullptr, 0) == hipSuccess;
            (void)hipStreamDestroy(cs);
            if (!ok) {
                if (gph) (void)hipGraphDestroy(gph);
                (void)hipFree(C->dmem);
                delete C;
                return SG_ERR_HIP;
            }
            C->graph = gph;
        }
        g_cache[key] = C;
    } else {
        C = it->second;
    }
    if (C->exec) {
        SG_HIP(hipGraphLaunch(C->exec, s));
        return SG_OK;
    }
    return enqueue(*C, s);
}

// Per-pass timing: enqueue the passes (no graph) `reps` times with HIP events
// at the pass boundaries on `s`, wait, and return the mean milliseconds of
// each pass (ms[0..2]).
sg_status sg_fft_profile(const sg_disc *discs, int n, void *ws, hipStream_t s, int reps, float *ms)
{
    Cached *C;
    {
        // make sure the plan exists (first call builds it, like sg_fft_run)
        std::lock_guard<std::mutex> lk(g_mu);
        auto key = signature(discs, n, ws);
        auto it = g_cache.find(key);
        if (it == g_cache.end()) C = nullptr;
        else C = it->second;
    }
    if (!C) {
        sg_status st = sg_fft_run(discs, n, ws, s);
        if (st != SG_OK) return st;
        std::lock_guard<std::mutex> lk(g_mu);
        C = g_cache[signature(discs, n, ws)];
    }
    std::vector<hipEvent_t> ev(4 * reps);
    for (auto &e : ev) SG_HIP(hipEventCreate(&e));
    for (int r = 0; r < reps; ++r) {
        SG_HIP(hipEventRecord(ev[4 * r], s));
        for (int pass = 1; pass <= 3; ++pass) {
            for (const Launch &L : C->plan.launches) {
                if (L.pass != pass) continue;
                const sg_status st = launch(*C, L, s);
                if (st != SG_OK) return st;
            }
            SG_HIP(hipEventRecord(ev[4 * r + pass], s));
        }
    }
    SG_HIP(hipEventSynchronize(ev[4 * reps - 1]));
    for (int p = 0; p < 3; ++p) ms[p] = 0.f;
    for (int r = 0; r < reps; ++r)
        for (int p = 0; p < 3; ++p) {
            float t = 0.f;
            SG_HIP(hipEventElapsedTime(&t, ev[4 * r + p], ev[4 * r + p + 1]));
            ms[p] += t / reps;
        }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return SG_OK;
}

void sg_fft_release()
{
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipDeviceSynchronize();
    for (auto &kv : g_cache) {
        Cached *C = kv.second;
        if (C->exec) (void)hipGraphExecDestroy(C->exec);
        if (C->graph) (void)hipGraphDestroy(C->graph);
        if (C->dmem) (void)hipFree(C->dmem);
        delete C;
    }
    g_cache.clear();
}
