// sg_fftpath.hip -- sg_field_fft: batched three-pass log-polar FFT
// convolution, one HIP graph per batch signature.
#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "sg_fftpath.h"
#include "sg_passes.h"

// ---------------------------------------------------------------- kernels
template <int N, int NF>
__global__ void __launch_bounds__(PassShape<N>::WGS)
k_pass1(const DiscDev *discs, const Job *jobs, const float2 *tw_default)
{
    using S = PassShape<N>;
    constexpr int W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t = threadIdx.x % S::T;
    const int wl = sg_xcd_remap(blockIdx.x, S::K);
    // whole padding workgroup: leave before any barrier
    if (jobs[wl * S::G].disc < 0) return;
    const Job J = jobs[wl * S::G + g];
    const bool valid = J.disc >= 0;
    DiscDev D;
    if (valid) D = discs[J.disc];
    else { D = discs[jobs[wl * S::G].disc]; D.tw_phi = tw_default; }
    LdsPlane<float> pl{lds + W * g};
    const int nr = D.nr;
    const size_t fs = sg_blk_field_elems(N, nr);
    const size_t plane = (size_t)nr * N;
    // two fluids: (fluid 0, fluid 1) of row idx; one fluid: rows 2 idx, 2 idx + 1
    const int i1 = NF == 2 ? J.idx : 2 * J.idx, i2 = NF == 2 ? J.idx : 2 * J.idx + 1;
    const int f2 = NF == 2 ? 1 : 0;
    TwRegC<N> tw;
    tw.load(D.tw_phi, t);
    phi_fwd_pair<N>(D.sigma + (size_t)i1 * N, D.sigma + f2 * plane + (size_t)i2 * N, D.st, i1,
                    D.st + f2 * fs, i2, nr, tw, t, pl, valid);
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

// Pass 2, one column job of one disc per group of NF * T threads (half h
// owns fluid h; NF = 1 has one half):
//   1. issue all loads at once: Sigma~_h (rows t + T p, p < P/2) and the kernel
//      spectra for target b = h at the thread's own frequencies
//      k_lo = t + T j (j < P/2), for every source a and component c; the
//      spectra arrive while the forward transform runs;
//   2. zero-padded forward u transform of Sigma~_h;
//   3. both halves put their natural-order spectra in LDS; thread t reads
//      Sigma^_a at k_lo and at the mirrors k_hi = NU - k_lo (k_hi = NU/2 for
//      t = 0, j = 0) for every a.  K(k_hi) is K(k_lo) conjugated (negated
//      too for K_phi), so every stored spectrum value is loaded exactly once;
//   4. multiply-accumulate g^_{h,c}(k) = sum_a K_c^{a h}(k) Sigma^_a(k) at the
//      2 (P/2) frequencies, write them to LDS in natural order and read them
//      back in the transform distribution;
//   5. inverse u transforms of the (r, phi) pair; the first n_r outputs are
//      stored.  One twiddle per stage and butterfly stays in registers.
template <int NU, int NF>
__global__ void __launch_bounds__((P2Shape<NU, NF>::WGS)) __attribute__((amdgpu_waves_per_eu(4)))
k_pass2(const DiscDev *discs, const Job *jobs, const float2 *tw_default)
{
    using S = P2Shape<NU, NF>;
    constexpr int P = S::P, T = S::T, H = P / 2;
    constexpr int NR = NU / 2;
    constexpr int W = LdsPlane<float>::elems(NU);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G * 2 * NF];
    const int g = threadIdx.x / S::CT;
    const int h = (threadIdx.x % S::CT) / T;
    const int t = threadIdx.x % T;
    const int wl = sg_xcd_remap(blockIdx.x, S::K);
    if (jobs[wl * S::G].disc < 0) return;
    const Job J = jobs[wl * S::G + g];
    const bool valid = J.disc >= 0;
    float2 *base = lds + W * g * 2 * NF;
    // planes: F_h (forward / output r) and X_h (spectrum / output phi)
    const LdsPlane<float> pl[2] = {LdsPlane<float>{base + W * (2 * h)},
                                   LdsPlane<float>{base + W * (2 * h + 1)}};
    const DiscDev D = discs[valid ? J.disc : jobs[wl * S::G].disc];
    TwRegC<NU> tw;
    tw.load(valid ? D.tw_u : tw_default, t);
    const int m = valid ? J.idx : 0;
    const size_t fs = sg_blk_field_elems(D.nphi, NR);
    const size_t kk = NR + 1;
    const size_t cstride = (size_t)(NF * NF) * 2 * kk;
    const float2 *col = D.spec + (size_t)m * cstride;

    // 1. loads
    float2 sh[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        sh[p] = make_float2(0.f, 0.f);
        if (valid && p < H) {
            const size_t row = h * fs;
            sh[p] = gload2(D.st, row + sg_blk_index(m, t + T * p, NR));
        }
    }
    // unique spectrum values K(k_lo) and K(NU/2) of every source fluid
    float2 K[NF][2][H], KN[NF][2];
#pragma unroll
    for (int a = 0; a < NF; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float2 *kc = col + ((a * NF + h) * 2 + c) * kk;
#pragma unroll
            for (int j = 0; j < H; ++j) K[a][c][j] = valid ? gload2(kc, t + T * j) : make_float2(0.f, 0.f);
            KN[a][c] = valid ? gload2(kc, NR) : make_float2(0.f, 0.f);
        }
    // 2. forward transform of the own fluid
    {
        float2(&own)[1][P] = *reinterpret_cast<float2(*)[1][P]>(&sh);
        const LdsPlane<float> p1[1] = {pl[0]};
        fft_m<NU, false, 1>(own, t, p1, tw);
    }
    // 3. spectra of all fluids at k_lo and k_hi
#pragma unroll
    for (int p = 0; p < P; ++p) pl[1].st(t + T * p, sh[p]);
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
    // 4. multiply-accumulate at k_lo and k_hi, back to the transform distribution
    float2 olo[2][H], ohi[2][H];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float2 a1 = make_float2(0.f, 0.f), a2 = make_float2(0.f, 0.f);
#pragma unroll
            for (int a = 0; a < NF; ++a) {
                const float2 k1 = K[a][c][j];
                // mirror: conj (K_r) or minus conj (K_phi); Nyquist reads K(NU/2)
                float2 k2 = (j == 0 && t == 0) ? KN[a][c] : k1;
                k2 = c == 0 ? make_float2(k2.x, -k2.y) : make_float2(-k2.x, k2.y);
                const float2 lo = slo[a][j], hi = shi[a][j];
                a1.x += k1.x * lo.x - k1.y * lo.y;
                a1.y += k1.x * lo.y + k1.y * lo.x;
                a2.x += k2.x * hi.x - k2.y * hi.y;
                a2.y += k2.x * hi.y + k2.y * hi.x;
            }
            olo[c][j] = a1;
            ohi[c][j] = a2;
        }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int klo = t + T * j;
            const int khi = (j == 0 && t == 0) ? NR : NU - klo;
            pl[c].st(klo, olo[c][j]);
            pl[c].st(khi, ohi[c][j]);
        }
    __syncthreads();
    float2 acc[2][P];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int p = 0; p < P; ++p) acc[c][p] = pl[c].ld(t + T * p);
    __syncthreads();
    // 5. inverse pair, first n_r outputs
    fft_m<NU, true, 2>(acc, t, pl, tw);
    if (valid) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int p = 0; p < H; ++p) {
                const size_t o = (h * 2 + c) * fs;
                gstore2(D.gh, o + sg_blk_index(m, t + T * p, NR), acc[c][p]);
            }
    }
}

template <int N, int NF>
__global__ void __launch_bounds__(PassShape<N>::WGS)
k_pass3(const DiscDev *discs, const Job *jobs, const float2 *tw_default)
{
    using S = PassShape<N>;
    constexpr int W = LdsPlane<float>::elems(N);
    __shared__ __attribute__((aligned(16))) float2 lds[W * S::G];
    const int g = threadIdx.x / S::T, t = threadIdx.x % S::T;
    const int wl = sg_xcd_remap(blockIdx.x, S::K);
    if (jobs[wl * S::G].disc < 0) return;
    const Job J = jobs[wl * S::G + g];
    const bool valid = J.disc >= 0;
    LdsPlane<float> pl{lds + W * g};
    const DiscDev D = discs[valid ? J.disc : jobs[wl * S::G].disc];
    const int nr = D.nr;
    const int b = valid ? J.idx / nr : 0, i = valid ? J.idx % nr : 0;
    const size_t fs = sg_blk_field_elems(N, nr);
    const size_t plane = (size_t)nr * N;
    TwRegC<N> tw;
    tw.load(valid ? D.tw_phi : tw_default, t);
    phi_inv_pair<N>(D.gh + (b * 2 + 0) * fs, i, D.gh + (b * 2 + 1) * fs, i, nr, tw,
                    D.gr + b * plane + (size_t)i * N, D.gp + b * plane + (size_t)i * N, t, pl,
                    valid);
}

// ------------------------------------------------------------- launching

using KernelFn = void (*)(const DiscDev *, const Job *, const float2 *);

struct PassKernel {
    KernelFn fn;
    int wgs, G, K;
};

template <int N, int NF> static PassKernel pk1()
{
    using S = PassShape<N>;
    return {k_pass1<N, NF>, S::WGS, S::G, S::K};
}
template <int N, int NF> static PassKernel pk2()
{
    using S = P2Shape<N, NF>;
    return {k_pass2<N, NF>, S::WGS, S::G, S::K};
}
template <int N, int NF> static PassKernel pk3()
{
    using S = PassShape<N>;
    return {k_pass3<N, NF>, S::WGS, S::G, S::K};
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
    PassKernel k{nullptr, 0, 0, 0};
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
        return PassKernel{nullptr, 0, 0, 0};
    };
    k = pick();
    out = k;
    return k.fn != nullptr;
}

// ------------------------------------------------------------- batch plan
struct Launch {
    PassKernel k;
    size_t job_off;   // offset (in Job units) into the job table
    int nwg;
    size_t tw_disc;   // disc whose twiddles serve padding groups
    int pass;
};

struct Plan {
    std::vector<DiscDev> discs;
    std::vector<Job> jobs;
    std::vector<Launch> launches;
};

size_t sg_fft_disc_ws_bytes(const sg_disc &d)
{
    const size_t fs = sg_blk_field_elems(d.grid.n_phi, d.grid.n_r);
    return sg_align256(sizeof(float2) * fs * d.fluids.n_fluids) +
           sg_align256(sizeof(float2) * fs * 2 * d.fluids.n_fluids);
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
            const int nf = kv.first.second;
            std::vector<Job> list;
            for (int di : kv.second) {
                const sg_disc &d = discs[di];
                int cnt;
                if (pass == 1) cnt = nf == 2 ? d.grid.n_r : d.grid.n_r / 2;
                else if (pass == 2) cnt = d.grid.n_phi / 2 + 1;
                else cnt = nf * d.grid.n_r;
                for (int j = 0; j < cnt; ++j) list.push_back({di, j});
                // keep each disc's jobs aligned to whole XCD clusters of
                // G*K jobs so that cache-line sharing stays inside one disc
                const size_t unit = (size_t)k.G * k.K;
                while (list.size() % unit) list.push_back({-1, 0});
            }
            const size_t per_round = (size_t)k.G * 8 * k.K;
            while (list.size() % per_round) list.push_back({-1, 0});
            Launch La;
            La.k = k;
            La.job_off = P.jobs.size();
            La.nwg = (int)(list.size() / k.G);
            La.tw_disc = kv.second[0];
            La.pass = pass;
            P.jobs.insert(P.jobs.end(), list.begin(), list.end());
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

static sg_status enqueue(const Cached &C, hipStream_t s)
{
    const DiscDev *dd = (const DiscDev *)C.dmem;
    const Job *jj = (const Job *)((const char *)C.dmem + sg_align256(sizeof(DiscDev) * C.plan.discs.size()));
    for (const Launch &L : C.plan.launches) {
        const float2 *twd = L.pass == 2 ? C.plan.discs[L.tw_disc].tw_u : C.plan.discs[L.tw_disc].tw_phi;
        hipLaunchKernelGGL(L.k.fn, dim3(L.nwg), dim3(L.k.wgs), 0, s, dd, jj + L.job_off, twd);
        SG_HIP(hipGetLastError());
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
        const size_t bytes = bd + sizeof(Job) * C->plan.jobs.size();
        if (hipMalloc(&C->dmem, bytes) != hipSuccess) {
            delete C;
            return SG_ERR_HIP;
        }
        if (hipMemcpy(C->dmem, C->plan.discs.data(), sizeof(DiscDev) * n, hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy((char *)C->dmem + bd, C->plan.jobs.data(), sizeof(Job) * C->plan.jobs.size(),
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
    const DiscDev *dd = (const DiscDev *)C->dmem;
    const Job *jj = (const Job *)((const char *)C->dmem + sg_align256(sizeof(DiscDev) * C->plan.discs.size()));
    std::vector<hipEvent_t> ev(4 * reps);
    for (auto &e : ev) SG_HIP(hipEventCreate(&e));
    for (int r = 0; r < reps; ++r) {
        SG_HIP(hipEventRecord(ev[4 * r], s));
        for (int pass = 1; pass <= 3; ++pass) {
            for (const Launch &L : C->plan.launches) {
                if (L.pass != pass) continue;
                const float2 *twd = L.pass == 2 ? C->plan.discs[L.tw_disc].tw_u : C->plan.discs[L.tw_disc].tw_phi;
                hipLaunchKernelGGL(L.k.fn, dim3(L.nwg), dim3(L.k.wgs), 0, s, dd, jj + L.job_off, twd);
                SG_HIP(hipGetLastError());
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
