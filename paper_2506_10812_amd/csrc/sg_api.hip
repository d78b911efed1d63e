// sg_api.hip -- the C ABI (include/sg.h): argument validation, workspace
// sizing and dispatch.  No device work is enqueued before validation passes.
#include <math.h>

#include <mutex>

#include "sg_adjoint.h"
#include "sg_direct.h"
#include "sg_fftpath.h"
#include "sg_semispec.h"
#include "sg_table.h"

static bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

static sg_status check_grid(const sg_grid *g)
{
    if (!g) return SG_ERR_ARG;
    if (g->n_r < 1 || g->n_phi < 1) return SG_ERR_ARG;
    if (!finite_pos(g->r_min) || !isfinite(g->r_max) || !(g->r_max > g->r_min)) return SG_ERR_ARG;
    return SG_OK;
}

static sg_status check_fft_grid(const sg_grid *g)
{
    sg_status s = check_grid(g);
    if (s != SG_OK) return s;
    if (!sg_is_pow2(g->n_r) || !sg_is_pow2(g->n_phi)) return SG_ERR_UNSUPPORTED;
    if (g->n_r < 2 || g->n_r > 2048 || g->n_phi < 4 || g->n_phi > 2048) return SG_ERR_UNSUPPORTED;
    return SG_OK;
}

static sg_status check_fluids(const sg_fluids *f)
{
    if (!f) return SG_ERR_ARG;
    if (f->n_fluids < 1 || f->n_fluids > 4) return SG_ERR_ARG;
    for (int i = 0; i < f->n_fluids; ++i)
        if (!finite_pos(f->h[i])) return SG_ERR_ARG;
    return SG_OK;
}

// FFT path beyond two groups: a pass-2 column job takes n_fluids x 2 n_r / 8
// threads, at most 1024, so n_r <= 1024 there.
static bool fft_groups_ok(const sg_grid *g, const sg_fluids *f)
{
    return f->n_fluids <= 2 || g->n_r <= 1024;
}

static bool flags_ok(uint32_t flags)
{
    return (flags & ~(uint32_t)(SG_SELF_CELL_EXCLUDE | SG_WITH_DH | SG_INDIRECT | SG_SECOND_ORDER)) == 0;
}

// SG_SECOND_ORDER tables have no separate own-cell term to drop
static bool second_order_ok(uint32_t flags)
{
    return !(flags & SG_SECOND_ORDER) || !(flags & SG_SELF_CELL_EXCLUDE);
}

// Semi-spectral path: n_phi a power of two in [4, 2048], 1 <= n_r <= 2048.
static sg_status check_ss_grid(const sg_grid *g)
{
    sg_status s = check_grid(g);
    if (s != SG_OK) return s;
    if (!sg_is_pow2(g->n_phi) || g->n_phi < 4 || g->n_phi > 2048) return SG_ERR_UNSUPPORTED;
    if (g->n_r > sg_ss_max_nr()) return SG_ERR_UNSUPPORTED;
    return SG_OK;
}

// Semi-spectral fluid (scale-height group) count: 1..4, and n_r <= 1024
// beyond two groups (the middle pass stages every group's column in LDS).
static bool ss_fluids_ok(const sg_grid *g, int nf)
{
    return nf >= 1 && nf <= 4 && (nf <= 2 || g->n_r <= 1024);
}

static bool ss_flags_ok(uint32_t flags)
{
    if ((flags & SG_POTENTIAL) && (flags & SG_INDIRECT)) return false;
    // second-order operators: the force on a log grid, own cell included
    if ((flags & SG_SECOND_ORDER) && (flags & (SG_POTENTIAL | SG_LINEAR_R | SG_SELF_CELL_EXCLUDE))) return false;
    return (flags & ~(uint32_t)(SG_SELF_CELL_EXCLUDE | SG_INDIRECT | SG_SEMI_SPECTRAL | SG_SS_FULL |
                                SG_POTENTIAL | SG_LINEAR_R | SG_SECOND_ORDER)) == 0;
}

extern "C" {

size_t sg_kernel_table_bytes(const sg_grid *grid, const sg_fluids *fluids, uint32_t flags)
{
    if (check_fft_grid(grid) != SG_OK || check_fluids(fluids) != SG_OK || !flags_ok(flags)) return 0;
    if (!second_order_ok(flags)) return 0;
    if (!fft_groups_ok(grid, fluids)) return 0;
    return sg_table_layout(grid->n_r, grid->n_phi, fluids->n_fluids, flags).total;
}

size_t sg_kernel_table_workspace_bytes(const sg_grid *grid, const sg_fluids *fluids, uint32_t flags)
{
    if (check_fft_grid(grid) != SG_OK || check_fluids(fluids) != SG_OK || !flags_ok(flags)) return 0;
    if (!fft_groups_ok(grid, fluids) || !second_order_ok(flags)) return 0;
    return sg_table_ws_bytes(grid->n_r, grid->n_phi);
}

sg_status sg_kernel_table(const sg_grid *grid, const sg_fluids *fluids, uint32_t flags,
                          void *d_table, void *d_ws, size_t ws_bytes, void *stream)
{
    sg_status s = check_fft_grid(grid);
    if (s != SG_OK) return s;
    if ((s = check_fluids(fluids)) != SG_OK) return s;
    if (!fft_groups_ok(grid, fluids)) return SG_ERR_UNSUPPORTED;
    if (!flags_ok(flags)) return SG_ERR_ARG;
    if (!second_order_ok(flags)) return SG_ERR_UNSUPPORTED;
    if (!d_table || ((uintptr_t)d_table & 255)) return SG_ERR_ARG;
    if (!d_ws || ws_bytes < sg_table_ws_bytes(grid->n_r, grid->n_phi) || ((uintptr_t)d_ws & 255))
        return SG_ERR_WORKSPACE;
    return sg_table_build(grid, fluids, flags, d_table, d_ws, (hipStream_t)stream);
}

size_t sg_ss_table_bytes(const sg_grid *grid, int n_fluids, uint32_t flags)
{
    if (check_ss_grid(grid) != SG_OK || !ss_fluids_ok(grid, n_fluids) || !ss_flags_ok(flags)) return 0;
    return sg_ss_layout(grid->n_r, grid->n_phi, n_fluids, sg_ss_du(*grid, flags), (flags & SG_SS_FULL) != 0).total;
}

size_t sg_ss_table_workspace_bytes(const sg_grid *grid, int n_fluids)
{
    if (check_ss_grid(grid) != SG_OK || !ss_fluids_ok(grid, n_fluids)) return 0;
    return sg_ss_ws_bytes(grid->n_r, grid->n_phi, n_fluids);
}

sg_status sg_ss_table(const sg_grid *grid, int n_fluids, const double *d_H, uint32_t flags, void *d_table,
                      void *d_ws, size_t ws_bytes, void *stream)
{
    sg_status s = check_ss_grid(grid);
    if (s != SG_OK) return s;
    if (n_fluids < 1 || n_fluids > 4 || !d_H) return SG_ERR_ARG;
    if (!ss_fluids_ok(grid, n_fluids)) return SG_ERR_UNSUPPORTED;
    if (!ss_flags_ok(flags)) return SG_ERR_ARG;
    if (!d_table || ((uintptr_t)d_table & 255)) return SG_ERR_ARG;
    if (!d_ws || ws_bytes < sg_ss_ws_bytes(grid->n_r, grid->n_phi, n_fluids) || ((uintptr_t)d_ws & 255))
        return SG_ERR_WORKSPACE;
    return sg_ss_table_build(grid, n_fluids, d_H, flags, d_table, d_ws, (hipStream_t)stream);
}

// Species summed into kernel groups: 0 (one density per fluid) or 1..8
// species, each in a group < n_fluids.
static bool species_ok(const sg_disc &d)
{
    if (d.n_species < 0 || d.n_species > 8) return false;
    for (int s = 0; s < d.n_species; ++s)
        if (d.species_group[s] >= d.fluids.n_fluids) return false;
    return true;
}

static sg_status check_disc(const sg_disc &d)
{
    if (!species_ok(d)) return SG_ERR_ARG;
    if (d.flags & SG_SEMI_SPECTRAL) {
        sg_status s = check_ss_grid(&d.grid);
        if (s != SG_OK) return s;
        if (d.fluids.n_fluids < 1 || d.fluids.n_fluids > 4) return SG_ERR_ARG;
        if (!ss_fluids_ok(&d.grid, d.fluids.n_fluids)) return SG_ERR_UNSUPPORTED;
        if (!ss_flags_ok(d.flags)) return SG_ERR_ARG;
        if (!d.sigma || !d.g_r || !d.g_phi || !d.table) return SG_ERR_ARG;
        if ((uintptr_t)d.table & 255) return SG_ERR_ARG;
        return SG_OK;
    }
    sg_status s = check_fft_grid(&d.grid);
    if (s != SG_OK) return s;
    if ((s = check_fluids(&d.fluids)) != SG_OK) return s;
    if (!fft_groups_ok(&d.grid, &d.fluids)) return SG_ERR_UNSUPPORTED;
    if (!flags_ok(d.flags)) return SG_ERR_ARG;
    if (!second_order_ok(d.flags)) return SG_ERR_UNSUPPORTED;
    if (!d.sigma || !d.g_r || !d.g_phi || !d.table) return SG_ERR_ARG;
    if ((uintptr_t)d.table & 255) return SG_ERR_ARG;
    return SG_OK;
}

size_t sg_field_fft_workspace_bytes(const sg_disc *discs, int n_discs)
{
    if (!discs || n_discs < 1 || n_discs > 4096) return 0;
    size_t total = 0;
    for (int i = 0; i < n_discs; ++i) {
        if (check_disc(discs[i]) != SG_OK) return 0;
        total += sg_fft_disc_ws_bytes(discs[i]);
    }
    return total;
}

sg_status sg_field_fft(const sg_disc *discs, int n_discs, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!discs || n_discs < 1 || n_discs > 4096) return SG_ERR_ARG;
    size_t need = 0;
    for (int i = 0; i < n_discs; ++i) {
        sg_status s = check_disc(discs[i]);
        if (s != SG_OK) return s;
        need += sg_fft_disc_ws_bytes(discs[i]);
    }
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255)) return SG_ERR_WORKSPACE;
    return sg_fft_run(discs, n_discs, d_ws, (hipStream_t)stream);
}

sg_status sg_field_fft_profile(const sg_disc *discs, int n_discs, void *d_ws, size_t ws_bytes,
                               void *stream, int reps, float *ms_per_pass)
{
    if (!discs || n_discs < 1 || n_discs > 4096 || reps < 1 || reps > 10000 || !ms_per_pass)
        return SG_ERR_ARG;
    size_t need = 0;
    for (int i = 0; i < n_discs; ++i) {
        sg_status s = check_disc(discs[i]);
        if (s != SG_OK) return s;
        need += sg_fft_disc_ws_bytes(discs[i]);
    }
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255)) return SG_ERR_WORKSPACE;
    return sg_fft_profile(discs, n_discs, d_ws, (hipStream_t)stream, reps, ms_per_pass);
}

sg_status sg_field_fft_tune(const sg_disc *discs, int n_discs, void *d_ws, size_t ws_bytes,
                            void *stream, sg_tune_result *results, int capacity, int *n_results)
{
    if (!discs || n_discs < 1 || n_discs > 4096 || capacity < 0 || (capacity > 0 && !results))
        return SG_ERR_ARG;
    size_t need = 0;
    for (int i = 0; i < n_discs; ++i) {
        sg_status s = check_disc(discs[i]);
        if (s != SG_OK) return s;
        need += sg_fft_disc_ws_bytes(discs[i]);
    }
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255)) return SG_ERR_WORKSPACE;
    return sg_fft_tune(discs, n_discs, d_ws, (hipStream_t)stream, results, capacity, n_results);
}

size_t sg_field_direct_workspace_bytes(const sg_grid *grid, int n_fluids, sg_dtype dtype,
                                       int per_cell_H)
{
    if (check_grid(grid) != SG_OK || n_fluids < 1 || n_fluids > 4) return 0;
    if (dtype != SG_F32 && dtype != SG_F64) return 0;
    if ((int64_t)grid->n_r * grid->n_phi > ((int64_t)1 << 26)) return 0;
    return sg_direct_ws_bytes(grid->n_r, grid->n_phi, n_fluids, dtype, per_cell_H ? 1 : 0);
}

size_t sg_potential_direct_workspace_bytes(const sg_grid *grid, int n_fluids, sg_dtype dtype,
                                           int per_cell_H)
{
    if (check_grid(grid) != SG_OK || n_fluids < 1 || n_fluids > 4) return 0;
    if (dtype != SG_F32 && dtype != SG_F64) return 0;
    return sg_potential_ws_bytes(grid->n_r, grid->n_phi, n_fluids, dtype, per_cell_H ? 1 : 0);
}

sg_status sg_potential_direct(const sg_grid *grid, int n_fluids, const double *h, const void *d_sigma,
                              const void *d_H, void *d_pot, sg_dtype dtype, uint32_t flags, void *d_ws,
                              size_t ws_bytes, void *stream)
{
    sg_status s = check_grid(grid);
    if (s != SG_OK) return s;
    if (n_fluids < 1 || n_fluids > 4) return SG_ERR_ARG;
    if (dtype != SG_F32 && dtype != SG_F64) return SG_ERR_ARG;
    if ((int64_t)grid->n_r * grid->n_phi > ((int64_t)1 << 26)) return SG_ERR_UNSUPPORTED;
    if (!d_sigma || !d_pot) return SG_ERR_ARG;
    if ((flags & ~(uint32_t)SG_SELF_CELL_EXCLUDE) != 0) return SG_ERR_ARG;
    if (!d_H) {
        if (!h) return SG_ERR_ARG;
        for (int f = 0; f < n_fluids; ++f)
            if (!finite_pos(h[f])) return SG_ERR_ARG;
    }
    const size_t need = sg_potential_ws_bytes(grid->n_r, grid->n_phi, n_fluids, dtype, d_H ? 1 : 0);
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255)) return SG_ERR_WORKSPACE;
    return sg_potential_launch(grid, n_fluids, d_H ? nullptr : h, d_sigma, d_H, d_pot, dtype, flags, d_ws,
                               (hipStream_t)stream);
}

sg_status sg_hsg(int64_t n, int n_fluids, const double *d_H, const double *d_Q, double *d_Hsg, void *stream)
{
    if (n < 0 || n_fluids < 1 || n_fluids > 4 || !d_H || !d_Q || !d_Hsg) return SG_ERR_ARG;
    if (n == 0) return SG_OK;
    return sg_hsg_launch(n, n_fluids, d_H, d_Q, d_Hsg, (hipStream_t)stream);
}

sg_status sg_eval_G0(const void *d_x, void *d_G, int64_t n, sg_dtype dtype, void *stream)
{
    if (!d_x || !d_G || n < 0 || (dtype != SG_F32 && dtype != SG_F64)) return SG_ERR_ARG;
    if (n == 0) return SG_OK;
    return sg_eval_G0_launch(d_x, d_G, n, dtype, (hipStream_t)stream);
}

}  // extern "C"

// Arguments of sg_field_direct other than the workspace; *need receives the
// workspace size the call takes.
static sg_status check_direct(const sg_grid *grid, int n_fluids, const double *h, const void *d_sigma,
                              const void *d_H, const void *d_g_r, const void *d_g_phi, sg_dtype dtype,
                              uint32_t flags, size_t *need)
{
    sg_status s = check_grid(grid);
    if (s != SG_OK) return s;
    if (n_fluids < 1 || n_fluids > 4) return SG_ERR_ARG;
    if (dtype != SG_F32 && dtype != SG_F64) return SG_ERR_ARG;
    if ((int64_t)grid->n_r * grid->n_phi > ((int64_t)1 << 26)) return SG_ERR_UNSUPPORTED;
    if (!d_sigma || !d_g_r || !d_g_phi) return SG_ERR_ARG;
    if ((flags & ~(uint32_t)(SG_SELF_CELL_EXCLUDE | SG_INDIRECT | SG_LINEAR_R)) != 0) return SG_ERR_ARG;
    if (!d_H) {
        if (!h) return SG_ERR_ARG;
        for (int f = 0; f < n_fluids; ++f)
            if (!finite_pos(h[f])) return SG_ERR_ARG;
    }
    *need = sg_direct_ws_bytes(grid->n_r, grid->n_phi, n_fluids, dtype, d_H ? 1 : 0);
    return SG_OK;
}

static const double k_ones[4] = {1.0, 1.0, 1.0, 1.0};  // h placeholder when d_H is given

// The no-allocation variant's workspace: one static device array per GPU,
// held from the library's load until the process ends.  In host code the
// name `scratch` is a host-side stand-in, not a device address: the device
// address is resolved once per device with hipGetSymbolAddress and only that
// pointer is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SG_NOALLOC_SCRATCH_BYTES];

#define SG_MAX_DEVICES 64
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SG_MAX_DEVICES];

// Device address of the current device's scratch array (resolved on the
// first call on that device, with that device current).
static sg_status scratch_of_current_device(void **out)
{
    int dev = -1;
    SG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= SG_MAX_DEVICES) return SG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SG_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SG_OK;
}

extern "C" {

sg_status sg_field_direct(const sg_grid *grid, int n_fluids, const double *h, const void *d_sigma,
                          const void *d_H, void *d_g_r, void *d_g_phi, sg_dtype dtype,
                          uint32_t flags, void *d_ws, size_t ws_bytes, void *stream)
{
    size_t need = 0;
    sg_status s = check_direct(grid, n_fluids, h, d_sigma, d_H, d_g_r, d_g_phi, dtype, flags, &need);
    if (s != SG_OK) return s;
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255)) return SG_ERR_WORKSPACE;
    return sg_direct_launch(grid, n_fluids, d_H ? k_ones : h, d_sigma, d_H, d_g_r, d_g_phi, dtype,
                            flags, d_ws, (hipStream_t)stream);
}

sg_status sg_field_direct_noalloc(const sg_grid *grid, int n_fluids, const double *h, const void *d_sigma,
                                  const void *d_H, void *d_g_r, void *d_g_phi, sg_dtype dtype,
                                  uint32_t flags, void *stream)
{
    size_t need = 0;
    sg_status s = check_direct(grid, n_fluids, h, d_sigma, d_H, d_g_r, d_g_phi, dtype, flags, &need);
    if (s != SG_OK) return s;
    if (need > SG_NOALLOC_SCRATCH_BYTES) return SG_ERR_SCRATCH;
    void *ws = nullptr;
    s = scratch_of_current_device(&ws);
    if (s != SG_OK) return s;
    // same kernels and workspace layout as sg_field_direct, on the static
    // array: nothing in the direct sum reads workspace it has not written in
    // the same call, so the previous call's contents need no clearing
    return sg_direct_launch(grid, n_fluids, d_H ? k_ones : h, d_sigma, d_H, d_g_r, d_g_phi, dtype,
                            flags, ws, (hipStream_t)stream);
}

// the FFT-path adjoint takes the forward's group counts (beyond two groups
// n_r <= 1024, as the forward)
static bool adjoint_groups_ok(const sg_disc &d)
{
    return (d.flags & SG_SEMI_SPECTRAL) || fft_groups_ok(&d.grid, &d.fluids);
}

size_t sg_field_adjoint_workspace_bytes(const sg_disc *disc)
{
    if (!disc || check_disc(*disc) != SG_OK || !adjoint_groups_ok(*disc)) return 0;
    return sg_adjoint_ws_bytes(*disc);
}

sg_status sg_field_adjoint(const sg_disc *disc, const float *d_lam_r, const float *d_lam_phi,
                           float *d_dsigma, double *d_dh, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!disc) return SG_ERR_ARG;
    sg_status s = check_disc(*disc);
    if (s != SG_OK) return s;
    if (!d_lam_r || !d_lam_phi || !d_dsigma) return SG_ERR_ARG;
    if (!adjoint_groups_ok(*disc)) return SG_ERR_UNSUPPORTED;
    if (disc->flags & SG_SEMI_SPECTRAL) {
        if (d_dh) return SG_ERR_UNSUPPORTED;  // dL/dSigma only
    } else {
        if (d_dh && !(disc->flags & SG_WITH_DH)) return SG_ERR_TABLE;
    }
    if (!d_ws || ws_bytes < sg_adjoint_ws_bytes(*disc) || ((uintptr_t)d_ws & 255))
        return SG_ERR_WORKSPACE;
    return sg_adjoint_run(*disc, d_lam_r, d_lam_phi, d_dsigma, d_dh, d_ws, (hipStream_t)stream);
}

static bool ss_grad_ok(const sg_disc *d)
{
    return d && check_disc(*d) == SG_OK && (d->flags & SG_SEMI_SPECTRAL);
}

// species discs also hold their group densities
static size_t ss_grad_bytes(const sg_disc &d)
{
    const int nr = d.grid.n_r, nphi = d.grid.n_phi, nf = d.fluids.n_fluids;
    size_t b = sg_ss_grad_ws_bytes(nr, nphi, nf);
    if (d.n_species) b += sg_align256(sizeof(float) * nf * (size_t)nr * nphi);
    return b;
}

size_t sg_ss_grad_H_workspace_bytes(const sg_disc *disc)
{
    if (!ss_grad_ok(disc)) return 0;
    return ss_grad_bytes(*disc);
}

sg_status sg_ss_grad_H(const sg_disc *disc, const double *d_H, const float *d_lam_r, const float *d_lam_phi,
                       double *d_dH, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!disc) return SG_ERR_ARG;
    sg_status s = check_disc(*disc);
    if (s != SG_OK) return s;
    if (!d_H || !d_lam_r || !d_lam_phi || !d_dH) return SG_ERR_ARG;
    if (!ss_grad_ok(disc)) return SG_ERR_UNSUPPORTED;
    const size_t need = ss_grad_bytes(*disc);
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws & 255)) return SG_ERR_WORKSPACE;
    return sg_ss_grad_run(*disc, d_H, d_lam_r, d_lam_phi, d_dH, d_ws, (hipStream_t)stream);
}

sg_status sg_eval_F(const void *d_x, void *d_F, void *d_dF, int64_t n, sg_dtype dtype, void *stream)
{
    if (!d_x || !d_F || n < 0 || (dtype != SG_F32 && dtype != SG_F64)) return SG_ERR_ARG;
    if (n == 0) return SG_OK;
    return sg_eval_F_launch(d_x, d_F, d_dF, n, dtype, (hipStream_t)stream);
}

sg_status sg_self_cell(const sg_grid *grid, const double *ha, const double *hb, int n, int which,
                       double *d_out, void *stream)
{
    sg_status s = check_grid(grid);
    if (s != SG_OK) return s;
    if (!ha || !hb || !d_out || n < 1 || n > SG_SELF_MAX || which < 0 || which > 2) return SG_ERR_ARG;
    for (int i = 0; i < n; ++i)
        if (!finite_pos(ha[i]) || !finite_pos(hb[i])) return SG_ERR_ARG;
    return sg_self_cell_launch(grid, ha, hb, n, which, d_out, (hipStream_t)stream);
}

void sg_release(void) { sg_fft_release(); }

int sg_field_fft_cache_entries(void) { return sg_fft_cache_entries(); }

const char *sg_status_string(sg_status s)
{
    switch (s) {
    case SG_OK: return "SG_OK";
    case SG_ERR_ARG: return "SG_ERR_ARG: invalid argument";
    case SG_ERR_UNSUPPORTED: return "SG_ERR_UNSUPPORTED: not supported by this path";
    case SG_ERR_HIP: return "SG_ERR_HIP: HIP runtime error";
    case SG_ERR_WORKSPACE: return "SG_ERR_WORKSPACE: workspace missing or too small";
    case SG_ERR_TABLE: return "SG_ERR_TABLE: kernel table does not match";
    case SG_ERR_SCRATCH:
        return "SG_ERR_SCRATCH: the call needs more workspace than the no-allocation entry point's "
               "static scratch (SG_NOALLOC_SCRATCH_BYTES per GPU)";
    }
    return "unknown sg_status";
}

int sg_version(void) { return 1; }

}  // extern "C"
