// sg_semispec.h -- internal entry points of the semi-spectral path.
#pragma once
#include "sg_passes.h"

// Middle pass of a semi-spectral disc (replaces pass 2 of the FFT path):
// fn has the pass-kernel signature; a workgroup of wgs threads takes one job
// (column m, target fluid b, block of tb target rows) and needs
// lds_per_row * c + lds_fixed bytes of dynamic LDS, c the longest staged
// column of a mode (n_r, or n_r + 2 w + 4 for a banded mode).
struct SsPassInfo {
    void (*fn)(const DiscDev *, const WJob *, int, const float2 *, int);
    int wgs, tb, lds_per_row, lds_fixed;
};

// variant 1, 2, 3: (targets per lane, row splits) = (2, 4), (2, 1), (4, 1),
// 1 with non-temporal operator loads; variant 4: as 1 with ordinary loads
bool sg_ss_pass_kernel(int nf, int variant, SsPassInfo &out);
int sg_ss_default_variant(int nr);
int sg_ss_max_nr();

size_t sg_ss_ws_bytes(int nr, int nphi, int nf);
size_t sg_ss_grad_ws_bytes(int nr, int nphi, int nf);
sg_status sg_ss_grad_run(const sg_disc &d, const double *d_H, const float *lam_r, const float *lam_p, double *dH,
                         void *d_ws, hipStream_t s);
sg_status sg_ss_table_build(const sg_grid *grid, int nf, const double *d_H, uint32_t flags, void *d_table,
                            void *d_ws, hipStream_t s);
