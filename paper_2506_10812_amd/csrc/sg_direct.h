// sg_direct.h -- internal entry points of the direct-sum path.
#pragma once
#include "sg_internal.h"

size_t sg_direct_ws_bytes(int nr, int nphi, int nf, sg_dtype dt, int percell);
sg_status sg_direct_launch(const sg_grid *g, int nf, const double *h, const void *sigma,
                           const void *H, void *gr, void *gp, sg_dtype dt, uint32_t flags,
                           void *ws, hipStream_t s);
size_t sg_potential_ws_bytes(int nr, int nphi, int nf, sg_dtype dt, int percell);
sg_status sg_potential_launch(const sg_grid *g, int nf, const double *h, const void *sigma,
                              const void *H, void *pot, sg_dtype dt, uint32_t flags, void *ws,
                              hipStream_t s);
sg_status sg_hsg_launch(int64_t n, int nf, const double *H, const double *Q, double *Hsg, hipStream_t s);
