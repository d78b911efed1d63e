// sg_adjoint.h -- internal entry points of the adjoint.
#pragma once
#include "sg_internal.h"

size_t sg_adjoint_ws_bytes(const sg_disc &d);
// Group densities of a species disc ([n_fluids][n_r][n_phi] float), summed
// in the forward's order (species order, from zero).
sg_status sg_species_group_sums(const sg_disc &d, float *gsig, hipStream_t s);
sg_status sg_adjoint_run(const sg_disc &d, const float *lam_r, const float *lam_p, float *dsig,
                         double *dh, void *ws, hipStream_t s);
