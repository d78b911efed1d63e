// sg_table.h -- internal declarations shared by the library's translation units.
#pragma once
#include "sg_internal.h"

#define SG_GL_N 48          // Gauss-Legendre order across the self cell (eta)
#define SG_GLX_N 16         // Gauss-Legendre order per radial panel (xi)
#define SG_PANELS 7         // geometric xi panels [0,4^-6], [4^-(j+1), 4^-j]
#define SG_SELF_MAX 64      // items per self-cell launch

struct GLNodes {
    double x[SG_GL_N], w[SG_GL_N];
    double xr[SG_GLX_N], wr[SG_GLX_N];
};

struct SelfItems {
    double ha[SG_SELF_MAX], hb[SG_SELF_MAX];
    int which[SG_SELF_MAX];
};

void sg_gl_nodes(GLNodes &gl);
size_t sg_table_ws_bytes(int nr, int nphi);
sg_status sg_table_build(const sg_grid *grid, const sg_fluids *fl, uint32_t flags, void *d_table,
                         void *d_ws, hipStream_t s);
sg_status sg_self_cell_launch(const sg_grid *grid, const double *ha, const double *hb, int n,
                              int which, double *d_out, hipStream_t s);
sg_status sg_eval_F_launch(const void *x, void *F, void *dF, int64_t n, sg_dtype dt, hipStream_t s);
sg_status sg_eval_G0_launch(const void *x, void *G, int64_t n, sg_dtype dt, hipStream_t s);

__global__ void k_twiddles(float2 *tw_u, int nu, float2 *tw_phi, int nphi);
__global__ void k_self_cell(SelfItems items, double *out, double du, double dphi, GLNodes gl);
// Own-cell integrals on a uniform radial grid (defined with the semi-spectral
// path): item = pair * n_r * per + cell, H double [F][n_r * per].
__global__ void k_ss_self_lin(const double *H, int nf, int nr, int per, double rmin, double dr, double dphi,
                              int pot, int which, double *out, GLNodes gl);
__global__ void k_self_cell_ring(const double *H, int nf, int nr, double lnrmin, double du, double dphi, int which,
                                 double *out, GLNodes gl);
template <typename T>
__global__ void k_self_cell_percell(const T *H, int nf, int nr, int nphi, double lnrmin, double du,
                                    double dphi, double *out, GLNodes gl);
template <typename T>
__global__ void k_pot_self(const T *H, const double *h, int nf, int nr, int nphi, double lnrmin,
                           double du, double dphi, int per_row, double *out, GLNodes gl, int which);
__global__ void k_fill_f64(double *p, int64_t n, double v);
