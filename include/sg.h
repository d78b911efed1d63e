/*
 * sg.h -- C ABI of the MI355X (gfx950) library for the exact thin-disc
 * self-gravity kernel of arXiv 2506.10812 (Rendon Restrepo, Rometsch,
 * Ziegler & Gressel, "Self-gravity in thin protoplanetary discs 1").
 *
 * The library sums the exact Bessel kernel
 *     K_ab(s) = pi^{-1/2} H_ab^{-2} (d/8) e^x [K1(x) - K0(x)],  x = d^2/8,
 *     d = s/H_ab,  H_ab^2 = (H_a^2 + H_b^2)/2          (Sect. 2.2, kernel and
 *                                                      r.m.s. scale height)
 * against surface density on a log-r x uniform-phi grid and returns the
 * in-plane gravitational acceleration of each fluid,
 *     g_b(x_i) = - sum_a sum_{k != i} Sigma_a[k] A_k K_ab(s_ik) e_s + self term
 * (Sect. 2.2, the 2D force divided by Sigma_b), projected on e_r and e_phi.
 *
 * Conventions shared by every call
 *   units      G = 1; outputs are accelerations g (not force densities); the
 *              field is attractive (points towards mass).
 *   grid       radial cell edges are log-spaced from r_min to r_max; cell
 *              centres u_i = ln r_min + (i + 1/2) du, du = ln(r_max/r_min)/n_r;
 *              phi_j = (j + 1/2) dphi, dphi = 2 pi / n_phi; cell area
 *              A_i = r_i^2 du dphi.
 *   layout     every device array is row-major [fluid][i_r][j_phi] with phi
 *              fastest; fluid 0 is gas, fluid 1 dust.  n_fluids is 1 to 4
 *              scale-height groups (the multi-fluid case of Sect. 5.2: all
 *              F^2 ordered pairs) on every path (adjoints included); on the
 *              FFT path beyond two groups n_r <= 1024.
 *   pairs      (a -> b) is source fluid a acting on target fluid b; a
 *              two-fluid disc has the four ordered pairs gg, dg, gd, dd
 *              (Sect. 2.2 lists the four combinations).
 *   self term  the own-cell contribution is the principal-value average of
 *              the log-polar radial kernel over the cell (the paper does not
 *              treat k = i); SG_SELF_CELL_EXCLUDE drops it.
 *   ownership  every device buffer is allocated and owned by the caller; the
 *              library reads and writes only the buffers passed in.  The only
 *              device memory the library owns is a per-signature cache of
 *              batch plans: descriptors and, for batches with several launch
 *              classes per pass, instantiated HIP graphs (sg_field_fft;
 *              sg_release() frees it) and the static scratch array of
 *              sg_field_direct_noalloc.
 *   streams    `stream` is a hipStream_t passed as void* (NULL = default
 *              stream).  Every call is asynchronous on that stream unless
 *              stated otherwise; buffers must stay valid until it completes.
 *   errors     calls return an sg_status; arguments are validated before any
 *              work is enqueued, so a non-SG_OK return (other than
 *              SG_ERR_HIP) has launched nothing.  No exception crosses the ABI.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sg_status {
    SG_OK = 0,
    SG_ERR_ARG = 1,         /* invalid argument (NULL pointer, size, range) */
    SG_ERR_UNSUPPORTED = 2, /* valid but not supported by this path        */
    SG_ERR_HIP = 3,         /* a HIP runtime call failed                    */
    SG_ERR_WORKSPACE = 4,   /* workspace pointer NULL or too small          */
    SG_ERR_TABLE = 5,       /* kernel table does not match the disc         */
    SG_ERR_SCRATCH = 6      /* larger than the no-allocation scratch array  */
} sg_status;

typedef enum sg_dtype { SG_F32 = 0, SG_F64 = 1 } sg_dtype;

enum {
    SG_SELF_CELL_EXCLUDE = 1u, /* drop the own-cell term                      */
    SG_WITH_DH = 2u,           /* table also holds d/dh spectra (adjoint)     */
    SG_INDIRECT = 4u,          /* add the indirect term (see below)           */
    SG_SEMI_SPECTRAL = 8u,     /* disc uses a semi-spectral table (below)     */
    SG_SS_FULL = 16u,          /* semi-spectral: keep every operator entry    */
    SG_POTENTIAL = 32u,        /* semi-spectral: operators of the potential   */
    SG_LINEAR_R = 64u,         /* uniform radial grid (semi-spectral, direct) */
    SG_SECOND_ORDER = 128u     /* kernel table: hat-weighted sources (below)  */
};

/* SG_SECOND_ORDER (sg_kernel_table, FFT path; an option beyond the paper,
 * whose convolution of Sect. 5.2 samples the App. C kernels at cell-centre
 * offsets): the sources are taken as the piecewise-bilinear interpolant of
 * the cell values on the (u, phi) grid (tensor-product hat functions on the
 * cell centres, periodic in phi; the first and last rings' hats reach half a
 * cell past the grid's edges), integrated exactly against the App. C
 * kernels.  The table then holds
 *   W_c(P, Q) = int int (1 - |s|)(1 - |t|) K_c((P + s) du, (Q + t) dphi) ds dt,
 * s, t in [-1, 1], in place of the point samples and the own-cell average:
 * the discrete field converges at second order in du, dphi to the field of
 * a smooth density, where the cell-centre sums converge at first order (the
 * ring kernel's 1/X and log|X| singularities).  The solve, its plan and its
 * cost are unchanged; the table build integrates each entry (Gauss-Legendre,
 * polar rules at the singular point), and with SG_WITH_DH the d/dh spectra
 * integrate the kernel's h derivatives the same way, so sg_field_adjoint's
 * dL/dh is that of the second-order field.  Not with SG_SELF_CELL_EXCLUDE
 * (SG_ERR_UNSUPPORTED: the own cell is an entry like any other); SG_INDIRECT
 * keeps its point-mass form.
 * sg_ss_table takes the flag too (log radial grid, force operators): each
 * ring pair's operator uses these weights with the pair's aspect ratios
 * h_a = H_a(r')/r', h_b = H_b(r)/r held across the hats, integrated within
 * 32 cells of the singular point and taken as K + (second differences)/12
 * beyond (remainder below 3e-6 of the entry).  Not with SG_POTENTIAL,
 * SG_LINEAR_R or SG_SELF_CELL_EXCLUDE; sg_field_adjoint gives their
 * dL/dSigma and sg_ss_grad_H their dL/dH (the h derivatives of the same
 * weights). */

/* SG_INDIRECT (Sect. 5.4 and the appendix "Indirect term"): every target
 * fluid also receives the acceleration -sum_a grad Phi_{a,ind} of the frame
 * centred on the star,
 *   g_r  += -(A cos phi + B sin phi),   g_phi += -(-A sin phi + B cos phi),
 *   A + i B = sum_a sqrt(2) sum_k Sigma_a[k] A_k K_a(d_k) e^{i phi_k},
 *   K_a(d) = pi^{-1/2} H_a^{-2} (d/4) e^{d^2/4} [K1 - K0](d^2/4),
 *   d_k = r_k / H_a at the source cell,
 * with the cell measure A_k = r_k^2 du dphi.  Accepted by sg_kernel_table
 * (no effect on the table), sg_field_fft, sg_field_direct and
 * sg_field_adjoint (which adds its transpose to dL/dSigma and its h
 * derivative to dL/dh). */

typedef struct sg_grid {
    int32_t n_r;    /* radial cells                                   */
    int32_t n_phi;  /* azimuthal cells                                */
    double r_min;   /* inner edge of the first radial cell (> 0)      */
    double r_max;   /* outer edge of the last radial cell (> r_min)   */
} sg_grid;

typedef struct sg_fluids {
    int32_t n_fluids; /* 1 to 4 scale-height groups (1: gas, 2: gas + dust) */
    int32_t pad_;
    double h[4];      /* aspect ratios h_f = H_f / r (constant per fluid)  */
} sg_fluids;

/* ---------------------------------------------------------------------
 * Kernel table (log-polar FFT path, H_f = h_f r).
 *
 * App. C writes the radial and azimuthal fields as convolutions in
 * (u = ln r, phi) with kernels K_r(X, phi), K_phi(X, phi) that depend only
 * on the offsets when every H_f is proportional to r; Sect. 5.2 notes the
 * kernel then needs computing only once.  sg_kernel_table samples both
 * kernels for every ordered pair on the wrapped 2 n_r x n_phi offset grid
 * (radial zero padding to 2 n_r, Sect. 5.2), puts the self term at offset
 * (0,0), transforms in double precision and stores the half spectrum
 * (k_u in [0, n_r], m in [0, n_phi/2]) rounded to float, pre-scaled by
 * -du dphi / (2 n_r n_phi).  With SG_WITH_DH it also stores the spectra of
 * dK/dh_a and dK/dh_b for sg_field_adjoint.
 *
 * Requirements: n_r and n_phi powers of two with 2 <= n_r <= 2048 and
 * 4 <= n_phi <= 2048 (SG_ERR_UNSUPPORTED otherwise); h_f > 0; 1 to 4
 * fluids (n_r <= 1024 for three or four, SG_ERR_UNSUPPORTED otherwise).
 * d_table: device buffer of sg_kernel_table_bytes() bytes, 256-byte aligned,
 * written completely.  d_ws: device scratch of sg_kernel_table_workspace_bytes()
 * bytes, contents undefined afterwards.  Asynchronous on `stream`.
 * The table is position independent: it may be copied, saved and reloaded.
 * --------------------------------------------------------------------- */
size_t sg_kernel_table_bytes(const sg_grid *grid, const sg_fluids *fluids, uint32_t flags);
size_t sg_kernel_table_workspace_bytes(const sg_grid *grid, const sg_fluids *fluids,
                                       uint32_t flags);
sg_status sg_kernel_table(const sg_grid *grid, const sg_fluids *fluids, uint32_t flags,
                          void *d_table, void *d_ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * Semi-spectral table (any scale height profile H_f(r)).
 *
 * Sect. 5.2 pairs an FFT in azimuth with a direct sum in radius, at cost
 * N_r N_phi log N_phi + N_phi N_r^2, to drop the H/r = const condition of
 * the full FFT method (App. D shows what that condition costs).  Between
 * source ring i' and target ring i the kernel depends on the azimuths only
 * through their difference, so each azimuthal mode m decouples into an
 * n_r x n_r radial operator per ordered fluid pair.  sg_ss_table samples
 * the App. C convolution-form kernels with h_a = H_a(r_i')/r_i' at the
 * source ring and h_b = H_b(r_i)/r_i at the target ring (so that
 * H_ab^2 = (H_a(r_i')^2 + H_b(r_i)^2)/2, the definition of Sect. 2.2),
 * puts the own-cell average (h = H/r of the ring) at zero offset, transforms
 * every ring pair in azimuth in double precision and stores the operators
 * rounded to float.  Refreshing H every few steps (Sect. 5.2) means calling
 * it again into the same table.
 *
 * Banded modes: the kernels are analytic in phi for |Im phi| < |X|
 * (X = u_i - u_i'), so the mode-m coupling of two rings decays like
 * e^{-m |X|}.  Mode m keeps only the ring pairs with |i - i'| <= w_m,
 * w_m = ceil(30 ln 2 / (m du)) (the dropped couplings are below about 2^-30
 * of the axisymmetric coupling of the same pair), and is stored as 2 w_m + 1
 * diagonals when 4 w_m + 2 <= n_r; m = 0 and wider modes are stored whole.
 * On fine radial grids this shrinks the table and the solve's traffic from
 * N_phi N_r^2 towards N_phi N_r log N_phi.  SG_SS_FULL stores every mode
 * whole (the exact operators).
 *
 * d_H: device double [n_fluids][n_r], H_f at the ring centres r_i
 * (r_i = r_min e^{(i + 1/2) du}), every value > 0 (not checked on the
 * device).  flags: SG_SELF_CELL_EXCLUDE, SG_INDIRECT (the indirect term,
 * with K_a at d = r_i'/H_a(r_i'), folded into mode 1 of the table; no cost
 * at solve time), SG_SS_FULL, SG_POTENTIAL, SG_LINEAR_R (below).  Grid:
 * n_phi a power of two in [4, 2048], n_r in [1, 2048], any n_r.  n_fluids:
 * 1 to 4 scale-height groups (the multi-fluid case of Sect. 5.2; n_r <= 1024
 * beyond two), d_H then [n_fluids][n_r], the operators covering all
 * n_fluids^2 ordered pairs; a disc's fluids.n_fluids is that count (its h
 * is not read).  Size: sg_ss_table_bytes() (at most
 * 8 (n_phi/2 + 1) F^2 n_r n_rt bytes, n_rt = n_r rounded up to even, plus a
 * few KB); d_table 256-byte aligned, written completely.
 * d_ws: sg_ss_table_workspace_bytes() bytes (<= about 130 MB), contents
 * undefined afterwards.  Asynchronous on `stream`.  The table is position
 * independent.
 *
 * SG_LINEAR_R: the radial grid is uniform instead of log-spaced (the
 * semi-spectral method allows linear radial grids, Sect. 5.2; NIRVANA's
 * tests use one, Sect. 4.1): edges r_min + k dr, dr = (r_max - r_min)/n_r,
 * centres r_i = r_min + (i + 1/2) dr, cell areas A_i = r_i dr dphi (the
 * exact sector areas); d_H holds H_f at these centres; the own-cell terms
 * integrate the cell's own X = ln(r'/r_i) range, [ln(1 - dr/(2 r_i)),
 * ln(1 + dr/(2 r_i))]; the band rule uses the smallest log spacing of
 * adjacent centres (at the outer edge).  The solve itself does not depend
 * on the radii.  Discs built from such a table carry SG_LINEAR_R too.
 *
 * SG_POTENTIAL: the table holds the operators of the potential of Sect. 5.5
 * and the appendix "Conservative force" instead of the field's,
 *   Phi_b(x_i) = sum_a sum_k Sigma_a[k] A_k P_ab(s_ik),
 *   P_ab(s) = -e^y K0(y) / (2 sqrt(pi) H_ab),  y = s^2 / (8 H_ab^2),
 * with the own-cell integral of P_ab (cell's ring H) unless excluded; a disc
 * with this table receives Phi in g_r (g_phi holds only the rounding of the
 * inverse transform, about 1e-7 of |Phi|).  With constant H
 * (the case the paper derives) -grad Phi is the field; not combinable with
 * SG_INDIRECT.
 *
 * SG_SECOND_ORDER: the operators of the hat-weighted (second-order) field,
 * see SG_SECOND_ORDER above; log radial grid and field operators only.
 *
 * Solve with sg_field_fft: a disc whose flags hold SG_SEMI_SPECTRAL (plus
 * the flags the table was built with) and whose table is an sg_ss_table
 * runs the phi transforms of the FFT path and, in place of the u-transform
 * pass, one pass over the radial operators; fluids.h is not used.  Such
 * discs mix freely with FFT-path discs in one batch.  sg_field_adjoint
 * gives their dL/dSigma (not dL/dH).
 * --------------------------------------------------------------------- */
size_t sg_ss_table_bytes(const sg_grid *grid, int n_fluids, uint32_t flags);
size_t sg_ss_table_workspace_bytes(const sg_grid *grid, int n_fluids);
sg_status sg_ss_table(const sg_grid *grid, int n_fluids, const double *d_H, uint32_t flags,
                      void *d_table, void *d_ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * One disc for the FFT path.  sigma, g_r, g_phi: float device arrays
 * [n_fluids][n_r][n_phi]; table: built by sg_kernel_table for the same grid,
 * fluids and flags (checked on the host from the arguments, not the device),
 * or, with SG_SEMI_SPECTRAL in flags, by sg_ss_table for the same grid and
 * fluid count.
 *
 * Species sharing kernels (Sect. 5.2, multi-fluid case): the kernels depend
 * on the scale heights only, so species with a common scale height share
 * one kernel group; the paper's example is gas plus two dust species of
 * equal H_d (four kernels, six convolutions).  With n_species = S in
 * [1, 8], sigma holds S species [S][n_r][n_phi] and species s belongs to
 * group species_group[s] < n_fluids (the fluids of sg_fluids are then the
 * kernel groups); each group's source density is the sum of its species
 * (formed while the densities are read), and g_r, g_phi [n_fluids][...]
 * are per group: every species of a group receives that group's
 * acceleration.  n_species = 0: one density per fluid, species_group
 * unused.  sg_field_adjoint of a species disc returns one dL/dSigma per
 * species (that of its group).
 * --------------------------------------------------------------------- */
typedef struct sg_disc {
    sg_grid grid;
    sg_fluids fluids;
    uint32_t flags;      /* flags the table was built with                 */
    int32_t n_species;   /* 0, or species summed into kernel groups (above) */
    const float *sigma;  /* device, [F][n_r][n_phi] (or [S][n_r][n_phi])   */
    float *g_r;          /* device, [F][n_r][n_phi], overwritten           */
    float *g_phi;        /* device, [F][n_r][n_phi], overwritten           */
    const void *table;   /* device, from sg_kernel_table or sg_ss_table    */
    uint8_t species_group[8]; /* kernel group of each species              */
} sg_disc;

/* ---------------------------------------------------------------------
 * sg_field_fft: g_r, g_phi of every disc in `discs` by the zero-padded
 * log-polar FFT convolution (App. C convolution form, Sect. 5.2 zero
 * padding).  Float arithmetic, float accumulation.  All discs of the batch
 * (any mix of supported sizes, one to four fluids, all ordered pairs fused
 * per spectral point) run as three passes: phi transform of Sigma, fused
 * u-transform / spectral multiply / inverse u-transform, inverse phi
 * transform.  A batch whose discs fall into several launch classes of one
 * pass (transform lengths, fluid counts) runs as one HIP-graph launch whose
 * branches run those classes side by side; a batch with one class per pass
 * enqueues its three kernels directly (a graph launch would only add
 * latency).  The plan, the graph where used and a device copy of the batch
 * descriptors are cached per (sizes, pointers) signature on the first call
 * (that call allocates and synchronises once); later calls with the same
 * signature only launch.  At most 256 signatures are kept; a new one
 * beyond that releases the least recently used (after a device
 * synchronisation).  d_ws: sg_field_fft_workspace_bytes(discs, n)
 * bytes, 256-byte aligned; its address is part of the signature.
 * n_discs in [1, 4096].  Outputs overwritten.
 * --------------------------------------------------------------------- */
size_t sg_field_fft_workspace_bytes(const sg_disc *discs, int n_discs);
sg_status sg_field_fft(const sg_disc *discs, int n_discs, void *d_ws, size_t ws_bytes,
                       void *stream);

/* Per-pass timing of the sg_field_fft launches (no graph): one complete run,
 * then pass 1's launches `reps` times back to back, then pass 2's, then
 * pass 3's, with HIP events between the groups on `stream`; waits for
 * completion (synchronous) and writes the mean milliseconds per launch of
 * pass 1 (phi transform), pass 2 (u transform + spectral multiply + inverse
 * u transform) and pass 3 (inverse phi transform) to ms_per_pass[3].  With
 * reps == 1 the preliminary complete run is left out and every launch of
 * one step runs once, in order, with events attached to the launch itself
 * (the kernel's own start and end): ms_per_pass then holds each pass's
 * summed kernel time, and a caller that evicts the caches first times one
 * cold step pass by pass.  The outputs hold a complete result afterwards.
 * For measurement; reps in [1, 10000]. */
sg_status sg_field_fft_profile(const sg_disc *discs, int n_discs, void *d_ws, size_t ws_bytes,
                               void *stream, int reps, float *ms_per_pass);

/* ---------------------------------------------------------------------
 * sg_field_fft_tune: autotuner of the batched FFT path.  For every launch
 * class of the batch (one pass over the discs that share a transform length
 * and a fluid count) it runs the default launch as the reference, then every
 * candidate: radix order of the transforms (small radix last or first, where
 * the length is not a power of 8), tile shape (the default number of
 * transforms per workgroup or twice it, up to 1024 threads) and XCD cluster
 * size (1, 2, 4 or 8 consecutive workgroups on one XCD); for the middle pass
 * of semi-spectral discs (a class of its own per n_r and fluid count,
 * length = n_r) the shape is one of four (1: four row splits, 2 targets per
 * lane, non-temporal operator loads, the default; 2, 3: whole operator rows
 * with 2 or 4 targets per lane; 4: as 1 with ordinary loads) times the
 * cluster size.
 * A candidate is timed
 * only if its output matches the reference (relative RMS <= 1e-5 over the
 * class's output buffers); the fastest wins.  Choices are cached per class
 * shape for the life of the process (and in the text file named by the
 * environment variable SG_TUNE_CACHE, if set, read on the first tuning call
 * and rewritten after each); later sg_field_fft calls of any batch with the
 * same class shapes use them.  Synchronous; allocates temporary device
 * memory; releases the cached plans.  On return the outputs hold a complete
 * sg_field_fft result.  results (may be NULL) receives up to `capacity`
 * entries, one per class in pass order; *n_results (may be NULL) the number
 * of classes.  Arguments as for sg_field_fft.
 * --------------------------------------------------------------------- */
typedef struct sg_tune_result {
    int32_t pass;              /* 1, 2, 3 */
    int32_t length;            /* transform length of the class */
    int32_t n_fluids;
    int32_t n_jobs;            /* workgroup jobs of the chosen launch */
    int32_t small_radix_first; /* chosen radix order */
    int32_t groups_per_wg;     /* chosen transforms per workgroup (middle
                                  pass of semi-spectral discs: the shape) */
    int32_t cluster;           /* chosen XCD cluster size */
    int32_t candidates;        /* candidates tried besides the reference */
    int32_t rejected;          /* candidates that failed the output check */
    float rel_best;            /* relative RMS of the choice against the reference */
    float ms_default;          /* mean launch time of the reference */
    float ms_best;             /* mean launch time of the choice */
} sg_tune_result;

sg_status sg_field_fft_tune(const sg_disc *discs, int n_discs, void *d_ws, size_t ws_bytes,
                            void *stream, sg_tune_result *results, int capacity, int *n_results);

/* ---------------------------------------------------------------------
 * sg_field_direct: the O(N^2) pairwise sum of the definition (Sect. 2.2,
 * 2D force through the kernel) for any grid size and general per-cell
 * scale heights.  d_H: device array [F][n_r][n_phi] of H (same dtype as
 * sigma), or NULL for H_f = h[f] r.  With per-cell H the self term of cell i
 * uses h_a = H_a[i]/r_i and h_b = H_b[i]/r_i.  dtype SG_F64: double inputs,
 * outputs and arithmetic; SG_F32: float inputs, outputs, arithmetic and
 * accumulation (the self term and the indirect term are computed in double
 * and rounded).  flags: SG_SELF_CELL_EXCLUDE, SG_INDIRECT (with the source
 * cell's own H in K_a), SG_LINEAR_R (uniform radial grid: centres
 * r_min + (i + 1/2) dr, sector areas r dr dphi, one-sided own-cell
 * integrals, as on the semi-spectral path).  n_r, n_phi >= 1, n_r * n_phi <= 2^26.  F (the
 * fluid count) 1 to 4.  h: host array [F], read when d_H == NULL.  d_ws:
 * sg_field_direct_workspace_bytes() bytes.
 * --------------------------------------------------------------------- */
size_t sg_field_direct_workspace_bytes(const sg_grid *grid, int n_fluids, sg_dtype dtype,
                                       int per_cell_H);
sg_status sg_field_direct(const sg_grid *grid, int n_fluids, const double *h,
                          const void *d_sigma, const void *d_H, void *d_g_r, void *d_g_phi,
                          sg_dtype dtype, uint32_t flags, void *d_ws, size_t ws_bytes,
                          void *stream);

/* ---------------------------------------------------------------------
 * sg_field_direct_noalloc: sg_field_direct without a workspace argument,
 * for callers that cannot allocate device memory (code under HIP stream
 * capture, serving loops, harnesses that forbid hipMalloc).  It calls no
 * allocating routine: its workspace is a static device array of
 * SG_NOALLOC_SCRATCH_BYTES (64 MiB) in the library, one per GPU, held from
 * the library's load until the process ends.  The first call on a device
 * resolves that array's address (hipGetSymbolAddress, not a stream
 * operation); make one call before capturing a stream.  Every call on a GPU
 * uses that GPU's one array, so calls that overlap on the same GPU (other
 * streams, other host threads) race: the caller serialises them.  Inputs,
 * outputs, flags and results as for sg_field_direct (same kernels, same
 * arithmetic, bitwise equal outputs).  SG_ERR_SCRATCH (nothing launched)
 * when sg_field_direct_workspace_bytes() for the arguments exceeds
 * SG_NOALLOC_SCRATCH_BYTES: float, h r scale heights, up to about 2.8e6
 * cells for one fluid (24 bytes per cell) and 1.4e6 for two (48 bytes).
 * --------------------------------------------------------------------- */
#define SG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
sg_status sg_field_direct_noalloc(const sg_grid *grid, int n_fluids, const double *h,
                                  const void *d_sigma, const void *d_H, void *d_g_r, void *d_g_phi,
                                  sg_dtype dtype, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------
 * sg_potential_direct: the conservative 2D potential of Sect. 5.5 (appendix
 * "Conservative force"), summed directly:
 *   Phi_b(x_i) = sum_a sum_{k != i} Sigma_a[k] A_k P_ab(|x_i - x_k|)
 *              + sum_a Sigma_a[i] int_{own cell} P_ab dA,
 *   P_ab(s)    = -e^y K0(y) / (2 sqrt(pi) H_ab),  y = s^2 / (8 H_ab^2),
 * with H_ab^2 = (H_a^2 + H_b^2)/2 from the source cell's H_a and the
 * target cell's H_b (the own-cell integral, a reading, uses the cell's
 * H_a and H_b).  The paper derives Phi for spatially constant H, where
 * -grad Phi_ab is the field of sg_field_direct; pass d_H filled with
 * constants for that case (d_H == NULL uses H_f = h[f] r).  d_pot: device
 * array [F][n_r][n_phi] of sigma's dtype.  Float: float arithmetic and
 * accumulation, self integrals in double.  flags: SG_SELF_CELL_EXCLUDE.
 * Sizes and workspace as for sg_field_direct.
 * --------------------------------------------------------------------- */
size_t sg_potential_direct_workspace_bytes(const sg_grid *grid, int n_fluids, sg_dtype dtype,
                                           int per_cell_H);
sg_status sg_potential_direct(const sg_grid *grid, int n_fluids, const double *h,
                              const void *d_sigma, const void *d_H, void *d_pot, sg_dtype dtype,
                              uint32_t flags, void *d_ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------
 * sg_hsg: self-gravitating scale heights (Sect. 2.1, stratification
 * parameters) for the H input of sg_field_direct / sg_potential_direct:
 *   H_f^sg = sqrt(2/pi) H_f f(Qt),  Qt = (sum_f 1/Q_f)^-1,
 *   f(x) = pi/(4x) [sqrt(1 + 8 x^2/pi) - 1],
 * H_f the thermal (gas) or diffusive (dust) scale height, Q_f the Toomre
 * parameter c_f Omega_K / (pi G Sigma_f) of each fluid.  Device double
 * arrays [n_fluids][n] (n cells), n_fluids 1 to 4; Q_f > 0.  Double
 * arithmetic.
 * --------------------------------------------------------------------- */
sg_status sg_hsg(int64_t n, int n_fluids, const double *d_H, const double *d_Q, double *d_Hsg,
                 void *stream);

/* ---------------------------------------------------------------------
 * sg_field_adjoint: reverse-mode derivative of sg_field_fft for one disc.
 * Given lam_r = dL/dg_r and lam_phi = dL/dg_phi (float device arrays
 * [F][n_r][n_phi]) it returns
 *   d_dsigma[a][i] = dL/dSigma_a[i]
 *                  = -du dphi sum_b sum_c sum_j lam_{b,c}[j] K_c^{ab}(j - i)
 * (the transposed convolution: conjugate kernel spectra) and, when d_dh is
 * not NULL, d_dh[f] = dL/dh_f (double, device, [F]) by a Parseval reduction
 * of lam against (dK/dh) (*) Sigma accumulated in double.  d_dh needs a
 * table built with SG_WITH_DH (SG_ERR_TABLE otherwise).
 * Semi-spectral discs: d_dsigma = M^T lam with the stored radial operators
 * transposed mode by mode (the folded indirect term and SG_POTENTIAL
 * operators included); d_dh must be NULL (SG_ERR_UNSUPPORTED otherwise).
 * Species discs (n_species = S > 0): lam is per group [F][n_r][n_phi] and
 * d_dsigma per species [S][n_r][n_phi], each species receiving its
 * group's dL/dSigma (the forward sums a group's species before the
 * transform); d_dh is taken at the group densities, summed in the
 * forward's order.  SG_INDIRECT (FFT path): the transpose of the star's pull
 * is added to d_dsigma (its coefficient's h_a derivative to d_dh), from two
 * double reductions over lam and Sigma in a fixed order.  Every group count
 * of the forward (one to four) is taken.
 * d_ws: sg_field_adjoint_workspace_bytes() bytes.  Asynchronous.
 * --------------------------------------------------------------------- */
size_t sg_field_adjoint_workspace_bytes(const sg_disc *disc);
sg_status sg_field_adjoint(const sg_disc *disc, const float *d_lam_r, const float *d_lam_phi,
                           float *d_dsigma, double *d_dh, void *d_ws, size_t ws_bytes,
                           void *stream);

/* ---------------------------------------------------------------------
 * sg_ss_grad_H: derivative of L with respect to the ring scale heights of
 * a semi-spectral disc (Sect. 5.2 operators with h_a = H_a(r_i')/r_i' at
 * the source ring and h_b = H_b(r_i)/r_i at the target ring), for
 * dL/dg_r = lam_r, dL/dg_phi = lam_phi (float device [F][n_r][n_phi]):
 *   d_dH[f][i] = dL/dH_f(r_i)   (double, device, [F][n_r]).
 * Every operator entry is differentiated through both of its scale heights
 * (the kernels' h derivatives, the own-cell integral's derivatives, and the
 * folded indirect term through H_a at the source ring; for SG_POTENTIAL
 * operators the potential kernel's, dP/dH_ab = -(2 y F(y) - e^y K0(y)) /
 * (2 sqrt(pi) H_ab^2), and its own-cell integral's) and contracted with
 * the phi spectra of lam and Sigma, mode by mode, in double; the derivative
 * operators are sampled and transformed on the fly and never stored, so a
 * call costs about twice a table build.  d_H: the H the disc's table was
 * built from.  disc->table supplies the phi twiddles only.  Species discs
 * (n_species > 0): the derivative at the group densities, summed in the
 * forward's order.  Discs without SG_SEMI_SPECTRAL return
 * SG_ERR_UNSUPPORTED.  d_ws: sg_ss_grad_H_workspace_bytes() bytes,
 * 256-byte aligned (it holds two doubles per ring pair and group pair,
 * 16 nf^2 n_r^2 bytes, besides the phi spectra).  Asynchronous; each ring
 * pair's partial sums are stored and added up in a fixed order, so the
 * result is the same, bit for bit, on every call.
 * --------------------------------------------------------------------- */
size_t sg_ss_grad_H_workspace_bytes(const sg_disc *disc);
sg_status sg_ss_grad_H(const sg_disc *disc, const double *d_H, const float *d_lam_r,
                       const float *d_lam_phi, double *d_dH, void *d_ws, size_t ws_bytes,
                       void *stream);

/* ---------------------------------------------------------------------
 * Device-side evaluation of F(x) = e^x [K1(x) - K0(x)] (the function of
 * App. A at argument x) for testing: d_x, d_F device arrays of n values in
 * `dtype`.  F'(x) too when d_dF is not NULL.
 * --------------------------------------------------------------------- */
sg_status sg_eval_F(const void *d_x, void *d_F, void *d_dF, int64_t n, sg_dtype dtype,
                    void *stream);

/* Device-side evaluation of G0(y) = e^y K0(y) (the kernel of the
 * conservative potential, sg_potential_direct) for testing: d_x, d_G device
 * arrays of n values in `dtype`. */
sg_status sg_eval_G0(const void *d_x, void *d_G, int64_t n, sg_dtype dtype, void *stream);

/* Self-cell term for a list of (h_a, h_b) pairs on one grid: d_out[i] =
 * principal-value average of the log-polar radial kernel K_r over the own
 * cell (double), the value sg_kernel_table places at offset (0,0) before
 * scaling.  which = 0 for the kernel, 1 for d/dh_a, 2 for d/dh_b.  ha, hb:
 * HOST arrays of n values, 1 <= n <= 64; d_out: device double array of n. */
sg_status sg_self_cell(const sg_grid *grid, const double *ha, const double *hb, int n, int which,
                       double *d_out, void *stream);

/* Frees the cached plans: graphs and descriptor tables (synchronises the device). */
void sg_release(void);

/* Number of batch signatures (discs' shapes and buffer addresses, workspace,
 * device) whose plan (and graph, where used) sg_field_fft currently caches; a caller that
 * keeps its buffers sees it stay constant after the first call. */
int sg_field_fft_cache_entries(void);

const char *sg_status_string(sg_status s);
int sg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SG_H */
