/*
 * conker.h -- C ABI of the MI355X (gfx950) ConKer hot path.
 *
 * ConKer (Brown, Mishtaku & Demina, arXiv:2108.00015) estimates isotropic
 * n-point correlation functions of tracer catalogs in three stages:
 *   mapping      (Sec. 2.2, Eq. bgsubtracted_map)  conker_grid_assign, conker_form_delta
 *   kernels      (Sec. 2.3)                         conker_make_shell_kernels
 *   convolution  (Sec. 2.4, Eqs. countconv/randconv) conker_convolve_shells
 *   summation    (Sec. 2.5, Eq. ksin_delta)         conker_contract_npt, conker_ratio
 *   both at once, maps never returned               conker_convolve_contract
 * and the paper's other forms: equidistant sums (Eq. ksinDiag,
 * conker_convolve_diag / conker_contract_diag), cross-correlations (Sec. 2.8,
 * *_cross), continuous delta fields (Sec. 2.7, conker_delta_field), n = 2 in
 * Fourier space (conker_pair_spectral), regions combined (Eq. ksi3combined,
 * conker_ratio_combined), maps and their distributions (Sec. 4.2,
 * conker_map_ratio, conker_value_histogram), the survey front end (Sec. 2.2,
 * conker_sky_to_cartesian, conker_analytic_randoms) and batches of catalogs
 * replayed as one HIP graph (conker_batch_*), whose launch shapes can be
 * tuned per job shape by timing them (conker_batch_autotune, conker_set_tune).
 *
 * Conventions shared by every call
 * --------------------------------
 * - d_* arguments are device pointers, h_* arguments host pointers.  The caller
 *   owns every buffer it passes; the library never frees or retains them past
 *   the call's stream work.
 * - Grids are C order [nx][ny][nz] (z fastest), real float32 or float64 per
 *   the conker_dtype argument.  Supported axis lengths for every call that
 *   transforms: 32, 64, 96, 128, 192, 256, 384, 512, 1024.
 * - Every call enqueues work on the context's HIP stream and returns without
 *   waiting for it (except where noted).  A context serves one stream and is
 *   not thread-safe.
 * - Every call returns CONKER_OK or a negative conker_status; nothing is
 *   thrown.  Invalid arguments are rejected before any launch, and
 *   conker_last_error() describes the last failure.
 * - The context owns internal workspace (FFT spectra, partial sums, twiddle
 *   tables), bounded by workspace_max_bytes; it is freed by conker_destroy.
 */
#ifndef CONKER_H
#define CONKER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct conker_ctx conker_ctx;

typedef enum {
    CONKER_OK = 0,
    CONKER_EINVAL = -1,       /* bad pointer, size or enum value              */
    CONKER_ENOMEM = -2,       /* workspace above the cap, or allocation failed */
    CONKER_EUNSUPPORTED = -3, /* axis length or order outside what is built   */
    CONKER_EHIP = -4,         /* a HIP runtime call failed                     */
    CONKER_ERANGE = -5        /* shell radius below half a cell or too large   */
} conker_status;

typedef enum { CONKER_F32 = 1, CONKER_F64 = 2 } conker_dtype;

/* Arithmetic of the summation stage. */
typedef enum {
    CONKER_MM_F64 = 0,        /* float64 maps, float64 matrix cores            */
    CONKER_MM_F32 = 1,        /* float32 maps, float32 matrix cores            */
    CONKER_MM_SPLIT_BF16 = 2, /* float32 maps split into three bfloat16 terms,
                                 bf16 matrix cores, float32 accumulation over
                                 short chains, float64 across chains          */
    CONKER_MM_SPLIT_F16 = 3   /* float32 operands scaled by powers of two from
                                 the largest |value| of each map and of the
                                 field, split into two float16 terms (22
                                 significant bits), three of the four term
                                 products on fp16 matrix cores; accumulation
                                 as for split-bf16; n >= 3 (n = 2: float32)   */
} conker_mmprec;

/* Grid of spacing `cell` whose cell (0,0,0) has its lower corner at `origin`
 * (Sec. 2.2).  Cell index of a point x: floor((x - origin) / cell) per axis,
 * evaluated in float64. */
typedef struct {
    int32_t dims[3];
    double origin[3];
    double cell;
} conker_grid;

/* ---- context -------------------------------------------------------------
 * conker_create: binds a context to HIP device `device` and stream
 * `hip_stream` (a hipStream_t; NULL = the default stream).
 * workspace_max_bytes caps internal allocations (0 = no cap).
 * On success *out holds the context; on failure *out is NULL. */
int conker_create(conker_ctx **out, int device, void *hip_stream, size_t workspace_max_bytes);
void conker_destroy(conker_ctx *ctx);
int conker_set_stream(conker_ctx *ctx, void *hip_stream);
/* Message of the last failure on this context ("" if none).  With ctx NULL,
 * the message of the last conker_create failure in this thread. */
const char *conker_last_error(const conker_ctx *ctx);
/* Bytes of internal workspace currently held by the context. */
size_t conker_workspace_bytes(const conker_ctx *ctx);

/* ---- mapping (Sec. 2.2) ----------------------------------------------------
 * conker_grid_assign: nearest-grid-point histogram of a catalog.
 *   d_pos        float32 [n][3] positions (x, y, z).
 *   d_w          float32 [n] weights, or NULL for unit weights.
 *   grid_dtype   dtype of d_grid; d_grid is ACCUMULATED into (zero it first).
 *   d_wsum       float64 scalar, += sum of the weights of in-grid points
 *                (may be NULL).
 *   d_n_outside  int64 scalar, += number of points outside the grid or with a
 *                non-finite coordinate or weight (may be NULL).  Such points
 *                are skipped.
 * Accumulation order is unspecified: float32 grids with non-integer weights
 * are exact only up to rounding; unit weights give exact integer counts. */
int conker_grid_assign(conker_ctx *ctx, const conker_grid *grid,
                       const float *d_pos, const float *d_w, int64_t n,
                       conker_dtype grid_dtype, void *d_grid,
                       double *d_wsum, int64_t *d_n_outside);

/* conker_form_delta: the density-variation histogram N = D - alpha R_raw with
 * alpha = wsum_data / wsum_rand (R normalised to the data total,
 * Eq. bgsubtracted_map).  d_grid holds D on entry and N on exit; d_rand holds
 * R_raw (unchanged).  alpha is computed on the device in float64 and written
 * to d_alpha (float64 scalar).  The subtraction is done in float64 and
 * rounded once to the grid dtype. */
int conker_form_delta(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                      void *d_grid, const void *d_rand,
                      const double *d_wsum_data, const double *d_wsum_rand,
                      double *d_alpha);

/* ---- kernels (Sec. 2.3) ----------------------------------------------------
 * A shell of radius s (length units) holds the lattice offsets delta with
 * r - 1/2 <= |delta| < r + 1/2, r = s / cell.  It must satisfy r >= 1/2 and
 * 2M + 1 <= min(dims), M = ceil(r + 1/2) - 1 (CONKER_ERANGE otherwise).
 *
 * conker_shell_size: number of offsets in the shell of r cells (host only). */
int conker_shell_size(double r_cells, int64_t *h_size);

/* Elements per radius of the stored kernel spectrum:
 * (nx/2+1) * (ny/2+1) * (nz/2+1). */
int64_t conker_kspec_elems(const conker_grid *grid);

/* conker_make_shell_kernels: spectra of the shell indicators, K_hat_m / N_c,
 * for n_radii radii h_radii[] (length units).  The spectrum of a
 * point-symmetric shell is real and even in each axis, so only the octant
 * 0 <= k <= n/2 per axis is stored, x fastest:
 *   d_kspec  dtype [n_radii][ny/2+1][nz/2+1][nx/2+1].
 * The transform is done in float64 and rounded once to dtype.
 * h_shell_sizes (may be NULL) receives |S_m| per radius. */
int conker_make_shell_kernels(conker_ctx *ctx, const conker_grid *grid,
                              const double *h_radii, int n_radii, conker_dtype dtype,
                              void *d_kspec, int64_t *h_shell_sizes);

/* ---- convolution (Sec. 2.4, Eqs. countconv, randconv) ---------------------
 * conker_convolve_shells: per-radius shell-sum maps of one or two real fields,
 *   maps_a[m](x) = sum over delta in S_m of field_a((x + delta) mod dims),
 * i.e. the circular 3D convolution field *** K_m done with FFTs.  The two
 * fields (typically N and R_raw) share every transform: they travel as the
 * real and imaginary parts of one complex field, a + i s b, which the real,
 * even kernel spectrum keeps apart.  s is a power of two chosen on the device
 * from the two fields' sums of squares (s b about a quarter of a in root mean
 * square), so that the rounding of the larger field does not swamp the
 * smaller one; it is undone exactly (maps_b are returned unscaled).  Every
 * call taking two fields does the same.
 *   d_field_a, d_field_b   dtype [nx][ny][nz]; d_field_b may be NULL.
 *   d_kspec                from conker_make_shell_kernels (same grid, dtype).
 *   d_maps_a, d_maps_b     dtype [n_radii][nx][ny][nz]; d_maps_b must be NULL
 *                          exactly when d_field_b is. */
int conker_convolve_shells(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                           const void *d_field_a, const void *d_field_b,
                           const void *d_kspec, int n_radii,
                           void *d_maps_a, void *d_maps_b);

/* ---- summation (Sec. 2.5, Eqs. ksin_delta, ksi2_delta, ksi3; Sec. 2.6) -----
 * Number of radius tuples of order n: multisets a_1 <= ... <= a_{n-1} of
 * n_radii shell indices, C(n_radii + n - 2, n - 1).  Returns -1 if n < 2. */
int64_t conker_num_tuples(int n_radii, int n);

/* conker_contract_npt:
 *   W[t] = sum over all cells x of field(x) * prod_i maps[a_i](x)
 * for every tuple t = (a_1 <= ... <= a_{n-1}), in lexicographic order.
 *   d_field  dtype [nx][ny][nz];  d_maps dtype [n_radii][nx][ny][nz].
 *   n        2..5;  n_radii 1..64.
 *   prec     CONKER_MM_F64 needs dtype F64; CONKER_MM_F32,
 *            CONKER_MM_SPLIT_BF16 and CONKER_MM_SPLIT_F16 need dtype F32.
 *   d_W      float64 [conker_num_tuples(n_radii, n)], overwritten. */
int conker_contract_npt(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                        const void *d_field, const void *d_maps, int n_radii, int n,
                        conker_mmprec prec, double *d_W);

/* conker_convolve_contract: conker_convolve_shells followed by
 * conker_contract_npt, without returning the maps:
 *   W_a[t] = sum_x field_a(x) prod_i maps_a[a_i](x), and likewise W_b for
 *   field_b, maps as defined for conker_convolve_shells, tuples in the order
 *   of conker_contract_npt.
 *   d_field_b and d_W_b: both given or both NULL.
 * Arguments as for conker_contract_npt (n 2..5, n_radii 1..64, dtype and prec
 * alike).  Since every term carries field(x), z-lines on which both fields
 * vanish add nothing: the inverse transforms are carried out only where a
 * line holds field.
 * - dtype CONKER_F32 with prec CONKER_MM_F32 or CONKER_MM_SPLIT_BF16, n = 2
 *   or 3, nz = 512, n_radii <= 30: one pass that never writes the maps to
 *   memory (each line of cells is transformed back for every radius in
 *   on-chip memory and summed at once); the context holds the spectra of all
 *   radii at once (n_radii * N_c * 8 bytes).
 * - every other case: the maps are written to the context's workspace
 *   (fields * n_radii * N_c * element size bytes) on the carrying lines only,
 *   and summed as conker_contract_npt does; the spectra are batched over the
 *   radii as in conker_convolve_shells.
 * The fields must be 16-byte aligned (CONKER_EINVAL otherwise). */
int conker_convolve_contract(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                             const void *d_field_a, const void *d_field_b, const void *d_kspec,
                             int n_radii, int n, conker_mmprec prec, double *d_W_a, double *d_W_b);

/* ---- equidistant configurations (Sec. 2.6, Eq. ksinDiag) -------------------
 * The diagonal entries a_1 = ... = a_{n-1} = m of Eq. ksin_delta, for every
 * order n = 2 .. n_max at once:
 *   out[(n - 2) * n_radii + m] = sum over all cells x of field(x) * C_m(x)^(n-1)
 * with C_m the shell map of radius m (conker_convolve_shells).  n_max 2..5.
 * Outputs are float64 device arrays of (n_max - 1) * n_radii, overwritten.
 *
 * conker_contract_diag: from stored maps, d_maps dtype [n_radii][nx][ny][nz].
 * Any dtype (F32 products are formed in float32 and summed in float64). */
int conker_contract_diag(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                         const void *d_field, const void *d_maps, int n_radii, int n_max,
                         double *d_out);

/* conker_contract_diag_noalloc: conker_contract_diag for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results; it
 * calls no hipMalloc, hipFree or allocating routine.  Its partial sums live in
 * a fixed device array of 2^19 doubles (4 MiB) per GPU, held from the first
 * conker_create on that GPU until the process ends: calls needing more
 * (n_radii x workgroups x (n_max - 1), at most 64 radii on grids of 2^21
 * cells and more) fail with CONKER_ERANGE.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other streams, other contexts)
 * race; calls in one stream are ordered and safe.  Each call overwrites every
 * partial it reads, so nothing needs clearing between calls. */
int conker_contract_diag_noalloc(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                                 const void *d_field, const void *d_maps, int n_radii, int n_max,
                                 double *d_out);

/* conker_convolve_diag: the same sums for field_a (and field_b) straight from
 * the kernel bank, without storing any map: the last inverse FFT pass of each
 * radius feeds the sums instead of memory, so the device holds only the
 * spectra of one radius batch.  Every supported grid and both dtypes.
 *   d_field_b and d_out_b: both given or both NULL.
 * Fields 16-byte aligned (CONKER_EINVAL otherwise); as for
 * conker_convolve_contract, lines on which both fields vanish are skipped. */
int conker_convolve_diag(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                         const void *d_field_a, const void *d_field_b, const void *d_kspec,
                         int n_radii, int n_max, double *d_out_a, double *d_out_b);

/* ---- cross-correlation of two tracers (Sec. 2.8) ----------------------------
 * Vertex 0 weighs with one field (the "centre" field Delta_0), the shells with
 * the maps of another (Delta_1).  From stored maps this is conker_contract_npt
 * called with d_field = Delta_0 and d_maps = the maps of Delta_1.  Without
 * storing maps:
 *
 * conker_convolve_contract_cross: as conker_convolve_contract, but the maps of
 * d_field_a (d_field_b) are summed against d_centre_a (d_centre_b):
 *   W_a[t] = sum_x centre_a(x) prod_i maps_a[a_i](x).
 * d_field_b, d_centre_b and d_W_b: all given or all NULL.  Same support and
 * alignment rules; lines where the centre fields vanish are skipped. */
int conker_convolve_contract_cross(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                                   const void *d_field_a, const void *d_field_b,
                                   const void *d_centre_a, const void *d_centre_b, const void *d_kspec,
                                   int n_radii, int n, conker_mmprec prec, double *d_W_a, double *d_W_b);

/* conker_convolve_diag_cross: conker_convolve_diag with centre fields:
 *   out_a[(n - 2) * n_radii + m] = sum_x centre_a(x) C_m[field_a](x)^(n-1). */
int conker_convolve_diag_cross(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                               const void *d_field_a, const void *d_field_b,
                               const void *d_centre_a, const void *d_centre_b, const void *d_kspec,
                               int n_radii, int n_max, double *d_out_a, double *d_out_b);

/* conker_ratio_cross: xi = W_cross / (alpha0 alpha1^(n-1) W_rand) in float64,
 * the two-tracer estimator with common randoms normalised to each tracer
 * (B_0 = alpha0 R_raw for vertex 0, alpha1 R_raw in the shells).  d_alpha0,
 * d_alpha1: device float64 scalars (from conker_form_delta of each tracer). */
int conker_ratio_cross(conker_ctx *ctx, const double *d_W_cross, const double *d_W_rand,
                       const double *d_alpha0, const double *d_alpha1, int n, int64_t count,
                       double *d_xi);

/* ---- n = 2 in Fourier space (Sec. 2.5, Eq. ksi2_delta; Sec. 2.8) ------------
 * conker_pair_spectral: for every radius m, from the forward spectra alone
 * (Parseval, K_m real and even):
 *   W_aa[m] = sum_x a(x) (K_m *** a)(x),  W_bb[m] likewise for b,
 *   W_ab[m] = sum_x a(x) (K_m *** b)(x)   (the cross-correlation of a and b),
 * i.e. conker_contract_npt with n = 2, in one pass over the spectrum and one
 * read of each kernel octant instead of an inverse transform per radius.
 * d_field_b may be NULL (then d_W_bb and d_W_ab must be NULL); d_W_bb and
 * d_W_ab may be NULL when not wanted.  Every supported grid, both dtypes. */
int conker_pair_spectral(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                         const void *d_field_a, const void *d_field_b, const void *d_kspec,
                         int n_radii, double *d_W_aa, double *d_W_bb, double *d_W_ab);

/* ---- continuous tracers (Sec. 2.7, Eqs. densitycont, ksin_cont) -------------
 * conker_delta_field: delta = (D - alpha R) / (alpha R) on cells where
 * alpha R != 0, and 0 on cells without random coverage.  d_alpha: device
 * float64 scalar, or NULL for 1.  d_delta may alias d_D.  The estimator of a
 * continuous tracer is then the plain sum W[t] = sum_x delta prod_i C_{a_i}[delta]
 * (conker_contract_npt / conker_convolve_contract on delta), with no ratio. */
int conker_delta_field(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype, const void *d_D,
                       const void *d_R, const double *d_alpha, void *d_delta);

/* ---- regions, maps and distributions (Sec. 3.4, Eq. ksi3combined; Sec. 4.2) ---
 * conker_ratio_combined: regions (or mocks) measured separately, combined by
 * adding numerators and denominators:
 *   num[t] = sum_j W_delta[j][t],  den[t] = sum_j alpha_j^n W_rand[j][t],
 *   xi[t] = num[t] / den[t]   (float64; regions summed in order j = 0, 1, ...).
 * d_W_delta, d_W_rand: [n_regions][count] contiguous; d_alpha: [n_regions].
 * d_num and d_den may be NULL. */
int conker_ratio_combined(conker_ctx *ctx, int n_regions, const double *d_W_delta,
                          const double *d_W_rand, const double *d_alpha, int n, int64_t count,
                          double *d_xi, double *d_num, double *d_den);

/* conker_map_ratio: the per-cell map W_0 W_1 / <B_0 B_1> of one radius,
 *   out(x) = N(x) C^N(x) / (alpha^2 W_R2 / N_c),
 * with C^N the map of N for that radius (conker_convolve_shells), W_R2 the
 * n = 2 sum of R_raw for that radius and alpha the normalisation (device
 * float64 scalars).  Its average over the cells is xi_2 of that radius.
 * d_N, d_map, d_out: dtype [nx][ny][nz]; d_out may alias either input. */
int conker_map_ratio(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype, const void *d_N,
                     const void *d_map, const double *d_W_R2, const double *d_alpha, void *d_out);

/* conker_value_histogram: counts of n values (dtype) in n_bins equal bins of
 * [lo, hi) (bin = floor((v - lo) / (hi - lo) * n_bins) in float64), then the
 * count below lo, then the count at or above hi (NaN included).
 * d_counts: int64 [n_bins + 2], overwritten.  1 <= n_bins <= 16000, lo < hi. */
int conker_value_histogram(conker_ctx *ctx, conker_dtype dtype, const void *d_values, int64_t n,
                           double lo, double hi, int n_bins, int64_t *d_counts);

/* ---- survey front end (Sec. 2.2, Eqs. hubbleint, cartesianx-z, factorizablility)
 * Fiducial cosmology: E(z) = sqrt(omega_m (1+z)^3 + omega_k (1+z)^2 +
 * omega_lambda), comoving distance r(z) = c/h0 int_0^z dz'/E(z') (with
 * h0 = 100 and c in km/s the unit is Mpc/h).  r(z) is tabulated on [0, z_max]
 * for each call. */
typedef struct {
    double omega_m, omega_k, omega_lambda;
    double h0, c;
    double z_max;   /* largest redshift converted; E(z)^2 must stay positive on [0, z_max] */
} conker_cosmology;

/* conker_sky_to_cartesian: X = r cos(dec) cos(ra), Y = r cos(dec) sin(ra),
 * Z = r sin(dec) with r = r(z).  d_ra_deg, d_dec_deg, d_z: float64 [n] device
 * arrays (degrees); d_pos: float32 [n][3], ready for conker_grid_assign.
 * Redshifts outside [0, z_max] (or NaN) give NaN positions, which
 * conker_grid_assign skips and counts. */
int conker_sky_to_cartesian(conker_ctx *ctx, const conker_cosmology *cosmo, const double *d_ra_deg,
                            const double *d_dec_deg, const double *d_z, int64_t n, float *d_pos);

/* conker_analytic_randoms: the expected random count per cell for
 * factorizable selection functions, instead of a random catalog:
 *   R(cell) = N_tot P_ang(ra, dec) P_z(z) / (r^2 dr/dz) * cell^3
 * at the cell centre, with dr/dz = c/(h0 E(z)).  P_ang: density per steradian
 * on an equal-angle table d_p_ang[n_dec][n_ra] over ra_range x dec_range
 * (degrees, host arrays of 2); P_z: density in z on n_z equal bins of z_range
 * (inside [0, z_max]).  Cells whose centre falls outside a table get 0.
 * d_R: dtype [nx][ny][nz], overwritten. */
int conker_analytic_randoms(conker_ctx *ctx, const conker_grid *grid, conker_dtype dtype,
                            const conker_cosmology *cosmo, double n_tot, const double *d_p_ang,
                            int n_dec, int n_ra, const double *h_ra_range, const double *h_dec_range,
                            const double *d_p_z, int n_z, const double *h_z_range, void *d_R);

/* conker_ratio: the estimator xi = W_delta / (alpha^n W_rand) in float64
 * (Eq. ksin_delta with B_i built on R = alpha R_raw).  All pointers are
 * device float64; d_alpha is a scalar. */
int conker_ratio(conker_ctx *ctx, const double *d_Wd, const double *d_Wr,
                 const double *d_alpha, int n, int64_t count, double *d_xi);

/* ---- batches of catalogs ---------------------------------------------------
 * One job = the whole path for one catalog pair (data, randoms) on its own
 * grid: zero the grids, grid_assign both catalogs, form_delta, convolution and
 * summation of both fields (conker_convolve_contract when the map pointers
 * are NULL, else convolve_shells + contract_npt), and ratio.
 * Independent catalogs (mocks, survey regions) combine afterwards by adding
 * numerators and denominators (Eq. ksi3combined).  All pointers are caller
 * owned device memory; jobs may share grid and map buffers (they run in
 * order on the context's stream) but not outputs. */
typedef struct {
    conker_grid grid;
    conker_dtype dtype;
    conker_mmprec prec;
    int n;                          /* correlation order 2..5 */
    int n_radii;
    const void *d_kspec;            /* from conker_make_shell_kernels for this grid */
    const float *d_data_pos;        /* [n_data][3] */
    const float *d_data_w;          /* [n_data] or NULL */
    int64_t n_data;
    const float *d_rand_pos;        /* [n_rand][3] */
    const float *d_rand_w;          /* [n_rand] or NULL */
    int64_t n_rand;
    void *d_N;                      /* dtype grid: N on exit */
    void *d_R;                      /* dtype grid: R_raw on exit */
    void *d_maps_N;                 /* dtype [n_radii][grid] or NULL (conker_convolve_contract) */
    void *d_maps_R;                 /* likewise, NULL exactly when d_maps_N is */
    double *d_wsum;                 /* [2]: in-grid weight sums of data, randoms */
    int64_t *d_n_outside;           /* [2]: rejected tracers of data, randoms */
    double *d_alpha;                /* [1] */
    double *d_W_delta;              /* [num_tuples(n_radii, n)] */
    double *d_W_rand;               /* [num_tuples]: sums on R_raw */
    double *d_xi;                   /* [num_tuples] */
} conker_job;

/* conker_batch_plan: validates and stores the job list, then runs it once
 * (synchronously) so that every workspace buffer, table and kernel attribute
 * the jobs need exists.  Replaces any earlier batch and captured graph.
 * conker_batch_run: enqueues every job again, in order.
 * conker_batch_capture: records the whole batch into one HIP graph (the
 * context stream must not be the default stream); nothing is allocated or
 * zeroed with memset nodes inside the capture.
 * conker_batch_launch: replays the captured graph on the context stream.
 *   The graph holds the addresses of the context's workspace buffers: any
 *   later call on the context that has to grow one of them (a larger grid,
 *   more radii, a larger catalog) frees it and drops the captured graph, and
 *   conker_batch_launch then fails with CONKER_EINVAL ("no captured batch")
 *   until the batch is captured again. */
int conker_batch_plan(conker_ctx *ctx, const conker_job *jobs, int n_jobs);
int conker_batch_run(conker_ctx *ctx);
int conker_batch_capture(conker_ctx *ctx);
int conker_batch_launch(conker_ctx *ctx);

/* Size classes.  Mock batches hold many catalogs on a few grid sizes; run one
 * by one, a small grid leaves most of the device idle in every stage.  So
 * conker_batch_plan groups the jobs that share the grid (dimensions, origin,
 * cell), the kernel bank pointer and n_radii (at most 64), with dtype float32,
 * n = 3, split or float32 summation (CONKER_MM_SPLIT_BF16, _SPLIT_F16 or
 * _F32; float32 only where the fused form below applies), 16-byte aligned
 * grids, a grid whose cell count is a multiple of 64 and whose x length has a
 * resident first inverse pass, and buffers (grids, maps, outputs) that no
 * other job of the group touches.  Such a group runs in chunks: every stage
 * of the path (mapping, binned by brick as for large catalogs where the grid
 * splits into bricks of 16 x 16 x 32 cells, else zeroing and atomics, N = D -
 * alpha R, the packed forward transform, the inverse transforms in radius
 * batches of 8, the order-3 summation from stored maps, the ratio) is one
 * launch for all jobs of a chunk, the job taken from the launch grid.  The
 * results are those of the job-by-job path up to the order of float
 * additions (mapping atomics, partial sums).  Jobs with NULL maps keep their
 * maps in a workspace of the chunk, except where every job of the group has
 * NULL maps, CONKER_MM_SPLIT_BF16 or CONKER_MM_F32, at most 16 radii and a z
 * length of 32, 64, 96, 128, 192 or 256: there the last inverse pass and the
 * summation run as one kernel that never stores the maps (all radii
 * transformed at once; float32 products on v_mfma_f32_16x16x4f32).  A
 * chunk's workspace is bounded by 16 GiB
 * (a class of large grids runs in several chunks) and is held by the context
 * until it is destroyed.  A group whose chunks would hold one job each, every
 * other job, and every job when the workspace cannot be allocated run job by
 * job.  Chunks run first, then the other jobs in order (see
 * conker_batch_autotune for how chunks are tuned).
 * conker_batch_classes: on != 0 (the default) enables the grouping for later
 *   conker_batch_plan calls on the context; 0 runs every job alone.
 * conker_batch_layout: for each planned job, the index of the chunk it runs
 *   in, or -1 when it runs alone (h_chunk: n_jobs ints, host memory). */
int conker_batch_classes(conker_ctx *ctx, int on);
int conker_batch_layout(const conker_ctx *ctx, int *h_chunk);

/* ---- launch shapes and their tuning ---------------------------------------
 * Not part of the method: how the convolution and summation stages are cut
 * into workgroups.  Every choice computes the same sums (the same arithmetic
 * in a different order of tiles); 0 in any field means the built-in default,
 * which an environment switch of the same meaning may override.
 *   x_tile, y_tile  columns per tile of the x- and y-axis inverse passes and
 *                   of the forward passes of those axes:
 *                   1 narrow (16 float32 / 8 float64 columns), 2 wide (twice
 *                   that: 256-byte runs).  Default: wide.
 *   x_resident      x-axis inverse pass: 1 streamed, 2 kernel-multiply tile
 *                   kept resident on chip across the batch's radii, its
 *                   stages alternating between two LDS exchange buffers
 *                   where both fit, 3 as 2 with one exchange buffer.
 *                   Default: 2 where the pass stores only the slabs
 *                   carrying field, else 3.
 *   mm_kernel       matrix-core summation: 1 one output tile per wave,
 *                   2 operand sharing across a workgroup, 3 (n = 3 with
 *                   split operands and at most 64 radii) every output tile
 *                   in each wave from one load of the maps.  Default: 3
 *                   where it applies, else 2 above four 32 x 32 output
 *                   tiles, else 1.
 *   radius_batch    radii (or radius pairs) per inverse batch, 1..64.
 *                   Default: as many as half of the free device memory holds.
 *   axis_order      map-free summations (conker_convolve_contract*,
 *                   conker_convolve_diag*) on grids with equal axis lengths:
 *                   the order of the axes the transforms run in, which sets
 *                   how much of the work outside the field's support is
 *                   skipped: 1 the given order (x,y,z), 2 (x,z,y),
 *                   3 (y,x,z), 4 (y,z,x), 5 (z,x,y), 6 (z,y,x) (the first
 *                   axis listed is transformed first after the kernel
 *                   multiply, the last one is the contiguous axis of the
 *                   summation); 0 (default) chosen on the device from the
 *                   support.  Other than 1, the fields are copied into the
 *                   permuted layout in workspace.
 *   radix           radix schedule of the float32 transform passes (not the
 *                   resident first inverse pass): 1 radix 8 first (32 = 8 4,
 *                   64 = 8 8, 128 = 8 4 4, 256 = 8 8 4, 512 = 8 8 8,
 *                   1024 = 8 8 4 4, 96 = 8 4 3, 192 = 8 8 3, 384 = 8 8 2 3),
 *                   2 radix 16 first where that saves a stage (64 = 16 4,
 *                   128 = 16 8, 256 = 16 16, 1024 = 16 16 4; other lengths
 *                   as 1).  Default: 1.
 *   ms              conker_batch_autotune only: the measured time of one run
 *                   of the job with this setting (milliseconds).
 * conker_set_tune: the setting used by every later call on the context
 *   (NULL: all defaults); rejects values outside the ranges above.
 * conker_get_tune: the current setting. */
typedef struct {
    int32_t x_tile;
    int32_t y_tile;
    int32_t x_resident;
    int32_t mm_kernel;
    int32_t radius_batch;
    int32_t axis_order;
    int32_t radix;
    float ms;
} conker_tune;

int conker_set_tune(conker_ctx *ctx, const conker_tune *h_tune);
int conker_get_tune(const conker_ctx *ctx, conker_tune *h_tune);

/* conker_axis_order_used: the axis order (1..6, numbered as axis_order above)
 * that the last map-free summation on this context ran in, 0 if none has run.
 * Waits for the context's stream when the order was chosen on the device. */
int conker_axis_order_used(conker_ctx *ctx, int *h_order);

/* conker_batch_autotune: after conker_batch_plan, picks a setting per job
 * shape (grid dimensions, dtype, order, number of radii, summation arithmetic,
 * fused or not) by timing the first job of that shape with HIP events: start
 * from the defaults and, one field at a time, keep the alternative that is
 * faster than the best so far (the minimum of `reps` timed runs, 1..16, after
 * one untimed run per candidate).  The fields searched: the column tiles, the
 * resident first pass, the summation kernel (n >= 3 from maps), the axis
 * order (map-free, cubic grids), the radius batch, and the radix schedule
 * (float32 grids with an axis of 64, 128, 256 or 1024).  Each chunk of a size
 * class is tuned as a whole over the column tiles and the radix schedule (its
 * jobs report the chunk's setting and the chunk's time divided by its number
 * of jobs).  Later conker_batch_run / conker_batch_capture use the chosen
 * settings; the jobs' outputs are recomputed with them before returning.
 * h_chosen (or NULL) receives n_jobs settings with their times.
 * Synchronous. */
int conker_batch_autotune(conker_ctx *ctx, int reps, conker_tune *h_chosen);

/* Blocks until all work queued on the context's stream has finished. */
int conker_synchronize(conker_ctx *ctx);

/* ---- per-launch timing ----------------------------------------------------
 * Not part of the method; used to report where the time goes, as the paper's
 * timing study splits it into mapping, convolution and summation (Sec. 3.2).
 * conker_profile_enable: with enable != 0, every later kernel launch of the
 *   library is bracketed by HIP events on the context stream; any previous
 *   records are dropped.  Waits for the stream first.
 * conker_profile_read: number of launches and their summed event time (ms)
 *   recorded for one launch kind; waits for the stream.
 * conker_profile_kind_name: name of a launch kind (0 .. count-1), NULL past
 *   the last one. */
int conker_profile_enable(conker_ctx *ctx, int enable);
int conker_profile_read(conker_ctx *ctx, int kind, int64_t *launches, double *total_ms);
const char *conker_profile_kind_name(int kind);

#ifdef __cplusplus
}
#endif

#endif /* CONKER_H */
