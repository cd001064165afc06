// Internal declarations shared by the ConKer HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/conker.h"

namespace conker {

// ---------------------------------------------------------------------------
// device buffers owned by a context
// ---------------------------------------------------------------------------
struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Power-of-two scale s = 2^k of the field packed into the imaginary part of
// the forward transform (a + i s b, fft.hip), in both float widths, written
// on the device by every packed forward transform and read by the passes and
// reductions that undo it.  Lives at offset 0 of conker_ctx::scal; the
// per-workgroup sums it is chosen from follow at SCAL_PART_OFF.
struct PackScale {
    double s, s_inv;
    float sf, sf_inv;
    int k;
    int pad;
};
constexpr size_t SCAL_PART_OFF = 256;
constexpr int SCAL_MAX_PART = 4096;   // workgroups of the sums (two doubles each)
constexpr size_t SCAL_BYTES = SCAL_PART_OFF + (size_t)SCAL_MAX_PART * 2 * sizeof(double);

// A chunk of one size class of a planned batch (batch.hip): the planned jobs
// `jobs`, run stage by stage; their device table at conker_ctx::cls + tab_off,
// radii transformed nb at a time.
struct ClassChunk {
    std::vector<int> jobs;
    size_t tab_off = 0;
    int nb = 0;
    bool fused = false;   // maps never stored: inverse z pass and summation in one kernel
    bool tuned = false;   // conker_batch_autotune chose `tune` for the chunk
    conker_tune tune{};
};

}  // namespace conker

struct conker_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    size_t ws_cap = 0;      // 0 = unlimited
    size_t ws_bytes = 0;    // bytes currently held
    std::string err;
    // twiddle tables exp(-2 pi i t / L), t in [0, L), keyed by L
    std::map<int, conker::Buf> tw32, tw64;
    conker::Buf spec;       // forward spectrum of the packed field pair
    conker::Buf tspec;      // per-radius spectra of one radius batch
    conker::Buf partial;    // per-workgroup partial sums of the summation stage
    conker::Buf full;       // reduced block matrices of the summation stage
    conker::Buf support;    // line mask, per-slab counts and list of lines carrying field
    conker::Buf scales;     // split-f16 summation: largest |value| per map and of the field
    conker::Buf cosmo;      // comoving-distance table of the survey front end
    conker::Buf order;      // support projections, chosen axis order and permuted fields
    conker::Buf bins;       // binned mapping: per-brick counts and starts, per-workgroup histograms, placed points
    conker::Buf blocks;     // summation: list of the 64-cell blocks where the field is non-zero
    conker::Buf maps;       // convolve-contract without the fused kernel: maps of carrying lines
    conker::Buf scal;       // allocated once by conker_create: PackScale and its partial sums
    int order_last = 0;             // axis order of the last map-free summation (1..6), -1: on the device
    const int *order_dev = nullptr; // with order_last -1: the chosen permutation index (0..5)
    std::map<uint64_t, conker::Buf> tables;  // item / tuple tables, keyed by (n_radii, n, prec)
    // per-launch event timing (conker_profile_enable)
    int n_cu = 0;
    bool prof = false;
    bool capturing = false;            // inside conker_batch_capture
    std::vector<conker_job> jobs;      // planned batch
    conker_tune tune{};                // launch shapes of the calls now enqueued (0 = default)
    conker_tune user_tune{};           // set by conker_set_tune
    std::vector<conker_tune> job_tune; // per planned job (conker_batch_autotune), else empty
    bool batch_classes = true;         // conker_batch_classes
    std::vector<conker::ClassChunk> chunks;  // size classes of the planned batch
    std::vector<int> seq_jobs;         // planned jobs run one at a time
    conker::Buf cls;                   // size classes: job tables, then the workspace of one chunk
    size_t cls_ws_off = 0;
    hipGraphExec_t graph_exec = nullptr;
    struct Rec {
        int kind;
        hipEvent_t e0, e1;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace conker {

// ---------------------------------------------------------------------------
// launch kinds reported by conker_profile_read
// ---------------------------------------------------------------------------
enum ProfKind {
    PK_SCATTER = 0,
    PK_FORM_DELTA,
    PK_FFT_FWD_Z,
    PK_FFT_FWD_Y,
    PK_FFT_FWD_X,
    PK_FFT_INV_X_MUL,
    PK_FFT_INV_Y,
    PK_FFT_INV_Z,
    PK_BANK_Z,
    PK_BANK_Y,
    PK_BANK_X,
    PK_CONTRACT_DOT,
    PK_CONTRACT_MM,
    PK_CONTRACT_REDUCE,
    PK_RATIO,
    PK_FUSED_ZC,
    PK_DIAG_Z,
    PK_DIAG_MAPS,
    PK_DIAG_REDUCE,
    PK_SUPPORT,
    PK_SPECTRAL,
    PK_SURVEY,
    PK_ORDER,
    PK_BLOCKS,
    PK_PACK_SCALE,
    PK_PACK_SCALE_REDUCE,
    PK_COUNT
};

// Brackets the launches of one kind with events on the context stream while
// profiling is enabled; free otherwise.
struct ProfScope {
    conker_ctx *c;
    int kind;
    hipEvent_t e0 = nullptr;
    ProfScope(conker_ctx *ctx, int k);
    ~ProfScope();
};

// ---------------------------------------------------------------------------
// status helpers
// ---------------------------------------------------------------------------
int fail(conker_ctx *ctx, int code, const char *fmt, ...);

#define CK_HIP(ctx, expr)                                                           \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::conker::fail((ctx), CONKER_EHIP, "%s failed: %s (%s:%d)", #expr, \
                                  hipGetErrorString(e_), __FILE__, __LINE__);       \
    } while (0)

#define CK_LAUNCH(ctx)                                                              \
    do {                                                                            \
        hipError_t e_ = hipGetLastError();                                          \
        if (e_ != hipSuccess)                                                       \
            return ::conker::fail((ctx), CONKER_EHIP, "kernel launch failed: %s (%s:%d)", \
                                  hipGetErrorString(e_), __FILE__, __LINE__);       \
    } while (0)

#define CK_OK(expr)                   \
    do {                              \
        int s_ = (expr);              \
        if (s_ != CONKER_OK) return s_; \
    } while (0)

// Grows `b` to at least `bytes` (contents are not preserved).  Respects the
// context's workspace cap.  Waits for the stream before releasing memory.
int ws_reserve(conker_ctx *ctx, Buf &b, size_t bytes);

// Looks up this device's copy of the allocation-free call's scratch array
// (diag.hip); the device must be current.  Once per device.
int noalloc_init(int device);

// Number of compute units of the context's device (cached).
int cu_count(conker_ctx *ctx);

// Device twiddle table of length L (float2 or double2), built on first use.
int twiddles(conker_ctx *ctx, int L, bool f64, const void **out);

// Validates ctx / grid pointers and the FFT-supported axis lengths.
int check_grid(conker_ctx *ctx, const conker_grid *g, bool need_fft);

inline size_t ncells(const conker_grid *g) {
    return (size_t)g->dims[0] * (size_t)g->dims[1] * (size_t)g->dims[2];
}

inline bool fft_length_ok(int L) {
    return L == 32 || L == 64 || L == 96 || L == 128 || L == 192 || L == 256 || L == 384 || L == 512 ||
           L == 1024;
}

// Largest offset component of a shell of radius r cells: ceil(r + 1/2) - 1.
int shell_reach(double r);
// Validates a shell radius (cells) against the grid; CONKER_ERANGE if it does not fit.
int check_shell(conker_ctx *ctx, const conker_grid *g, double r_cells);

// Lines (x, y) on which field_a or field_b is non-zero (support.hip).  The
// fields must be 16-byte aligned (CONKER_EINVAL otherwise).
struct Support {
    const unsigned char *mask = nullptr;   // [nx * ny] 0 / 1
    const int *xcount = nullptr;           // [nx] carrying lines per x-slab
    const int *list = nullptr;             // carrying lines x * ny + y, increasing
    const int *count = nullptr;            // device scalar: length of list
    // sums of squares of the two fields the support was taken from, as
    // sums_n per-workgroup partial pairs (sum a^2, sum b^2), added in a fixed
    // order by the packed forward transform of those same fields
    const double *sums = nullptr;
    int sums_n = 0;
};
int support_lines(conker_ctx *c, const conker_grid *g, bool f64, const void *fa, const void *fb, Support *out);
// The same outputs from a mask and per-slab counts computed elsewhere:
// support_alloc reserves the buffers (mask [nx * ny], xcount [nx]; room for
// nx pairs of sums in *sums_slot when it is given) to fill, support_list then
// builds the ordered list and its count.
int support_alloc(conker_ctx *c, int nx, int ny, Support *out, unsigned char **mask, int **xcount,
                  double **sums_slot = nullptr);
int support_list(conker_ctx *c, int nx, int ny, const Support &s);

// FFT passes (fft.hip) ------------------------------------------------------
// Forward 3D FFT of the complex field packed from two real fields
// (a + i s b) into the spectrum buffer `spec` (natural order, unnormalised).
// With b, s = 2^k is first chosen on the device from the sums of squares of
// a and b (taken from sup->sums when given, else by a pass over both fields)
// and written to the context's PackScale; without b, nothing is scaled and
// the PackScale is left as it was.
// With `sup`, the line support of a and b themselves (both zero on every other
// line): inputs known to be zero are neither written between the passes nor
// read.
int fft_forward_pair(conker_ctx *ctx, const conker_grid *g, bool f64,
                     const void *a, const void *b, void *spec, const Support *sup = nullptr);
// Forward 3D FFT of two shell indicators packed as (K_ra + i K_rb), float64,
// followed by extraction of the real octant spectra (scaled by 1/N_c) into
// kspec rows ma and mb (mb < 0: none) with dtype out_f64 ? double : float.
int fft_shell_pair(conker_ctx *ctx, const conker_grid *g, double lo_a, double hi_a,
                   double lo_b, double hi_b, void *work, void *kspec, bool out_f64,
                   int ma, int mb);
// Inverse passes for radii [m0, m0 + nb): multiply spectrum by K_m, inverse
// 3D FFT, write real parts to maps_a[m] and imaginary parts to maps_b[m].
// With maps_a NULL only the x and y passes run, leaving tspec[m - m0] holding
// the spectra transformed back along x and y (still along kz).
// With `sup` (and maps_a NULL, or sup_maps): outputs are needed on carrying
// lines only; the x pass writes carrying x-slabs, the y pass skips empty slabs
// and writes carrying lines, and with sup_maps the z pass writes the maps of
// carrying lines only (z-line tiles without one are skipped; the maps of other
// lines keep whatever they held).
// With pair_ns > 0 (one real field, maps_b NULL): radius pairing.  m0 and nb
// count slots; slot j is multiplied by K_{2j} + i K_{2j+1} (K_{2j} alone when
// 2j + 1 = pair_ns) and unpacked into maps_a rows 2j and 2j + 1.
int fft_inverse_batch(conker_ctx *ctx, const conker_grid *g, bool f64,
                      const void *spec, const void *kspec, int m0, int nb, void *tspec,
                      void *maps_a, void *maps_b, const Support *sup = nullptr, int pair_ns = 0,
                      bool sup_maps = false);
// Inverse z pass of tspec[0 .. nb) (after fft_inverse_batch with maps_a NULL)
// with the equidistant sums sum_x F(x) C_m(x)^p, p = 1 .. pmax (1..4), of the
// real part against fa and the imaginary part against fb (NULL: none), in
// place of storing the maps.  `blocks` workgroups per radius (at most
// fft_z_tiles) each write one row of 2 * pmax doubles to
// part[(m * blocks + block) * 2 * pmax], field a first.  With `sup`, only its
// list of carrying lines is transformed and summed (in tiles of listed lines).
int fft_inverse_z_diag(conker_ctx *ctx, const conker_grid *g, bool f64, const void *tspec, int nb,
                       const void *fa, const void *fb, int pmax, int blocks, void *part,
                       const Support *sup = nullptr);

// ---------------------------------------------------------------------------
// Size classes of a batch (batch.hip): jobs on one grid with one kernel bank,
// order and arithmetic run every stage as one launch over all of them, the job
// taken from blockIdx.y (or z).  ClassJob is one entry of the device table of
// their buffers (float32 grids).
// ---------------------------------------------------------------------------
struct ClassJob {
    float *N, *R, *mapsN, *mapsR;
    const float *dpos, *dw, *rpos, *rw;
    long long nd, nr;
    long long ioff_d, ioff_r;  // binned mapping: offsets of the catalogs' placed points
    double *wsum;              // [2]
    long long *nout;           // [2]
    double *alpha;             // [1]
    double *Wd, *Wr, *xi;      // [tuples]
};
// Forward transforms of all M jobs: spec[j] (complex [nc], contiguous by job)
// of N_j + i s_j R_j, s_j into scales[j] chosen from the sums of squares in
// part (sums_G pairs per job, as map_jobs leaves them).
int fft_forward_jobs(conker_ctx *ctx, const conker_grid *g, int M, const ClassJob *tab, void *spec,
                     PackScale *scales, const double *part, int sums_G);
// Inverse transforms of radii [m0, m0 + nb) of all M jobs: tspec[j][0 .. nb)
// (contiguous), then the maps of job j into tab[j].mapsN / mapsR rows m0 ..
// (maps of R multiplied by 1 / s_j).
int fft_inverse_jobs(conker_ctx *c, const conker_grid *g, int M, const ClassJob *tab, const void *kspec, int m0,
                     int nb, const void *spec, void *tspec, const PackScale *scales);
// Whether the size-class transforms support grid g (float32): a resident
// first inverse pass exists for its x length and fits its z length.
bool fft_jobs_ok(const conker_grid *g);
// Maps both catalogs of all M jobs and forms N = D - alpha R.  With a
// workspace of map_jobs_bytes (non-zero where the grid splits into the
// binned mapping's bricks; n_total: all points of the table) the points are
// binned by brick and summed in LDS, each brick written whole; else the grids
// are zeroed and the points added with atomics (n_max: the largest catalog).
// Both fields' sums of squares go to part (pairs per workgroup, *sums_G
// workgroups per job, at most 4 cu_count / M + 1) for fft_forward_jobs.
size_t map_jobs_bytes(const conker_grid *g, int M, int64_t n_total);
int map_jobs(conker_ctx *c, const conker_grid *g, int M, const ClassJob *tab, int64_t n_max, int64_t n_total,
             void *ws, double *part, int *sums_G);
// xi of every job of the table (count tuples of order n).
int ratio_jobs(conker_ctx *c, int M, const ClassJob *tab, int n, int64_t count);
// Whether the fused inverse z pass + order-3 summation (k_zinv_mm3_jobs)
// serves grid g with n_radii = ns (split bfloat16 or float32, maps never stored).
bool fft_mm3_jobs_ok(const conker_grid *g, int ns);
// Its workgroups per job (partial tiles: 2 M of them per workgroup column).
int fft_mm3_jobs_blocks(conker_ctx *ctx, int M);
// Inverse transforms of all ns radii of all M jobs (tspec: M ns spectra) and
// the order-3 summation on the fly: partial[(2 job + field) G + workgroup]
// 32 x 32 float64 tiles, G = fft_mm3_jobs_blocks.
int fft_inverse_mm3_jobs(conker_ctx *ctx, const conker_grid *g, int M, const ClassJob *tab, const void *kspec, int ns,
                         const void *spec, void *tspec, const PackScale *scales, double *partial, conker_mmprec prec);
// The reduction and gather of W_delta and W_R of order 3 from such partials
// (full: 2 M 1024 (RED_S + 1) doubles).
int reduce3_jobs(conker_ctx *c, int M, const ClassJob *tab, int ns, int G, const double *partial, double *full);
// W_delta and W_R of order 3 of all M jobs from their maps (split arithmetic,
// n_radii <= 64), into tab[j].Wd / Wr.  ws: workspace of contract3_jobs_bytes.
size_t contract3_jobs_bytes(conker_ctx *c, const conker_grid *g, int M, int ns);
int contract3_jobs(conker_ctx *c, const conker_grid *g, int M, const ClassJob *tab, int ns, conker_mmprec prec,
                   void *ws);

// The context's PackScale (device memory, valid on the context's stream after
// the last packed forward transform).
inline const PackScale *pack_scale_dev(const conker_ctx *c) { return (const PackScale *)c->scal.p; }

// Device list of the 64-cell blocks (cells 64 k .. 64 k + 63) holding a cell
// where F != 0, ascending (blocks.hip): *list = int[*count], both in device
// memory in the context's workspace, valid until the next call.  nc % 16 == 0.
int block_list(conker_ctx *c, const void *F, bool f64, size_t nc, const int **list, const int **count);

// Axis order of map-free summations (order.hip): with the context's
// axis_order setting (0 auto, 1 as given, 2..6 a fixed permutation) and a
// cubic grid, copies the distinct non-NULL fields in[0 .. n_in) into the
// permuted layout and points out[k] at the copies; otherwise out = in.  With
// n_in = 4, in[2] and in[3] are the centre fields that decide the support.
// When the fields are permuted, *sup receives the line support of the
// permuted centre fields (from the same projections) and *have_sup is set;
// otherwise the caller computes it with support_lines.
int order_fields(conker_ctx *c, const conker_grid *g, bool f64, int ns, const void *const *in, int n_in,
                 const void **out, Support *sup, bool *have_sup);

// Radii per inverse batch given the bytes one radius's spectrum takes
// (conv.hip); fixed_bytes is the workspace needed beside the batch.
int batch_radii(conker_ctx *c, size_t per_radius_bytes, int n_radii, size_t fixed_bytes);
// Number of z-line tiles of the inverse z pass of this grid.
int fft_z_tiles(const conker_grid *g, bool f64);

}  // namespace conker
