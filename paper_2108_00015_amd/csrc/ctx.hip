// Context, workspace, error reporting, twiddle tables and the float64 ratio.
#include <cmath>
#include <cstdarg>
#include <cstring>

#include "common.h"

namespace {
thread_local std::string g_create_err;
}

namespace conker {

int fail(conker_ctx *ctx, int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_err = buf;
    return code;
}

int ws_reserve(conker_ctx *ctx, Buf &b, size_t bytes) {
    if (bytes <= b.bytes) return CONKER_OK;
    if (ctx->capturing)
        return fail(ctx, CONKER_ENOMEM, "workspace would grow to %zu bytes inside a graph capture", bytes);
    size_t next = ctx->ws_bytes - b.bytes + bytes;
    if (ctx->ws_cap && next > ctx->ws_cap)
        return fail(ctx, CONKER_ENOMEM, "workspace of %zu bytes needed, cap is %zu", next, ctx->ws_cap);
    if (b.p) {
        CK_HIP(ctx, hipStreamSynchronize(ctx->stream));
        // a captured batch replays kernels on this buffer's address: it is
        // dropped with the buffer (conker_batch_launch then reports that no
        // batch is captured)
        if (ctx->graph_exec) {
            CK_HIP(ctx, hipGraphExecDestroy(ctx->graph_exec));
            ctx->graph_exec = nullptr;
        }
        CK_HIP(ctx, hipFree(b.p));
        ctx->ws_bytes -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, CONKER_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    b.p = p;
    b.bytes = bytes;
    ctx->ws_bytes += bytes;
    return CONKER_OK;
}

// cos and sin of 2 pi t / L in float64, reduced to the first octant so that the
// eighth-turn symmetries of the table hold exactly.
static void unit_root(long t, long L, double *c, double *s) {
    // L is a multiple of 4.  theta = 2 pi t / L = q pi/2 + phi, phi in [0, pi/2).
    t %= L;
    if (t < 0) t += L;
    long q = (4 * t) / L;
    long u = t - q * (L / 4);
    double cp, sp;
    if (8 * u > L) {            // phi > pi/4: use the complementary angle
        double a = 2.0 * M_PI * (double)(L / 4 - u) / (double)L;
        cp = std::sin(a);
        sp = std::cos(a);
    } else {
        double a = 2.0 * M_PI * (double)u / (double)L;
        cp = std::cos(a);
        sp = std::sin(a);
    }
    switch (q) {
        case 0: *c = cp; *s = sp; break;
        case 1: *c = -sp; *s = cp; break;
        case 2: *c = -cp; *s = -sp; break;
        default: *c = sp; *s = -cp; break;
    }
}

int twiddles(conker_ctx *ctx, int L, bool f64, const void **out) {
    auto &tab = f64 ? ctx->tw64 : ctx->tw32;
    auto it = tab.find(L);
    if (it != tab.end()) {
        *out = it->second.p;
        return CONKER_OK;
    }
    std::vector<double> h(2 * (size_t)L);
    for (int t = 0; t < L; ++t) {
        double c, s;
        unit_root(t, L, &c, &s);
        h[2 * t] = c;
        h[2 * t + 1] = -s;     // exp(-2 pi i t / L)
    }
    Buf b;
    size_t bytes = (size_t)L * (f64 ? 16 : 8);
    CK_OK(ws_reserve(ctx, b, bytes));
    if (f64) {
        CK_HIP(ctx, hipMemcpy(b.p, h.data(), bytes, hipMemcpyHostToDevice));
    } else {
        std::vector<float> hf(2 * (size_t)L);
        for (size_t i = 0; i < hf.size(); ++i) hf[i] = (float)h[i];
        CK_HIP(ctx, hipMemcpy(b.p, hf.data(), bytes, hipMemcpyHostToDevice));
    }
    tab[L] = b;
    *out = b.p;
    return CONKER_OK;
}

int check_grid(conker_ctx *ctx, const conker_grid *g, bool need_fft) {
    if (!ctx) return CONKER_EINVAL;
    if (!g) return fail(ctx, CONKER_EINVAL, "grid is NULL");
    for (int k = 0; k < 3; ++k) {
        if (g->dims[k] <= 0) return fail(ctx, CONKER_EINVAL, "grid dims must be positive");
        if (need_fft && !fft_length_ok(g->dims[k]))
            return fail(ctx, CONKER_EUNSUPPORTED,
                        "axis length %d not supported (32, 64, 96, 128, 192, 256, 384, 512 or 1024)", g->dims[k]);
    }
    if ((double)g->dims[0] * g->dims[1] * g->dims[2] > (double)(1u << 30))
        return fail(ctx, CONKER_EUNSUPPORTED, "grid larger than 2^30 cells");
    if (!(g->cell > 0.0) || !std::isfinite(g->cell))
        return fail(ctx, CONKER_EINVAL, "cell size must be positive and finite");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(g->origin[k])) return fail(ctx, CONKER_EINVAL, "origin must be finite");
    return CONKER_OK;
}

int cu_count(conker_ctx *c) {
    if (c->n_cu <= 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || v <= 0)
            v = 256;
        c->n_cu = v;
    }
    return c->n_cu;
}

static hipEvent_t take_event(conker_ctx *c) {
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(conker_ctx *ctx, int k) : c(ctx), kind(k) {
    if (c && c->prof) {
        e0 = take_event(c);
        if (e0) (void)hipEventRecord(e0, c->stream);
    }
}

ProfScope::~ProfScope() {
    if (c && c->prof && e0) {
        hipEvent_t e1 = take_event(c);
        if (e1) {
            (void)hipEventRecord(e1, c->stream);
            c->recs.push_back({kind, e0, e1});
        } else {
            c->pool.push_back(e0);
        }
    }
}

static void recycle_records(conker_ctx *c) {
    for (auto &r : c->recs) {
        c->pool.push_back(r.e0);
        c->pool.push_back(r.e1);
    }
    c->recs.clear();
}

int shell_reach(double r) { return (int)std::ceil(r + 0.5) - 1; }

int check_shell(conker_ctx *ctx, const conker_grid *g, double r) {
    if (!(r >= 0.5) || !std::isfinite(r))
        return fail(ctx, CONKER_ERANGE, "shell radius %g cells is below half a cell", r);
    int M = shell_reach(r);
    int mn = g->dims[0];
    if (g->dims[1] < mn) mn = g->dims[1];
    if (g->dims[2] < mn) mn = g->dims[2];
    if (2 * M + 1 > mn)
        return fail(ctx, CONKER_ERANGE, "shell radius %g cells (reach %d) does not fit axis length %d", r, M, mn);
    return CONKER_OK;
}

}  // namespace conker

using namespace conker;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" int conker_create(conker_ctx **out, int device, void *stream, size_t cap) {
    if (!out) return fail(nullptr, CONKER_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0)
        return fail(nullptr, CONKER_EHIP, "no HIP device: %s", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, CONKER_EINVAL, "device %d out of range", device);
    e = hipSetDevice(device);
    if (e != hipSuccess) return fail(nullptr, CONKER_EHIP, "hipSetDevice: %s", hipGetErrorString(e));
    {
        const int st = noalloc_init(device);   // device current: its copy of the scratch array
        if (st != CONKER_OK) return st;
    }
    conker_ctx *c = new conker_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->ws_cap = cap;
    // the packed-pair scale and its partial sums: held for the context's life
    // (never regrown, so graphs may record its address); s = 1 until the first
    // packed forward transform
    e = hipMalloc(&c->scal.p, SCAL_BYTES);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(nullptr, CONKER_ENOMEM, "hipMalloc(%zu) failed: %s", SCAL_BYTES, hipGetErrorString(e));
    }
    c->scal.bytes = SCAL_BYTES;
    const PackScale one{1.0, 1.0, 1.0f, 1.0f, 0, 0};
    e = hipMemcpy(c->scal.p, &one, sizeof one, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(c->scal.p);
        delete c;
        return fail(nullptr, CONKER_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    *out = c;
    return CONKER_OK;
}

extern "C" void conker_destroy(conker_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    auto rel = [](Buf &b) {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    };
    for (auto &kv : c->tw32) rel(kv.second);
    for (auto &kv : c->tw64) rel(kv.second);
    for (auto &kv : c->tables) rel(kv.second);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    recycle_records(c);
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    c->pool.clear();
    rel(c->spec);
    rel(c->tspec);
    rel(c->cls);
    rel(c->partial);
    rel(c->full);
    rel(c->support);
    rel(c->scales);
    rel(c->cosmo);
    rel(c->order);
    rel(c->bins);
    rel(c->blocks);
    rel(c->maps);
    rel(c->scal);
    delete c;
}

extern "C" int conker_set_stream(conker_ctx *c, void *stream) {
    if (!c) return CONKER_EINVAL;
    c->stream = (hipStream_t)stream;
    return CONKER_OK;
}

extern "C" const char *conker_last_error(const conker_ctx *c) {
    return c ? c->err.c_str() : g_create_err.c_str();
}

extern "C" size_t conker_workspace_bytes(const conker_ctx *c) { return c ? c->ws_bytes : 0; }

extern "C" int conker_synchronize(conker_ctx *c) {
    if (!c) return CONKER_EINVAL;
    CK_HIP(c, hipStreamSynchronize(c->stream));
    return CONKER_OK;
}

extern "C" int conker_profile_enable(conker_ctx *c, int enable) {
    if (!c) return CONKER_EINVAL;
    CK_HIP(c, hipStreamSynchronize(c->stream));
    recycle_records(c);
    c->prof = enable != 0;
    return CONKER_OK;
}

extern "C" int conker_profile_read(conker_ctx *c, int kind, int64_t *launches, double *total_ms) {
    if (!c) return CONKER_EINVAL;
    if (kind < 0 || kind >= PK_COUNT || !launches || !total_ms)
        return fail(c, CONKER_EINVAL, "bad profile kind or NULL pointer");
    CK_HIP(c, hipStreamSynchronize(c->stream));
    int64_t n = 0;
    double ms = 0.0;
    for (auto &r : c->recs) {
        if (r.kind != kind) continue;
        float t = 0.f;
        CK_HIP(c, hipEventElapsedTime(&t, r.e0, r.e1));
        ms += t;
        ++n;
    }
    *launches = n;
    *total_ms = ms;
    return CONKER_OK;
}

extern "C" const char *conker_profile_kind_name(int kind) {
    static const char *names[PK_COUNT] = {
        "scatter", "form_delta", "fft_fwd_z", "fft_fwd_y", "fft_fwd_x", "fft_inv_x_mul", "fft_inv_y",
        "fft_inv_z", "bank_z", "bank_y", "bank_x", "contract_dot", "contract_mm", "contract_reduce", "ratio",
        "fused_zinv_contract", "diag_zinv", "diag_maps", "diag_reduce", "support", "pair_spectral", "survey_front_end",
        "axis_order", "cell_blocks", "pack_scale", "pack_scale_reduce"};
    return (kind >= 0 && kind < PK_COUNT) ? names[kind] : nullptr;
}

extern "C" int64_t conker_num_tuples(int n_radii, int n) {
    if (n < 2 || n_radii < 0) return -1;
    // C(n_radii + n - 2, n - 1)
    int64_t k = n - 1, top = n_radii + n - 2;
    int64_t r = 1;
    for (int64_t i = 1; i <= k; ++i) r = r * (top - k + i) / i;
    return r;
}

extern "C" int conker_shell_size(double r, int64_t *out) {
    if (!out) return CONKER_EINVAL;
    if (!(r >= 0.5) || !std::isfinite(r)) return CONKER_ERANGE;
    int M = shell_reach(r);
    double lo = (r - 0.5) * (r - 0.5), hi = (r + 0.5) * (r + 0.5);
    int64_t cnt = 0;
    for (int x = -M; x <= M; ++x)
        for (int y = -M; y <= M; ++y)
            for (int z = -M; z <= M; ++z) {
                double d2 = (double)(x * x + y * y + z * z);
                if (d2 >= lo && d2 < hi) ++cnt;
            }
    *out = cnt;
    return CONKER_OK;
}

extern "C" int64_t conker_kspec_elems(const conker_grid *g) {
    if (!g) return -1;
    return (int64_t)(g->dims[0] / 2 + 1) * (g->dims[1] / 2 + 1) * (g->dims[2] / 2 + 1);
}

// ---------------------------------------------------------------------------
// estimator ratio (float64)
// ---------------------------------------------------------------------------
__global__ void k_ratio(const double *Wd, const double *Wr, const double *alpha, int n,
                        int64_t count, double *xi) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double a = *alpha, an = 1.0;
    for (int k = 0; k < n; ++k) an *= a;
    xi[i] = Wd[i] / (an * Wr[i]);
}

// Size classes: the ratio of every job of the table (job = blockIdx.y).
__global__ void k_ratio_jobs(const ClassJob *__restrict__ tab, int n, int64_t count) {
    const ClassJob &j = tab[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double a = *j.alpha, an = 1.0;
    for (int k = 0; k < n; ++k) an *= a;
    j.xi[i] = j.Wd[i] / (an * j.Wr[i]);
}

namespace conker {
int ratio_jobs(conker_ctx *c, int M, const ClassJob *tab, int n, int64_t count) {
    if (count <= 0) return CONKER_OK;
    ProfScope ps(c, PK_RATIO);
    hipLaunchKernelGGL(k_ratio_jobs, dim3((unsigned)((count + 255) / 256), (unsigned)M), dim3(256), 0, c->stream,
                       tab, n, count);
    CK_LAUNCH(c);
    return CONKER_OK;
}
}  // namespace conker

extern "C" int conker_ratio(conker_ctx *c, const double *Wd, const double *Wr, const double *alpha,
                            int n, int64_t count, double *xi) {
    if (!c) return CONKER_EINVAL;
    if (!Wd || !Wr || !alpha || !xi) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (n < 2 || n > 5) return fail(c, CONKER_EINVAL, "order n=%d outside 2..5", n);
    if (count < 0) return fail(c, CONKER_EINVAL, "negative count");
    if (count == 0) return CONKER_OK;
    CK_HIP(c, hipSetDevice(c->device));
    int threads = 256;
    int64_t blocks = (count + threads - 1) / threads;
    ProfScope ps(c, PK_RATIO);
    hipLaunchKernelGGL(k_ratio, dim3((unsigned)blocks), dim3(threads), 0, c->stream, Wd, Wr, alpha, n,
                       count, xi);
    CK_LAUNCH(c);
    return CONKER_OK;
}
