// Batches of independent catalogs (mock catalogs, survey regions): each job is
// the whole path -- mapping, convolution, summation, ratio -- on its own grid
// and kernel bank.  The batch is planned once (validation, and one eager run
// that allocates every workspace buffer and table the jobs need), then can be
// run eagerly again, or captured into one HIP graph and replayed.  Regions or
// mocks are combined afterwards by adding numerators and denominators
// (Eq. ksi3combined).
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "common.h"

using namespace conker;

namespace {

// Zeroes a buffer with a kernel (graph-safe, unlike a memset node).
__global__ void k_zero(unsigned long long *__restrict__ p, size_t n_words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

int zero_bytes(conker_ctx *c, void *p, size_t bytes) {
    if (bytes % 8) return fail(c, CONKER_EINVAL, "zeroed buffers must be a multiple of 8 bytes");
    const size_t words = bytes / 8;
    const int threads = 256;
    const size_t want = (words + threads - 1) / threads;
    const int blocks = (int)(want < 4096 ? (want ? want : 1) : 4096);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(threads), 0, c->stream, (unsigned long long *)p, words);
    CK_LAUNCH(c);
    return CONKER_OK;
}

bool fused_ok(const conker_job &j) {
    return j.dtype == CONKER_F32 && (j.prec == CONKER_MM_F32 || j.prec == CONKER_MM_SPLIT_BF16) &&
           (j.n == 2 || j.n == 3) && j.grid.dims[2] == 512 && j.n_radii >= 1 && j.n_radii <= 30;
}

int run_job(conker_ctx *c, const conker_job &j) {
    const size_t esz = j.dtype == CONKER_F64 ? 8 : 4;
    const size_t nc = ncells(&j.grid);
    CK_OK(zero_bytes(c, j.d_N, nc * esz));
    CK_OK(zero_bytes(c, j.d_R, nc * esz));
    CK_OK(zero_bytes(c, j.d_wsum, 2 * sizeof(double)));
    CK_OK(zero_bytes(c, j.d_n_outside, 2 * sizeof(int64_t)));
    CK_OK(conker_grid_assign(c, &j.grid, j.d_data_pos, j.d_data_w, j.n_data, j.dtype, j.d_N, j.d_wsum,
                             j.d_n_outside));
    CK_OK(conker_grid_assign(c, &j.grid, j.d_rand_pos, j.d_rand_w, j.n_rand, j.dtype, j.d_R, j.d_wsum + 1,
                             j.d_n_outside + 1));
    CK_OK(conker_form_delta(c, &j.grid, j.dtype, j.d_N, j.d_R, j.d_wsum, j.d_wsum + 1, j.d_alpha));
    if (!j.d_maps_N) {
        CK_OK(conker_convolve_contract(c, &j.grid, j.dtype, j.d_N, j.d_R, j.d_kspec, j.n_radii, j.n, j.prec,
                                       j.d_W_delta, j.d_W_rand));
    } else {
        CK_OK(conker_convolve_shells(c, &j.grid, j.dtype, j.d_N, j.d_R, j.d_kspec, j.n_radii, j.d_maps_N,
                                     j.d_maps_R));
        CK_OK(conker_contract_npt(c, &j.grid, j.dtype, j.d_N, j.d_maps_N, j.n_radii, j.n, j.prec, j.d_W_delta));
        CK_OK(conker_contract_npt(c, &j.grid, j.dtype, j.d_R, j.d_maps_R, j.n_radii, j.n, j.prec, j.d_W_rand));
    }
    const int64_t cnt = conker_num_tuples(j.n_radii, j.n);
    CK_OK(conker_ratio(c, j.d_W_delta, j.d_W_rand, j.d_alpha, j.n, cnt, j.d_xi));
    return CONKER_OK;
}

// Launch shapes of job k while it is enqueued; the context setting again after.
struct TuneScope {
    conker_ctx *c;
    TuneScope(conker_ctx *ctx, const conker_tune &t) : c(ctx) { c->tune = t; }
    ~TuneScope() { c->tune = c->user_tune; }
};

const conker_tune &tune_of(const conker_ctx *c, size_t k) {
    return c->job_tune.size() == c->jobs.size() ? c->job_tune[k] : c->user_tune;
}

int run_all(conker_ctx *c) {
    for (size_t k = 0; k < c->jobs.size(); ++k) {
        TuneScope ts(c, tune_of(c, k));
        CK_OK(run_job(c, c->jobs[k]));
    }
    return CONKER_OK;
}

bool tune_ok(const conker_tune &t) {
    auto in = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
    return in(t.x_tile, 0, 2) && in(t.y_tile, 0, 2) && in(t.x_resident, 0, 3) && in(t.mm_kernel, 0, 3) &&
           in(t.radius_batch, 0, 64) && in(t.axis_order, 0, 6);
}

// Shortest of `reps` timed runs of job j with setting t (after one untimed run
// that also grows any workspace the setting needs).  Infeasible settings
// (workspace above the cap or the device's memory) time as infinity.
int time_job(conker_ctx *c, const conker_job &j, const conker_tune &t, int reps, hipEvent_t e0, hipEvent_t e1,
             float *ms) {
    TuneScope ts(c, t);
    int st = run_job(c, j);
    if (st == CONKER_ENOMEM) {
        (void)hipGetLastError();   // a failed allocation leaves its status behind
        CK_HIP(c, hipStreamSynchronize(c->stream));
        c->err.clear();
        *ms = 3.0e38f;
        return CONKER_OK;
    }
    CK_OK(st);
    float best = 3.0e38f;
    for (int r = 0; r < reps; ++r) {
        CK_HIP(c, hipEventRecord(e0, c->stream));
        CK_OK(run_job(c, j));
        CK_HIP(c, hipEventRecord(e1, c->stream));
        CK_HIP(c, hipEventSynchronize(e1));
        float v = 0.f;
        CK_HIP(c, hipEventElapsedTime(&v, e0, e1));
        best = std::min(best, v);
    }
    *ms = best;
    return CONKER_OK;
}

// One sweep over the fields: keep an alternative when it beats the best time
// so far by more than 1 % (timing noise keeps the earlier choice).
int tune_job(conker_ctx *c, const conker_job &j, int reps, hipEvent_t e0, hipEvent_t e1, conker_tune *out) {
    conker_tune best = c->user_tune;
    float best_ms;
    CK_OK(time_job(c, j, best, reps, e0, e1, &best_ms));
    const bool nomaps = j.d_maps_N == nullptr;   // conker_convolve_contract
    const bool fused = nomaps && fused_ok(j);     // ... with its fused kernel
    const int slots = j.n_radii;
    struct Knob {
        int32_t conker_tune::*field;
        std::vector<int> alt;
    };
    std::vector<Knob> knobs = {{&conker_tune::y_tile, {1, 2}},
                               {&conker_tune::x_tile, {1, 2}},
                               {&conker_tune::x_resident, {1, 2, 3}}};
    if (!fused && j.n >= 3 && j.prec != CONKER_MM_F64)
        knobs.push_back({&conker_tune::mm_kernel,
                         (j.n == 3 && j.prec != CONKER_MM_F32) ? std::vector<int>{1, 2, 3} : std::vector<int>{1, 2}});
    if (nomaps && j.grid.dims[0] == j.grid.dims[1] && j.grid.dims[1] == j.grid.dims[2])
        knobs.push_back({&conker_tune::axis_order, {1}});   // the given order against the chosen one
    if (!fused && slots >= 4) {
        std::vector<int> rb = {(slots + 1) / 2};
        if (slots >= 8) rb.push_back((slots + 3) / 4);
        knobs.push_back({&conker_tune::radius_batch, rb});
    }
    for (const auto &k : knobs) {
        const int start = best.*(k.field);
        for (int v : k.alt) {
            if (v == start) continue;
            conker_tune cand = best;
            cand.*(k.field) = v;
            float ms;
            CK_OK(time_job(c, j, cand, reps, e0, e1, &ms));
            if (ms < 0.99f * best_ms) {
                best = cand;
                best_ms = ms;
            }
        }
    }
    if (!(best_ms < 1.0e38f)) return fail(c, CONKER_ENOMEM, "no launch setting of the job fits in memory");
    best.ms = best_ms;
    *out = best;
    return CONKER_OK;
}

int check_job(conker_ctx *c, const conker_job &j, int k) {
    CK_OK(check_grid(c, &j.grid, true));
    if (j.dtype != CONKER_F32 && j.dtype != CONKER_F64) return fail(c, CONKER_EINVAL, "job %d: bad dtype", k);
    if (j.n < 2 || j.n > 5) return fail(c, CONKER_EINVAL, "job %d: order %d outside 2..5", k, j.n);
    if (j.n_radii < 1 || j.n_radii > 64) return fail(c, CONKER_EINVAL, "job %d: n_radii outside 1..64", k);
    if (!j.d_kspec || !j.d_N || !j.d_R || !j.d_wsum || !j.d_n_outside || !j.d_alpha || !j.d_W_delta ||
        !j.d_W_rand || !j.d_xi || (j.n_data > 0 && !j.d_data_pos) || (j.n_rand > 0 && !j.d_rand_pos))
        return fail(c, CONKER_EINVAL, "job %d: NULL pointer", k);
    if ((j.d_maps_N == nullptr) != (j.d_maps_R == nullptr))
        return fail(c, CONKER_EINVAL, "job %d: maps_N and maps_R must both be given or both be NULL", k);
    return CONKER_OK;
}

}  // namespace

extern "C" int conker_batch_plan(conker_ctx *c, const conker_job *jobs, int n_jobs) {
    if (!c) return CONKER_EINVAL;
    if (!jobs || n_jobs <= 0) return fail(c, CONKER_EINVAL, "empty job list");
    for (int k = 0; k < n_jobs; ++k) CK_OK(check_job(c, jobs[k], k));
    CK_HIP(c, hipSetDevice(c->device));
    if (c->graph_exec) {
        CK_HIP(c, hipGraphExecDestroy(c->graph_exec));
        c->graph_exec = nullptr;
    }
    c->jobs.assign(jobs, jobs + n_jobs);
    c->job_tune.clear();
    // one eager pass allocates every buffer and table the jobs use
    CK_OK(run_all(c));
    CK_HIP(c, hipStreamSynchronize(c->stream));
    return CONKER_OK;
}

extern "C" int conker_batch_run(conker_ctx *c) {
    if (!c) return CONKER_EINVAL;
    if (c->jobs.empty()) return fail(c, CONKER_EINVAL, "no batch planned");
    CK_HIP(c, hipSetDevice(c->device));
    return run_all(c);
}

extern "C" int conker_batch_capture(conker_ctx *c) {
    if (!c) return CONKER_EINVAL;
    if (c->jobs.empty()) return fail(c, CONKER_EINVAL, "no batch planned");
    if (!c->stream) return fail(c, CONKER_EINVAL, "graph capture needs a context stream other than the default");
    CK_HIP(c, hipSetDevice(c->device));
    if (c->graph_exec) {
        CK_HIP(c, hipGraphExecDestroy(c->graph_exec));
        c->graph_exec = nullptr;
    }
    const bool prof = c->prof;
    c->prof = false;
    c->capturing = true;
    CK_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int st = run_all(c);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->capturing = false;
    c->prof = prof;
    if (st != CONKER_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(c, CONKER_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->graph_exec = nullptr;
        return fail(c, CONKER_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return CONKER_OK;
}

extern "C" int conker_batch_launch(conker_ctx *c) {
    if (!c) return CONKER_EINVAL;
    if (!c->graph_exec) return fail(c, CONKER_EINVAL, "no captured batch");
    CK_HIP(c, hipSetDevice(c->device));
    CK_HIP(c, hipGraphLaunch(c->graph_exec, c->stream));
    return CONKER_OK;
}

extern "C" int conker_set_tune(conker_ctx *c, const conker_tune *t) {
    if (!c) return CONKER_EINVAL;
    conker_tune v{};
    if (t) v = *t;
    v.ms = 0.f;
    if (!tune_ok(v))
        return fail(c, CONKER_EINVAL,
                    "launch setting out of range (tiles 0..2, resident 0..3, kernel 0..3; radius batch 0..64; axis order 0..6)");
    c->user_tune = v;
    c->tune = v;
    return CONKER_OK;
}

extern "C" int conker_get_tune(const conker_ctx *c, conker_tune *t) {
    if (!c || !t) return CONKER_EINVAL;
    *t = c->user_tune;
    return CONKER_OK;
}

extern "C" int conker_batch_autotune(conker_ctx *c, int reps, conker_tune *h_chosen) {
    if (!c) return CONKER_EINVAL;
    if (c->jobs.empty()) return fail(c, CONKER_EINVAL, "no batch planned");
    if (reps < 1 || reps > 16) return fail(c, CONKER_EINVAL, "reps %d outside 1..16", reps);
    CK_HIP(c, hipSetDevice(c->device));
    if (c->graph_exec) {   // recorded with the earlier settings
        CK_HIP(c, hipGraphExecDestroy(c->graph_exec));
        c->graph_exec = nullptr;
    }
    const bool prof = c->prof;
    c->prof = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess
                 ? CONKER_OK
                 : fail(c, CONKER_EHIP, "hipEventCreate failed");
    using Key = std::tuple<int, int, int, int, int, int, int, bool>;
    std::map<Key, conker_tune> seen;
    std::vector<conker_tune> chosen(c->jobs.size());
    for (size_t k = 0; k < c->jobs.size() && st == CONKER_OK; ++k) {
        const conker_job &j = c->jobs[k];
        const Key key{j.grid.dims[0], j.grid.dims[1], j.grid.dims[2], (int)j.dtype, (int)j.prec, j.n, j.n_radii,
                      j.d_maps_N == nullptr};
        auto it = seen.find(key);
        if (it != seen.end()) {
            chosen[k] = it->second;
            continue;
        }
        st = tune_job(c, j, reps, e0, e1, &chosen[k]);
        if (st == CONKER_OK) seen[key] = chosen[k];
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->prof = prof;
    c->tune = c->user_tune;
    if (st != CONKER_OK) {
        c->job_tune.clear();
        return st;
    }
    c->job_tune = chosen;
    // outputs and workspace as the chosen settings leave them
    CK_OK(run_all(c));
    CK_HIP(c, hipStreamSynchronize(c->stream));
    if (h_chosen) std::memcpy(h_chosen, chosen.data(), chosen.size() * sizeof(conker_tune));
    return CONKER_OK;
}
