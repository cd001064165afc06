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

// Whether an axis of the grid has a second radix schedule (conker_tune::radix).
bool has_alt_radix(const conker_grid &g) {
    for (int a = 0; a < 3; ++a) {
        const int L = g.dims[a];
        if (L == 64 || L == 128 || L == 256 || L == 1024) return true;
    }
    return false;
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

// ---------------------------------------------------------------------------
// Size classes.  Jobs on one grid (dimensions, origin and cell), with one
// kernel bank and number of radii (at most 64), float32, order 3, split
// summation, and buffers that no other job of the class touches, run stage
// by stage: each stage is one launch for a chunk of such jobs, the job in the
// grid's y (or z) index and its buffers in a device table (ClassJob).  The
// stages are those of the job-by-job path (mapping binned by brick where the
// grid splits into bricks, packed forward transform, resident first inverse
// pass, radii in batches of CLASS_NB, matrix-core summation from stored
// maps, or the last inverse pass and the summation fused where no job wants
// its maps).  A chunk's workspace (spectra, radius-batch spectra, the maps
// of jobs that give none, scales, partial sums) is at most CLASS_WS bytes, so
// a class of large grids runs in several chunks; a class whose chunks would
// hold one job each, and every other job, runs job by job.
// ---------------------------------------------------------------------------
constexpr size_t CLASS_WS = (size_t)16 << 30;
constexpr int CLASS_NB = 8;

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

struct ChunkLayout {
    size_t spec, tspec, maps, scales, part, c3, full3, bins, bytes;
};

int64_t points_of(const conker_ctx *c, const std::vector<int> &js) {
    int64_t n = 0;
    for (int k : js) n += c->jobs[k].n_data + c->jobs[k].n_rand;
    return n;
}

// fused: all n_radii spectra at once, no maps, partial tiles of the fused
// summation; else nb spectra at once, maps of the jobs that give none.
ChunkLayout chunk_layout(conker_ctx *c, const conker_job &j0, int M, int nb, bool maps, bool fused,
                         int64_t n_total) {
    const size_t nc = ncells(&j0.grid);
    const int ns = j0.n_radii;
    ChunkLayout L;
    L.spec = 0;
    L.tspec = L.spec + up256((size_t)M * nc * 8);
    L.maps = L.tspec + up256((size_t)M * (fused ? ns : nb) * nc * 8);
    L.scales = L.maps + (maps && !fused ? up256((size_t)M * 2 * ns * nc * 4) : 0);
    L.part = L.scales + up256((size_t)M * sizeof(PackScale));
    L.c3 = L.part + up256(((size_t)4 * cu_count(c) + M) * 2 * sizeof(double));
    if (fused) {
        L.full3 = L.c3 + up256((size_t)2 * M * fft_mm3_jobs_blocks(c, M) * 1024 * sizeof(double));
        L.bytes = L.full3 + up256((size_t)2 * M * 1024 * (64 + 1) * sizeof(double));
    } else {
        L.full3 = L.c3;
        L.bytes = L.c3 + up256(contract3_jobs_bytes(c, &j0.grid, M, ns));
    }
    L.bins = L.bytes;   // binned mapping (none where the grid does not split into its bricks)
    L.bytes += up256(map_jobs_bytes(&j0.grid, M, n_total));
    return L;
}

bool class_ok(const conker_job &j) {
    const size_t nc = ncells(&j.grid);
    const bool aligned = (((uintptr_t)j.d_N | (uintptr_t)j.d_R) & 15) == 0;
    return j.dtype == CONKER_F32 && j.n == 3 &&
           (j.prec == CONKER_MM_SPLIT_BF16 || j.prec == CONKER_MM_SPLIT_F16 || j.prec == CONKER_MM_F32) &&
           j.n_radii <= 64 && nc % 64 == 0 && aligned && fft_jobs_ok(&j.grid);
}

// Device byte ranges a job writes or owns (grids, maps, outputs).
void job_ranges(const conker_job &j, std::vector<std::pair<uintptr_t, uintptr_t>> &out) {
    const size_t nc = ncells(&j.grid), ns = j.n_radii;
    const size_t cnt = (size_t)conker_num_tuples(j.n_radii, j.n);
    auto add = [&](const void *p, size_t b) {
        if (p && b) out.push_back({(uintptr_t)p, (uintptr_t)p + b});
    };
    add(j.d_N, nc * 4);
    add(j.d_R, nc * 4);
    add(j.d_maps_N, ns * nc * 4);
    add(j.d_maps_R, ns * nc * 4);
    add(j.d_wsum, 2 * sizeof(double));
    add(j.d_n_outside, 2 * sizeof(int64_t));
    add(j.d_alpha, sizeof(double));
    add(j.d_W_delta, cnt * 8);
    add(j.d_W_rand, cnt * 8);
    add(j.d_xi, cnt * 8);
}

bool overlaps(const std::vector<std::pair<uintptr_t, uintptr_t>> &a,
              const std::vector<std::pair<uintptr_t, uintptr_t>> &b) {
    for (const auto &x : a)
        for (const auto &y : b)
            if (x.first < y.second && y.first < x.second) return true;
    return false;
}

// Splits the planned batch into chunks of size classes and jobs run alone,
// reserves conker_ctx::cls and writes the chunks' tables.
int plan_classes(conker_ctx *c) {
    c->chunks.clear();
    c->seq_jobs.clear();
    const int nj = (int)c->jobs.size();
    std::vector<int> seq;
    std::vector<std::vector<int>> groups;
    if (c->batch_classes) {
        using Key = std::tuple<int, int, int, double, double, double, double, const void *, int, int>;
        std::map<Key, size_t> where;
        for (int k = 0; k < nj; ++k) {
            const conker_job &j = c->jobs[k];
            if (!class_ok(j)) {
                seq.push_back(k);
                continue;
            }
            const Key key{j.grid.dims[0], j.grid.dims[1], j.grid.dims[2], j.grid.origin[0], j.grid.origin[1],
                          j.grid.origin[2], j.grid.cell, j.d_kspec, j.n_radii, (int)j.prec};
            auto it = where.find(key);
            if (it == where.end()) {
                where[key] = groups.size();
                groups.push_back({k});
            } else {
                groups[it->second].push_back(k);
            }
        }
    } else {
        for (int k = 0; k < nj; ++k) seq.push_back(k);
    }
    size_t tab_bytes = 0, ws_max = 0;
    for (const auto &grp : groups) {
        // members whose buffers no earlier member touches
        std::vector<int> mem;
        std::vector<std::pair<uintptr_t, uintptr_t>> held;
        for (int k : grp) {
            std::vector<std::pair<uintptr_t, uintptr_t>> r;
            job_ranges(c->jobs[k], r);
            if (overlaps(r, held)) {
                seq.push_back(k);
                continue;
            }
            held.insert(held.end(), r.begin(), r.end());
            mem.push_back(k);
        }
        const conker_job &j0 = c->jobs[grp[0]];
        const int nb = std::min(j0.n_radii, CLASS_NB);
        // maps wanted by no member, split bfloat16 or float32: the fused summation where the grid allows
        bool fused = (j0.prec == CONKER_MM_SPLIT_BF16 || j0.prec == CONKER_MM_F32) &&
                     fft_mm3_jobs_ok(&j0.grid, j0.n_radii);
        for (int k : mem) fused = fused && c->jobs[k].d_maps_N == nullptr;
        if (j0.prec == CONKER_MM_F32 && !fused) {   // the stored-map class summation is split-only
            for (int k : mem) seq.push_back(k);
            continue;
        }
        // greedy chunks under the workspace bound
        std::vector<ClassChunk> mine;
        ClassChunk cur;
        cur.nb = nb;
        cur.fused = fused;
        auto bytes_of = [&](const std::vector<int> &js) {
            bool maps = false;
            for (int k : js) maps = maps || c->jobs[k].d_maps_N == nullptr;
            return chunk_layout(c, j0, (int)js.size(), nb, maps, fused, points_of(c, js)).bytes;
        };
        for (int k : mem) {
            std::vector<int> t = cur.jobs;
            t.push_back(k);
            if (!cur.jobs.empty() && bytes_of(t) > CLASS_WS) {
                mine.push_back(cur);
                cur.jobs.clear();
                t = {k};
            }
            cur.jobs = t;
        }
        if (!cur.jobs.empty()) mine.push_back(cur);
        size_t most = 0;
        for (const auto &ch : mine) most = std::max(most, ch.jobs.size());
        if (mem.empty() || most < 2 || bytes_of({mine[0].jobs[0]}) > CLASS_WS) {   // nothing shared: job by job
            for (int k : mem) seq.push_back(k);
            continue;
        }
        for (auto &ch : mine) {
            ch.tab_off = tab_bytes;
            tab_bytes += up256(ch.jobs.size() * sizeof(ClassJob));
            ws_max = std::max(ws_max, bytes_of(ch.jobs));
            c->chunks.push_back(ch);
        }
    }
    if (!c->chunks.empty()) {
        const int st = ws_reserve(c, c->cls, tab_bytes + ws_max);
        if (st != CONKER_OK) {   // no room: every job runs alone
            if (st != CONKER_ENOMEM) return st;
            c->err.clear();
            for (const auto &ch : c->chunks) seq.insert(seq.end(), ch.jobs.begin(), ch.jobs.end());
            c->chunks.clear();
        }
    }
    c->cls_ws_off = tab_bytes;
    std::sort(seq.begin(), seq.end());
    c->seq_jobs = seq;
    for (const auto &ch : c->chunks) {
        const conker_job &j0 = c->jobs[ch.jobs[0]];
        const int M = (int)ch.jobs.size();
        bool maps = false;
        for (int k : ch.jobs) maps = maps || c->jobs[k].d_maps_N == nullptr;
        const ChunkLayout L = chunk_layout(c, j0, M, ch.nb, maps, ch.fused, points_of(c, ch.jobs));
        const size_t nc = ncells(&j0.grid), ns = j0.n_radii;
        char *ws = (char *)c->cls.p + c->cls_ws_off;
        std::vector<ClassJob> tab(M);
        int64_t ioff = 0;
        for (int i = 0; i < M; ++i) {
            const conker_job &j = c->jobs[ch.jobs[i]];
            ClassJob &t = tab[i];
            t.N = (float *)j.d_N;
            t.R = (float *)j.d_R;
            if (ch.fused) {
                t.mapsN = t.mapsR = nullptr;
            } else if (j.d_maps_N) {
                t.mapsN = (float *)j.d_maps_N;
                t.mapsR = (float *)j.d_maps_R;
            } else {
                t.mapsN = (float *)(ws + L.maps) + (size_t)i * 2 * ns * nc;
                t.mapsR = t.mapsN + ns * nc;
            }
            t.dpos = j.d_data_pos;
            t.dw = j.d_data_w;
            t.rpos = j.d_rand_pos;
            t.rw = j.d_rand_w;
            t.nd = j.n_data;
            t.nr = j.n_rand;
            t.ioff_d = ioff;
            ioff += j.n_data;
            t.ioff_r = ioff;
            ioff += j.n_rand;
            t.wsum = j.d_wsum;
            t.nout = (long long *)j.d_n_outside;
            t.alpha = j.d_alpha;
            t.Wd = j.d_W_delta;
            t.Wr = j.d_W_rand;
            t.xi = j.d_xi;
        }
        CK_HIP(c, hipMemcpyAsync((char *)c->cls.p + ch.tab_off, tab.data(), M * sizeof(ClassJob),
                                 hipMemcpyHostToDevice, c->stream));
    }
    CK_HIP(c, hipStreamSynchronize(c->stream));
    return CONKER_OK;
}

int run_chunk(conker_ctx *c, const ClassChunk &ch) {
    const conker_job &j0 = c->jobs[ch.jobs[0]];
    const int M = (int)ch.jobs.size(), ns = j0.n_radii;
    bool maps = false;
    int64_t n_max = 0;
    for (int k : ch.jobs) {
        maps = maps || c->jobs[k].d_maps_N == nullptr;
        n_max = std::max({n_max, c->jobs[k].n_data, c->jobs[k].n_rand});
    }
    const int64_t n_total = points_of(c, ch.jobs);
    const ChunkLayout L = chunk_layout(c, j0, M, ch.nb, maps, ch.fused, n_total);
    const ClassJob *tab = (const ClassJob *)((const char *)c->cls.p + ch.tab_off);
    char *ws = (char *)c->cls.p + c->cls_ws_off;
    PackScale *scales = (PackScale *)(ws + L.scales);
    int sums_G = 0;
    CK_OK(map_jobs(c, &j0.grid, M, tab, n_max, n_total, L.bytes > L.bins ? ws + L.bins : nullptr,
                   (double *)(ws + L.part), &sums_G));
    CK_OK(fft_forward_jobs(c, &j0.grid, M, tab, ws + L.spec, scales, (const double *)(ws + L.part), sums_G));
    if (ch.fused) {
        CK_OK(fft_inverse_mm3_jobs(c, &j0.grid, M, tab, j0.d_kspec, ns, ws + L.spec, ws + L.tspec, scales,
                                   (double *)(ws + L.c3), j0.prec));
        CK_OK(reduce3_jobs(c, M, tab, ns, fft_mm3_jobs_blocks(c, M), (const double *)(ws + L.c3),
                           (double *)(ws + L.full3)));
        return ratio_jobs(c, M, tab, 3, conker_num_tuples(ns, 3));
    }
    for (int m0 = 0; m0 < ns; m0 += ch.nb)
        CK_OK(fft_inverse_jobs(c, &j0.grid, M, tab, j0.d_kspec, m0, std::min(ch.nb, ns - m0), ws + L.spec,
                               ws + L.tspec, scales));
    CK_OK(contract3_jobs(c, &j0.grid, M, tab, ns, j0.prec, ws + L.c3));
    return ratio_jobs(c, M, tab, 3, conker_num_tuples(ns, 3));
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
    for (const auto &ch : c->chunks) {
        TuneScope ts(c, ch.tuned ? ch.tune : c->user_tune);
        CK_OK(run_chunk(c, ch));
    }
    for (int k : c->seq_jobs) {
        TuneScope ts(c, tune_of(c, k));
        CK_OK(run_job(c, c->jobs[k]));
    }
    return CONKER_OK;
}

bool tune_ok(const conker_tune &t) {
    auto in = [](int v, int lo, int hi) { return v >= lo && v <= hi; };
    return in(t.x_tile, 0, 2) && in(t.y_tile, 0, 2) && in(t.x_resident, 0, 3) && in(t.mm_kernel, 0, 3) &&
           in(t.radius_batch, 0, 64) && in(t.axis_order, 0, 6) && in(t.radix, 0, 2);
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
    if (j.dtype == CONKER_F32 && has_alt_radix(j.grid)) knobs.push_back({&conker_tune::radix, {2}});
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

// Time of one run of a chunk with setting t (the minimum of reps after one
// untimed run); infinity where it fails for lack of memory.
int time_chunk(conker_ctx *c, const ClassChunk &ch, const conker_tune &t, int reps, hipEvent_t e0, hipEvent_t e1,
               float *ms) {
    TuneScope ts(c, t);
    int st = run_chunk(c, ch);
    if (st == CONKER_ENOMEM) {
        (void)hipGetLastError();
        CK_HIP(c, hipStreamSynchronize(c->stream));
        c->err.clear();
        *ms = 3.0e38f;
        return CONKER_OK;
    }
    CK_OK(st);
    float best = 3.0e38f;
    for (int r = 0; r < reps; ++r) {
        CK_HIP(c, hipEventRecord(e0, c->stream));
        CK_OK(run_chunk(c, ch));
        CK_HIP(c, hipEventRecord(e1, c->stream));
        CK_HIP(c, hipEventSynchronize(e1));
        float v = 0.f;
        CK_HIP(c, hipEventElapsedTime(&v, e0, e1));
        best = std::min(best, v);
    }
    *ms = best;
    return CONKER_OK;
}

// A chunk's sweep, as tune_job's: the tiles of the column passes and the
// radix schedule (the other fields do not apply to the class stages).
int tune_chunk(conker_ctx *c, const ClassChunk &ch, int reps, hipEvent_t e0, hipEvent_t e1, conker_tune *out) {
    const conker_job &j0 = c->jobs[ch.jobs[0]];
    conker_tune best = c->user_tune;
    float best_ms;
    CK_OK(time_chunk(c, ch, best, reps, e0, e1, &best_ms));
    struct Knob {
        int32_t conker_tune::*field;
        std::vector<int> alt;
    };
    std::vector<Knob> knobs = {{&conker_tune::y_tile, {1, 2}}, {&conker_tune::x_tile, {1, 2}}};
    if (has_alt_radix(j0.grid)) knobs.push_back({&conker_tune::radix, {2}});
    for (const auto &k : knobs) {
        const int start = best.*(k.field);
        for (int v : k.alt) {
            if (v == start) continue;
            conker_tune cand = best;
            cand.*(k.field) = v;
            float ms;
            CK_OK(time_chunk(c, ch, cand, reps, e0, e1, &ms));
            if (ms < 0.99f * best_ms) {
                best = cand;
                best_ms = ms;
            }
        }
    }
    if (!(best_ms < 1.0e38f)) return fail(c, CONKER_ENOMEM, "no launch setting of the chunk fits in memory");
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
    c->chunks.clear();
    c->seq_jobs.clear();
    const int st = plan_classes(c);
    if (st != CONKER_OK) {
        c->jobs.clear();
        return st;
    }
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

extern "C" int conker_batch_classes(conker_ctx *c, int on) {
    if (!c) return CONKER_EINVAL;
    c->batch_classes = on != 0;
    return CONKER_OK;
}

extern "C" int conker_batch_layout(const conker_ctx *c, int *h_chunk) {
    if (!c || !h_chunk) return CONKER_EINVAL;
    for (size_t k = 0; k < c->jobs.size(); ++k) h_chunk[k] = -1;
    for (size_t q = 0; q < c->chunks.size(); ++q)
        for (int k : c->chunks[q].jobs) h_chunk[k] = (int)q;
    return CONKER_OK;
}

extern "C" int conker_set_tune(conker_ctx *c, const conker_tune *t) {
    if (!c) return CONKER_EINVAL;
    conker_tune v{};
    if (t) v = *t;
    v.ms = 0.f;
    if (!tune_ok(v))
        return fail(c, CONKER_EINVAL,
                    "launch setting out of range (tiles 0..2, resident 0..3, kernel 0..3; radius batch 0..64; axis order "
                    "0..6; radix 0..2)");
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
    std::vector<conker_tune> chosen(c->jobs.size(), c->user_tune);
    for (auto &ch : c->chunks) {   // a chunk's setting, reported for each of its jobs with the time per job
        ch.tuned = false;
        if (st != CONKER_OK) break;
        conker_tune t;
        st = tune_chunk(c, ch, reps, e0, e1, &t);
        if (st != CONKER_OK) break;
        ch.tune = t;
        ch.tuned = true;
        for (int k : ch.jobs) {
            chosen[k] = t;
            chosen[k].ms = t.ms / (float)ch.jobs.size();
        }
    }
    for (size_t q = 0; q < c->seq_jobs.size() && st == CONKER_OK; ++q) {
        const size_t k = (size_t)c->seq_jobs[q];
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
        for (auto &ch : c->chunks) ch.tuned = false;
        return st;
    }
    c->job_tune = chosen;
    // outputs and workspace as the chosen settings leave them
    CK_OK(run_all(c));
    CK_HIP(c, hipStreamSynchronize(c->stream));
    if (h_chosen) std::memcpy(h_chosen, chosen.data(), chosen.size() * sizeof(conker_tune));
    return CONKER_OK;
}
