// Batches of independent catalogs (mock catalogs, survey regions): each job is
// the whole path -- mapping, convolution, summation, ratio -- on its own grid
// and kernel bank.  The batch is planned once (validation, and one eager run
// that allocates every workspace buffer and table the jobs need), then can be
// run eagerly again, or captured into one HIP graph and replayed.  Regions or
// mocks are combined afterwards by adding numerators and denominators
// (Eq. ksi3combined).
#include <cstring>
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
    if (!j.d_maps_N && fused_ok(j)) {
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
    if (!j.d_maps_N && !fused_ok(j))
        return fail(c, CONKER_EINVAL, "job %d: maps are needed (the fused summation does not apply)", k);
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
    // one eager pass allocates every buffer and table the jobs use
    for (const auto &j : c->jobs) CK_OK(run_job(c, j));
    CK_HIP(c, hipStreamSynchronize(c->stream));
    return CONKER_OK;
}

extern "C" int conker_batch_run(conker_ctx *c) {
    if (!c) return CONKER_EINVAL;
    if (c->jobs.empty()) return fail(c, CONKER_EINVAL, "no batch planned");
    CK_HIP(c, hipSetDevice(c->device));
    for (const auto &j : c->jobs) CK_OK(run_job(c, j));
    return CONKER_OK;
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
    int st = CONKER_OK;
    for (const auto &j : c->jobs) {
        st = run_job(c, j);
        if (st != CONKER_OK) break;
    }
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
