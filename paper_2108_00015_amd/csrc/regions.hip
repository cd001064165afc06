// Regions, maps and distributions.
//
// * Several regions or mocks measured separately (for instance the two
//   galactic caps, Sec. 3.4) are combined by adding numerators and
//   denominators (Eq. ksi3combined): xi = sum_j W_delta_j / sum_j alpha_j^n W_R_j.
// * The maps keep the location information (Sec. 4.2): the per-cell map
//   W_0 W_1 / <B_0 B_1> of one radius is N(x) C^N(x) over the cell average of
//   alpha^2 R_raw C^R, i.e. alpha^2 W_R2 / N_c; its cell average is the 2pcf.
// * Distributions of map values: equal-width bins of [lo, hi) plus one bin
//   below and one at or above (NaN included), counted in integers, so the
//   result does not depend on scheduling.
#include "common.h"

using namespace conker;

namespace {

__global__ void k_ratio_combined(const double *__restrict__ Wd, const double *__restrict__ Wr,
                                 const double *__restrict__ alpha, int n_regions, int n, int64_t count,
                                 double *__restrict__ xi, double *__restrict__ num_out, double *__restrict__ den_out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    double num = 0.0, den = 0.0;
    for (int j = 0; j < n_regions; ++j) {
        double an = 1.0;
        for (int k = 0; k < n; ++k) an *= alpha[j];
        num += Wd[(size_t)j * count + t];
        den += an * Wr[(size_t)j * count + t];
    }
    xi[t] = num / den;
    if (num_out) num_out[t] = num;
    if (den_out) den_out[t] = den;
}

template <typename T>
__global__ __launch_bounds__(256) void k_map_ratio(const T *__restrict__ N, const T *__restrict__ C, size_t nc,
                                                   const double *WR2, const double *alpha, T *__restrict__ out) {
    const double a = *alpha;
    const double norm = a * a * (*WR2) / (double)nc;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride)
        out[i] = (T)((double)N[i] * (double)C[i] / norm);
}

__global__ void k_zero_i64(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Workgroup-private counts in LDS, added to the global counts once per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_value_hist(const T *__restrict__ v, size_t n, double lo, double hi,
                                                    int n_bins, unsigned long long *__restrict__ counts) {
    extern __shared__ unsigned int sh[];
    const int nb = n_bins + 2;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sh[b] = 0u;
    __syncthreads();
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double x = (double)v[i];
        int b;
        if (x >= lo && x < hi) {
            b = (int)floor((x - lo) / (hi - lo) * (double)n_bins);
            if (b > n_bins - 1) b = n_bins - 1;
        } else {
            b = x < lo ? n_bins : n_bins + 1;   // NaN fails both tests: above
        }
        atomicAdd(&sh[b], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        if (sh[b]) atomicAdd(&counts[b], (unsigned long long)sh[b]);
}

}  // namespace

extern "C" int conker_ratio_combined(conker_ctx *c, int n_regions, const double *Wd, const double *Wr,
                                     const double *alpha, int n, int64_t count, double *xi, double *num,
                                     double *den) {
    if (!c) return CONKER_EINVAL;
    if (n_regions < 1) return fail(c, CONKER_EINVAL, "n_regions must be positive");
    if (!Wd || !Wr || !alpha || !xi) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (n < 2 || n > 5) return fail(c, CONKER_EINVAL, "order n=%d outside 2..5", n);
    if (count < 0) return fail(c, CONKER_EINVAL, "negative count");
    if (count == 0) return CONKER_OK;
    CK_HIP(c, hipSetDevice(c->device));
    const int threads = 256;
    ProfScope ps(c, PK_RATIO);
    hipLaunchKernelGGL(k_ratio_combined, dim3((unsigned)((count + threads - 1) / threads)), dim3(threads), 0,
                       c->stream, Wd, Wr, alpha, n_regions, n, count, xi, num, den);
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_map_ratio(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *N, const void *C,
                                const double *WR2, const double *alpha, void *out) {
    CK_OK(check_grid(c, g, false));
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (!N || !C || !WR2 || !alpha || !out) return fail(c, CONKER_EINVAL, "NULL pointer");
    CK_HIP(c, hipSetDevice(c->device));
    const size_t nc = ncells(g);
    const int threads = 256;
    const size_t want = (nc + threads - 1) / threads;
    const int blocks = (int)(want < 4096 ? want : 4096);
    ProfScope ps(c, PK_FORM_DELTA);
    if (dt == CONKER_F32)
        hipLaunchKernelGGL(k_map_ratio<float>, dim3(blocks), dim3(threads), 0, c->stream, (const float *)N,
                           (const float *)C, nc, WR2, alpha, (float *)out);
    else
        hipLaunchKernelGGL(k_map_ratio<double>, dim3(blocks), dim3(threads), 0, c->stream, (const double *)N,
                           (const double *)C, nc, WR2, alpha, (double *)out);
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_value_histogram(conker_ctx *c, conker_dtype dt, const void *values, int64_t n, double lo,
                                      double hi, int n_bins, int64_t *counts) {
    if (!c) return CONKER_EINVAL;
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (!counts || (n > 0 && !values)) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (n < 0) return fail(c, CONKER_EINVAL, "negative count");
    if (n_bins < 1 || n_bins > 16000) return fail(c, CONKER_EINVAL, "n_bins %d outside 1..16000", n_bins);
    if (!(hi > lo)) return fail(c, CONKER_EINVAL, "need lo < hi");
    CK_HIP(c, hipSetDevice(c->device));
    const int nb = n_bins + 2;
    ProfScope ps(c, PK_SUPPORT);
    hipLaunchKernelGGL(k_zero_i64, dim3((nb + 255) / 256), dim3(256), 0, c->stream, (unsigned long long *)counts,
                       nb);
    CK_LAUNCH(c);
    if (n == 0) return CONKER_OK;
    const int threads = 256;
    const int64_t want = (n + threads - 1) / threads;
    const int blocks = (int)(want < 2048 ? want : 2048);
    const size_t lds = (size_t)nb * sizeof(unsigned int);
    if (dt == CONKER_F32)
        hipLaunchKernelGGL(k_value_hist<float>, dim3(blocks), dim3(threads), lds, c->stream, (const float *)values,
                           (size_t)n, lo, hi, n_bins, (unsigned long long *)counts);
    else
        hipLaunchKernelGGL(k_value_hist<double>, dim3(blocks), dim3(threads), lds, c->stream,
                           (const double *)values, (size_t)n, lo, hi, n_bins, (unsigned long long *)counts);
    CK_LAUNCH(c);
    return CONKER_OK;
}
