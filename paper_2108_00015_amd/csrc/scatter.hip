// Mapping stage (Sec. 2.2): nearest-grid-point histograms and N = D - alpha R.
#include <cmath>

#include "common.h"

namespace {

struct GridGeom {
    double ox, oy, oz, cell;
    int nx, ny, nz;
};

template <typename T>
__device__ inline void atomic_add_grid(T *p, float w);

template <>
__device__ inline void atomic_add_grid<float>(float *p, float w) {
    unsafeAtomicAdd(p, w);
}

template <>
__device__ inline void atomic_add_grid<double>(double *p, float w) {
    unsafeAtomicAdd(p, (double)w);
}

__device__ inline int cell_of(float x, double o, double cell, int n, bool &ok) {
    // floor((x - origin) / cell) in float64 with IEEE division
    double c = floor(((double)x - o) / cell);
    ok = ok && (c >= 0.0) && (c < (double)n);
    return ok ? (int)c : 0;
}

// Each thread handles a strided subset of points; one float64 atomic per
// block for the weight sum and one int64 atomic for the rejected count.
template <typename T>
__global__ __launch_bounds__(256) void k_scatter(const float *__restrict__ pos,
                                                 const float *__restrict__ w, int64_t n, GridGeom g,
                                                 T *__restrict__ grid, double *wsum,
                                                 unsigned long long *n_out) {
    double my_w = 0.0;
    unsigned long long my_out = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        float x = pos[3 * p + 0];
        float y = pos[3 * p + 1];
        float z = pos[3 * p + 2];
        float wt = w ? w[p] : 1.0f;
        bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(wt);
        int cx = cell_of(x, g.ox, g.cell, g.nx, ok);
        int cy = cell_of(y, g.oy, g.cell, g.ny, ok);
        int cz = cell_of(z, g.oz, g.cell, g.nz, ok);
        if (ok) {
            size_t lin = ((size_t)cx * g.ny + cy) * g.nz + cz;
            atomic_add_grid<T>(grid + lin, wt);
            my_w += (double)wt;
        } else {
            ++my_out;
        }
    }
    // block reduction
    __shared__ double sw[256];
    __shared__ unsigned long long so[256];
    sw[threadIdx.x] = my_w;
    so[threadIdx.x] = my_out;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sw[threadIdx.x] += sw[threadIdx.x + s];
            so[threadIdx.x] += so[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (wsum) unsafeAtomicAdd(wsum, sw[0]);
        if (n_out && so[0]) atomicAdd(n_out, so[0]);
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_form_delta(T *__restrict__ D, const T *__restrict__ R,
                                                    size_t n, const double *wd, const double *wr,
                                                    double *alpha_out) {
    const double alpha = *wd / *wr;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    if (i == 0 && alpha_out) *alpha_out = alpha;
    for (; i < n; i += stride) D[i] = (T)((double)D[i] - alpha * (double)R[i]);
}

}  // namespace

using namespace conker;

extern "C" int conker_grid_assign(conker_ctx *c, const conker_grid *g, const float *pos,
                                  const float *w, int64_t n, conker_dtype dt, void *grid,
                                  double *wsum, int64_t *n_out) {
    CK_OK(check_grid(c, g, false));
    if (n < 0) return fail(c, CONKER_EINVAL, "negative point count");
    if ((n > 0 && !pos) || !grid) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (n == 0) return CONKER_OK;
    CK_HIP(c, hipSetDevice(c->device));
    GridGeom gg{g->origin[0], g->origin[1], g->origin[2], g->cell, g->dims[0], g->dims[1], g->dims[2]};
    int threads = 256;
    int64_t want = (n + threads - 1) / threads;
    int blocks = (int)(want < 8192 ? want : 8192);
    auto *no = reinterpret_cast<unsigned long long *>(n_out);
    ProfScope ps(c, PK_SCATTER);
    if (dt == CONKER_F32)
        hipLaunchKernelGGL(k_scatter<float>, dim3(blocks), dim3(threads), 0, c->stream, pos, w, n, gg,
                           (float *)grid, wsum, no);
    else
        hipLaunchKernelGGL(k_scatter<double>, dim3(blocks), dim3(threads), 0, c->stream, pos, w, n, gg,
                           (double *)grid, wsum, no);
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_form_delta(conker_ctx *c, const conker_grid *g, conker_dtype dt, void *D,
                                 const void *R, const double *wd, const double *wr, double *alpha) {
    CK_OK(check_grid(c, g, false));
    if (!D || !R || !wd || !wr) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    CK_HIP(c, hipSetDevice(c->device));
    size_t n = ncells(g);
    int threads = 256;
    size_t want = (n + threads - 1) / threads;
    int blocks = (int)(want < 16384 ? want : 16384);
    ProfScope ps(c, PK_FORM_DELTA);
    if (dt == CONKER_F32)
        hipLaunchKernelGGL(k_form_delta<float>, dim3(blocks), dim3(threads), 0, c->stream, (float *)D,
                           (const float *)R, n, wd, wr, alpha);
    else
        hipLaunchKernelGGL(k_form_delta<double>, dim3(blocks), dim3(threads), 0, c->stream, (double *)D,
                           (const double *)R, n, wd, wr, alpha);
    CK_LAUNCH(c);
    return CONKER_OK;
}
