// Equidistant (diagonal) n-point sums, Eq. ksinDiag: for every radius m and
// order n, sum_x F(x) C_m(x)^(n-1) -- the tuple a_1 = ... = a_{n-1} = m of
// Eq. ksin_delta.  Two forms:
//   * conker_convolve_diag: streamed out of the last inverse FFT pass, so no
//     map is ever stored (memory: the spectra of one radius batch only);
//   * conker_contract_diag: from stored maps.
// Both write per-workgroup FP64 partial rows that one kernel reduces in a
// fixed order, so results do not depend on scheduling.
#include <algorithm>
#include <mutex>

#include "common.h"

using namespace conker;

// Partial rows of conker_contract_diag_noalloc: a file-scope device array (one
// copy per GPU, held until the process ends) in place of the context's
// workspace, so that the call allocates nothing.  Host code never passes this
// name to a kernel: the address of each device's copy is looked up once per
// device (noalloc_init) and that address is used.
constexpr size_t NOALLOC_DOUBLES = (size_t)1 << 19;   // 4 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

constexpr int DT = 256;   // threads of the map and reduce kernels

template <typename T>
struct Vec;
template <>
struct Vec<float> {
    static constexpr int V = 4;
    using type = float4;
};
template <>
struct Vec<double> {
    static constexpr int V = 2;
    using type = double2;
};

template <typename T, int P>
__device__ __forceinline__ void acc_pow(double (&acc)[P], T f, T c) {
    T pw = c;
    acc[0] += (double)(f * pw);
#pragma unroll
    for (int p = 1; p < P; ++p) {
        pw *= c;
        acc[p] += (double)(f * pw);
    }
}

// Block sum of P doubles into row[p] (thread 0 .. P-1 write); ends with a barrier.
template <int P>
__device__ __forceinline__ void block_sum(double (&acc)[P], double (*red)[P], double *row) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < P; ++p) {
        double v = acc[p];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wv][p] = v;
    }
    __syncthreads();
    if (threadIdx.x < P) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < DT / 64; ++w) v += red[w][threadIdx.x];
        row[threadIdx.x] = v;
    }
    __syncthreads();
}

// Workgroup b covers cells [b * chunk, min(nc, (b + 1) * chunk)) for every
// radius; the field chunk is re-read per radius from L2.
template <typename T, int P>
__global__ __launch_bounds__(DT) void k_diag_maps(const T *__restrict__ F, const T *__restrict__ maps, size_t nc,
                                                  int ns, size_t chunk, double *__restrict__ part) {
    using VT = typename Vec<T>::type;
    constexpr int V = Vec<T>::V;
    __shared__ double red[DT / 64][P];
    const size_t c0 = (size_t)blockIdx.x * chunk;
    const size_t c1 = c0 + chunk < nc ? c0 + chunk : nc;
    for (int m = 0; m < ns; ++m) {
        double acc[P];
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] = 0.0;
        const T *mp = maps + (size_t)m * nc;
        for (size_t i = c0 + (size_t)threadIdx.x * V; i < c1; i += (size_t)DT * V) {
            const VT f = *reinterpret_cast<const VT *>(F + i);
            const VT c = *reinterpret_cast<const VT *>(mp + i);
            if constexpr (V == 4) {
                acc_pow<T, P>(acc, f.x, c.x);
                acc_pow<T, P>(acc, f.y, c.y);
                acc_pow<T, P>(acc, f.z, c.z);
                acc_pow<T, P>(acc, f.w, c.w);
            } else {
                acc_pow<T, P>(acc, f.x, c.x);
                acc_pow<T, P>(acc, f.y, c.y);
            }
        }
        block_sum<P>(acc, red, part + ((size_t)m * gridDim.x + blockIdx.x) * P);
    }
}

// part rows [ns][blocks][nf * P] -> out_f[(p - 1) * ns + m], p = 1 .. P.
// With ps, field b was transformed times the pair's scale s: its sums of
// power p carry s^p.
__global__ __launch_bounds__(DT) void k_diag_reduce(const double *__restrict__ part, int blocks, int ns, int nf,
                                                    int P, double *__restrict__ out_a, double *__restrict__ out_b,
                                                    const PackScale *ps) {
    __shared__ double red[DT];
    const int m = blockIdx.x;
    const int W = nf * P;
    for (int j = 0; j < W; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < blocks; b += DT) v += part[((size_t)m * blocks + b) * W + j];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = DT / 2; s >= 1; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const int f = j / P, p = j - f * P;
            double *o = f == 0 ? out_a : out_b;
            double v = red[0];
            if (f == 1 && ps)
                for (int q = 0; q <= p; ++q) v *= ps->s_inv;   // a power of two: exact
            if (o) o[(size_t)p * ns + m] = v;
        }
        __syncthreads();
    }
}

template <typename T>
int launch_maps(conker_ctx *c, const T *F, const T *maps, size_t nc, int ns, int P, int G, size_t chunk,
                double *part) {
    switch (P) {
        case 1: hipLaunchKernelGGL((k_diag_maps<T, 1>), dim3(G), dim3(DT), 0, c->stream, F, maps, nc, ns, chunk, part); break;
        case 2: hipLaunchKernelGGL((k_diag_maps<T, 2>), dim3(G), dim3(DT), 0, c->stream, F, maps, nc, ns, chunk, part); break;
        case 3: hipLaunchKernelGGL((k_diag_maps<T, 3>), dim3(G), dim3(DT), 0, c->stream, F, maps, nc, ns, chunk, part); break;
        default: hipLaunchKernelGGL((k_diag_maps<T, 4>), dim3(G), dim3(DT), 0, c->stream, F, maps, nc, ns, chunk, part); break;
    }
    CK_LAUNCH(c);
    return CONKER_OK;
}

int reduce(conker_ctx *c, const double *part, int blocks, int ns, int nf, int P, double *oa, double *ob,
           const PackScale *scale) {
    ProfScope ps(c, PK_DIAG_REDUCE);
    hipLaunchKernelGGL(k_diag_reduce, dim3(ns), dim3(DT), 0, c->stream, part, blocks, ns, nf, P, oa, ob, scale);
    CK_LAUNCH(c);
    return CONKER_OK;
}

int check_common(conker_ctx *c, const conker_grid *g, conker_dtype dt, int ns, int n_max) {
    CK_OK(check_grid(c, g, true));
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (ns <= 0) return fail(c, CONKER_EINVAL, "n_radii must be positive");
    if (n_max < 2 || n_max > 5) return fail(c, CONKER_EINVAL, "n_max %d outside 2..5", n_max);
    return CONKER_OK;
}

// Workgroups of the map kernel and the cells each covers (a whole number of
// vector steps).
void diag_plan(size_t nc, bool f64, int *G_out, size_t *chunk_out) {
    const size_t step = (size_t)DT * (f64 ? 2 : 4);
    int G = (int)std::min<size_t>(2048, std::max<size_t>(1, nc / (4 * step)));
    size_t chunk = (nc + G - 1) / G;
    chunk = (chunk + step - 1) / step * step;
    *G_out = (int)((nc + chunk - 1) / chunk);
    *chunk_out = chunk;
}

}  // namespace

namespace conker {

// Address of this device's copy of `scratch`, looked up once per device with
// that device current (conker_create).
int noalloc_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return CONKER_OK;   // the call then reports it
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return CONKER_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(nullptr, CONKER_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                    hipGetErrorString(e));
    g_noalloc_ptr[device] = ptr;
    return CONKER_OK;
}

}  // namespace conker

extern "C" int conker_contract_diag(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *field,
                                    const void *maps, int n_radii, int n_max, double *out) {
    CK_OK(check_common(c, g, dt, n_radii, n_max));
    if (!field || !maps || !out) return fail(c, CONKER_EINVAL, "NULL pointer");
    CK_HIP(c, hipSetDevice(c->device));
    const size_t nc = ncells(g);
    const bool f64 = dt == CONKER_F64;
    int G;
    size_t chunk;
    diag_plan(nc, f64, &G, &chunk);
    const int P = n_max - 1;
    CK_OK(ws_reserve(c, c->partial, (size_t)n_radii * G * P * sizeof(double)));
    double *part = (double *)c->partial.p;
    {
        ProfScope ps(c, PK_DIAG_MAPS);
        if (f64) CK_OK(launch_maps<double>(c, (const double *)field, (const double *)maps, nc, n_radii, P, G, chunk, part));
        else CK_OK(launch_maps<float>(c, (const float *)field, (const float *)maps, nc, n_radii, P, G, chunk, part));
    }
    return reduce(c, part, G, n_radii, 1, P, out, nullptr, nullptr);
}

// The same sums with the partial rows in the file-scope `scratch` array: no
// allocation, no memset, no event; the maps kernel overwrites every row the
// reduction reads.  Calls that overlap on one GPU share the array and race.
extern "C" int conker_contract_diag_noalloc(conker_ctx *c, const conker_grid *g, conker_dtype dt,
                                            const void *field, const void *maps, int n_radii, int n_max,
                                            double *out) {
    CK_OK(check_common(c, g, dt, n_radii, n_max));
    if (!field || !maps || !out) return fail(c, CONKER_EINVAL, "NULL pointer");
    const size_t nc = ncells(g);
    const bool f64 = dt == CONKER_F64;
    int G;
    size_t chunk;
    diag_plan(nc, f64, &G, &chunk);
    const int P = n_max - 1;
    const size_t need = (size_t)n_radii * G * P;
    if (need > NOALLOC_DOUBLES)
        return fail(c, CONKER_ERANGE,
                    "allocation-free call: %d radii x %d workgroups x %d powers = %zu partial sums, above its "
                    "fixed %zu (n_radii <= %zu at n_max %d on this grid)",
                    n_radii, G, P, need, NOALLOC_DOUBLES, NOALLOC_DOUBLES / ((size_t)G * P), n_max);
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES || !g_noalloc_ptr[c->device])
        return fail(c, CONKER_EHIP, "allocation-free scratch of device %d not set up", c->device);
    double *part = (double *)g_noalloc_ptr[c->device];
    CK_HIP(c, hipSetDevice(c->device));
    if (f64) CK_OK(launch_maps<double>(c, (const double *)field, (const double *)maps, nc, n_radii, P, G, chunk, part));
    else CK_OK(launch_maps<float>(c, (const float *)field, (const float *)maps, nc, n_radii, P, G, chunk, part));
    hipLaunchKernelGGL(k_diag_reduce, dim3(n_radii), dim3(DT), 0, c->stream, part, G, n_radii, 1, P, out, nullptr,
                       nullptr);
    CK_LAUNCH(c);
    return CONKER_OK;
}

// Maps from fa (fb), summed against the centre fields ca (cb).
static int convolve_diag(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa, const void *fb,
                         const void *ca, const void *cb, const void *kspec, int n_radii, int n_max, double *out_a,
                         double *out_b) {
    CK_OK(check_common(c, g, dt, n_radii, n_max));
    if (!fa || !ca || !kspec || !out_a) return fail(c, CONKER_EINVAL, "NULL pointer");
    if ((fb == nullptr) != (out_b == nullptr) || (fb == nullptr) != (cb == nullptr))
        return fail(c, CONKER_EINVAL, "field_b, its centre field and out_b must all be given or all be NULL");
    CK_HIP(c, hipSetDevice(c->device));
    const bool f64 = dt == CONKER_F64;
    Support sup;
    bool have_sup = false;
    {   // axis order of the transforms (cubic grids): the passes run on permuted copies
        const void *in[4] = {fa, fb, ca, cb}, *out[4];
        CK_OK(order_fields(c, g, f64, n_radii, in, 4, out, &sup, &have_sup));
        fa = out[0]; fb = out[1]; ca = out[2]; cb = out[3];
    }
    const size_t nc = ncells(g);
    const size_t cbytes = nc * (f64 ? sizeof(double2) : sizeof(float2));
    const int B = batch_radii(c, cbytes, n_radii, cbytes);
    const int P = n_max - 1;
    const int blocks = std::min(fft_z_tiles(g, f64), 4 * cu_count(c));
    CK_OK(ws_reserve(c, c->spec, cbytes));
    CK_OK(ws_reserve(c, c->tspec, (size_t)B * cbytes));
    CK_OK(ws_reserve(c, c->partial, (size_t)n_radii * blocks * 2 * P * sizeof(double)));
    double *part = (double *)c->partial.p;
    if (!have_sup) CK_OK(support_lines(c, g, f64, ca, cb, &sup));
    // the convolved fields are the centre fields (auto-correlation): their
    // support also prunes the forward transform
    CK_OK(fft_forward_pair(c, g, f64, fa, fb, c->spec.p, (fa == ca && fb == cb) ? &sup : nullptr));
    for (int m0 = 0; m0 < n_radii; m0 += B) {
        const int nb = (m0 + B <= n_radii) ? B : n_radii - m0;
        CK_OK(fft_inverse_batch(c, g, f64, c->spec.p, kspec, m0, nb, c->tspec.p, nullptr, nullptr, &sup));
        CK_OK(fft_inverse_z_diag(c, g, f64, c->tspec.p, nb, ca, cb, P, blocks,
                                 part + (size_t)m0 * blocks * 2 * P, &sup));
    }
    return reduce(c, part, blocks, n_radii, 2, P, out_a, out_b, fb ? pack_scale_dev(c) : nullptr);
}

extern "C" int conker_convolve_diag(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa,
                                    const void *fb, const void *kspec, int n_radii, int n_max, double *out_a,
                                    double *out_b) {
    return convolve_diag(c, g, dt, fa, fb, fa, fb, kspec, n_radii, n_max, out_a, out_b);
}

extern "C" int conker_convolve_diag_cross(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa,
                                          const void *fb, const void *ca, const void *cb, const void *kspec,
                                          int n_radii, int n_max, double *out_a, double *out_b) {
    return convolve_diag(c, g, dt, fa, fb, ca, cb, kspec, n_radii, n_max, out_a, out_b);
}
