// Two further forms of the estimator:
//
// * Continuous tracers (Sec. 2.7, Eq. densitycont): the field is the relative
//   over-density delta = (D - R) / R of two continuous maps on the grid; it is
//   convolved and summed like N (Eq. ksin_cont) with no normalisation after.
//
// * n = 2 in Fourier space: with K_m real and even and an unnormalised DFT,
//     sum_x a(x) (K_m *** b)(x) = N_c^-1 sum_k conj(a^(k)) b^(k) K_m^(k)
//   (Parseval).  The forward spectrum S = a^ + i b^ of the packed field pair is
//   read once and each radius costs one read of its kernel octant, instead of
//   a full inverse transform per radius.  a^ and b^ are separated with
//   a^(k) = (S(k) + conj S(-k)) / 2 and b^(k) = (S(k) - conj S(-k)) / (2i).
//   The sum over all k is folded onto the stored octant: every octant point
//   (kx <= nx/2, ky <= ny/2, kz <= nz/2) stands for its 1, 2, 4 or 8 sign
//   mirrors, which share the value of K_m^ and hold -k for each of their k.
//   Cross-correlations of the two fields (Sec. 2.8) come out of the same pass.
#include <algorithm>

#include "common.h"

using namespace conker;

namespace {

constexpr int NT = 256;

template <typename T>
__global__ __launch_bounds__(256) void k_delta_field(const T *__restrict__ D, const T *__restrict__ R, size_t n,
                                                     const double *alpha, T *__restrict__ out) {
    const double a = alpha ? *alpha : 1.0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double r = a * (double)R[i];
        out[i] = r != 0.0 ? (T)(((double)D[i] - r) / r) : (T)0;
    }
}

__global__ void k_ratio_cross(const double *Wd, const double *Wr, const double *a0, const double *a1, int n,
                              int64_t count, double *xi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double s = *a0;
    for (int k = 1; k < n; ++k) s *= *a1;
    xi[i] = Wd[i] / (s * Wr[i]);
}

constexpr size_t SPEC_LDS = 64 * 1024;   // bytes of folded powers per workgroup

__device__ __forceinline__ int mirrors(int k, int n, int (&out)[2]) {
    out[0] = k;
    if (k != 0 && 2 * k != n) {
        out[1] = n - k;
        return 2;
    }
    return 1;
}

// Workgroup (zb, oy): octant rows ky = oy, kz in [zb * TZ, zb * TZ + TZ), all kx;
// the folded powers are kept in LDS as T (float32 on the mixed path).
// Phase 1 folds |a^|^2, |b^|^2 and Re(conj a^ b^) over each point's mirrors
// into LDS; phase 2 walks the radii, reading each octant row of K_m once.
// part[((m * blocks) + block) * 3 + {aa, bb, ab}].
template <typename T>
__global__ __launch_bounds__(NT) void k_pair_spectral(const typename std::conditional<
                                                          std::is_same<T, float>::value, float2, double2>::type *spec,
                                                      const T *__restrict__ kspec, int nx, int ny, int nz, size_t kel,
                                                      int ns, int TZ, double *__restrict__ part) {
    using C = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;
    using P = T;
    const int OX = nx / 2 + 1, OZ = nz / 2 + 1;
    extern __shared__ __align__(16) unsigned char smem[];
    P *pw = reinterpret_cast<P *>(smem);   // [3][TZ][OX]
    __shared__ double red[NT / 64][3];
    const int oy = blockIdx.y, z0 = blockIdx.x * TZ;
    const int nzl = std::min(TZ, OZ - z0);
    int ys[2], zs[2], xs[2];
    const int ny_m = mirrors(oy, ny, ys);
    // ---- phase 1: folded powers ------------------------------------------------
    for (int e = threadIdx.x; e < OX * TZ; e += NT) {
        const int zl = e % TZ, ox = e / TZ;
        double aa = 0.0, bb = 0.0, ab = 0.0;
        if (zl < nzl) {
            const int nz_m = mirrors(z0 + zl, nz, zs);
            const int nx_m = mirrors(ox, nx, xs);
            for (int ix = 0; ix < nx_m; ++ix)
                for (int iy = 0; iy < ny_m; ++iy)
                    for (int iz = 0; iz < nz_m; ++iz) {
                        const int x = xs[ix], y = ys[iy], z = zs[iz];
                        const int xm = x ? nx - x : 0, ym = y ? ny - y : 0, zm = z ? nz - z : 0;
                        const C s = spec[((size_t)x * ny + y) * nz + z];
                        const C t = spec[((size_t)xm * ny + ym) * nz + zm];   // S(-k)
                        // a^ = (s + conj t) / 2, b^ = (s - conj t) / (2i)
                        const double ar = 0.5 * ((double)s.x + (double)t.x), ai = 0.5 * ((double)s.y - (double)t.y);
                        const double br = 0.5 * ((double)s.y + (double)t.y), bi = -0.5 * ((double)s.x - (double)t.x);
                        aa += ar * ar + ai * ai;
                        bb += br * br + bi * bi;
                        ab += ar * br + ai * bi;
                    }
        }
        pw[(0 * TZ + zl) * OX + ox] = (P)aa;
        pw[(1 * TZ + zl) * OX + ox] = (P)bb;
        pw[(2 * TZ + zl) * OX + ox] = (P)ab;
    }
    __syncthreads();
    // ---- phase 2: one pass over the kernel octant rows per radius --------------
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int blocks = gridDim.x * gridDim.y, bid = blockIdx.y * gridDim.x + blockIdx.x;
    for (int m = 0; m < ns; ++m) {
        const T *kb = kspec + (size_t)m * kel + ((size_t)oy * OZ + z0) * OX;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int e = threadIdx.x; e < OX * nzl; e += NT) {
            const int zl = e / OX, ox = e - zl * OX;
            const double k = (double)kb[(size_t)zl * OX + ox];
            s0 += (double)pw[(0 * TZ + zl) * OX + ox] * k;
            s1 += (double)pw[(1 * TZ + zl) * OX + ox] * k;
            s2 += (double)pw[(2 * TZ + zl) * OX + ox] * k;
        }
        for (int o = 32; o >= 1; o >>= 1) {
            s0 += __shfl_xor(s0, o);
            s1 += __shfl_xor(s1, o);
            s2 += __shfl_xor(s2, o);
        }
        if (lane == 0) {
            red[wv][0] = s0;
            red[wv][1] = s1;
            red[wv][2] = s2;
        }
        __syncthreads();
        if (threadIdx.x < 3) {
            double v = 0.0;
            for (int w = 0; w < NT / 64; ++w) v += red[w][threadIdx.x];
            part[((size_t)m * blocks + bid) * 3 + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

// part rows [ns][blocks][3] -> W_aa[m], W_bb[m], W_ab[m] (any may be NULL), fixed order.
// b was transformed times the pair's scale s: W_bb carries s^2, W_ab s.
__global__ __launch_bounds__(NT) void k_spectral_reduce(const double *__restrict__ part, int blocks, int ns,
                                                        double *Waa, double *Wbb, double *Wab,
                                                        const PackScale *ps) {
    __shared__ double red[NT];
    const int m = blockIdx.x;
    for (int j = 0; j < 3; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < blocks; b += NT) v += part[((size_t)m * blocks + b) * 3 + j];
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = NT / 2; s >= 1; s >>= 1) {
            if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double *o = j == 0 ? Waa : (j == 1 ? Wbb : Wab);
            double v = red[0];
            if (j == 1) v *= ps->s_inv * ps->s_inv;   // powers of two: exact
            if (j == 2) v *= ps->s_inv;
            if (o) o[m] = v;
        }
        __syncthreads();
    }
}

}  // namespace

extern "C" int conker_delta_field(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *D,
                                  const void *R, const double *alpha, void *delta) {
    CK_OK(check_grid(c, g, false));
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (!D || !R || !delta) return fail(c, CONKER_EINVAL, "NULL pointer");
    CK_HIP(c, hipSetDevice(c->device));
    const size_t n = ncells(g);
    const int threads = 256;
    const size_t want = (n + threads - 1) / threads;
    const int blocks = (int)(want < 4096 ? want : 4096);
    ProfScope ps(c, PK_FORM_DELTA);
    if (dt == CONKER_F32)
        hipLaunchKernelGGL(k_delta_field<float>, dim3(blocks), dim3(threads), 0, c->stream, (const float *)D,
                           (const float *)R, n, alpha, (float *)delta);
    else
        hipLaunchKernelGGL(k_delta_field<double>, dim3(blocks), dim3(threads), 0, c->stream, (const double *)D,
                           (const double *)R, n, alpha, (double *)delta);
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_ratio_cross(conker_ctx *c, const double *Wd, const double *Wr, const double *alpha0,
                                  const double *alpha1, int n, int64_t count, double *xi) {
    if (!c) return CONKER_EINVAL;
    if (!Wd || !Wr || !alpha0 || !alpha1 || !xi) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (n < 2 || n > 5) return fail(c, CONKER_EINVAL, "order n=%d outside 2..5", n);
    if (count < 0) return fail(c, CONKER_EINVAL, "negative count");
    if (count == 0) return CONKER_OK;
    CK_HIP(c, hipSetDevice(c->device));
    const int threads = 256;
    const int64_t blocks = (count + threads - 1) / threads;
    ProfScope ps(c, PK_RATIO);
    hipLaunchKernelGGL(k_ratio_cross, dim3((unsigned)blocks), dim3(threads), 0, c->stream, Wd, Wr, alpha0, alpha1,
                       n, count, xi);
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_pair_spectral(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa,
                                    const void *fb, const void *kspec, int n_radii, double *W_aa, double *W_bb,
                                    double *W_ab) {
    CK_OK(check_grid(c, g, true));
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (!fa || !kspec || !W_aa) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (!fb && (W_bb || W_ab)) return fail(c, CONKER_EINVAL, "W_bb and W_ab need field_b");
    if (n_radii <= 0) return fail(c, CONKER_EINVAL, "n_radii must be positive");
    CK_HIP(c, hipSetDevice(c->device));
    const bool f64 = dt == CONKER_F64;
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    const size_t nc = ncells(g);
    const size_t cbytes = nc * (f64 ? sizeof(double2) : sizeof(float2));
    const size_t kel = (size_t)(nx / 2 + 1) * (ny / 2 + 1) * (nz / 2 + 1);
    const size_t row = (size_t)3 * (nx / 2 + 1) * (f64 ? sizeof(double) : sizeof(float));
    int TZ = 16;
    while (TZ > 1 && (size_t)TZ * row > SPEC_LDS) TZ /= 2;
    const dim3 grid((unsigned)((nz / 2 + 1 + TZ - 1) / TZ), (unsigned)(ny / 2 + 1));
    const int blocks = (int)(grid.x * grid.y);
    const size_t lds = (size_t)TZ * row;
    CK_OK(ws_reserve(c, c->spec, cbytes));
    CK_OK(ws_reserve(c, c->partial, (size_t)n_radii * blocks * 3 * sizeof(double)));
    CK_OK(fft_forward_pair(c, g, f64, fa, fb, c->spec.p));
    {
        ProfScope ps(c, PK_SPECTRAL);
        if (f64)
            hipLaunchKernelGGL(k_pair_spectral<double>, grid, dim3(NT), lds, c->stream, (const double2 *)c->spec.p,
                               (const double *)kspec, nx, ny, nz, kel, n_radii, TZ, (double *)c->partial.p);
        else
            hipLaunchKernelGGL(k_pair_spectral<float>, grid, dim3(NT), lds, c->stream, (const float2 *)c->spec.p,
                               (const float *)kspec, nx, ny, nz, kel, n_radii, TZ, (double *)c->partial.p);
        CK_LAUNCH(c);
    }
    ProfScope ps(c, PK_DIAG_REDUCE);
    hipLaunchKernelGGL(k_spectral_reduce, dim3(n_radii), dim3(NT), 0, c->stream, (const double *)c->partial.p, blocks,
                       n_radii, W_aa, fb ? W_bb : nullptr, fb ? W_ab : nullptr, pack_scale_dev(c));
    CK_LAUNCH(c);
    return CONKER_OK;
}
