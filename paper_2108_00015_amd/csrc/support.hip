// Lines of cells that can contribute to a summation.
//
// Every term of Eq. ksin_delta carries the factor F(x) of the field at the
// tuple's central cell, so a z-line (x, y) on which both fields vanish adds
// nothing, whatever the maps hold there.  Survey volumes leave many such lines
// (a sky cap fills a cone of its box).  When the maps are only summed, never
// stored, the inverse passes therefore need their outputs only on the lines
// that carry field: the x pass writes only x-slabs with at least one such line,
// the y pass skips empty x-slabs and writes only carrying lines, and the z pass
// transforms only carrying lines.  The results are unchanged.
//
// A line carries field if any value is non-zero in either field, tested on
// the bits other than the sign (-0.0 counts as zero: it adds nothing to any
// sum; NaN counts as non-zero, which only keeps a line).  Outputs:
//   mask[x * ny + y]   1 or 0;
//   xcount[x]          carrying lines of slab x;
//   list[0 .. count)   carrying lines x * ny + y in increasing order;
//   count              their number.
#include "common.h"

using namespace conker;

namespace {

constexpr int ST = 256;   // threads per workgroup (4 waves)

// sm: the bits other than the sign of the four 32-bit words of 16 bytes
// (float32: every word; float64: the high word of each value).
// With `sums` (both fields given): also each field's sum of squares over the
// slab, written as the pair sums[2 x + {0, 1}] (the packed transform's scale
// is chosen from them).
template <typename T>
__device__ __forceinline__ double sq16(const uint4 &v) {   // sum of squares of the values in 16 bytes
    if constexpr (sizeof(T) == 4) {
        const float a = __uint_as_float(v.x), b = __uint_as_float(v.y), c = __uint_as_float(v.z),
                    d = __uint_as_float(v.w);
        return (double)a * a + (double)b * b + (double)c * c + (double)d * d;
    } else {
        const double a = __hiloint2double((int)v.y, (int)v.x), b = __hiloint2double((int)v.w, (int)v.z);
        return a * a + b * b;
    }
}

template <typename T>
__global__ __launch_bounds__(ST) void k_line_mask(const uint4 *__restrict__ fa, const uint4 *__restrict__ fb,
                                                  int ny, int units, uint4 sm, unsigned char *__restrict__ mask,
                                                  int *__restrict__ xcount, double *__restrict__ sums) {
    __shared__ int cnt[ST / 64];
    __shared__ double red[ST / 64][2];
    const int x = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int c = 0;
    double sa = 0.0, sb = 0.0;
    for (int y = w; y < ny; y += ST / 64) {
        const size_t base = ((size_t)x * ny + y) * units;
        unsigned any = 0;
        for (int u = lane; u < units; u += 64) {
            const uint4 a = fa[base + u];
            any |= (a.x & sm.x) | (a.y & sm.y) | (a.z & sm.z) | (a.w & sm.w);
            if (sums) sa += sq16<T>(a);
            if (fb) {
                const uint4 b = fb[base + u];
                any |= (b.x & sm.x) | (b.y & sm.y) | (b.z & sm.z) | (b.w & sm.w);
                if (sums) sb += sq16<T>(b);
            }
        }
        const bool on = __ballot(any != 0u) != 0ull;
        if (lane == 0) {
            mask[(size_t)x * ny + y] = on ? 1 : 0;
            c += on ? 1 : 0;
        }
    }
    if (lane == 0) cnt[w] = c;
    if (sums) {   // uniform
        for (int o = 32; o >= 1; o >>= 1) {
            sa += __shfl_xor(sa, o);
            sb += __shfl_xor(sb, o);
        }
        if (lane == 0) {
            red[w][0] = sa;
            red[w][1] = sb;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < ST / 64; ++i) s += cnt[i];
        xcount[x] = s;
    }
    if (sums && threadIdx.x < 2) {
        double v = 0.0;
        for (int i = 0; i < ST / 64; ++i) v += red[i][threadIdx.x];
        sums[2 * x + threadIdx.x] = v;
    }
}

// One workgroup per slab x: offset = carrying lines of slabs before x, then a
// block scan over the slab's mask writes its lines in order.
__global__ __launch_bounds__(ST) void k_line_list(const unsigned char *__restrict__ mask,
                                                  const int *__restrict__ xcount, int nx, int ny,
                                                  int *__restrict__ list, int *__restrict__ count) {
    __shared__ int red[ST];
    const int x = blockIdx.x, t = threadIdx.x;
    int s = 0;
    for (int i = t; i < x; i += ST) s += xcount[i];
    red[t] = s;
    __syncthreads();
    for (int h = ST / 2; h >= 1; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const int offset = red[0];
    const int mine = xcount[x];
    if (x == nx - 1 && t == 0) *count = offset + mine;
    if (mine == 0) return;   // uniform over the workgroup
    __syncthreads();
    const int per = (ny + ST - 1) / ST;
    const int y0 = t * per;
    int c = 0;
    for (int y = y0; y < y0 + per && y < ny; ++y) c += mask[(size_t)x * ny + y];
    red[t] = c;
    __syncthreads();
    for (int h = 1; h < ST; h <<= 1) {   // inclusive scan
        const int v = t >= h ? red[t - h] : 0;
        __syncthreads();
        red[t] += v;
        __syncthreads();
    }
    int pos = offset + red[t] - c;
    for (int y = y0; y < y0 + per && y < ny; ++y)
        if (mask[(size_t)x * ny + y]) list[pos++] = x * ny + y;
}

}  // namespace

namespace conker {

int support_alloc(conker_ctx *c, int nx, int ny, Support *out, unsigned char **mask, int **xcount,
                  double **sums_slot) {
    *out = Support{};
    const size_t nl = (size_t)nx * ny;
    const size_t mask_b = (nl + 255) / 256 * 256;
    const size_t xc_b = ((size_t)nx * sizeof(int) + 255) / 256 * 256;
    const size_t list_b = (nl * sizeof(int) + 255) / 256 * 256;
    const size_t sums_b = ((size_t)nx * 2 * sizeof(double) + 255) / 256 * 256;
    CK_OK(ws_reserve(c, c->support, mask_b + xc_b + list_b + 256 + sums_b));
    char *p = (char *)c->support.p;
    out->mask = *mask = (unsigned char *)p;
    out->xcount = *xcount = (int *)(p + mask_b);
    out->list = (int *)(p + mask_b + xc_b);
    out->count = (int *)(p + mask_b + xc_b + list_b);
    if (sums_slot) *sums_slot = (double *)(p + mask_b + xc_b + list_b + 256);   // room for nx pairs
    return CONKER_OK;
}

int support_list(conker_ctx *c, int nx, int ny, const Support &s) {
    ProfScope ps(c, PK_SUPPORT);
    hipLaunchKernelGGL(k_line_list, dim3(nx), dim3(ST), 0, c->stream, s.mask, s.xcount, nx, ny,
                       const_cast<int *>(s.list), const_cast<int *>(s.count));
    CK_LAUNCH(c);
    return CONKER_OK;
}

int support_lines(conker_ctx *c, const conker_grid *g, bool f64, const void *fa, const void *fb, Support *out) {
    const int nx = g->dims[0], ny = g->dims[1], nz = g->dims[2];
    *out = Support{};
    if (((uintptr_t)fa & 15) || ((uintptr_t)fb & 15))
        return fail(c, CONKER_EINVAL, "fields must be 16-byte aligned");
    unsigned char *mask;
    int *xcount;
    double *sums;
    CK_OK(support_alloc(c, nx, ny, out, &mask, &xcount, &sums));
    const int units = (int)((size_t)nz * (f64 ? 8 : 4) / 16);   // 16-byte words per line
    if (!fb) sums = nullptr;   // one field: nothing is packed beside it
    {
        ProfScope ps(c, PK_SUPPORT);
        const uint4 sm = f64 ? uint4{0xffffffffu, 0x7fffffffu, 0xffffffffu, 0x7fffffffu}
                             : uint4{0x7fffffffu, 0x7fffffffu, 0x7fffffffu, 0x7fffffffu};
        if (f64)
            hipLaunchKernelGGL(k_line_mask<double>, dim3(nx), dim3(ST), 0, c->stream, (const uint4 *)fa,
                               (const uint4 *)fb, ny, units, sm, mask, xcount, sums);
        else
            hipLaunchKernelGGL(k_line_mask<float>, dim3(nx), dim3(ST), 0, c->stream, (const uint4 *)fa,
                               (const uint4 *)fb, ny, units, sm, mask, xcount, sums);
        CK_LAUNCH(c);
    }
    out->sums = sums;
    out->sums_n = sums ? nx : 0;
    return support_list(c, nx, ny, *out);
}

}  // namespace conker
