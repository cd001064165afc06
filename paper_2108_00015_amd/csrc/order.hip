// Axis order of the transforms for map-free summations on cubic grids.
//
// The inverse passes after the kernel multiply skip work outside the support
// of the summed fields: the first pass writes only slabs (along the first
// transformed axis) that hold field, the middle pass reads those slabs and
// writes only lines along the last axis that carry field, and the last pass
// (fused with the summation) runs over those lines.  How much is skipped
// depends on which axis comes first and which last: a sky cap along z, for
// instance, spans few z-slabs but most x-slabs.  On a cubic grid every
// permutation of the axes maps the shell of radius r (Sec. 2.3) onto itself,
// so the stored kernel spectra serve the permuted grid unchanged and the sums
// of Eq. ksin_delta are the same; only the order in which they are added
// changes.  The fields are therefore copied into the permuted layout (on the
// device, graph-safe) and the passes run on the copies.
//
// The permutation is either fixed by the context's setting or chosen on the
// device from the field's support: the projections of the non-zero cells onto
// the three coordinate planes give, for each axis a, the fraction s_a of
// slabs with field and the fraction l_a of lines along a that carry field.
// With first axis A and last axis C the inverse passes move about
// 2 s_A + 2 l_C grid-units of complex values per radius; the permutation with
// the smallest figure is taken when it saves more than the copies cost.
#include "common.h"

using namespace conker;

namespace {

// Permutation p (0..5, lexicographic): new axis k is old axis PERM[p][k].
__constant__ int PERM[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

constexpr int OT = 256;   // threads per workgroup

// One wave per z-line (x, y) of an L^3 grid: bits[(x L + y) W + w] holds
// cells 32 w .. 32 w + 31 of the line (bit set: the cell holds field in
// either field), W = L / 32, and pxy[x L + y] = the line carries field.
// Non-zero is a bit test of everything but the sign, as for the line masks.
// Each lane reads 16 bytes (CPL cells) per step; the lanes' flags are packed
// into 32-bit words (LPW lanes a word) with shuffles.
// With `sums` (both fields given): also the sums of squares of each field
// over the workgroup's lines, written as the pair sums[2 blockIdx.x + {0, 1}]
// (the packed transform's scale is chosen from them).
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
__global__ __launch_bounds__(OT) void k_occ_bits(const T *__restrict__ fa, const T *__restrict__ fb, int L,
                                                 unsigned *__restrict__ bits, unsigned char *__restrict__ pxy,
                                                 double *__restrict__ sums) {
    constexpr int CPL = 16 / (int)sizeof(T), LPW = 32 / CPL;
    __shared__ double red[OT / 64][2];
    const int lane = threadIdx.x & 63;
    const size_t line = (size_t)blockIdx.x * (OT / 64) + (threadIdx.x >> 6);
    const bool valid = line < (size_t)L * L;   // uniform per wave
    const uint4 *a = reinterpret_cast<const uint4 *>(fa + (valid ? line : 0) * L);
    const uint4 *b = fb ? reinterpret_cast<const uint4 *>(fb + (valid ? line : 0) * L) : nullptr;
    const int W = L / 32, units = valid ? L / CPL : 0;
    unsigned any = 0;
    double sa = 0.0, sb = 0.0;
    for (int j = 0; j * 64 < units; ++j) {
        const int q = j * 64 + lane;
        unsigned fl = 0;
        if (q < units) {
            // sign bits cleared: -0.0 adds nothing to any sum and counts as zero
            constexpr unsigned MLO = CPL == 4 ? 0x7fffffffu : 0xffffffffu;
            uint4 v = a[q];
            if (sums) sa += sq16<T>(v);
            if (b) {
                const uint4 v2 = b[q];
                if (sums) sb += sq16<T>(v2);
                v = uint4{v.x | v2.x, v.y | v2.y, v.z | v2.z, v.w | v2.w};
            }
            v = uint4{v.x & MLO, v.y & 0x7fffffffu, v.z & MLO, v.w & 0x7fffffffu};
            if constexpr (CPL == 4) {
                fl = (v.x != 0u ? 1u : 0u) | (v.y != 0u ? 2u : 0u) | (v.z != 0u ? 4u : 0u) | (v.w != 0u ? 8u : 0u);
            } else {
                fl = ((v.x | v.y) != 0u ? 1u : 0u) | ((v.z | v.w) != 0u ? 2u : 0u);
            }
        }
        unsigned word = fl << (CPL * (lane % LPW));
#pragma unroll
        for (int o = 1; o < LPW; o <<= 1) word |= __shfl_xor(word, o);
        any |= word;
        const int wi = j * (64 / LPW) + lane / LPW;   // word of the line this lane group fills
        if (lane % LPW == 0 && wi < W) bits[line * W + wi] = word;
    }
    const bool carry = __ballot(any != 0u) != 0ull;
    if (lane == 0 && valid) pxy[line] = carry ? 1 : 0;
    if (sums) {   // uniform
        for (int o = 32; o >= 1; o >>= 1) {
            sa += __shfl_xor(sa, o);
            sb += __shfl_xor(sb, o);
        }
        if (lane == 0) {
            red[threadIdx.x >> 6][0] = sa;
            red[threadIdx.x >> 6][1] = sb;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            double v = 0.0;
            for (int w = 0; w < OT / 64; ++w) v += red[w][threadIdx.x];
            sums[2 * blockIdx.x + threadIdx.x] = v;
        }
    }
}

// Projections onto the (x, z) and (y, z) planes: workgroups 0 .. L-1 write
// row x of pxz (OR over y of the lines' words), workgroups L .. 2L-1 row y of
// pyz (OR over x).
__global__ __launch_bounds__(OT) void k_occ_planes(const unsigned *__restrict__ bits, int L,
                                                   unsigned *__restrict__ pxz, unsigned *__restrict__ pyz) {
    __shared__ unsigned acc[32];
    const int W = L / 32, t = threadIdx.x;
    const bool rows_x = (int)blockIdx.x < L;
    const int r = rows_x ? blockIdx.x : blockIdx.x - L;
    if (t < W) acc[t] = 0u;
    __syncthreads();
    for (int e = t; e < L * W; e += OT) {
        const int k = e / W, w = e - (e / W) * W;   // k: the other in-plane index (y for pxz, x for pyz)
        const size_t line = rows_x ? (size_t)r * L + k : (size_t)k * L + r;
        const unsigned v = bits[line * W + w];
        if (v) atomicOr(&acc[w], v);
    }
    __syncthreads();
    if (t < W) (rows_x ? pxz : pyz)[(size_t)r * W + t] = acc[t];
}

// One workgroup: fractions of slabs and lines per axis from the projections,
// then the permutation with the smallest pass traffic (ties: the lower index,
// so the given order wins).  Writes the chosen index to *perm.
__global__ __launch_bounds__(1024) void k_choose_order(const unsigned char *__restrict__ pxy,
                                                       const unsigned *__restrict__ pxz,
                                                       const unsigned *__restrict__ pyz, int L, int ns,
                                                       int *__restrict__ perm) {
    __shared__ unsigned col_z[32];                // OR over x of the rows of pxz (bits z)
    __shared__ unsigned long long cnt[6];         // slabs x, y, z; lines along x, y, z
    const int t = threadIdx.x, W = L / 32;
    if (t < 32) col_z[t] = 0u;
    if (t < 6) cnt[t] = 0ull;
    __syncthreads();
    unsigned long long sx = 0, sy = 0, lx = 0, ly = 0, lz = 0;
    for (int r = t; r < L; r += blockDim.x) {
        unsigned ox = 0, oy = 0;
        for (int w = 0; w < W; ++w) {
            const unsigned a = pxz[(size_t)r * W + w], b = pyz[(size_t)r * W + w];
            ox |= a;
            oy |= b;
            ly += __popc(a);   // (x, z) positions with field: lines along y
            lx += __popc(b);   // (y, z) positions: lines along x
            if (a) atomicOr(&col_z[w], a);
        }
        sx += ox != 0u;
        sy += oy != 0u;
    }
    const uint4 *p16 = reinterpret_cast<const uint4 *>(pxy);   // bytes 0 / 1, L^2 a multiple of 16
    for (size_t i = t; i < (size_t)L * L / 16; i += blockDim.x) {
        const uint4 v = p16[i];
        lz += __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w);
    }
    atomicAdd(&cnt[0], sx);
    atomicAdd(&cnt[1], sy);
    atomicAdd(&cnt[3], lx);
    atomicAdd(&cnt[4], ly);
    atomicAdd(&cnt[5], lz);
    __syncthreads();
    if (t == 0) {
        unsigned long long sz = 0;
        for (int w = 0; w < W; ++w) sz += __popc(col_z[w]);
        const double slab[3] = {(double)cnt[0] / L, (double)cnt[1] / L, (double)sz / L};
        const double lines[3] = {(double)cnt[3] / ((double)L * L), (double)cnt[4] / ((double)L * L),
                                 (double)cnt[5] / ((double)L * L)};
        double best = 0.0;
        int bp = 0;
        for (int p = 0; p < 6; ++p) {
            const double s = 2.0 * slab[PERM[p][0]] + 2.0 * lines[PERM[p][2]];
            if (p == 0 || s < best) {
                best = s;
                bp = p;
            }
        }
        const double id = 2.0 * slab[0] + 2.0 * lines[2];
        // copies of the fields cost about two grid-units; ask for a clear saving
        perm[0] = (ns * (id - best) > 3.0) ? bp : 0;
    }
}

// dst = src with its axes permuted: new axis k is old axis PERM[p][k], with p
// fixed (>= 0) or read from *pdev.  A workgroup moves a 32 x 32 tile spanned
// by old z (contiguous in src) and the old axis u that becomes contiguous in
// dst (u = y when z stays the contiguous axis), at one value of the third axis.
template <typename T>
__global__ __launch_bounds__(OT) void k_permute(const T *__restrict__ src, T *__restrict__ dst, int L, int pfix,
                                                const int *__restrict__ pdev) {
    __shared__ T tile[32][33];
    const int p = pfix >= 0 ? pfix : *pdev;
    const int b = PERM[p][2];
    const int u = b != 2 ? b : 1, w = 1 - u;   // the three old axes are z (2), u and w
    const size_t LL = (size_t)L * L;
    auto old_stride = [&](int a) -> size_t { return a == 0 ? LL : (a == 1 ? (size_t)L : 1); };
    auto new_stride = [&](int a) -> size_t {
        return PERM[p][0] == a ? LL : (PERM[p][1] == a ? (size_t)L : 1);
    };
    const size_t su_o = old_stride(u), sw_o = old_stride(w);
    const size_t sz_n = new_stride(2), su_n = new_stride(u), sw_n = new_stride(w);
    const int z0 = blockIdx.x * 32, u0 = blockIdx.y * 32, wv = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const T *s0 = src + (size_t)wv * sw_o;
    T *d0 = dst + (size_t)wv * sw_n;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int a = ty + 8 * r;
        tile[a][tx] = s0[(size_t)(z0 + tx) + (size_t)(u0 + a) * su_o];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int a = ty + 8 * r;
        if (b != 2)   // old u becomes contiguous: lanes run along u
            d0[(size_t)(z0 + a) * sz_n + (size_t)(u0 + tx) * su_n] = tile[tx][a];
        else          // z stays contiguous: lanes run along z
            d0[(size_t)(z0 + tx) * sz_n + (size_t)(u0 + a) * su_n] = tile[a][tx];
    }
}

// Line support of the permuted grid from the projections: workgroup n0 (a
// slab of the new first axis) writes mask[n0 L + n1] for the lines along the
// new last axis and xcount[n0], the number of those that carry field.
__global__ __launch_bounds__(OT) void k_support_planes(const unsigned char *__restrict__ pxy,
                                                       const unsigned *__restrict__ pxz,
                                                       const unsigned *__restrict__ pyz, int L, int pfix,
                                                       const int *__restrict__ pdev, unsigned char *__restrict__ mask,
                                                       int *__restrict__ xcount) {
    __shared__ int part[OT / 64];
    const int p = pfix >= 0 ? pfix : *pdev;
    const int a0 = PERM[p][0], a1 = PERM[p][1], C = PERM[p][2];
    const int n0 = blockIdx.x, W = L / 32;
    int cnt = 0;
    for (int n1 = threadIdx.x; n1 < L; n1 += OT) {
        // old coordinates fixed by the line (the one along C is free)
        const int ox = a0 == 0 ? n0 : (a1 == 0 ? n1 : 0);
        const int oy = a0 == 1 ? n0 : (a1 == 1 ? n1 : 0);
        const int oz = a0 == 2 ? n0 : (a1 == 2 ? n1 : 0);
        bool on;
        if (C == 2) on = pxy[(size_t)ox * L + oy] != 0;
        else if (C == 1) on = (pxz[(size_t)ox * W + (oz >> 5)] >> (oz & 31)) & 1u;
        else on = (pyz[(size_t)oy * W + (oz >> 5)] >> (oz & 31)) & 1u;
        mask[(size_t)n0 * L + n1] = on ? 1 : 0;
        cnt += on ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int i = 0; i < OT / 64; ++i) s += part[i];
        xcount[n0] = s;
    }
}

}  // namespace

namespace conker {

int order_fields(conker_ctx *c, const conker_grid *g, bool f64, int ns, const void *const *in, int n_in,
                 const void **out, Support *sup, bool *have_sup) {
    for (int k = 0; k < n_in; ++k) out[k] = in[k];
    if (have_sup) *have_sup = false;
    const int L = g->dims[0];
    const int mode = c->tune.axis_order;   // 0 auto, else permutation mode - 1 (1: as given)
    const int pfix = mode >= 1 ? mode - 1 : -1;
    c->order_last = 1;
    c->order_dev = nullptr;
    if (pfix == 0 || g->dims[1] != L || g->dims[2] != L || L % 32) return CONKER_OK;
    for (int k = 0; k < n_in; ++k)
        if ((uintptr_t)in[k] & 15) return fail(c, CONKER_EINVAL, "fields must be 16-byte aligned");
    // distinct non-NULL fields are copied; repeats share a copy
    int src_of[4], n_copy = 0;
    const void *uniq[4];
    for (int k = 0; k < n_in; ++k) {
        src_of[k] = -1;
        if (!in[k]) continue;
        for (int j = 0; j < n_copy; ++j)
            if (uniq[j] == in[k]) src_of[k] = j;
        if (src_of[k] < 0) {
            uniq[n_copy] = in[k];
            src_of[k] = n_copy++;
        }
    }
    const size_t nc = ncells(g), esz = f64 ? 8 : 4;
    const size_t W = (size_t)L / 32;
    const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t pxy_b = up((size_t)L * L), plane_b = up(W * L * sizeof(unsigned));
    const size_t bits_b = up((size_t)L * L * W * sizeof(unsigned));
    const unsigned blocks = (unsigned)(((size_t)L * L + OT / 64 - 1) / (OT / 64));
    const size_t sums_b = up((size_t)blocks * 2 * sizeof(double));
    const size_t head = pxy_b + 2 * plane_b + 256 + bits_b + sums_b;
    const size_t field_b = up(nc * esz);
    CK_OK(ws_reserve(c, c->order, head + (size_t)n_copy * field_b));
    char *base = (char *)c->order.p;
    unsigned char *pxy = (unsigned char *)base;
    unsigned *pxz = (unsigned *)(base + pxy_b);
    unsigned *pyz = (unsigned *)(base + pxy_b + plane_b);
    int *perm = (int *)(base + pxy_b + 2 * plane_b);
    unsigned *bits = (unsigned *)(base + pxy_b + 2 * plane_b + 256);
    double *sums = (double *)(base + pxy_b + 2 * plane_b + 256 + bits_b);
    // projections of the centre fields' support (they carry the factor F of every term)
    const void *sa = in[n_in >= 4 ? 2 : 0], *sb = in[n_in >= 4 ? 3 : 1];
    if (!sb) sums = nullptr;   // one field: nothing is packed beside it
    {
        ProfScope ps(c, PK_ORDER);
        if (f64)
            hipLaunchKernelGGL(k_occ_bits<double>, dim3(blocks), dim3(OT), 0, c->stream, (const double *)sa,
                               (const double *)sb, L, bits, pxy, sums);
        else
            hipLaunchKernelGGL(k_occ_bits<float>, dim3(blocks), dim3(OT), 0, c->stream, (const float *)sa,
                               (const float *)sb, L, bits, pxy, sums);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_occ_planes, dim3(2 * L), dim3(OT), 0, c->stream, bits, L, pxz, pyz);
        CK_LAUNCH(c);
        if (pfix < 0) {
            hipLaunchKernelGGL(k_choose_order, dim3(1), dim3(1024), 0, c->stream, pxy, pxz, pyz, L, ns, perm);
            CK_LAUNCH(c);
        }
        const dim3 grid((unsigned)(L / 32), (unsigned)(L / 32), (unsigned)L);
        for (int j = 0; j < n_copy; ++j) {
            void *dst = base + head + (size_t)j * field_b;
            if (f64)
                hipLaunchKernelGGL(k_permute<double>, grid, dim3(OT), 0, c->stream, (const double *)uniq[j],
                                   (double *)dst, L, pfix, perm);
            else
                hipLaunchKernelGGL(k_permute<float>, grid, dim3(OT), 0, c->stream, (const float *)uniq[j],
                                   (float *)dst, L, pfix, perm);
            CK_LAUNCH(c);
        }
    }
    for (int k = 0; k < n_in; ++k)
        if (in[k]) out[k] = base + head + (size_t)src_of[k] * field_b;
    c->order_last = pfix >= 0 ? pfix + 1 : -1;
    c->order_dev = pfix >= 0 ? nullptr : perm;
    if (sup) {   // line support of the permuted centre fields, from the same projections
        unsigned char *mask;
        int *xcount;
        CK_OK(support_alloc(c, L, L, sup, &mask, &xcount));
        {
            ProfScope ps(c, PK_SUPPORT);
            hipLaunchKernelGGL(k_support_planes, dim3(L), dim3(OT), 0, c->stream, pxy, pxz, pyz, L, pfix, perm, mask,
                               xcount);
            CK_LAUNCH(c);
        }
        CK_OK(support_list(c, L, L, *sup));
        sup->sums = sums;   // of the (unpermuted) centre fields: permutations keep them
        sup->sums_n = sums ? (int)blocks : 0;
        if (have_sup) *have_sup = true;
    }
    return CONKER_OK;
}

}  // namespace conker

extern "C" int conker_axis_order_used(conker_ctx *c, int *h_order) {
    if (!c || !h_order) return CONKER_EINVAL;
    if (c->order_last >= 0) {
        *h_order = c->order_last;
        return CONKER_OK;
    }
    CK_HIP(c, hipSetDevice(c->device));
    int v = 0;
    CK_HIP(c, hipMemcpyAsync(&v, c->order_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    CK_HIP(c, hipStreamSynchronize(c->stream));
    *h_order = v + 1;
    return CONKER_OK;
}
