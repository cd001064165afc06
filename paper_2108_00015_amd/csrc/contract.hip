// Summation stage (Sec. 2.5, Eq. ksin_delta):
//   W(a_1..a_{n-1}) = sum_x F(x) prod_i C_{a_i}(x)
// for every multiset a_1 <= ... <= a_{n-1} of shell indices.
//
// n = 2 is a set of dot products and runs on the vector ALUs.
// n = 3, 4, 5 are written as one matrix product over the cells:
//   rows    = left items  (F * C_a for n = 3; F * C_a * C_b, a <= b, for n = 4, 5)
//   columns = right items (C_c for n = 3, 4; C_c * C_d, c <= d, for n = 5)
//   M[row][col] = sum_x row(x) * col(x)
// and every tuple is one entry of M: (a, b) for n = 3, ((a, b), c) for n = 4,
// ((a, b), (c, d)) for n = 5.  M is computed in output tiles on the matrix
// cores; each lane builds its operand values on the fly from the maps, so no
// item product is ever stored.  Only the 64-cell blocks where F is non-zero
// are summed (the others add exactly nothing), from a list in ascending block
// order split evenly across workgroups (blocks.hip); each
// workgroup writes float64 partial tiles that a second kernel sums in a fixed
// order, and a third gathers the tuple entries.
//
// Matrix-core instructions (gfx950, wave64):
//   float64:  v_mfma_f64_16x16x4_f64    (16x16 tiles, 4 cells per instruction)
//   float32:  v_mfma_f32_32x32x2_f32    (32x32 tiles, 2 cells per instruction)
//   split:    v_mfma_f32_32x32x16_bf16  (32x32 tiles, 16 cells per instruction;
//             n = 3 with at most 16 radii: v_mfma_f32_16x16x32_bf16, one
//             16x16 tile, 32 cells per instruction);
//             each float32 operand is split into three bfloat16 terms
//             x = h + m + l and the six products of order <= 2^-16 relative
//             (hh, hm, mh, hl, mm, lh) are accumulated.
// float32 accumulators are flushed into float64 registers every ~128 cells.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "split3.h"

using namespace conker;

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int NT = 256;
constexpr int WAVES = NT / 64;

// Item code of one lane for one tile: maps (a, b) for the left item and
// (c, d) for the right item.  -1 = no factor (value 1), -2 = padding (value 0).
struct Items {
    int a, b, c, d;
};

// The 64-cell blocks of one workgroup: an equal share (one of gridDim.x) of
// list[0 .. *count) -- the blocks where F is non-zero, in ascending order --
// when a list is given, else of all blocks in order.  Block k starts at cell
// first(k); the last block of the grid may be partial (nc % 16 == 0).
struct Blocks {
    const int *list;
    int k0, k1;
    __device__ size_t first(int k) const { return (size_t)(list ? list[k] : k) * 64; }
};

__device__ __forceinline__ Blocks my_blocks(const int *list, const int *count, size_t nc) {
    const long nall = (long)((nc + 63) / 64);
    const long n = list ? (long)*count : nall;
    if (n == nall) list = nullptr;   // every block listed: they are 0 .. nall - 1 in order
    const long per = (n + (long)gridDim.x - 1) / (long)gridDim.x;
    const long k0 = (long)blockIdx.x * per;
    return Blocks{list, (int)(k0 < n ? k0 : n), (int)(k0 + per < n ? k0 + per : n)};
}

// V consecutive values starting at a 16-byte aligned address, as 16-byte loads
template <typename T, int V>
__device__ __forceinline__ void ld(const T *__restrict__ p, T (&v)[V]) {
    if constexpr (std::is_same<T, float>::value) {
        static_assert(V % 4 == 0, "float loads come in fours");
#pragma unroll
        for (int q = 0; q < V / 4; ++q) {
            const float4 u = reinterpret_cast<const float4 *>(p)[q];
            v[4 * q + 0] = u.x;
            v[4 * q + 1] = u.y;
            v[4 * q + 2] = u.z;
            v[4 * q + 3] = u.w;
        }
    } else {
        static_assert(V % 2 == 0, "double loads come in pairs");
#pragma unroll
        for (int q = 0; q < V / 2; ++q) {
            const double2 u = reinterpret_cast<const double2 *>(p)[q];
            v[2 * q + 0] = u.x;
            v[2 * q + 1] = u.y;
        }
    }
}

// ---------------------------------------------------------------------------
// n = 2: W(a) = sum_x F(x) C_a(x), float64 accumulation
// ---------------------------------------------------------------------------
template <typename T, int NS>
__global__ __launch_bounds__(NT) void k_dot(const T *__restrict__ F, const T *__restrict__ maps,
                                            size_t nc, int n_radii, const int *__restrict__ list,
                                            const int *__restrict__ count, double *__restrict__ partial) {
    constexpr int V = std::is_same<T, float>::value ? 4 : 2;   // cells per 16-byte load
    constexpr int TPB = 64 / V;                                  // threads per block
    double acc[NS];
#pragma unroll
    for (int a = 0; a < NS; ++a) acc[a] = 0.0;
    const Blocks bk = my_blocks(list, count, nc);
    for (int k = bk.k0 + (int)threadIdx.x / TPB; k < bk.k1; k += NT / TPB) {
        const size_t x = bk.first(k) + (size_t)(threadIdx.x % TPB) * V;
        if (x >= nc) continue;
        T f[V];
        ld<T, V>(F + x, f);
#pragma unroll
        for (int a = 0; a < NS; ++a) {
            if (a < n_radii) {
                T m[V];
                ld<T, V>(maps + (size_t)a * nc + x, m);
#pragma unroll
                for (int e = 0; e < V; ++e) acc[a] += (double)f[e] * (double)m[e];
            }
        }
    }
    __shared__ double red[WAVES][NS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < NS; ++a) {
        double v = acc[a];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[w][a] = v;
    }
    __syncthreads();
    if (threadIdx.x < n_radii) {
        double s = 0.0;
        for (int k = 0; k < WAVES; ++k) s += red[k][threadIdx.x];
        partial[(size_t)blockIdx.x * n_radii + threadIdx.x] = s;
    }
}

// One block per radius: strided partial sums, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void k_dot_reduce(const double *__restrict__ partial, int G, int n_radii,
                                                    double *W) {
    const int a = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) s += partial[(size_t)g * n_radii + a];
    __shared__ double t[256];
    t[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) t[threadIdx.x] += t[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) W[a] = t[0];
}

// ---------------------------------------------------------------------------
// operand values: product of up to two maps at V consecutive cells
// ---------------------------------------------------------------------------
template <typename T, int V>
__device__ __forceinline__ void item_vals(const T *__restrict__ maps, size_t nc, size_t x, int a, int b,
                                          T (&v)[V]) {
    if (a == -2) {
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = (T)0;
        return;
    }
    if (a >= 0) {
        ld<T, V>(maps + (size_t)a * nc + x, v);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = (T)1;
    }
    if (b >= 0) {
        T u[V];
        ld<T, V>(maps + (size_t)b * nc + x, u);
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] *= u[e];
    }
}

// ---------------------------------------------------------------------------
// matrix-core kernels.  Grid: (workgroups, tile groups).  Each workgroup of
// four waves handles its share of the summed 64-cell blocks for NBW output
// tiles; the waves split each block, then combine their float64 tiles through
// LDS.
// ---------------------------------------------------------------------------
template <int TS>
__device__ void wave_combine_store(double (&acc)[TS * TS / 64], double *lds, double *out) {
    // acc holds this lane's share of one TS x TS tile in instruction layout
    constexpr int PL = TS * TS / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < PL; ++v) lds[(w * PL + v) * 64 + lane] = acc[v];
    __syncthreads();
    for (int e = threadIdx.x; e < TS * TS; e += NT) {
        // element e = (row i, col j) of the tile; locate its (lane, reg)
        const int i = e / TS, j = e - (e / TS) * TS;
        int l, v;
        if constexpr (TS == 16) {          // f64 16x16x4: lane = j + 16 (i % 4), reg = i / 4
            l = j + 16 * (i & 3);
            v = i >> 2;
        } else {                           // 32x32: lane = j + 32 ((i / 4) % 2), reg = i % 4 + 4 (i / 8)
            l = j + 32 * ((i >> 2) & 1);
            v = (i & 3) + 4 * (i >> 3);
        }
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < WAVES; ++k) s += lds[(k * PL + v) * 64 + l];
        out[e] = s;
    }
    __syncthreads();
}

// float64: 16x16 tiles, each lane feeds row (lane % 16) with the cell of k-slot lane / 16
template <int NBW>
__global__ __launch_bounds__(NT) void k_mm_f64(const double *__restrict__ F, const double *__restrict__ maps,
                                               size_t nc, const int *__restrict__ list,
                                               const int *__restrict__ count, const Items *__restrict__ tab,
                                               int n_tiles, double *__restrict__ partial) {
    constexpr int TS = 16, CPI = 8;   // 4 k-slots x 2 cells per iteration
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, h = lane >> 4;
    Items it[NBW];
    bool live[NBW], same[NBW];
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int tile = blockIdx.y * NBW + s;
        live[s] = tile < n_tiles;
        it[s] = live[s] ? tab[(size_t)tile * TS + r] : Items{-2, -1, -2, -1};
        same[s] = (it[s].a == it[s].c) && (it[s].b == it[s].d);
    }
    doublex4 acc[NBW];
#pragma unroll
    for (int s = 0; s < NBW; ++s) acc[s] = doublex4{0, 0, 0, 0};
    const Blocks bk = my_blocks(list, count, nc);
    size_t xb = bk.k0 < bk.k1 ? bk.first(bk.k0) : 0;
    for (int k = bk.k0; k < bk.k1; ++k) {
    const size_t xn = k + 1 < bk.k1 ? bk.first(k + 1) : 0;
#pragma unroll
    for (int u = 0; u < 64 / (WAVES * CPI); ++u) {   // this wave's cells of the block
        const size_t x0 = xb + (size_t)(u * WAVES + w) * CPI;
        if (x0 >= nc) break;   // the last block of the grid may be partial
        const size_t x = x0 + 2 * h;
        double fv[2];
        ld<double, 2>(F + x, fv);
        const double f0 = fv[0], f1 = fv[1];
#pragma unroll
        for (int s = 0; s < NBW; ++s) {
            if (!live[s]) continue;
            double av[2], bv[2];
            item_vals<double, 2>(maps, nc, x, it[s].a, it[s].b, av);
            if (same[s]) { bv[0] = av[0]; bv[1] = av[1]; }
            else item_vals<double, 2>(maps, nc, x, it[s].c, it[s].d, bv);
            acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0] * f0, bv[0], acc[s], 0, 0, 0);
            acc[s] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1] * f1, bv[1], acc[s], 0, 0, 0);
        }
    }
    xb = xn;
    }
    __shared__ double lds[WAVES * 4 * 64];
    const int G = gridDim.x;
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int tile = blockIdx.y * NBW + s;
        if (tile >= n_tiles) break;
        double a4[4] = {acc[s][0], acc[s][1], acc[s][2], acc[s][3]};
        wave_combine_store<16>(a4, lds, partial + ((size_t)tile * G + blockIdx.x) * (TS * TS));
    }
}

// float32: 32x32 tiles, v_mfma_f32_32x32x2_f32, lane feeds row lane % 32 in k-slot lane / 32
template <int NBW>
__global__ __launch_bounds__(NT) void k_mm_f32(const float *__restrict__ F, const float *__restrict__ maps,
                                               size_t nc, const int *__restrict__ list,
                                               const int *__restrict__ count, const Items *__restrict__ tab,
                                               int n_tiles, double *__restrict__ partial) {
    constexpr int TS = 32, CPI = 8, FLUSH = 16;   // 2 k-slots x 4 cells per iteration
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    Items it[NBW];
    bool live[NBW], same[NBW];
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int tile = blockIdx.y * NBW + s;
        live[s] = tile < n_tiles;
        it[s] = live[s] ? tab[(size_t)tile * TS + r] : Items{-2, -1, -2, -1};
        same[s] = (it[s].a == it[s].c) && (it[s].b == it[s].d);
    }
    floatx16 acc[NBW];
    double accd[NBW][16];
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        acc[s] = floatx16{0};
#pragma unroll
        for (int v = 0; v < 16; ++v) accd[s][v] = 0.0;
    }
    const Blocks bk = my_blocks(list, count, nc);
    size_t xb = bk.k0 < bk.k1 ? bk.first(bk.k0) : 0;
    int cnt = 0;
    for (int k = bk.k0; k < bk.k1; ++k) {
    const size_t xn = k + 1 < bk.k1 ? bk.first(k + 1) : 0;
#pragma unroll
    for (int u = 0; u < 64 / (WAVES * CPI); ++u) {   // this wave's cells of the block
        const size_t x0 = xb + (size_t)(u * WAVES + w) * CPI;
        if (x0 >= nc) break;   // the last block of the grid may be partial
        const size_t x = x0 + 4 * h;
        float f[4];
        ld<float, 4>(F + x, f);
#pragma unroll
        for (int s = 0; s < NBW; ++s) {
            if (!live[s]) continue;
            float av[4], bv[4];
            item_vals<float, 4>(maps, nc, x, it[s].a, it[s].b, av);
            if (same[s]) {
#pragma unroll
                for (int e = 0; e < 4; ++e) bv[e] = av[e];
            } else {
                item_vals<float, 4>(maps, nc, x, it[s].c, it[s].d, bv);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e] * f[e], bv[e], acc[s], 0, 0, 0);
        }
        if (++cnt == FLUSH) {
            cnt = 0;
#pragma unroll
            for (int s = 0; s < NBW; ++s) {
#pragma unroll
                for (int v = 0; v < 16; ++v) accd[s][v] += (double)acc[s][v];
                acc[s] = floatx16{0};
            }
        }
    }
    xb = xn;
    }
    __shared__ double lds[WAVES * 16 * 64];
    const int G = gridDim.x;
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int tile = blockIdx.y * NBW + s;
        if (tile >= n_tiles) break;
        double a16[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) a16[v] = accd[s][v] + (double)acc[s][v];
        wave_combine_store<32>(a16, lds, partial + ((size_t)tile * G + blockIdx.x) * (TS * TS));
    }
}

// split-fp16: each factor x of an operand (the field, or a map of one radius)
// is normalised by 2^s_x, s_x = -(floor(log2 max|x|) + 1), so that it lies
// below 1 in magnitude; an operand (a product of factors) is then scaled by
// 2^(14 + sum s_x) < 2^14, inside the float16 range with room for rounding,
// and split into hi = fp16(v), lo = fp16(v - hi).  All scales are powers of
// two, so scaling and unscaling are exact.  maxabs[m] holds the bits of
// max|maps[m]| (m < ns) and of max|F| (m = ns).
__device__ __forceinline__ int norm_exp(unsigned bits) {
    if (bits == 0u) return 0;
    const int e = (int)((bits >> 23) & 255u) - 127;   // floor(log2) for normal values
    const int s = -(e + 1);
    return s < -100 ? -100 : (s > 100 ? 100 : s);
}

__device__ __forceinline__ int item_exp(const unsigned *maxabs, int ns, int2 it, bool with_f) {
    if (it.x < 0) return 0;
    int s = 14 + norm_exp(maxabs[it.x]);
    if (it.y >= 0) s += norm_exp(maxabs[it.y]);
    if (with_f) s += norm_exp(maxabs[ns]);
    return s;
}

__device__ __forceinline__ void split2h(const float (&v)[8], f16x8 &hi, f16x8 &lo) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const _Float16 h = (_Float16)v[e];
        hi[e] = h;
        lo[e] = (_Float16)(v[e] - (float)h);
    }
}

// max |x| of every map row and of F over the summed blocks (the cells that
// enter any sum), as float bits (non-negative floats order like their bit
// patterns): grid (workgroups, ns + 1).
// With tab (size classes): field z = blockIdx.z is N (z even) or R (z odd) of
// job z / 2, its rows at out + z (ns + 1).
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ F, const float *__restrict__ maps,
                                                size_t nc, int ns, const int *__restrict__ list,
                                                const int *__restrict__ count, unsigned *__restrict__ out,
                                                const ClassJob *__restrict__ tab) {
    __shared__ float red[4];
    if (tab) {
        const ClassJob &j = tab[blockIdx.z >> 1];
        const bool r = blockIdx.z & 1;
        F = r ? j.R : j.N;
        maps = r ? j.mapsR : j.mapsN;
        out += (size_t)blockIdx.z * (ns + 1);
    }
    const int row = blockIdx.y;
    const float *src = row < ns ? maps + (size_t)row * nc : F;
    const Blocks bk = my_blocks(list, count, nc);
    float m = 0.f;
    for (int k = bk.k0 + (int)threadIdx.x / 16; k < bk.k1; k += 256 / 16) {
        const size_t i = bk.first(k) + (size_t)(threadIdx.x & 15) * 4;
        if (i >= nc) continue;
        const float4 v = *reinterpret_cast<const float4 *>(src + i);
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        atomicMax(out + row, __float_as_uint(m));
    }
}

__global__ void k_zero_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Scale exponent of a per-wave item (a, b): constant-1 (-1) and absent factors
// add nothing; padding (-2) holds zeros.
__device__ __forceinline__ int items_exp(const unsigned *maxabs, int ns, int a, int b, bool with_f) {
    if (a == -2) return 0;
    int s = 14;
    if (a >= 0) s += norm_exp(maxabs[a]);
    if (b >= 0) s += norm_exp(maxabs[b]);
    if (with_f) s += norm_exp(maxabs[ns]);
    return s;
}

// split bfloat16 (three terms, six products) or split float16 (scaled, two
// terms, three products): 32x32 tiles, 32x32x16 matrix instructions, lane feeds
// row lane % 32 with the 8 cells of k-slot lane / 32
template <int NBW, int PREC>
__global__ __launch_bounds__(NT) void k_mm_split(const float *__restrict__ F, const float *__restrict__ maps,
                                                 size_t nc, const int *__restrict__ list,
                                                 const int *__restrict__ count, const Items *__restrict__ tab,
                                                 int n_tiles, double *__restrict__ partial, int ns,
                                                 const unsigned *__restrict__ maxabs) {
    constexpr bool F16 = PREC == CONKER_MM_SPLIT_F16;
    constexpr int TS = 32, CPI = 16, FLUSH = 8;   // 2 k-slots x 8 cells per iteration
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    Items it[NBW];
    bool live[NBW], same[NBW];
    int er[NBW], ec[NBW];   // split-f16 scale exponents of this lane's row and column items
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int tile = blockIdx.y * NBW + s;
        live[s] = tile < n_tiles;
        it[s] = live[s] ? tab[(size_t)tile * TS + r] : Items{-2, -1, -2, -1};
        same[s] = (it[s].a == it[s].c) && (it[s].b == it[s].d);
        er[s] = ec[s] = 0;
        if constexpr (F16) {
            er[s] = items_exp(maxabs, ns, it[s].a, it[s].b, true);
            ec[s] = items_exp(maxabs, ns, it[s].c, it[s].d, false);
        }
    }
    floatx16 acc[NBW];
    double accd[NBW][16];
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        acc[s] = floatx16{0};
#pragma unroll
        for (int v = 0; v < 16; ++v) accd[s][v] = 0.0;
    }
    const Blocks bk = my_blocks(list, count, nc);
    size_t xb = bk.k0 < bk.k1 ? bk.first(bk.k0) : 0;
    int cnt = 0;
    for (int k = bk.k0; k < bk.k1; ++k) {
    const size_t xn = k + 1 < bk.k1 ? bk.first(k + 1) : 0;
#pragma unroll
    for (int u = 0; u < 64 / (WAVES * CPI); ++u) {   // this wave's cells of the block
        const size_t x0 = xb + (size_t)(u * WAVES + w) * CPI;
        if (x0 >= nc) break;   // the last block of the grid may be partial
        const size_t x = x0 + 8 * h;
        float f[8];
        ld<float, 8>(F + x, f);
#pragma unroll
        for (int s = 0; s < NBW; ++s) {
            if (!live[s]) continue;
            float cv[8], av[8], bv[8];
            item_vals<float, 8>(maps, nc, x, it[s].a, it[s].b, cv);
            if (same[s]) {
#pragma unroll
                for (int e = 0; e < 8; ++e) bv[e] = cv[e];
            } else {
                item_vals<float, 8>(maps, nc, x, it[s].c, it[s].d, bv);
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) av[e] = cv[e] * f[e];
            if constexpr (F16) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    av[e] = ldexpf(av[e], er[s]);
                    bv[e] = ldexpf(bv[e], ec[s]);
                }
                f16x8 ah, al, bh, bl;
                split2h(av, ah, al);
                split2h(bv, bh, bl);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, acc[s], 0, 0, 0);
            } else {
                bf16x8 ah, am, al, bh, bm, bl;
                split3(av, ah, am, al);
                split3(bv, bh, bm, bl);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc[s], 0, 0, 0);
                acc[s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[s], 0, 0, 0);
            }
        }
        if (++cnt == FLUSH) {
            cnt = 0;
#pragma unroll
            for (int s = 0; s < NBW; ++s) {
#pragma unroll
                for (int v = 0; v < 16; ++v) accd[s][v] += (double)acc[s][v];
                acc[s] = floatx16{0};
            }
        }
    }
    xb = xn;
    }
    __shared__ double lds[WAVES * 16 * 64];
    const int G = gridDim.x;
#pragma unroll
    for (int s = 0; s < NBW; ++s) {
        const int tile = blockIdx.y * NBW + s;
        if (tile >= n_tiles) break;
        double a16[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) a16[v] = accd[s][v] + (double)acc[s][v];
        if constexpr (F16) {   // element (i, j = lane % 32): row exponent from lane i, column exponent ours
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                a16[v] = ldexp(a16[v], -(__shfl(er[s], i) + ec[s]));
            }
        }
        wave_combine_store<32>(a16, lds, partial + ((size_t)tile * G + blockIdx.x) * (TS * TS));
    }
}

// ---------------------------------------------------------------------------
// float32 / split-bf16 matrix-core summation with operands built once per
// chunk.  A workgroup owns a share of the summed 64-cell blocks and a group of up to 24 output
// tiles (a rectangle of row tiles x column tiles).  For every 64 cells it
// stages the maps and F in LDS; for every 16 of those it builds each row item
// (F C_a [C_b]) and column item (C_c [C_d]) of its rectangle once, as three
// bf16 planes (or one float32 plane), in LDS; then each wave runs the matrix
// instructions of its (at most three) tiles from LDS.  Each group stages the
// maps and builds its items anew, so fewer, larger groups cost less: with
// three tiles per wave the 19 tiles of 20 radii at n = 5 are one group.  float32 accumulators are
// flushed into float64 registers every 128 cells.
// ---------------------------------------------------------------------------
struct Group {
    int rt0, nrt, ct0, nct, t0, nt;
};

constexpr int V2_NT = 512, V2_WAVES = V2_NT / 64, V2_MAXU = 4;   // tiles per wave: MAXT, 2 or 3
constexpr int V2_PRE = 3;                       // staged float4 per thread: (64 + 1) * 16 <= 3 * 512
constexpr int V2_LDS_MAX = 150 * 1024;          // dynamic LDS of one k_mm2 workgroup
constexpr int V2_SROW = 68;                     // staged row stride (floats): 64 cells + 4 of padding


template <int PREC, int MAXT>
__global__ __launch_bounds__(V2_NT) void k_mm2(const float *__restrict__ F, const float *__restrict__ maps, size_t nc,
                                              int ns, const int *__restrict__ list, const int *__restrict__ count,
                                              const int2 *__restrict__ ritems,
                                              const int2 *__restrict__ citems, const int2 *__restrict__ tiles,
                                              const Group *__restrict__ groups, int G, double *__restrict__ partial,
                                              const unsigned *__restrict__ maxabs) {
    constexpr bool SPLIT = PREC == CONKER_MM_SPLIT_BF16;
    constexpr bool F16 = PREC == CONKER_MM_SPLIT_F16;
    constexpr int NP = SPLIT ? 3 : (F16 ? 2 : 1);           // operand planes
    constexpr int EB = (SPLIT || F16) ? 2 : 4;              // bytes per operand element
    extern __shared__ __align__(16) unsigned char smem[];
    const Group gr = groups[blockIdx.y];
    // LDS: two staging buffers [2 ns + 3][V2_SROW] (maps, F, a constant row,
    // a row of zeros, then the products P_a = F C_a; rows padded against bank
    // conflicts) and two operand buffers (A planes, then B planes), so that the
    // next 64 cells load while these are summed and the next 16-cell operands
    // build while these multiply.
    const int SZ = (2 * ns + 3) * V2_SROW;
    const int ROW_F = ns, ROW_ONE = ns + 1, ROW_ZERO = ns + 2, ROW_P = ns + 3;
    float *stg0 = reinterpret_cast<float *>(smem);
    const int na = gr.nrt * 32, nb = gr.nct * 32;
    const size_t abytes = (size_t)NP * na * 16 * EB;
    const size_t opb = abytes + (size_t)NP * nb * 16 * EB;
    unsigned char *ops0 = reinterpret_cast<unsigned char *>(stg0 + 2 * SZ);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    // build units of this thread: unit u -> (item, half); items of A first, then B
    // Each unit builds v = S[r0] * S[r1] over 8 cells from two staged rows
    // (P_a, a map or zeros; a map or ones) and stores it at
    // operand offset uoff = 2 item + half (-1: no such unit).  The 32 lanes of
    // a half-wave take the same half of 32 consecutive items, so that their
    // stores are contiguous.
    // Operand layout (bf16 / fp16): planes, then halves, then rows: element
    // (plane p, half h, row i) at (p * 2 + h) * rows + i, 16 bytes each, so the
    // 32 lanes that load one half of a 32-row tile read 512 contiguous bytes.
    const int a_units = na * 2;   // operand offsets below this are rows of A, the rest of B
    int urow[V2_MAXU][2];
    int uoff[V2_MAXU];
    int uexp[V2_MAXU];   // split-fp16 operand scale exponents
#pragma unroll
    for (int k = 0; k < V2_MAXU; ++k) {
        const int u = threadIdx.x + k * V2_NT;
        const int item = ((u >> 6) << 5) | (u & 31), half = (u >> 5) & 1;
        int2 it;
        if (item < na) it = ritems[gr.rt0 * 32 + item];
        else if (item < na + nb) it = citems[gr.ct0 * 32 + (item - na)];
        else it = int2{-3, -1};
        const bool isA = item < na;
        urow[k][0] = it.x >= 0 ? (isA ? ROW_P + it.x : it.x) : ROW_ZERO;
        urow[k][1] = (it.x >= 0 && it.y >= 0) ? it.y : ROW_ONE;
        uoff[k] = it.x == -3 ? -1 : item * 2 + half;   // B rows follow the A rows
        uexp[k] = 0;
        if constexpr (F16) {
            if (it.x >= 0) uexp[k] = item_exp(maxabs, ns, it, isA);
        }
    }
    // tiles of this wave
    int ta[MAXT], tb[MAXT];
    bool tl[MAXT];
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
        const int lt = w + k * V2_WAVES;
        tl[k] = lt < gr.nt;
        const int2 t = tl[k] ? tiles[gr.t0 + lt] : int2{gr.rt0, gr.ct0};
        ta[k] = (t.x - gr.rt0) * 32 + r;
        tb[k] = (t.y - gr.ct0) * 32 + r;
    }
    floatx16 acc[MAXT];
    double dacc[MAXT][16];
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
        acc[k] = floatx16{0};
#pragma unroll
        for (int v = 0; v < 16; ++v) dacc[k][v] = 0.0;
    }
    const Blocks bk = my_blocks(list, count, nc);
    // constant rows of both staging buffers
    for (int e = threadIdx.x; e < 2 * 64; e += V2_NT) {
        const int b = e >> 6, c = e & 63;
        stg0[b * SZ + ROW_ONE * V2_SROW + c] = 1.f;
        stg0[b * SZ + ROW_ZERO * V2_SROW + c] = 0.f;
    }
    // staging of 64 cells: (ns + 1) * 16 float4, at most V2_PRE per thread
    const int nst = (ns + 1) * 16;
    // Three named registers rather than an array: an array that the loads
    // and stores reach through these lambdas ends up in scratch memory,
    // where each load is waited for on the spot instead of in flight while
    // the previous 64 cells are summed.
    static_assert(V2_PRE == 3, "staging registers");
    float4 pre0, pre1, pre2;
    auto load1 = [&](int k, size_t x) {
        const int e = min((int)threadIdx.x + k * V2_NT, nst - 1);   // past the end: repeat the last entry
        const int row = e >> 4, q = e & 15;
        const float *src = row < ns ? maps + (size_t)row * nc + x + 4 * q : F + x + 4 * q;
        return *reinterpret_cast<const float4 *>(src);
    };
    auto fetch = [&](size_t x) {
        pre0 = load1(0, x);
        pre1 = load1(1, x);
        pre2 = load1(2, x);
    };
    auto put1 = [&](float *dst, int k, float4 v) {
        const int e = threadIdx.x + k * V2_NT;
        if (e < nst) reinterpret_cast<float4 *>(dst + (e >> 4) * V2_SROW)[e & 15] = v;
    };
    auto put = [&](float *dst) {
        put1(dst, 0, pre0);
        put1(dst, 1, pre1);
        put1(dst, 2, pre2);
    };
    // rows P_a = F C_a of a staged buffer (after its maps and F are visible)
    auto products = [&](float *buf) {
        for (int e = threadIdx.x; e < ns * 16; e += V2_NT) {
            const int a = e >> 4, q = e & 15;
            const float4 c = reinterpret_cast<const float4 *>(buf + a * V2_SROW)[q];
            const float4 f = reinterpret_cast<const float4 *>(buf + ROW_F * V2_SROW)[q];
            reinterpret_cast<float4 *>(buf + (ROW_P + a) * V2_SROW)[q] =
                float4{f.x * c.x, f.y * c.y, f.z * c.z, f.w * c.w};
        }
    };
    if (bk.k0 < bk.k1) {
        fetch(bk.first(bk.k0));
        put(stg0);
    }
    __syncthreads();
    int since = 0, sb = 0, ob = 0;
    for (int k = bk.k0; k < bk.k1; ++k) {
        const bool more = k + 1 < bk.k1;
        if (more) fetch(bk.first(k + 1));   // in flight while these 64 cells are summed
        products(stg0 + sb * SZ);
        __syncthreads();
        const float *sm_maps = stg0 + sb * SZ;
#pragma unroll 1
        for (int sub = 0; sub < 4; ++sub) {
            unsigned char *sA = ops0 + ob * opb;
            unsigned char *sB = sA + abytes;
            // build the operands of 16 cells
#pragma unroll
            for (int k = 0; k < V2_MAXU; ++k) {
                // a wave's units of one k are 32 consecutive items and the
                // item count is a multiple of 32, so this skips whole waves
                const int o = uoff[k];
                if (o < 0) continue;
                const int half = ((threadIdx.x + k * V2_NT) >> 5) & 1;
                const int cb = sub * 16 + half * 8;
                float v[8];
                {
                    const float4 *p0 = reinterpret_cast<const float4 *>(sm_maps + urow[k][0] * V2_SROW + cb);
                    const float4 *p1 = reinterpret_cast<const float4 *>(sm_maps + urow[k][1] * V2_SROW + cb);
                    const float4 a0 = p0[0], a1 = p0[1], b0 = p1[0], b1 = p1[1];
                    v[0] = a0.x * b0.x; v[1] = a0.y * b0.y; v[2] = a0.z * b0.z; v[3] = a0.w * b0.w;
                    v[4] = a1.x * b1.x; v[5] = a1.y * b1.y; v[6] = a1.z * b1.z; v[7] = a1.w * b1.w;
                }
                const bool isA = o < a_units;
                unsigned char *dst = isA ? sA : sB;
                const int ro = isA ? o : o - a_units;   // (row * 2 + half) within its operand
                const int nrows = isA ? na : nb;
                const int hr = (ro & 1) * nrows + (ro >> 1);   // (half, row) within a plane
                if constexpr (SPLIT) {
                    bf16x8 hi, mi, lo;
                    split3(v, hi, mi, lo);
                    bf16x8 *d = reinterpret_cast<bf16x8 *>(dst);
                    d[0 * nrows * 2 + hr] = hi;
                    d[1 * nrows * 2 + hr] = mi;
                    d[2 * nrows * 2 + hr] = lo;
                } else if constexpr (F16) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = ldexpf(v[e], uexp[k]);
                    f16x8 hi, lo;
                    split2h(v, hi, lo);
                    f16x8 *d = reinterpret_cast<f16x8 *>(dst);
                    d[0 * nrows * 2 + hr] = hi;
                    d[1 * nrows * 2 + hr] = lo;
                } else {
                    float4 *d = reinterpret_cast<float4 *>(dst) + ro * 2;
                    d[0] = float4{v[0], v[1], v[2], v[3]};
                    d[1] = float4{v[4], v[5], v[6], v[7]};
                }
            }
            __syncthreads();
            // matrix instructions of this wave's tiles
#pragma unroll
            for (int k = 0; k < MAXT; ++k) {
                if (!tl[k]) continue;
                if constexpr (SPLIT) {
                    const bf16x8 *A = reinterpret_cast<const bf16x8 *>(sA);
                    const bf16x8 *B = reinterpret_cast<const bf16x8 *>(sB);
                    const bf16x8 ah = A[(0 * 2 + h) * na + ta[k]], am = A[(1 * 2 + h) * na + ta[k]],
                                 al = A[(2 * 2 + h) * na + ta[k]];
                    const bf16x8 bh = B[(0 * 2 + h) * nb + tb[k]], bm = B[(1 * 2 + h) * nb + tb[k]],
                                 bl = B[(2 * 2 + h) * nb + tb[k]];
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[k], 0, 0, 0);
                } else if constexpr (F16) {
                    const f16x8 *A = reinterpret_cast<const f16x8 *>(sA);
                    const f16x8 *B = reinterpret_cast<const f16x8 *>(sB);
                    const f16x8 ah = A[(0 * 2 + h) * na + ta[k]], al = A[(1 * 2 + h) * na + ta[k]];
                    const f16x8 bh = B[(0 * 2 + h) * nb + tb[k]], bl = B[(1 * 2 + h) * nb + tb[k]];
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, acc[k], 0, 0, 0);
                    acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, acc[k], 0, 0, 0);
                } else {
                    const float4 *A = reinterpret_cast<const float4 *>(sA) + (ta[k] * 2 + h) * 2;
                    const float4 *B = reinterpret_cast<const float4 *>(sB) + (tb[k] * 2 + h) * 2;
                    const float4 a0 = A[0], a1 = A[1], b0 = B[0], b1 = B[1];
                    const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                    const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        acc[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[e], bv[e], acc[k], 0, 0, 0);
                }
            }
            ob ^= 1;   // the next sub-step builds into the other operand buffer
        }
        if (more) put(stg0 + (sb ^ 1) * SZ);
        __syncthreads();
        sb ^= 1;
        if (++since == 2) {
            since = 0;
#pragma unroll
            for (int k = 0; k < MAXT; ++k) {
#pragma unroll
                for (int v = 0; v < 16; ++v) dacc[k][v] += (double)acc[k][v];
                acc[k] = floatx16{0};
            }
        }
    }
    // write this wave's tiles: lane l, reg v holds (i = 8 (v / 4) + 4 (l / 32) + v % 4, j = l % 32)
#pragma unroll
    for (int k = 0; k < MAXT; ++k) {
        if (!tl[k]) continue;
        const int tile = gr.t0 + w + k * V2_WAVES;
        double *out = partial + ((size_t)tile * G + blockIdx.x) * 1024;
        int ecol = 0;
        if constexpr (F16) ecol = item_exp(maxabs, ns, citems[(gr.ct0 * 32) + tb[k]], false);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), j = lane & 31;
            double x = dacc[k][v] + (double)acc[k][v];
            if constexpr (F16) {
                const int erow = item_exp(maxabs, ns, ritems[gr.rt0 * 32 + (ta[k] - r) + i], true);
                x = ldexp(x, -(erow + ecol));
            }
            out[i * 32 + j] = x;
        }
    }
}

// Sum the per-workgroup partial tiles in a fixed order, in two levels:
// slice s of every tile element sums workgroups [s*G/S, (s+1)*G/S), then the
// S slice sums are added.  full[tile][e].
constexpr int RED_S = 64;
__global__ void k_tile_reduce1(const double *__restrict__ partial, int n_tiles, int G, int te,
                               double *__restrict__ slices) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // (tile, s, e), e fastest
    if (idx >= (size_t)n_tiles * RED_S * te) return;
    const size_t e = idx % te;
    const size_t s = (idx / te) % RED_S;
    const size_t tile = idx / ((size_t)te * RED_S);
    const int g0 = (int)((long)G * s / RED_S), g1 = (int)((long)G * (s + 1) / RED_S);
    const double *p = partial + tile * (size_t)G * te + e;
    double acc = 0.0;
    for (int g = g0; g < g1; ++g) acc += p[(size_t)g * te];
    slices[idx] = acc;
}

__global__ void k_tile_reduce2(const double *__restrict__ slices, int n_tiles, int te,
                               double *__restrict__ full) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;   // (tile, e)
    if (idx >= (size_t)n_tiles * te) return;
    const size_t e = idx % te, tile = idx / te;
    const double *p = slices + tile * (size_t)RED_S * te + e;
    double acc = 0.0;
    for (int s = 0; s < RED_S; ++s) acc += p[(size_t)s * te];
    full[idx] = acc;
}

__global__ void k_gather(const double *__restrict__ full, const int *__restrict__ where, int64_t count,
                         double *__restrict__ W) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) W[t] = full[where[t]];
}

// Size classes: field z = blockIdx.y (N of job z / 2 for even z, R for odd)
// gathers from its tiles, tile_elems doubles apart.
__global__ void k_gather_jobs(const double *__restrict__ full, size_t tile_elems, const int *__restrict__ where,
                              int64_t count, const ClassJob *__restrict__ tab) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const ClassJob &j = tab[blockIdx.y >> 1];
    double *W = (blockIdx.y & 1) ? j.Wr : j.Wd;
    W[t] = full[(size_t)blockIdx.y * tile_elems + where[t]];
}

// ---------------------------------------------------------------------------
// host-side planning: items, needed tiles, tuple locations
// ---------------------------------------------------------------------------
struct Plan {
    int TS = 0;
    int n_tiles = 0;
    int64_t count = 0;
    Buf *items = nullptr;   // Items [n_tiles][TS]
    Buf *where = nullptr;   // int [count]: index into full[n_tiles][TS*TS]
};

void enumerate_tuples(int ns, int k, std::vector<std::vector<int>> &out) {
    std::vector<int> t(k, 0);
    if (k == 0) return;
    while (true) {
        out.push_back(t);
        int i = k - 1;
        while (i >= 0 && t[i] == ns - 1) --i;
        if (i < 0) break;
        ++t[i];
        for (int j = i + 1; j < k; ++j) t[j] = t[i];
    }
}

// Row and column items of the order-n summation as one matrix product (Eq.
// ksin_delta): rows F C_a (n = 3) or F C_a C_b (a <= b), columns C_b (n = 3,
// 4) or C_c C_d (c <= d).  The tuple a <= b <= c <= d takes row (a, b) and
// column (c, d), so rows are ordered by their larger radius b (then a) and
// columns by their smaller radius c (then d): the needed entries then fill a
// staircase of whole tiles (for 20 radii at n = 5, 19 tiles of 32 x 32 instead
// of 28 in lexicographic order).  row_of / col_of: position of pair (x, y) at
// x ns + y, or of single x at x.
struct ItemLists {
    std::vector<std::pair<int, int>> left, right;
    std::vector<int> row_of, col_of;
};

void item_lists(int ns, int n, ItemLists &L) {
    std::vector<std::vector<int>> pairs;   // lexicographic: by c, then d
    enumerate_tuples(ns, 2, pairs);
    auto singles = [&](std::vector<std::pair<int, int>> &v, std::vector<int> &at) {
        at.assign(ns, -1);
        for (int a = 0; a < ns; ++a) {
            at[a] = (int)v.size();
            v.push_back({a, -1});
        }
    };
    auto pair_list = [&](std::vector<std::pair<int, int>> &v, std::vector<int> &at, bool by_second) {
        std::vector<std::pair<int, int>> ps;
        for (auto &p : pairs) ps.push_back({p[0], p[1]});
        if (by_second)
            std::stable_sort(ps.begin(), ps.end(), [](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                return x.second != y.second ? x.second < y.second : x.first < y.first;
            });
        at.assign((size_t)ns * ns, -1);
        for (auto &p : ps) {
            at[(size_t)p.first * ns + p.second] = (int)v.size();
            v.push_back(p);
        }
    };
    if (n == 3) singles(L.left, L.row_of);
    else pair_list(L.left, L.row_of, true);
    if (n == 5) pair_list(L.right, L.col_of, false);
    else singles(L.right, L.col_of);
}

// row and column position of tuple u (a_1 <= ... <= a_{n-1})
inline std::pair<int, int> tuple_rc(const ItemLists &L, int ns, int n, const std::vector<int> &u) {
    if (n == 3) return {L.row_of[u[0]], L.col_of[u[1]]};
    if (n == 4) return {L.row_of[(size_t)u[0] * ns + u[1]], L.col_of[u[2]]};
    return {L.row_of[(size_t)u[0] * ns + u[1]], L.col_of[(size_t)u[2] * ns + u[3]]};
}

int make_plan(conker_ctx *c, int ns, int n, int TS, Plan &pl) {
    const uint64_t key = ((uint64_t)ns << 16) | ((uint64_t)n << 8) | (uint64_t)TS;
    Buf &bi = c->tables[key * 2];
    Buf &bw = c->tables[key * 2 + 1];
    ItemLists IL;
    item_lists(ns, n, IL);
    const auto &left = IL.left, &right = IL.right;
    const int LT = ((int)left.size() + TS - 1) / TS, RT = ((int)right.size() + TS - 1) / TS;
    std::vector<std::vector<int>> tuples;
    enumerate_tuples(ns, n - 1, tuples);
    pl.count = (int64_t)tuples.size();
    std::vector<int> tile_id(LT * RT, -1);
    std::vector<std::pair<int, int>> tiles;
    std::vector<std::pair<int, int>> rc(tuples.size());
    for (size_t t = 0; t < tuples.size(); ++t) {
        const auto [li, ri] = tuple_rc(IL, ns, n, tuples[t]);
        rc[t] = {li, ri};
        int &id = tile_id[(li / TS) * RT + ri / TS];
        if (id < 0) {
            id = (int)tiles.size();
            tiles.push_back({li / TS, ri / TS});
        }
    }
    pl.n_tiles = (int)tiles.size();
    pl.TS = TS;
    if (!bi.p) {
        std::vector<Items> hi((size_t)pl.n_tiles * TS);
        for (int k = 0; k < pl.n_tiles; ++k)
            for (int r = 0; r < TS; ++r) {
                const int li = tiles[k].first * TS + r, ri = tiles[k].second * TS + r;
                Items &x = hi[(size_t)k * TS + r];
                if (li < (int)left.size()) { x.a = left[li].first; x.b = left[li].second; }
                else { x.a = -2; x.b = -1; }
                if (ri < (int)right.size()) { x.c = right[ri].first; x.d = right[ri].second; }
                else { x.c = -2; x.d = -1; }
            }
        std::vector<int> hw(tuples.size());
        for (size_t t = 0; t < tuples.size(); ++t) {
            const int li = rc[t].first, ri = rc[t].second;
            const int k = tile_id[(li / TS) * RT + ri / TS];
            hw[t] = k * TS * TS + (li % TS) * TS + (ri % TS);
        }
        CK_OK(ws_reserve(c, bi, hi.size() * sizeof(Items)));
        CK_OK(ws_reserve(c, bw, hw.size() * sizeof(int)));
        CK_HIP(c, hipMemcpy(bi.p, hi.data(), hi.size() * sizeof(Items), hipMemcpyHostToDevice));
        CK_HIP(c, hipMemcpy(bw.p, hw.data(), hw.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    pl.items = &bi;
    pl.where = &bw;
    return CONKER_OK;
}

// Plan of the operand-sharing kernel: item tables per row / column tile, the
// needed tiles (same order as make_plan, so `where` from make_plan applies),
// and groups of at most three tiles per wave whose row and column rectangles
// fit LDS.
struct Plan2 {
    int n_tiles = 0, n_groups = 0, max_lds = 0;
    Buf *ritems = nullptr, *citems = nullptr, *tiles = nullptr, *groups = nullptr;
};

int make_plan2(conker_ctx *c, int ns, int n, bool split, int maxt, Plan2 &p2) {
    constexpr int TS = 32;
    const uint64_t key = (((uint64_t)ns << 16) | ((uint64_t)n << 8) | 32u) * 16 + (split ? 8 : 9) + (maxt == 3 ? 2 : 0);
    Buf &bri = c->tables[key * 4 + 0], &bci = c->tables[key * 4 + 1];
    Buf &bti = c->tables[key * 4 + 2], &bgr = c->tables[key * 4 + 3];
    ItemLists IL;
    item_lists(ns, n, IL);
    const auto &left = IL.left, &right = IL.right;
    const int LT = ((int)left.size() + TS - 1) / TS, RT = ((int)right.size() + TS - 1) / TS;
    std::vector<std::vector<int>> tuples;
    enumerate_tuples(ns, n - 1, tuples);
    std::vector<int> tile_id(LT * RT, -1);
    std::vector<std::pair<int, int>> tiles;
    for (auto &u : tuples) {
        const auto [li, ri] = tuple_rc(IL, ns, n, u);
        int &id = tile_id[(li / TS) * RT + ri / TS];
        if (id < 0) {
            id = (int)tiles.size();
            tiles.push_back({li / TS, ri / TS});
        }
    }
    const int eb = split ? 6 : 4;   // LDS bytes per operand element over all planes
    auto lds_of = [&](int nrt, int nct) { return 2 * (2 * ns + 3) * V2_SROW * 4 + 2 * (nrt + nct) * TS * 16 * eb; };
    std::vector<Group> groups;
    int i = 0;
    p2.max_lds = 0;
    while (i < (int)tiles.size()) {
        Group g{tiles[i].first, 1, tiles[i].second, 1, i, 1};
        int rlo = tiles[i].first, rhi = rlo, clo = tiles[i].second, chi = clo;
        int j = i + 1;
        while (j < (int)tiles.size() && j - i < V2_WAVES * maxt) {
            const int nrlo = std::min(rlo, tiles[j].first), nrhi = std::max(rhi, tiles[j].first);
            const int nclo = std::min(clo, tiles[j].second), nchi = std::max(chi, tiles[j].second);
            const int nrt = nrhi - nrlo + 1, nct = nchi - nclo + 1;
            if ((nrt + nct) * TS * 2 > V2_NT * V2_MAXU || lds_of(nrt, nct) > V2_LDS_MAX) break;
            rlo = nrlo; rhi = nrhi; clo = nclo; chi = nchi;
            ++j;
        }
        g.rt0 = rlo; g.nrt = rhi - rlo + 1; g.ct0 = clo; g.nct = chi - clo + 1; g.t0 = i; g.nt = j - i;
        p2.max_lds = std::max(p2.max_lds, lds_of(g.nrt, g.nct));
        groups.push_back(g);
        i = j;
    }
    p2.n_tiles = (int)tiles.size();
    p2.n_groups = (int)groups.size();
    if (!bri.p) {
        std::vector<int2> hr((size_t)LT * TS), hc((size_t)RT * TS), ht(tiles.size());
        for (int k = 0; k < LT * TS; ++k)
            hr[k] = k < (int)left.size() ? int2{left[k].first, left[k].second} : int2{-2, -1};
        for (int k = 0; k < RT * TS; ++k)
            hc[k] = k < (int)right.size() ? int2{right[k].first, right[k].second} : int2{-2, -1};
        for (size_t k = 0; k < tiles.size(); ++k) ht[k] = int2{tiles[k].first, tiles[k].second};
        CK_OK(ws_reserve(c, bri, hr.size() * sizeof(int2)));
        CK_OK(ws_reserve(c, bci, hc.size() * sizeof(int2)));
        CK_OK(ws_reserve(c, bti, ht.size() * sizeof(int2)));
        CK_OK(ws_reserve(c, bgr, groups.size() * sizeof(Group)));
        CK_HIP(c, hipMemcpy(bri.p, hr.data(), hr.size() * sizeof(int2), hipMemcpyHostToDevice));
        CK_HIP(c, hipMemcpy(bci.p, hc.data(), hc.size() * sizeof(int2), hipMemcpyHostToDevice));
        CK_HIP(c, hipMemcpy(bti.p, ht.data(), ht.size() * sizeof(int2), hipMemcpyHostToDevice));
        CK_HIP(c, hipMemcpy(bgr.p, groups.data(), groups.size() * sizeof(Group), hipMemcpyHostToDevice));
    }
    p2.ritems = &bri;
    p2.citems = &bci;
    p2.tiles = &bti;
    p2.groups = &bgr;
    return CONKER_OK;
}

template <typename T>
int contract_dot(conker_ctx *c, const T *F, const T *maps, size_t nc, int ns, const int *list, const int *count,
                 double *W) {
    const int G = (int)std::min<size_t>(2048, std::max<size_t>(1, nc / 4096));
    CK_OK(ws_reserve(c, c->partial, (size_t)G * ns * sizeof(double)));
    double *part = (double *)c->partial.p;
    {
    ProfScope ps(c, PK_CONTRACT_DOT);
    if (ns <= 16)
        hipLaunchKernelGGL((k_dot<T, 16>), dim3(G), dim3(NT), 0, c->stream, F, maps, nc, ns, list, count, part);
    else if (ns <= 32)
        hipLaunchKernelGGL((k_dot<T, 32>), dim3(G), dim3(NT), 0, c->stream, F, maps, nc, ns, list, count, part);
    else
        hipLaunchKernelGGL((k_dot<T, 64>), dim3(G), dim3(NT), 0, c->stream, F, maps, nc, ns, list, count, part);
    CK_LAUNCH(c);
    }
    ProfScope ps(c, PK_CONTRACT_REDUCE);
    hipLaunchKernelGGL(k_dot_reduce, dim3(ns), dim3(256), 0, c->stream, part, G, ns, W);
    CK_LAUNCH(c);
    return CONKER_OK;
}

// ---------------------------------------------------------------------------
// n = 3 with at most 64 radii, split operands: every output tile of the
// product from one load of each map value.  For a 32x32x16 matrix
// instruction lane l holds A[row l % 32][8 cells] and B[8 cells][column l % 32]:
// with row items F C_a and column items C_b these are the same map values, so
// one wave loads C_r and C_{32 + r} (r = l % 32) and F for 16 cells and feeds
// the tiles (0,0) = (F C_r, C_r), (0,1) = (F C_r, C_{32+r}), (1,1) =
// (F C_{32+r}, C_{32+r}) (only the first for ns <= 32), the order in which
// make_plan numbers them.  The loads of the next 16 cells are issued before
// the current ones are used, so a wave keeps one step of loads in flight.
// Cells: each wave takes 16 of every 64-cell block of its workgroup's share.
// ---------------------------------------------------------------------------
// With tab (size classes): field z = blockIdx.y is N (z even) or R (z odd) of
// job z / 2, its scales at maxabs + z (ns + 1) and its tiles after the
// z NTL G partial tiles of the fields before it.
template <int RT, int PREC, bool NEST>
__global__ __launch_bounds__(NT) void k_mm3(const float *__restrict__ F, const float *__restrict__ maps, size_t nc,
                                            const int *__restrict__ list, const int *__restrict__ count, int ns,
                                            double *__restrict__ partial, const unsigned *__restrict__ maxabs,
                                            const ClassJob *__restrict__ tab) {
    constexpr bool F16 = PREC == CONKER_MM_SPLIT_F16;
    constexpr int NTL = RT == 1 ? 1 : 3, TS = 32, CPI = 16, FLUSH = 8;
    if (tab) {
        const ClassJob &jb = tab[blockIdx.y >> 1];
        const bool fr = blockIdx.y & 1;
        F = fr ? jb.R : jb.N;
        maps = fr ? jb.mapsR : jb.mapsN;
        if (maxabs) maxabs += (size_t)blockIdx.y * (ns + 1);
        partial += (size_t)blockIdx.y * NTL * gridDim.x * (TS * TS);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int m0 = r < ns ? r : -1;
    const int m1 = (RT == 2 && 32 + r < ns) ? 32 + r : -1;
    const float *p0 = maps + (size_t)(m0 < 0 ? 0 : m0) * nc;
    const float *p1 = maps + (size_t)(m1 < 0 ? 0 : m1) * nc;
    // split-f16 scale exponents: row items F C_m (with F), column items C_m
    int eA0 = 0, eB0 = 0, eA1 = 0, eB1 = 0;
    if constexpr (F16) {
        eA0 = items_exp(maxabs, ns, m0 < 0 ? -2 : m0, -1, true);
        eB0 = items_exp(maxabs, ns, m0 < 0 ? -2 : m0, -1, false);
        eA1 = items_exp(maxabs, ns, m1 < 0 ? -2 : m1, -1, true);
        eB1 = items_exp(maxabs, ns, m1 < 0 ? -2 : m1, -1, false);
    }
    floatx16 acc[NTL];
    double accd[NTL][16];
#pragma unroll
    for (int s = 0; s < NTL; ++s) {
        acc[s] = floatx16{0};
#pragma unroll
        for (int v = 0; v < 16; ++v) accd[s][v] = 0.0;
    }
    auto mma = [&](floatx16 &a, const float (&av)[8], const float (&bv)[8], int ea, int eb) {
        if constexpr (F16) {
            float sa[8], sb[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                sa[e] = ldexpf(av[e], ea);
                sb[e] = ldexpf(bv[e], eb);
            }
            f16x8 ah, al, bh, bl;
            split2h(sa, ah, al);
            split2h(sb, bh, bl);
            a = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, a, 0, 0, 0);
        } else {
            bf16x8 ah, am, al, bh, bm, bl;
            split3(av, ah, am, al);
            split3(bv, bh, bm, bl);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, a, 0, 0, 0);
        }
    };
    // this wave's 8 cells of a block: x = first(k) + 16 w + 8 h; the last
    // block of the grid may be partial (nc % 16 == 0, so a wave's 16 cells are
    // either all in the grid or all beyond it)
    // Lanes without a map (rows beyond ns) and cells beyond the grid read a
    // valid address (cell 0) and are zeroed by a select: no branches.
    const bool h0 = m0 >= 0, h1 = m1 >= 0;
    float f[8], c0[8], c1[8];
    const Blocks bk = my_blocks(list, count, nc);
    const size_t off = (size_t)w * CPI + 8 * h;
    auto load = [&](int k) {
        const size_t xw = bk.first(k) + (size_t)w * CPI;   // the wave's 16 cells: all in or all out
        const bool in = xw < nc;
        const size_t x = in ? xw + 8 * h : 0;
        ld<float, 8>(F + x, f);
        ld<float, 8>(p0 + x, c0);
        if constexpr (RT == 2) ld<float, 8>(p1 + x, c1);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            f[e] = in ? f[e] : 0.f;
            c0[e] = h0 ? c0[e] : 0.f;
            c1[e] = (RT == 2 && h1) ? c1[e] : 0.f;
        }
    };
    (void)off;
    if (bk.k0 < bk.k1) load(bk.k0);
    auto step = [&](int k) {
        float fc[8], c0c[8], c1c[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            fc[e] = f[e];
            c0c[e] = c0[e];
            c1c[e] = c1[e];
        }
        load(k + 1 < bk.k1 ? k + 1 : k);   // the next block (this one again at the end: no branch)
        float a0[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) a0[e] = fc[e] * c0c[e];
        mma(acc[0], a0, c0c, eA0, eB0);
        if constexpr (RT == 2) {
            float a1[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) a1[e] = fc[e] * c1c[e];
            mma(acc[1], a0, c1c, eA0, eB1);
            mma(acc[2], a1, c1c, eA1, eB1);
        }
    };
    auto flush = [&]() {
#pragma unroll
        for (int s = 0; s < NTL; ++s) {
#pragma unroll
            for (int v = 0; v < 16; ++v) accd[s][v] += (double)acc[s][v];
            acc[s] = floatx16{0};
        }
    };
    if constexpr (NEST) {
        // FLUSH blocks into the float32 accumulators, then float64: the inner
        // loop keeps them in the matrix-core registers (with a flush counter in
        // a single loop the compiler copies them out and back every block).
        // One tile only: with three (NEST false) the nested form measured
        // slower (127 -> 155 ms on 1024^3 x 40 radii), the flat one stays.
        for (int k = bk.k0; k < bk.k1;) {
            const int kend = k + FLUSH < bk.k1 ? k + FLUSH : bk.k1;
            for (; k < kend; ++k) step(k);
            flush();
        }
    } else {
        int cnt = 0;
        for (int k = bk.k0; k < bk.k1; ++k) {
            step(k);
            if (++cnt == FLUSH) {
                cnt = 0;
                flush();
            }
        }
    }
    __shared__ double lds[WAVES * 16 * 64];
    const int G = gridDim.x;
#pragma unroll
    for (int s = 0; s < NTL; ++s) {
        double a16[16];
#pragma unroll
        for (int v = 0; v < 16; ++v) a16[v] = accd[s][v] + (double)acc[s][v];
        if constexpr (F16) {   // element (i, j = lane % 32): row exponent of lane i, column exponent ours
            const int er = s == 2 ? eA1 : eA0, ec = s == 0 ? eB0 : eB1;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                a16[v] = ldexp(a16[v], -(__shfl(er, i) + ec));
            }
        }
        wave_combine_store<32>(a16, lds, partial + ((size_t)s * G + blockIdx.x) * (TS * TS));
    }
}

// n = 3 with at most 16 radii: one 16 x 16 tile (v_mfma_f32_16x16x32_bf16 /
// _f16, 32 cells per instruction), so no lane carries a padding row as it
// would in a 32 x 32 tile.  Lane: row and column r = lane % 16, cells
// 8 (lane / 16) .. + 7 of its wave's 32; two waves per 64-cell block, two
// blocks per step of the workgroup.  Output element (i, j) of the tile sits
// in lane j + 16 (i / 4), register i % 4.  The tile is written into the
// upper-left corner of a 32 x 32 partial tile (zeros elsewhere), the layout
// the reduction and gather of the 32 x 32 plan read.
template <int PREC>
__global__ __launch_bounds__(NT) void k_mm3s(const float *__restrict__ F, const float *__restrict__ maps, size_t nc,
                                             const int *__restrict__ list, const int *__restrict__ count, int ns,
                                             double *__restrict__ partial, const unsigned *__restrict__ maxabs,
                                             const ClassJob *__restrict__ tab) {
    constexpr bool F16 = PREC == CONKER_MM_SPLIT_F16;
    constexpr int FLUSH = 4;   // float32 sums over 128 cells per lane, then float64
    typedef float floatx4 __attribute__((ext_vector_type(4)));
    if (tab) {
        const ClassJob &jb = tab[blockIdx.y >> 1];
        const bool fr = blockIdx.y & 1;
        F = fr ? jb.R : jb.N;
        maps = fr ? jb.mapsR : jb.mapsN;
        if (maxabs) maxabs += (size_t)blockIdx.y * (ns + 1);
        partial += (size_t)blockIdx.y * gridDim.x * 1024;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, h = lane >> 4;
    const int m0 = r < ns ? r : -1;
    const float *p0 = maps + (size_t)(m0 < 0 ? 0 : m0) * nc;
    int eA = 0, eB = 0;
    if constexpr (F16) {
        eA = items_exp(maxabs, ns, m0 < 0 ? -2 : m0, -1, true);
        eB = items_exp(maxabs, ns, m0 < 0 ? -2 : m0, -1, false);
    }
    floatx4 acc = floatx4{0};
    double accd[4] = {0.0, 0.0, 0.0, 0.0};
    const bool hm = m0 >= 0;
    float f[8], c0[8];
    const Blocks bk = my_blocks(list, count, nc);
    const int half = w & 1, pairw = w >> 1;
    // Blocks beyond the workgroup's share, cells beyond the grid (nc % 16 == 0:
    // a lane's 8 cells are all in or all out) and lanes without a map read a
    // valid address and are zeroed by a select.
    auto load = [&](int k) {
        const int kb = k + pairw;
        const bool inb = kb < bk.k1;
        const size_t xw = bk.first(inb ? kb : k) + (size_t)half * 32 + 8 * h;
        const bool in = inb && xw < nc;
        const size_t x = in ? xw : 0;
        ld<float, 8>(F + x, f);
        ld<float, 8>(p0 + x, c0);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            f[e] = in ? f[e] : 0.f;
            c0[e] = hm ? c0[e] : 0.f;
        }
    };
    if (bk.k0 < bk.k1) load(bk.k0);
    int cnt = 0;
    for (int k = bk.k0; k < bk.k1; k += 2) {
        float a[8], b[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            a[e] = f[e] * c0[e];
            b[e] = c0[e];
        }
        load(k + 2 < bk.k1 ? k + 2 : k);
        if constexpr (F16) {
            float sa[8], sb[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                sa[e] = ldexpf(a[e], eA);
                sb[e] = ldexpf(b[e], eB);
            }
            f16x8 ah, al, bh, bl;
            split2h(sa, ah, al);
            split2h(sb, bh, bl);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, acc, 0, 0, 0);
        } else {
            bf16x8 ah, am, al, bh, bm, bl;
            split3(a, ah, am, al);
            split3(b, bh, bm, bl);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
        }
        if (++cnt == FLUSH) {
            cnt = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) accd[v] += (double)acc[v];
            acc = floatx4{0};
        }
    }
    __shared__ double lds[WAVES * 4 * 64];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double t = accd[v] + (double)acc[v];
        if constexpr (F16) t = ldexp(t, -(__shfl(eA, 4 * h + v) + eB));   // row 4 h + v, column r
        lds[(w * 4 + v) * 64 + lane] = t;
    }
    __syncthreads();
    double *out = partial + (size_t)blockIdx.x * 1024;
    for (int e = threadIdx.x; e < 1024; e += NT) {
        const int i = e >> 5, j = e & 31;
        double s = 0.0;
        if (i < 16 && j < 16) {
            const int l = j + 16 * (i >> 2), v = i & 3;
#pragma unroll
            for (int q = 0; q < WAVES; ++q) s += lds[(q * 4 + v) * 64 + l];
        }
        out[e] = s;
    }
}

// n = 3, split bfloat16, 33..16 NG radii (NG = 3): NG groups of 16 radii, one 16 x 16
// tile (v_mfma_f32_16x16x32_bf16) for every pair of groups gi <= gj, 32 cells
// per instruction (the 32 x 32 tiles of k_mm3 carry up to 31 rows of padding
// here and twice the instruction cycles per cell).  Lane (r, h) holds map
// 16 g + r of every group at cells 8 h .. 8 h + 7 of its wave's 32; each map
// is split once as a column operand and once (times F) as a row operand.  The
// 16 x 16 tiles are written into the three 32 x 32 partial tiles of the
// summation plan (rows a, columns b >= a: tile 0 = (a, b) < 32, tile 1 =
// a < 32 <= b, tile 2 = 32 <= a, b), zeros elsewhere.
template <int NG>
__global__ __launch_bounds__(NT) void k_mm3g(const float *__restrict__ F, const float *__restrict__ maps, size_t nc,
                                             const int *__restrict__ list, const int *__restrict__ count, int ns,
                                             double *__restrict__ partial, const ClassJob *__restrict__ tab) {
    constexpr int NTT = NG * (NG + 1) / 2, FLUSH = 4;
    if (tab) {
        const ClassJob &jb = tab[blockIdx.y >> 1];
        const bool fr = blockIdx.y & 1;
        F = fr ? jb.R : jb.N;
        maps = fr ? jb.mapsR : jb.mapsN;
        partial += (size_t)blockIdx.y * 3 * gridDim.x * 1024;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, h = lane >> 4;
    const float *pg[NG];
    bool hg[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int m = 16 * g + r;
        hg[g] = m < ns;
        pg[g] = maps + (size_t)(hg[g] ? m : 0) * nc;
    }
    floatx4_t acc[NTT];
    double accd[NTT][4];
#pragma unroll
    for (int t = 0; t < NTT; ++t) {
        acc[t] = floatx4_t{0};
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[t][v] = 0.0;
    }
    float f[8], c[NG][8];
    const Blocks bk = my_blocks(list, count, nc);
    const int half = w & 1, pairw = w >> 1;
    auto load = [&](int k) {   // as k_mm3s: two waves per block, two blocks per step
        const int kb = k + pairw;
        const bool inb = kb < bk.k1;
        const size_t xw = bk.first(inb ? kb : k) + (size_t)half * 32 + 8 * h;
        const bool in = inb && xw < nc;
        const size_t x = in ? xw : 0;
        ld<float, 8>(F + x, f);
#pragma unroll
        for (int g = 0; g < NG; ++g) ld<float, 8>(pg[g] + x, c[g]);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            f[e] = in ? f[e] : 0.f;
#pragma unroll
            for (int g = 0; g < NG; ++g) c[g][e] = hg[g] ? c[g][e] : 0.f;
        }
    };
    if (bk.k0 < bk.k1) load(bk.k0);
    for (int k = bk.k0; k < bk.k1;) {
        const int kend = k + 2 * FLUSH < bk.k1 ? k + 2 * FLUSH : bk.k1;
        for (; k < kend; k += 2) {
            float fc[8], cc[NG][8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                fc[e] = f[e];
#pragma unroll
                for (int g = 0; g < NG; ++g) cc[g][e] = c[g][e];
            }
            load(k + 2 < bk.k1 ? k + 2 : k);
            bf16x8_t bh[NG], bm[NG], bl[NG];
#pragma unroll
            for (int g = 0; g < NG; ++g) split3(cc[g], bh[g], bm[g], bl[g]);
            int t = 0;
#pragma unroll
            for (int gi = 0; gi < NG; ++gi) {
                float a[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) a[e] = fc[e] * cc[gi][e];
                bf16x8_t ah, am, al;
                split3(a, ah, am, al);
#pragma unroll
                for (int gj = gi; gj < NG; ++gj, ++t) {
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[gj], acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm[gj], acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[gj], acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh[gj], acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm[gj], acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[gj], acc[t], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NTT; ++t) {
#pragma unroll
            for (int v = 0; v < 4; ++v) accd[t][v] += (double)acc[t][v];
            acc[t] = floatx4_t{0};
        }
    }
    // the workgroup's three 32 x 32 partial tiles: zeros, then each 16 x 16
    // tile summed over the waves (element (i, j) of a tile: lane j + 16 (i / 4),
    // register i % 4) at rows 16 gi + i, columns 16 gj + j
    __shared__ double red[WAVES * 4 * 64];
    const int G = gridDim.x;
    for (int e = threadIdx.x; e < 3 * 1024; e += NT) partial[((size_t)(e >> 10) * G + blockIdx.x) * 1024 + (e & 1023)] = 0.0;
    int t = 0;
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
#pragma unroll
        for (int gj = gi; gj < NG; ++gj, ++t) {
            __syncthreads();   // the previous tile's reads of red (and the zeros) are done
#pragma unroll
            for (int v = 0; v < 4; ++v) red[(w * 4 + v) * 64 + lane] = accd[t][v];
            __syncthreads();
            const int tile = gi < 2 ? (gj < 2 ? 0 : 1) : 2;
            double *out = partial + ((size_t)tile * G + blockIdx.x) * 1024;
            const int r0 = (gi & 1) * 16, c0 = (gj & 1) * 16;
            for (int e = threadIdx.x; e < 256; e += NT) {
                const int i = e >> 4, j = e & 15;
                const int l = j + 16 * (i >> 2), v = i & 3;
                double sum = 0.0;
#pragma unroll
                for (int q = 0; q < WAVES; ++q) sum += red[(q * 4 + v) * 64 + l];
                out[(r0 + i) * 32 + c0 + j] = sum;
            }
        }
    }
}

template <int NBW>
int launch_mm(conker_ctx *c, conker_mmprec prec, dim3 grid, const void *F, const void *maps, size_t nc,
              const int *list, const int *count, const Items *tab, int n_tiles, double *part, int ns,
              const unsigned *maxabs) {
    if (prec == CONKER_MM_F64)
        hipLaunchKernelGGL((k_mm_f64<NBW>), grid, dim3(NT), 0, c->stream, (const double *)F,
                           (const double *)maps, nc, list, count, tab, n_tiles, part);
    else if (prec == CONKER_MM_F32)
        hipLaunchKernelGGL((k_mm_f32<NBW>), grid, dim3(NT), 0, c->stream, (const float *)F,
                           (const float *)maps, nc, list, count, tab, n_tiles, part);
    else if (prec == CONKER_MM_SPLIT_F16)
        hipLaunchKernelGGL((k_mm_split<NBW, CONKER_MM_SPLIT_F16>), grid, dim3(NT), 0, c->stream, (const float *)F,
                           (const float *)maps, nc, list, count, tab, n_tiles, part, ns, maxabs);
    else
        hipLaunchKernelGGL((k_mm_split<NBW, CONKER_MM_SPLIT_BF16>), grid, dim3(NT), 0, c->stream,
                           (const float *)F, (const float *)maps, nc, list, count, tab, n_tiles, part, ns,
                           (const unsigned *)nullptr);
    CK_LAUNCH(c);
    return CONKER_OK;
}

}  // namespace

extern "C" int conker_contract_npt(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *F,
                                   const void *maps, int ns, int n, conker_mmprec prec, double *W) {
    CK_OK(check_grid(c, g, false));
    if (!F || !maps || !W) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (n < 2 || n > 5) return fail(c, CONKER_EINVAL, "order n=%d outside 2..5", n);
    if (ns < 1 || ns > 64) return fail(c, CONKER_EINVAL, "n_radii=%d outside 1..64", ns);
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (prec == CONKER_MM_F64 && dt != CONKER_F64)
        return fail(c, CONKER_EINVAL, "float64 summation needs float64 maps");
    if ((prec == CONKER_MM_F32 || prec == CONKER_MM_SPLIT_BF16 || prec == CONKER_MM_SPLIT_F16) && dt != CONKER_F32)
        return fail(c, CONKER_EINVAL, "float32, split-bf16 and split-f16 summation need float32 maps");
    if (prec != CONKER_MM_F64 && prec != CONKER_MM_F32 && prec != CONKER_MM_SPLIT_BF16 &&
        prec != CONKER_MM_SPLIT_F16)
        return fail(c, CONKER_EINVAL, "bad precision");
    const size_t nc = ncells(g);
    if (nc % 16) return fail(c, CONKER_EUNSUPPORTED, "cell count must be a multiple of 16");
    CK_HIP(c, hipSetDevice(c->device));
    // only the 64-cell blocks holding a non-zero F are summed
    const int *blist = nullptr, *bcount = nullptr;
    CK_OK(block_list(c, F, dt == CONKER_F64, nc, &blist, &bcount));
    if (n == 2) {
        if (dt == CONKER_F64)
            return contract_dot<double>(c, (const double *)F, (const double *)maps, nc, ns, blist, bcount, W);
        return contract_dot<float>(c, (const float *)F, (const float *)maps, nc, ns, blist, bcount, W);
    }
    const int TS = prec == CONKER_MM_F64 ? 16 : 32;
    Plan pl;
    CK_OK(make_plan(c, ns, n, TS, pl));
    // Operand-sharing kernel (k_mm2) for many tiles (pair products, n >= 4, and
    // split-f16); per-wave tiles (k_mm_*) when the tuples fit a few 32 x 32
    // tiles, where k_mm2 would leave most waves of a workgroup idle.
    static const int mm_env = [] {
        const char *e = std::getenv("CONKER_MM_KERNEL");
        return e ? std::atoi(e) : 0;   // 0 auto, 1 per-wave tiles, 2 operand sharing, 3 n = 3 all tiles per wave
    }();
    const int mm_kernel = c->tune.mm_kernel ? c->tune.mm_kernel : mm_env;
    const bool use_v2 = prec != CONKER_MM_F64 && (mm_kernel == 2 || (mm_kernel == 0 && pl.n_tiles > 4)) &&
                        !(mm_kernel == 3 && n == 3);
    unsigned *maxabs = nullptr;
    if (prec == CONKER_MM_SPLIT_F16) {   // largest |value| of every map and of F, after the workspace below
        CK_OK(ws_reserve(c, c->scales, 256 * sizeof(unsigned)));
        ProfScope ps(c, PK_CONTRACT_DOT);
        maxabs = (unsigned *)c->scales.p;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(128), 0, c->stream, maxabs, ns + 1);
        CK_LAUNCH(c);
        const size_t mchunk = 64 * 1024;
        const dim3 mg((unsigned)((nc + mchunk - 1) / mchunk), (unsigned)(ns + 1));
        hipLaunchKernelGGL(k_absmax, mg, dim3(256), 0, c->stream, (const float *)F, (const float *)maps, nc, ns,
                           blist, bcount, maxabs, (const ClassJob *)nullptr);
        CK_LAUNCH(c);
    }
    if (use_v2) {
        // operand-sharing matrix-core kernel: three tiles per wave where that
        // makes fewer groups (each group stages the maps and builds its items
        // anew), else two (fewer registers)
        const bool split = prec == CONKER_MM_SPLIT_BF16;
        Plan2 p2;
        int maxt = 2;
        CK_OK(make_plan2(c, ns, n, split, 2, p2));
        {
            Plan2 p3;
            CK_OK(make_plan2(c, ns, n, split, 3, p3));
            if (p3.n_groups < p2.n_groups) {
                p2 = p3;
                maxt = 3;
            }
        }
        if (nc % 64) return fail(c, CONKER_EUNSUPPORTED, "cell count must be a multiple of 64");
        const size_t G = std::max<size_t>(1, std::min<size_t>(nc / 512, 1024 / (size_t)p2.n_groups));
        const int te = 1024;
        const size_t full_b = (size_t)p2.n_tiles * te * (RED_S + 1) * sizeof(double);
        CK_OK(ws_reserve(c, c->partial, (size_t)p2.n_tiles * G * te * sizeof(double)));
        CK_OK(ws_reserve(c, c->full, full_b));
        double *part = (double *)c->partial.p;
        {
            ProfScope ps(c, PK_CONTRACT_MM);
            dim3 grid((unsigned)G, (unsigned)p2.n_groups);
            static bool attr_set = false;
            if (!attr_set) {
                const void *ks[] = {(const void *)k_mm2<CONKER_MM_SPLIT_BF16, 2>, (const void *)k_mm2<CONKER_MM_F32, 2>,
                                    (const void *)k_mm2<CONKER_MM_SPLIT_F16, 2>, (const void *)k_mm2<CONKER_MM_SPLIT_BF16, 3>,
                                    (const void *)k_mm2<CONKER_MM_F32, 3>, (const void *)k_mm2<CONKER_MM_SPLIT_F16, 3>};
                for (const void *k : ks)
                    CK_HIP(c, hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, V2_LDS_MAX));
                attr_set = true;
            }
            auto launch = [&](auto kern) {
                hipLaunchKernelGGL(kern, grid, dim3(V2_NT), p2.max_lds, c->stream, (const float *)F,
                                   (const float *)maps, nc, ns, blist, bcount, (const int2 *)p2.ritems->p,
                                   (const int2 *)p2.citems->p, (const int2 *)p2.tiles->p,
                                   (const Group *)p2.groups->p, (int)G, part, (const unsigned *)maxabs);
            };
            if (prec == CONKER_MM_SPLIT_BF16)
                maxt == 3 ? launch(k_mm2<CONKER_MM_SPLIT_BF16, 3>) : launch(k_mm2<CONKER_MM_SPLIT_BF16, 2>);
            else if (prec == CONKER_MM_SPLIT_F16)
                maxt == 3 ? launch(k_mm2<CONKER_MM_SPLIT_F16, 3>) : launch(k_mm2<CONKER_MM_SPLIT_F16, 2>);
            else
                maxt == 3 ? launch(k_mm2<CONKER_MM_F32, 3>) : launch(k_mm2<CONKER_MM_F32, 2>);
            CK_LAUNCH(c);
        }
        ProfScope ps(c, PK_CONTRACT_REDUCE);
        const size_t tot = (size_t)p2.n_tiles * te;
        double *full = (double *)c->full.p;
        double *slices = full + tot;
        hipLaunchKernelGGL(k_tile_reduce1, dim3((unsigned)((tot * RED_S + 255) / 256)), dim3(256), 0, c->stream,
                           part, p2.n_tiles, (int)G, te, slices);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_tile_reduce2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, slices,
                           p2.n_tiles, te, full);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_gather, dim3((unsigned)((pl.count + 255) / 256)), dim3(256), 0, c->stream,
                           (const double *)full, (const int *)pl.where->p, pl.count, W);
        CK_LAUNCH(c);
        return CONKER_OK;
    }
    // n = 3, at most 64 radii, split operands: every tile from one load of the maps
    const bool use_mm3 = n == 3 && ns <= 64 && (prec == CONKER_MM_SPLIT_BF16 || prec == CONKER_MM_SPLIT_F16) &&
                         (mm_kernel == 3 || mm_kernel == 0);
    if (use_mm3) {
        const int RT = ns <= 16 ? 0 : (ns <= 32 ? 1 : 2);
        if (pl.n_tiles != (RT <= 1 ? 1 : 3)) return fail(c, CONKER_EINVAL, "unexpected tile plan");
        const size_t G = std::max<size_t>(1, std::min<size_t>(nc / 1024, (size_t)8 * cu_count(c)));
        const int te = TS * TS;
        CK_OK(ws_reserve(c, c->partial, (size_t)pl.n_tiles * G * te * sizeof(double)));
        CK_OK(ws_reserve(c, c->full, (size_t)pl.n_tiles * te * (RED_S + 1) * sizeof(double)));
        double *part = (double *)c->partial.p;
        {
            ProfScope ps(c, PK_CONTRACT_MM);
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(NT), 0, c->stream, (const float *)F,
                                   (const float *)maps, nc, blist, bcount, ns, part, (const unsigned *)maxabs,
                                   (const ClassJob *)nullptr);
            };
            if (RT == 0) {
                if (prec == CONKER_MM_SPLIT_F16) go(k_mm3s<CONKER_MM_SPLIT_F16>);
                else go(k_mm3s<CONKER_MM_SPLIT_BF16>);
            } else if (RT == 1) {
                if (prec == CONKER_MM_SPLIT_F16) go(k_mm3<1, CONKER_MM_SPLIT_F16, true>);
                else go(k_mm3<1, CONKER_MM_SPLIT_BF16, true>);
            } else if (prec == CONKER_MM_SPLIT_BF16 && ns <= 48) {   // 16 x 16 tiles over three groups of radii
                hipLaunchKernelGGL(k_mm3g<3>, dim3((unsigned)G), dim3(NT), 0, c->stream, (const float *)F,
                                   (const float *)maps, nc, blist, bcount, ns, part, (const ClassJob *)nullptr);
            } else {   // four groups would need more registers than two waves per SIMD allow
                if (prec == CONKER_MM_SPLIT_F16) go(k_mm3<2, CONKER_MM_SPLIT_F16, false>);
                else go(k_mm3<2, CONKER_MM_SPLIT_BF16, false>);
            }
            CK_LAUNCH(c);
        }
        ProfScope ps(c, PK_CONTRACT_REDUCE);
        const size_t tot = (size_t)pl.n_tiles * te;
        double *full = (double *)c->full.p;
        double *slices = full + tot;
        hipLaunchKernelGGL(k_tile_reduce1, dim3((unsigned)((tot * RED_S + 255) / 256)), dim3(256), 0, c->stream,
                           part, pl.n_tiles, (int)G, te, slices);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_tile_reduce2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, slices,
                           pl.n_tiles, te, full);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_gather, dim3((unsigned)((pl.count + 255) / 256)), dim3(256), 0, c->stream,
                           (const double *)full, (const int *)pl.where->p, pl.count, W);
        CK_LAUNCH(c);
        return CONKER_OK;
    }
    const int NBW = pl.n_tiles == 1 ? 1 : (prec == CONKER_MM_F64 ? 4 : 2);
    const int groups = (pl.n_tiles + NBW - 1) / NBW;
    // ~4096 workgroups in total, each with an equal share of the summed blocks
    const size_t G = std::max<size_t>(1, std::min<size_t>(nc / 1024, 4096 / (size_t)groups));
    const int te = TS * TS;
    CK_OK(ws_reserve(c, c->partial, (size_t)pl.n_tiles * G * te * sizeof(double)));
    CK_OK(ws_reserve(c, c->full, (size_t)pl.n_tiles * te * (RED_S + 1) * sizeof(double)));
    double *part = (double *)c->partial.p;
    const Items *tab = (const Items *)pl.items->p;
    dim3 grid((unsigned)G, (unsigned)groups);
    {
    ProfScope ps(c, PK_CONTRACT_MM);
    if (NBW == 1) CK_OK(launch_mm<1>(c, prec, grid, F, maps, nc, blist, bcount, tab, pl.n_tiles, part, ns, maxabs));
    else if (NBW == 2) CK_OK(launch_mm<2>(c, prec, grid, F, maps, nc, blist, bcount, tab, pl.n_tiles, part, ns, maxabs));
    else CK_OK(launch_mm<4>(c, prec, grid, F, maps, nc, blist, bcount, tab, pl.n_tiles, part, ns, maxabs));
    }
    ProfScope ps(c, PK_CONTRACT_REDUCE);
    const size_t tot = (size_t)pl.n_tiles * te;
    double *full = (double *)c->full.p;
    double *slices = full + tot;
    hipLaunchKernelGGL(k_tile_reduce1, dim3((unsigned)((tot * RED_S + 255) / 256)), dim3(256), 0, c->stream,
                       part, pl.n_tiles, (int)G, te, slices);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_tile_reduce2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, slices,
                       pl.n_tiles, te, full);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((pl.count + 255) / 256)), dim3(256), 0, c->stream,
                       (const double *)full, (const int *)pl.where->p, pl.count, W);
    CK_LAUNCH(c);
    return CONKER_OK;
}

// ---------------------------------------------------------------------------
// Order 3 for every job of a size class (batch.hip): absmax (split-f16), one
// summation launch over all 2M fields (every 64-cell block: size classes are
// full boxes), one two-level reduction over all their tiles, one gather.
// ---------------------------------------------------------------------------
namespace {
struct Jobs3Layout {
    int G, ntl;
    size_t maxabs_off, part_off, full_off, bytes;
};
Jobs3Layout jobs3_layout(conker_ctx *c, size_t nc, int M, int ns) {
    Jobs3Layout L;
    L.ntl = ns <= 32 ? 1 : 3;
    L.G = (int)std::max<size_t>(1, std::min<size_t>(nc / 1024, (size_t)8 * cu_count(c) / (2 * (size_t)M)));
    const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t nf = 2 * (size_t)M, te = 1024;
    L.maxabs_off = 0;
    L.part_off = up(nf * (ns + 1) * sizeof(unsigned));
    L.full_off = L.part_off + up(nf * L.ntl * (size_t)L.G * te * sizeof(double));
    L.bytes = L.full_off + up(nf * L.ntl * te * (RED_S + 1) * sizeof(double));
    return L;
}
}  // namespace

namespace conker {

size_t contract3_jobs_bytes(conker_ctx *c, const conker_grid *g, int M, int ns) {
    return jobs3_layout(c, ncells(g), M, ns).bytes;
}

int reduce3_jobs(conker_ctx *c, int M, const ClassJob *tab, int ns, int G, const double *part, double *full) {
    Plan pl;
    CK_OK(make_plan(c, ns, 3, 32, pl));
    if (pl.n_tiles != 1) return fail(c, CONKER_EINVAL, "unexpected tile plan");
    ProfScope ps(c, PK_CONTRACT_REDUCE);
    const int te = 1024, tiles = 2 * M;
    const size_t tot = (size_t)tiles * te;
    double *slices = full + tot;
    hipLaunchKernelGGL(k_tile_reduce1, dim3((unsigned)((tot * RED_S + 255) / 256)), dim3(256), 0, c->stream, part,
                       tiles, G, te, slices);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_tile_reduce2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, slices, tiles,
                       te, full);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_gather_jobs, dim3((unsigned)((pl.count + 255) / 256), (unsigned)tiles), dim3(256), 0,
                       c->stream, (const double *)full, (size_t)te, (const int *)pl.where->p, pl.count, tab);
    CK_LAUNCH(c);
    return CONKER_OK;
}

int contract3_jobs(conker_ctx *c, const conker_grid *g, int M, const ClassJob *tab, int ns, conker_mmprec prec,
                   void *ws) {
    if (ns < 1 || ns > 64) return fail(c, CONKER_EINVAL, "size class: n_radii=%d outside 1..64", ns);
    if (prec != CONKER_MM_SPLIT_BF16 && prec != CONKER_MM_SPLIT_F16)
        return fail(c, CONKER_EINVAL, "size class: split summation only");
    const size_t nc = ncells(g);
    if (nc % 64) return fail(c, CONKER_EUNSUPPORTED, "cell count must be a multiple of 64");
    const Jobs3Layout L = jobs3_layout(c, nc, M, ns);
    Plan pl;
    CK_OK(make_plan(c, ns, 3, 32, pl));
    if (pl.n_tiles != L.ntl) return fail(c, CONKER_EINVAL, "unexpected tile plan");
    char *base = (char *)ws;
    unsigned *maxabs = (unsigned *)(base + L.maxabs_off);
    double *part = (double *)(base + L.part_off);
    double *full = (double *)(base + L.full_off);
    const unsigned nf = 2u * (unsigned)M;
    if (prec == CONKER_MM_SPLIT_F16) {
        ProfScope ps(c, PK_CONTRACT_DOT);
        const int nz = (int)nf * (ns + 1);
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((nz + 127) / 128)), dim3(128), 0, c->stream, maxabs, nz);
        CK_LAUNCH(c);
        const size_t mchunk = 64 * 1024;
        const dim3 mg((unsigned)((nc + mchunk - 1) / mchunk), (unsigned)(ns + 1), nf);
        hipLaunchKernelGGL(k_absmax, mg, dim3(256), 0, c->stream, (const float *)nullptr, (const float *)nullptr, nc,
                           ns, (const int *)nullptr, (const int *)nullptr, maxabs, tab);
        CK_LAUNCH(c);
    }
    {
        ProfScope ps(c, PK_CONTRACT_MM);
        const dim3 grid((unsigned)L.G, nf);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(NT), 0, c->stream, (const float *)nullptr, (const float *)nullptr, nc,
                               (const int *)nullptr, (const int *)nullptr, ns, part,
                               prec == CONKER_MM_SPLIT_F16 ? (const unsigned *)maxabs : (const unsigned *)nullptr,
                               tab);
        };
        if (ns <= 16) {
            if (prec == CONKER_MM_SPLIT_F16) go(k_mm3s<CONKER_MM_SPLIT_F16>);
            else go(k_mm3s<CONKER_MM_SPLIT_BF16>);
        } else if (L.ntl == 1) {
            if (prec == CONKER_MM_SPLIT_F16) go(k_mm3<1, CONKER_MM_SPLIT_F16, true>);
            else go(k_mm3<1, CONKER_MM_SPLIT_BF16, true>);
        } else if (prec == CONKER_MM_SPLIT_BF16 && ns <= 48) {
            hipLaunchKernelGGL(k_mm3g<3>, grid, dim3(NT), 0, c->stream, (const float *)nullptr, (const float *)nullptr,
                               nc, (const int *)nullptr, (const int *)nullptr, ns, part, tab);
        } else {
            if (prec == CONKER_MM_SPLIT_F16) go(k_mm3<2, CONKER_MM_SPLIT_F16, false>);
            else go(k_mm3<2, CONKER_MM_SPLIT_BF16, false>);
        }
        CK_LAUNCH(c);
    }
    ProfScope ps(c, PK_CONTRACT_REDUCE);
    const int te = 1024;
    const int tiles = (int)nf * L.ntl;   // every field's tiles, one after the other
    const size_t tot = (size_t)tiles * te;
    double *slices = full + tot;
    hipLaunchKernelGGL(k_tile_reduce1, dim3((unsigned)((tot * RED_S + 255) / 256)), dim3(256), 0, c->stream, part,
                       tiles, L.G, te, slices);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_tile_reduce2, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, slices, tiles,
                       te, full);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_gather_jobs, dim3((unsigned)((pl.count + 255) / 256), nf), dim3(256), 0, c->stream,
                       (const double *)full, (size_t)L.ntl * te, (const int *)pl.where->p, pl.count, tab);
    CK_LAUNCH(c);
    return CONKER_OK;
}

}  // namespace conker
