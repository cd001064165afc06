// Mapping stage (Sec. 2.2): nearest-grid-point histograms and N = D - alpha R.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "common.h"

namespace {

struct GridGeom {
    double ox, oy, oz, cell;
    int nx, ny, nz;
};

__device__ inline int cell_of(float x, double o, double cell, int n, bool &ok);

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

// ---------------------------------------------------------------------------
// Binned mapping for large catalogs.  Points arrive in no spatial order, so
// one float atomic per point at a random address of a grid far larger than
// the caches turns into a memory read-modify-write per point.  Instead the
// grid is cut into bricks of BX x BY x BZ cells and the points are counted,
// placed in brick order, and summed one brick at a time in LDS:
//   k_bin_count  per-workgroup brick histogram (LDS) of a contiguous chunk of
//                points, written out and added to the per-brick totals; the
//                weight sum and rejected count as in k_scatter;
//   k_bin_scan   exclusive prefix sum of the totals: brick starts, cursors;
//   k_bin_place  each workgroup reserves its share of every brick with one
//                atomic, then writes (cell in brick, weight) of its points at
//                their brick's slots (ranks from LDS atomics);
//   k_bin_accum  one workgroup per brick holding points: LDS tile sums, then
//                the tile is added to the grid (the grid is accumulated into).
//                The tile sums are 64-bit integers of w 2^E (LDS integer
//                adds run several times faster than float ones), E chosen
//                per brick from its point count times the largest |w| (from
//                the count pass) so that no sum can leave 62 bits; each w is
//                rounded to nearest (unbiased), the sums are independent of
//                the order and rounded once when added to the grid.  Bricks
//                whose bound is not finite add floats.
// The sums are the same as the direct kernel's, in another order (exact for
// unit weights, which give integer counts).
// ---------------------------------------------------------------------------
constexpr int BX = 16, BY = 16, BZ = 32, BCELLS = BX * BY * BZ;
constexpr int MAX_BRICKS = 16384;   // LDS histogram of one workgroup: 64 KB
constexpr int BG = 512;             // workgroups of the count / place passes
constexpr int BT = 1024;            // their threads
constexpr int64_t BIN_MIN_POINTS = (int64_t)1 << 22;

struct BrickGeom {
    int bnx, bny, bnz;   // bricks per axis
};

__device__ __forceinline__ bool locate(const float *pos, const float *w, int64_t p, const GridGeom &g,
                                       const BrickGeom &bg, int &brick, int &inner, float &wt) {
    const float x = pos[3 * p + 0], y = pos[3 * p + 1], z = pos[3 * p + 2];
    wt = w ? w[p] : 1.0f;
    bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(wt);
    const int cx = cell_of(x, g.ox, g.cell, g.nx, ok);
    const int cy = cell_of(y, g.oy, g.cell, g.ny, ok);
    const int cz = cell_of(z, g.oz, g.cell, g.nz, ok);
    brick = ((cx / BX) * bg.bny + cy / BY) * bg.bnz + cz / BZ;
    inner = ((cx % BX) * BY + cy % BY) * BZ + cz % BZ;
    return ok;
}

__device__ __forceinline__ void bin_count_body(const float *__restrict__ pos, const float *__restrict__ w,
                                               int64_t n, int64_t chunk, GridGeom g, BrickGeom bg, int nb,
                                               unsigned *__restrict__ hist_out, unsigned *__restrict__ totals,
                                               double *wsum, unsigned long long *n_out,
                                               unsigned *__restrict__ wmax_bits) {
    __shared__ unsigned hist[MAX_BRICKS];
    __shared__ double sw[BT / 64];
    __shared__ unsigned long long so[BT / 64];
    __shared__ float sm[BT / 64];
    float my_max = 0.f;
    for (int b = threadIdx.x; b < nb; b += BT) hist[b] = 0u;
    __syncthreads();
    double my_w = 0.0;
    unsigned long long my_out = 0;
    const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = p0 + chunk < n ? p0 + chunk : n;
    // four points per thread and step, all located before any LDS update
    for (int64_t q = p0 + threadIdx.x; q < p1; q += 4 * BT) {
        int brick[4], inner[4];
        float wt[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t p = q + (int64_t)k * BT;
            ok[k] = p < p1 && locate(pos, w, p, g, bg, brick[k], inner[k], wt[k]);
            if (p < p1 && !ok[k]) ++my_out;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (ok[k]) {
                atomicAdd(&hist[brick[k]], 1u);
                my_w += (double)wt[k];
                my_max = fmaxf(my_max, fabsf(wt[k]));
            }
    }
    __syncthreads();
    unsigned *mine = hist_out + (size_t)blockIdx.x * nb;
    for (int b = threadIdx.x; b < nb; b += BT) {
        const unsigned h = hist[b];
        mine[b] = h;
        if (h) atomicAdd(&totals[b], h);
    }
    // weight sum and rejected count of the workgroup
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        my_w += __shfl_xor(my_w, o);
        my_out += __shfl_xor(my_out, o);
        my_max = fmaxf(my_max, __shfl_xor(my_max, o));
    }
    if ((threadIdx.x & 63) == 0) {
        sw[threadIdx.x >> 6] = my_w;
        so[threadIdx.x >> 6] = my_out;
        sm[threadIdx.x >> 6] = my_max;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
        unsigned long long b = 0;
        float m = 0.f;
        for (int i = 0; i < BT / 64; ++i) {
            a += sw[i];
            b += so[i];
            m = fmaxf(m, sm[i]);
        }
        if (wsum) unsafeAtomicAdd(wsum, a);
        if (n_out && b) atomicAdd(n_out, b);
        atomicMax(wmax_bits, __float_as_uint(m));   // |w| >= 0: float order = bit order
    }
}

__global__ __launch_bounds__(BT) void k_bin_count(const float *__restrict__ pos, const float *__restrict__ w,
                                                  int64_t n, int64_t chunk, GridGeom g, BrickGeom bg, int nb,
                                                  unsigned *__restrict__ hist_out, unsigned *__restrict__ totals,
                                                  double *wsum, unsigned long long *n_out,
                                                  unsigned *__restrict__ wmax_bits) {
    bin_count_body(pos, w, n, chunk, g, bg, nb, hist_out, totals, wsum, n_out, wmax_bits);
}

// ---------------------------------------------------------------------------
// The binned mapping for every catalog of a size class at once: field
// z = blockIdx.y = 2 job + {0 data, 1 randoms} has its own counts, starts and
// cursors at meta + z 3 SB (totals, with the largest |w| after them; starts;
// cursors), its workgroup histograms at hist + z gridDim.x nb and its placed
// points at items + the field's item offset.
// ---------------------------------------------------------------------------
struct JobField {
    const float *pos, *w;
    int64_t n, ioff;
    float *grid;
    double *wsum;
    unsigned long long *n_out;
};

__device__ __forceinline__ JobField job_field(const conker::ClassJob *tab, int z) {
    const conker::ClassJob &j = tab[z >> 1];
    const bool r = z & 1;
    return JobField{r ? j.rpos : j.dpos, r ? j.rw : j.dw, r ? j.nr : j.nd, r ? j.ioff_r : j.ioff_d, r ? j.R : j.N,
                    j.wsum + (r ? 1 : 0), reinterpret_cast<unsigned long long *>(j.nout + (r ? 1 : 0))};
}

// wsum, rejected counts and the brick totals (with the largest |w|) of every field
__global__ void k_bin_zero_jobs(const conker::ClassJob *__restrict__ tab, int M, unsigned *__restrict__ meta,
                                int sb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * M) {
        const JobField f = job_field(tab, t);
        *f.wsum = 0.0;
        *f.n_out = 0ull;
    }
    for (int i = t; i < 2 * M * sb; i += gridDim.x * blockDim.x) {
        const int z = i / sb, k = i - z * sb;
        meta[(size_t)z * 3 * sb + k] = 0u;
    }
}

__global__ __launch_bounds__(BT) void k_bin_count_jobs(const conker::ClassJob *__restrict__ tab, GridGeom g,
                                                       BrickGeom bg, int nb, unsigned *__restrict__ hist,
                                                       unsigned *__restrict__ meta, int sb) {
    const JobField f = job_field(tab, blockIdx.y);
    const int64_t chunk = (f.n + gridDim.x - 1) / gridDim.x;
    unsigned *totals = meta + (size_t)blockIdx.y * 3 * sb;
    bin_count_body(f.pos, f.w, f.n, chunk, g, bg, nb, hist + (size_t)blockIdx.y * gridDim.x * nb, totals, f.wsum,
                   f.n_out, totals + nb);
}

// One workgroup: start[b] = sum of totals before b (start[nb] = all), cursor = start.
__device__ __forceinline__ void bin_scan_body(const unsigned *__restrict__ totals, int nb,
                                              unsigned *__restrict__ start, unsigned *__restrict__ cursor) {
    __shared__ unsigned part[BT];
    const int t = threadIdx.x, per = (nb + BT - 1) / BT;
    const int b0 = t * per;
    unsigned s = 0;
    for (int b = b0; b < b0 + per && b < nb; ++b) s += totals[b];
    part[t] = s;
    __syncthreads();
    for (int h = 1; h < BT; h <<= 1) {   // inclusive scan of the thread sums
        const unsigned v = t >= h ? part[t - h] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned run = part[t] - s;
    for (int b = b0; b < b0 + per && b < nb; ++b) {
        start[b] = run;
        cursor[b] = run;
        run += totals[b];
    }
    if (t == BT - 1) start[nb] = part[t];
}

__global__ __launch_bounds__(BT) void k_bin_scan(const unsigned *__restrict__ totals, int nb,
                                                 unsigned *__restrict__ start, unsigned *__restrict__ cursor) {
    bin_scan_body(totals, nb, start, cursor);
}

__global__ __launch_bounds__(BT) void k_bin_scan_jobs(int nb, unsigned *__restrict__ meta, int sb) {
    unsigned *m = meta + (size_t)blockIdx.x * 3 * sb;
    bin_scan_body(m, nb, m + sb, m + 2 * sb);
}

__device__ __forceinline__ void bin_place_body(const float *__restrict__ pos, const float *__restrict__ w,
                                               int64_t n, int64_t chunk, GridGeom g, BrickGeom bg, int nb,
                                               const unsigned *__restrict__ hist_in, unsigned *__restrict__ cursor,
                                               uint2 *__restrict__ items) {
    __shared__ unsigned base[MAX_BRICKS];
    __shared__ unsigned rank[MAX_BRICKS];
    const unsigned *mine = hist_in + (size_t)blockIdx.x * nb;
    for (int b = threadIdx.x; b < nb; b += BT) {
        const unsigned h = mine[b];
        base[b] = h ? atomicAdd(&cursor[b], h) : 0u;
        rank[b] = 0u;
    }
    __syncthreads();
    const int64_t p0 = (int64_t)blockIdx.x * chunk, p1 = p0 + chunk < n ? p0 + chunk : n;
    for (int64_t q = p0 + threadIdx.x; q < p1; q += 4 * BT) {
        int brick[4], inner[4];
        float wt[4];
        bool ok[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t p = q + (int64_t)k * BT;
            ok[k] = p < p1 && locate(pos, w, p, g, bg, brick[k], inner[k], wt[k]);
        }
        unsigned slot[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (ok[k]) slot[k] = base[brick[k]] + atomicAdd(&rank[brick[k]], 1u);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (ok[k]) items[slot[k]] = uint2{(unsigned)inner[k], __float_as_uint(wt[k])};
    }
}

__global__ __launch_bounds__(BT) void k_bin_place(const float *__restrict__ pos, const float *__restrict__ w,
                                                  int64_t n, int64_t chunk, GridGeom g, BrickGeom bg, int nb,
                                                  const unsigned *__restrict__ hist_in, unsigned *__restrict__ cursor,
                                                  uint2 *__restrict__ items) {
    bin_place_body(pos, w, n, chunk, g, bg, nb, hist_in, cursor, items);
}

__global__ __launch_bounds__(BT) void k_bin_place_jobs(const conker::ClassJob *__restrict__ tab, GridGeom g,
                                                       BrickGeom bg, int nb, const unsigned *__restrict__ hist,
                                                       unsigned *__restrict__ meta, int sb, uint2 *__restrict__ items) {
    const JobField f = job_field(tab, blockIdx.y);
    const int64_t chunk = (f.n + gridDim.x - 1) / gridDim.x;
    bin_place_body(f.pos, f.w, f.n, chunk, g, bg, nb, hist + (size_t)blockIdx.y * gridDim.x * nb,
                   meta + (size_t)blockIdx.y * 3 * sb + 2 * sb, items + f.ioff);
}

// OVER: the brick's cells are written with its sums (every brick, empty ones
// with zeros), else its sums are added to the grid (bricks with points only).
template <typename T, bool OVER>
__device__ __forceinline__ void bin_accum_body(const uint2 *__restrict__ items, const unsigned *__restrict__ start,
                                               GridGeom g, BrickGeom bg, T *__restrict__ grid,
                                               const unsigned *__restrict__ wmax_bits) {
    __shared__ unsigned long long acc[BCELLS];   // fixed-point sums, or the T sums in its first bytes
    T *const tile = reinterpret_cast<T *>(acc);
    const int b = blockIdx.x;
    const unsigned i0 = start[b], i1 = start[b + 1];
    if (!OVER && i0 == i1) return;   // uniform: no point in this brick
    // Fixed point w 2^E with 2^E chosen per brick so that every cell sum stays
    // within (i1 - i0) max|w| 2^E <= 2^62 (int64): each w is rounded to the
    // nearest multiple of 2^-E, exactly for |w| >= 2^(23 - E) (unit weights
    // always; in a brick of 2^13 points every |w| >= 2^-26 max|w|), so the
    // sums are unbiased and independent of the order.  Bricks whose bound is
    // not finite add floats.  Uniform over the workgroup.
    const float bound = (float)(i1 - i0) * __uint_as_float(*wmax_bits);
    int eb = 0;
    (void)frexpf(bound, &eb);                       // bound < 2^eb
    const int E = bound > 0.f ? min(62 - eb, 126) : 0;   // eb <= 128: E >= -66
    const bool fixed = isfinite(bound);
    const float to_fixed = ldexpf(1.0f, E);
    const double from_fixed = ldexp(1.0, -E);
    for (int e = threadIdx.x; e < BCELLS; e += 256) acc[e] = 0ull;   // zero bits: 0 in every view
    __syncthreads();
    for (unsigned i = i0 + threadIdx.x; i < i1; i += 4 * 256) {
        uint2 it[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) it[k] = i + k * 256 < i1 ? items[i + k * 256] : uint2{0u, 0u};
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i + k * 256 < i1) {
                const float wv = __uint_as_float(it[k].y);
                if (fixed) atomicAdd(&acc[it[k].x], (unsigned long long)__float2ll_rn(wv * to_fixed));
                else atomicAdd(&tile[it[k].x], (T)wv);
            }
    }
    __syncthreads();
    // the brick's rows of BZ cells, 4 values a thread-step; every value read before any is written
    const int bz = b % bg.bnz, by = (b / bg.bnz) % bg.bny, bx = b / (bg.bnz * bg.bny);
    constexpr int V = 4, PER = BCELLS / V / 256;
    T v[PER][V];
    size_t lin[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = (threadIdx.x + k * 256) * V;
        const int lz = e % BZ, ly = (e / BZ) % BY, lx = e / (BZ * BY);
        lin[k] = ((size_t)(bx * BX + lx) * g.ny + (by * BY + ly)) * g.nz + (bz * BZ + lz);
#pragma unroll
        for (int j = 0; j < V; ++j) v[k][j] = OVER ? (T)0 : grid[lin[k] + j];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int e = (threadIdx.x + k * 256) * V;
#pragma unroll
        for (int j = 0; j < V; ++j) {
            const T s = fixed ? (T)((double)(long long)acc[e + j] * from_fixed) : tile[e + j];
            grid[lin[k] + j] = OVER ? s : v[k][j] + s;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bin_accum(const uint2 *__restrict__ items, const unsigned *__restrict__ start,
                                                   GridGeom g, BrickGeom bg, T *__restrict__ grid,
                                                   const unsigned *__restrict__ wmax_bits) {
    bin_accum_body<T, false>(items, start, g, bg, grid, wmax_bits);
}

// every brick (blockIdx.x) of field blockIdx.y, written whole
__global__ __launch_bounds__(256) void k_bin_accum_jobs(const conker::ClassJob *__restrict__ tab, GridGeom g,
                                                        BrickGeom bg, int nb, const unsigned *__restrict__ meta,
                                                        int sb, const uint2 *__restrict__ items) {
    const JobField f = job_field(tab, blockIdx.y);
    const unsigned *m = meta + (size_t)blockIdx.y * 3 * sb;
    bin_accum_body<float, true>(items + f.ioff, m + sb, g, bg, f.grid, m + nb);
}

__global__ void k_zero_u32(unsigned *__restrict__ p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// VEC (both fields 16-byte aligned): 16-byte loads and stores for the bulk,
// the same per-element arithmetic.
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_form_delta(T *__restrict__ D, const T *__restrict__ R,
                                                    size_t n, const double *wd, const double *wr,
                                                    double *alpha_out) {
    const double alpha = *wd / *wr;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    if (t0 == 0 && alpha_out) *alpha_out = alpha;
    size_t done = 0;
    if constexpr (VEC) {
        constexpr int V = 16 / (int)sizeof(T);
        using VT = std::conditional_t<std::is_same<T, float>::value, float4, double2>;
        const size_t nv = n / V;
        for (size_t i = t0; i < nv; i += stride) {
            VT d = reinterpret_cast<const VT *>(D)[i];
            const VT r = reinterpret_cast<const VT *>(R)[i];
            T *dp = reinterpret_cast<T *>(&d);
            const T *rp = reinterpret_cast<const T *>(&r);
#pragma unroll
            for (int k = 0; k < V; ++k) dp[k] = (T)((double)dp[k] - alpha * (double)rp[k]);
            reinterpret_cast<VT *>(D)[i] = d;
        }
        done = nv * V;
    }
    for (size_t i = done + t0; i < n; i += stride) D[i] = (T)((double)D[i] - alpha * (double)R[i]);
}

// Size classes (job table, float32 grids): blockIdx.y = 2 job + {0 data, 1
// randoms}, each catalog into its own grid as k_scatter does.
__global__ __launch_bounds__(256) void k_scatter_jobs(const conker::ClassJob *__restrict__ tab, GridGeom g) {
    const conker::ClassJob &j = tab[blockIdx.y >> 1];
    const bool r = blockIdx.y & 1;
    const float *pos = r ? j.rpos : j.dpos;
    const float *w = r ? j.rw : j.dw;
    const int64_t n = r ? j.nr : j.nd;
    float *grid = r ? j.R : j.N;
    double *wsum = j.wsum + (r ? 1 : 0);
    auto *n_out = reinterpret_cast<unsigned long long *>(j.nout + (r ? 1 : 0));
    double my_w = 0.0;
    unsigned long long my_out = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const float x = pos[3 * p + 0], y = pos[3 * p + 1], z = pos[3 * p + 2];
        const float wt = w ? w[p] : 1.0f;
        bool ok = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(wt);
        const int cx = cell_of(x, g.ox, g.cell, g.nx, ok);
        const int cy = cell_of(y, g.oy, g.cell, g.ny, ok);
        const int cz = cell_of(z, g.oz, g.cell, g.nz, ok);
        if (ok) {
            atomic_add_grid<float>(grid + ((size_t)cx * g.ny + cy) * g.nz + cz, wt);
            my_w += (double)wt;
        } else {
            ++my_out;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        my_w += __shfl_xor(my_w, o);
        my_out += __shfl_xor(my_out, o);
    }
    __shared__ double sw[4];
    __shared__ unsigned long long so[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        sw[wv] = my_w;
        so[wv] = my_out;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tw = sw[0] + sw[1] + sw[2] + sw[3];
        const unsigned long long to = so[0] + so[1] + so[2] + so[3];
        if (tw != 0.0) unsafeAtomicAdd(wsum, tw);
        if (to) atomicAdd(n_out, to);
    }
}

// Size classes: zeroes both grids (16-byte stores), the weight sums and the
// rejected counts of job blockIdx.y.
__global__ __launch_bounds__(256) void k_zero_jobs(const conker::ClassJob *__restrict__ tab, size_t nc) {
    const conker::ClassJob &j = tab[blockIdx.y];
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    float4 *a = reinterpret_cast<float4 *>(j.N), *b = reinterpret_cast<float4 *>(j.R);
    const float4 z{0.f, 0.f, 0.f, 0.f};
    for (size_t i = t0; i < nc / 4; i += stride) {
        a[i] = z;
        b[i] = z;
    }
    if (t0 < 2) {
        j.wsum[t0] = 0.0;
        j.nout[t0] = 0;
    }
}

// Size classes: N = D - alpha R of job blockIdx.y in place (as k_form_delta),
// and the sums of squares of N and R that the packed transform's scale is
// chosen from (the pair of workgroup x of job y at part + 2 (y gridDim.x + x)).
__global__ __launch_bounds__(256) void k_form_delta_jobs(const conker::ClassJob *__restrict__ tab, size_t nc,
                                                         double *__restrict__ part) {
    const conker::ClassJob &j = tab[blockIdx.y];
    const double alpha = j.wsum[0] / j.wsum[1];
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    if (t0 == 0) *j.alpha = alpha;
    float4 *D = reinterpret_cast<float4 *>(j.N);
    const float4 *R = reinterpret_cast<const float4 *>(j.R);
    double sa = 0.0, sb = 0.0;
    for (size_t i = t0; i < nc / 4; i += stride) {
        float4 d = D[i];
        const float4 r = R[i];
        d.x = (float)((double)d.x - alpha * (double)r.x);
        d.y = (float)((double)d.y - alpha * (double)r.y);
        d.z = (float)((double)d.z - alpha * (double)r.z);
        d.w = (float)((double)d.w - alpha * (double)r.w);
        D[i] = d;
        sa += (double)d.x * d.x + (double)d.y * d.y + (double)d.z * d.z + (double)d.w * d.w;
        sb += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
    }
    for (int o = 32; o >= 1; o >>= 1) {
        sa += __shfl_xor(sa, o);
        sb += __shfl_xor(sb, o);
    }
    __shared__ double red[4][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[wv][0] = sa;
        red[wv][1] = sb;
    }
    __syncthreads();
    if (threadIdx.x < 2)
        part[2 * ((size_t)blockIdx.y * gridDim.x + blockIdx.x) + threadIdx.x] =
            red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

}  // namespace

using namespace conker;

namespace conker {

namespace {
struct BinLayout {
    int nb, sb, bg;
    size_t meta, hist, items, bytes;
};
bool bin_layout(const conker_grid *g, int M, int64_t n_total, BinLayout *L) {
    if (g->dims[0] % BX || g->dims[1] % BY || g->dims[2] % BZ) return false;
    const int64_t nb = (int64_t)(g->dims[0] / BX) * (g->dims[1] / BY) * (g->dims[2] / BZ);
    if (nb > MAX_BRICKS || n_total > ((int64_t)1 << 32)) return false;
    const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    L->nb = (int)nb;
    L->sb = (int)((nb + 1 + 3) / 4 * 4);
    L->bg = std::max(8, 512 / (2 * M));   // workgroups per catalog in the count and place passes
    L->meta = 0;
    L->hist = up((size_t)2 * M * 3 * L->sb * sizeof(unsigned));
    L->items = L->hist + up((size_t)2 * M * L->bg * nb * sizeof(unsigned));
    L->bytes = L->items + up((size_t)n_total * sizeof(uint2));
    return true;
}
}  // namespace

size_t map_jobs_bytes(const conker_grid *g, int M, int64_t n_total) {
    BinLayout L;
    return bin_layout(g, M, n_total, &L) ? L.bytes : 0;
}

int map_jobs(conker_ctx *c, const conker_grid *g, int M, const ClassJob *tab, int64_t n_max, int64_t n_total,
             void *ws, double *part, int *sums_G) {
    const size_t nc = ncells(g);
    if (nc % 4) return fail(c, CONKER_EINVAL, "size class: cell count must be a multiple of 4");
    const GridGeom gg{g->origin[0], g->origin[1], g->origin[2], g->cell, g->dims[0], g->dims[1], g->dims[2]};
    const size_t cap = (size_t)4 * cu_count(c);
    const unsigned zb = (unsigned)std::max<size_t>(1, std::min<size_t>(cap / M + 1, (nc / 4 + 255) / 256));
    BinLayout L;
    if (ws && bin_layout(g, M, n_total, &L)) {   // binned: every grid written whole by its bricks
        ProfScope ps(c, PK_SCATTER);
        const BrickGeom bg{g->dims[0] / BX, g->dims[1] / BY, g->dims[2] / BZ};
        char *base = (char *)ws;
        unsigned *meta = (unsigned *)(base + L.meta), *hist = (unsigned *)(base + L.hist);
        uint2 *items = (uint2 *)(base + L.items);
        const unsigned nf = 2u * (unsigned)M;
        hipLaunchKernelGGL(k_bin_zero_jobs, dim3((unsigned)((nf * L.sb + 255) / 256)), dim3(256), 0, c->stream, tab, M,
                           meta, L.sb);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_count_jobs, dim3((unsigned)L.bg, nf), dim3(BT), 0, c->stream, tab, gg, bg, L.nb, hist,
                           meta, L.sb);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_scan_jobs, dim3(nf), dim3(BT), 0, c->stream, L.nb, meta, L.sb);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_place_jobs, dim3((unsigned)L.bg, nf), dim3(BT), 0, c->stream, tab, gg, bg, L.nb,
                           (const unsigned *)hist, meta, L.sb, items);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_accum_jobs, dim3((unsigned)L.nb, nf), dim3(256), 0, c->stream, tab, gg, bg, L.nb,
                           (const unsigned *)meta, L.sb, (const uint2 *)items);
        CK_LAUNCH(c);
    } else {
        ProfScope ps(c, PK_SCATTER);
        hipLaunchKernelGGL(k_zero_jobs, dim3(zb, (unsigned)M), dim3(256), 0, c->stream, tab, nc);
        CK_LAUNCH(c);
        if (n_max > 0) {
            const int64_t want = (n_max + 255) / 256;
            const unsigned sb = (unsigned)std::min<int64_t>(want, std::max<int64_t>(64, 16384 / M));
            hipLaunchKernelGGL(k_scatter_jobs, dim3(sb, 2u * (unsigned)M), dim3(256), 0, c->stream, tab, gg);
            CK_LAUNCH(c);
        }
    }
    ProfScope ps(c, PK_FORM_DELTA);
    hipLaunchKernelGGL(k_form_delta_jobs, dim3(zb, (unsigned)M), dim3(256), 0, c->stream, tab, nc, part);
    CK_LAUNCH(c);
    *sums_G = (int)zb;
    return CONKER_OK;
}

}  // namespace conker

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
    auto *no = reinterpret_cast<unsigned long long *>(n_out);
    ProfScope ps(c, PK_SCATTER);
    const BrickGeom bg{g->dims[0] / BX, g->dims[1] / BY, g->dims[2] / BZ};
    const int64_t nb64 = (int64_t)bg.bnx * bg.bny * bg.bnz;
    if (n >= BIN_MIN_POINTS && n <= (int64_t)0xffffffffu && g->dims[0] % BX == 0 && g->dims[1] % BY == 0 &&
        g->dims[2] % BZ == 0 && nb64 <= MAX_BRICKS) {
        const int nb = (int)nb64;
        const auto up = [](size_t b) { return (b + 255) / 256 * 256; };
        // totals[nb] (zeroed with the totals) holds the largest |w| as float bits
        const size_t tot_b = up((nb + 1) * sizeof(unsigned)), start_b = up((nb + 1) * sizeof(unsigned));
        const size_t hist_b = up((size_t)BG * nb * sizeof(unsigned)), items_b = up((size_t)n * sizeof(uint2));
        CK_OK(ws_reserve(c, c->bins, 3 * tot_b + start_b + hist_b + items_b));
        char *base = (char *)c->bins.p;
        unsigned *totals = (unsigned *)base;
        unsigned *cursor = (unsigned *)(base + tot_b);
        unsigned *start = (unsigned *)(base + 3 * tot_b);
        unsigned *hist = (unsigned *)(base + 3 * tot_b + start_b);
        uint2 *items = (uint2 *)(base + 3 * tot_b + start_b + hist_b);
        const int64_t chunk = (n + BG - 1) / BG;
        unsigned *wmax_bits = totals + nb;
        hipLaunchKernelGGL(k_zero_u32, dim3(64), dim3(256), 0, c->stream, totals, nb + 1);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_count, dim3(BG), dim3(BT), 0, c->stream, pos, w, n, chunk, gg, bg, nb, hist, totals,
                           wsum, no, wmax_bits);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(BT), 0, c->stream, totals, nb, start, cursor);
        CK_LAUNCH(c);
        hipLaunchKernelGGL(k_bin_place, dim3(BG), dim3(BT), 0, c->stream, pos, w, n, chunk, gg, bg, nb, hist, cursor,
                           items);
        CK_LAUNCH(c);
        if (dt == CONKER_F32)
            hipLaunchKernelGGL(k_bin_accum<float>, dim3(nb), dim3(256), 0, c->stream, items, start, gg, bg,
                               (float *)grid, (const unsigned *)wmax_bits);
        else
            hipLaunchKernelGGL(k_bin_accum<double>, dim3(nb), dim3(256), 0, c->stream, items, start, gg, bg,
                               (double *)grid, (const unsigned *)wmax_bits);
        CK_LAUNCH(c);
        return CONKER_OK;
    }
    int threads = 256;
    int64_t want = (n + threads - 1) / threads;
    int blocks = (int)(want < 8192 ? want : 8192);
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
    // a streaming pass: about four workgroups per CU looping over the cells
    int threads = 256;
    size_t want = (n + threads - 1) / threads;
    const size_t cap = (size_t)4 * cu_count(c);
    int blocks = (int)(want < cap ? want : cap);
    const bool vec = (((uintptr_t)D | (uintptr_t)R) & 15) == 0;
    ProfScope ps(c, PK_FORM_DELTA);
    if (dt == CONKER_F32) {
        if (vec)
            hipLaunchKernelGGL((k_form_delta<float, true>), dim3(blocks), dim3(threads), 0, c->stream, (float *)D,
                               (const float *)R, n, wd, wr, alpha);
        else
            hipLaunchKernelGGL((k_form_delta<float, false>), dim3(blocks), dim3(threads), 0, c->stream, (float *)D,
                               (const float *)R, n, wd, wr, alpha);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_form_delta<double, true>), dim3(blocks), dim3(threads), 0, c->stream, (double *)D,
                               (const double *)R, n, wd, wr, alpha);
        else
            hipLaunchKernelGGL((k_form_delta<double, false>), dim3(blocks), dim3(threads), 0, c->stream,
                               (double *)D, (const double *)R, n, wd, wr, alpha);
    }
    CK_LAUNCH(c);
    return CONKER_OK;
}
