// List of the 64-cell blocks where a field is non-zero.
//
// A cell where the field F is zero adds nothing to any sum of the summation
// stage, W = sum_x F(x) prod_i C_{a_i}(x) (Sec. 2.5, Eq. ksin_delta): outside
// a survey footprint most of the grid is such cells.  The summation kernels
// walk the list built here instead of every cell; it holds, in ascending
// order, each 64-cell block (cells 64 k .. 64 k + 63 of the flat grid) with at
// least one cell where F != 0 (either sign of zero counts as zero).  The order
// is fixed, so the split of the list over workgroups, and with it every
// floating-point sum, is the same from run to run.
//   k_blk_mark   one bit per block and the number of marked blocks per
//                workgroup (256 blocks each), from coalesced 16-byte loads;
//   k_blk_scan   exclusive prefix sum of the workgroup counts, and the total;
//   k_blk_place  one wave per 2048 blocks (64 words, eight mark workgroups)
//                writes the indices of its marked blocks from the offset of
//                its first mark workgroup.
// No memset: every word of the workspace read later is written first, so the
// three launches may be captured in a graph.
#include <cstdint>
#include <type_traits>

#include "common.h"

using namespace conker;

namespace {

constexpr int BK_T = 256;      // threads of the mark pass
constexpr int BK_PER = 256;    // blocks per mark workgroup: 8 words of 32 bits
constexpr int PL_WORDS = 64;   // words per place wave: 2048 blocks
constexpr int BK_S = 1024;     // threads of the scan

template <typename T>
__device__ __forceinline__ bool nonzero16(const T *p) {
    if constexpr (std::is_same<T, float>::value) {
        const uint4 u = *reinterpret_cast<const uint4 *>(p);
        return ((u.x << 1) | (u.y << 1) | (u.z << 1) | (u.w << 1)) != 0u;
    } else {
        const ulonglong2 u = *reinterpret_cast<const ulonglong2 *>(p);
        return ((u.x << 1) | (u.y << 1)) != 0ull;
    }
}

template <typename T>
__global__ __launch_bounds__(BK_T) void k_blk_mark(const T *__restrict__ F, size_t nc, unsigned *__restrict__ bits,
                                                   unsigned *__restrict__ wgcnt) {
    constexpr int CPL = 16 / (int)sizeof(T);   // cells per lane load
    constexpr int LPB = 64 / CPL;              // lanes per block: 16 (float), 32 (double)
    constexpr int BPS = 64 / LPB;              // blocks per wave load
    constexpr int WPB = BK_PER / (BK_T / 64);  // blocks per wave
    constexpr unsigned long long LMASK = LPB == 64 ? ~0ull : ((1ull << LPB) - 1ull);
    __shared__ unsigned wsum[BK_T / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const size_t b0 = (size_t)blockIdx.x * BK_PER + (size_t)wv * WPB;   // a multiple of 32
    unsigned word = 0u, cnt = 0u;
    for (int s = 0; s < WPB / BPS; ++s) {
        const size_t blk = b0 + (size_t)s * BPS + (size_t)(lane / LPB);
        const size_t x = blk * 64 + (size_t)(lane % LPB) * CPL;
        // nc is a multiple of 16: a lane's cells are all inside the grid or all past it
        const bool nz = x < nc && nonzero16<T>(F + x);
        const unsigned long long bal = __ballot(nz);
        unsigned nib = 0u;
#pragma unroll
        for (int j = 0; j < BPS; ++j) nib |= ((bal >> (j * LPB)) & LMASK) != 0ull ? (1u << j) : 0u;
        word |= nib << ((s * BPS) & 31);
        if ((((s + 1) * BPS) & 31) == 0) {   // word of blocks b0 + s BPS - (s BPS mod 32) .. + 31 done
            if (lane == 0) bits[(b0 + (size_t)s * BPS) / 32] = word;
            cnt += __popc(word);
            word = 0u;
        }
    }
    if (lane == 0) wsum[wv] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0u;
#pragma unroll
        for (int k = 0; k < BK_T / 64; ++k) t += wsum[k];
        wgcnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(BK_S) void k_blk_scan(const unsigned *__restrict__ wgcnt, int ng,
                                                   unsigned *__restrict__ wgoff, int *__restrict__ total) {
    __shared__ unsigned part[BK_S];
    const int t = threadIdx.x, per = (ng + BK_S - 1) / BK_S;
    const int g0 = t * per;
    unsigned s = 0u;
    for (int g = g0; g < g0 + per && g < ng; ++g) s += wgcnt[g];
    part[t] = s;
    __syncthreads();
    for (int h = 1; h < BK_S; h <<= 1) {   // inclusive scan of the thread sums
        const unsigned v = t >= h ? part[t - h] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    unsigned run = part[t] - s;
    for (int g = g0; g < g0 + per && g < ng; ++g) {
        wgoff[g] = run;
        run += wgcnt[g];
    }
    if (t == BK_S - 1) total[0] = (int)part[t];
}

__global__ __launch_bounds__(64) void k_blk_place(const unsigned *__restrict__ bits, size_t nwords,
                                                  const unsigned *__restrict__ wgoff, int *__restrict__ list) {
    static_assert(PL_WORDS * 32 % BK_PER == 0, "a place wave covers whole mark workgroups");
    const int lane = threadIdx.x;   // word `lane` of this range: blocks base .. base + 31
    const size_t wi = (size_t)blockIdx.x * PL_WORDS + lane;
    const unsigned word = wi < nwords ? bits[wi] : 0u;
    const int c = __popc(word);
    int incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o);
        if (lane >= o) incl += v;
    }
    int pos = (int)wgoff[(size_t)blockIdx.x * (PL_WORDS * 32 / BK_PER)] + incl - c;
    const int base = (int)(wi * 32);
    unsigned rest = word;
    while (rest) {
        const int j = __ffs(rest) - 1;
        rest &= rest - 1u;
        list[pos++] = base + j;
    }
}

}  // namespace

namespace conker {

int block_list(conker_ctx *c, const void *F, bool f64, size_t nc, const int **list, const int **count) {
    if (nc % 16) return fail(c, CONKER_EUNSUPPORTED, "cell count must be a multiple of 16");
    const size_t nblk = (nc + 63) / 64;
    const size_t ng = (nblk + BK_PER - 1) / BK_PER;
    // workspace: bits [ng * 8], wgcnt [ng], wgoff [ng], total [4], list [nblk]
    const size_t words = ng * (BK_PER / 32);
    const size_t bytes = (words + 2 * ng + 4) * sizeof(unsigned) + nblk * sizeof(int);
    CK_OK(ws_reserve(c, c->blocks, bytes));
    unsigned *bits = (unsigned *)c->blocks.p;
    unsigned *wgcnt = bits + words;
    unsigned *wgoff = wgcnt + ng;
    int *total = (int *)(wgoff + ng);
    int *lst = total + 4;
    ProfScope ps(c, PK_BLOCKS);
    if (f64)
        hipLaunchKernelGGL(k_blk_mark<double>, dim3((unsigned)ng), dim3(BK_T), 0, c->stream, (const double *)F, nc,
                           bits, wgcnt);
    else
        hipLaunchKernelGGL(k_blk_mark<float>, dim3((unsigned)ng), dim3(BK_T), 0, c->stream, (const float *)F, nc,
                           bits, wgcnt);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_blk_scan, dim3(1), dim3(BK_S), 0, c->stream, wgcnt, (int)ng, wgoff, total);
    CK_LAUNCH(c);
    const size_t np = (words + PL_WORDS - 1) / PL_WORDS;
    hipLaunchKernelGGL(k_blk_place, dim3((unsigned)np), dim3(64), 0, c->stream, (const unsigned *)bits, words, wgoff,
                       lst);
    CK_LAUNCH(c);
    *list = lst;
    *count = total;
    return CONKER_OK;
}

}  // namespace conker
