// 3D FFT passes for the convolution stage (Sec. 2.4: the shell convolutions
// are realised with FFTs) and for the shell-kernel spectra (Sec. 2.3).
//
// Layout: complex grids [nx][ny][nz], z fastest.  A 3D transform is three
// passes of 1D line transforms, one per axis.  Each workgroup owns a tile of
// TC lines: for the z axis TC whole contiguous lines, for the y and x axes TC
// adjacent z-columns (so that every global access is a run of TC consecutive
// complex values).  A line transform is a Stockham autosort FFT with radix-8/4
// stages: the first stage reads global memory straight into registers, the
// last writes global memory straight from registers, and the stages in
// between exchange through LDS.  Twiddles come from a host-built float64 table
// exp(-2 pi i t / L) copied into LDS.
//
// Loads and stores go through small operator structs so that the same line
// engine packs two real fields into one complex field, multiplies by a kernel
// spectrum, unpacks real maps, generates shell indicators on the fly, or
// extracts the stored octant of a kernel spectrum.
#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <utility>

#include "common.h"
#include "fft_math.h"
#include "split3.h"

using namespace conker;

namespace {

using namespace conker::fftm;

// Radix schedule per line length (product of the stage radices).
template <int L>
struct Plan;
template <> struct Plan<32>   { static constexpr int n = 2; static constexpr int r[4] = {8, 4, 1, 1}; };
template <> struct Plan<64>   { static constexpr int n = 2; static constexpr int r[4] = {8, 8, 1, 1}; };
template <> struct Plan<128>  { static constexpr int n = 3; static constexpr int r[4] = {8, 4, 4, 1}; };
template <> struct Plan<256>  { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 4, 1}; };
template <> struct Plan<512>  { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 8, 1}; };
template <> struct Plan<1024> { static constexpr int n = 4; static constexpr int r[4] = {8, 8, 4, 4}; };
// lengths with a factor 3: the radix-3 stage comes last, so that every earlier
// stage has a power-of-two span
template <> struct Plan<96>   { static constexpr int n = 3; static constexpr int r[4] = {8, 4, 3, 1}; };
template <> struct Plan<192>  { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 3, 1}; };
template <> struct Plan<384>  { static constexpr int n = 4; static constexpr int r[4] = {8, 8, 2, 3}; };

// The other schedule of a length (a launch setting, chosen per grid shape by
// the autotuner): radix 16 first, one stage fewer (64 = 16 4, 128 = 16 8,
// 256 = 16 16, 1024 = 16 16 4).  Carried in a pass's tile-mode parameter as
// MODE + 8 (TM_BASE strips it); lengths without one keep their schedule.
template <int L>
struct PlanAlt {
    static constexpr bool has = false;
};
template <> struct PlanAlt<64>   { static constexpr bool has = true; static constexpr int n = 2; static constexpr int r[4] = {16, 4, 1, 1}; };
template <> struct PlanAlt<128>  { static constexpr bool has = true; static constexpr int n = 2; static constexpr int r[4] = {16, 8, 1, 1}; };
template <> struct PlanAlt<256>  { static constexpr bool has = true; static constexpr int n = 2; static constexpr int r[4] = {16, 16, 1, 1}; };
template <> struct PlanAlt<1024> { static constexpr bool has = true; static constexpr int n = 3; static constexpr int r[4] = {16, 16, 4, 1}; };

constexpr int TM_BASE = 7, TM_ALT = 8;
template <int L, int MODE>
using PlanM = std::conditional_t<(MODE & TM_ALT) != 0 && PlanAlt<L>::has, PlanAlt<L>, Plan<L>>;

template <int L, int MODE, int S>
constexpr int stage_ns() {   // product of radices before stage S
    int p = 1;
    for (int s = 0; s < S; ++s) p *= PlanM<L, MODE>::r[s];
    return p;
}

// Tile modes.
//   TM_J: lanes run along a line; a tile is TC whole contiguous lines (z axis).
//   TM_C: lanes run across the TC columns of a tile of strided lines (y, x axes);
//         runs of TC consecutive complex values (128 bytes).
//   TM_W: as TM_C with twice the columns (256-byte runs); the default for the
//         x and y axes (a launch setting selects TM_C instead).
//   TM_R: as TM_C with up to 1024 threads; used by the x pass that keeps its
//         spectrum tile resident (in registers) across a batch of radii.
enum TileMode { TM_J = 0, TM_C = 1, TM_W = 2, TM_R = 3 };

template <typename T, int L, int MODE>
struct Shape {
    static constexpr int BM = MODE & TM_BASE;
    static constexpr bool f64 = std::is_same<T, double>::value;
    static constexpr int TC_C = f64 ? (L >= 1024 ? 4 : 8) : (L >= 1024 ? 8 : 16);
    static constexpr int TCJ0 = (f64 ? 2048 : 4096) / L;   // lines per z tile: a power of two
    static constexpr int TCJ = TCJ0 >= 256 ? 256 : TCJ0 >= 128 ? 128 : TCJ0 >= 64 ? 64 : TCJ0 >= 32 ? 32
                             : TCJ0 >= 16 ? 16 : TCJ0 >= 8 ? 8 : TCJ0 >= 4 ? 4 : TCJ0 >= 2 ? 2 : 1;
    static constexpr int TC = BM == TM_J ? TCJ : (BM == TM_W ? 2 * TC_C : TC_C);
    static constexpr int PAD = BM == TM_J ? 0 : (f64 ? 0 : 2);
    static constexpr int NB0 = (L / PlanM<L, MODE>::r[0]) * TC;   // first-stage butterflies per tile
    static constexpr int NT =
        BM == TM_J ? 256
                   : (((BM == TM_W || BM == TM_R) && NB0 >= 1024) ? 1024 : (NB0 >= 512 ? 512 : 256));
    static constexpr int LDS = BM == TM_J ? TC * (L + (L >> 3)) : L * (TC + PAD);
    // registers per thread must stay near 128 for four waves per SIMD
    static constexpr int MINW = NT >= 512 ? 4 : 2;
};

template <int MODE, int L, int TC, int PAD>
__device__ __forceinline__ int lds_addr(int i, int c) {
    if constexpr ((MODE & TM_BASE) == TM_J) return c * (L + (L >> 3)) + i + (i >> 3);
    else return i * (TC + PAD) + c;
}

// Butterfly q of this thread -> (j = butterfly index within a line, c = column).
// TM_C / TM_W: the column is fixed per thread (NT is a multiple of TC), j steps by NT/TC.
// TM_J: lanes run along j; the line index steps by NT/LR (or j by NT when LR > NT).
template <int NT, int MODE, int LR, int TC>
__device__ __forceinline__ void split_q(int q, int &j, int &c) {
    const int t = threadIdx.x;
    if constexpr ((MODE & TM_BASE) == TM_J) {
        if constexpr (NT % LR == 0) { j = t % LR; c = t / LR + q * (NT / LR); }
        else { const int b = t + q * NT; j = b % LR; c = b / LR; }
    } else {
        static_assert(NT % TC == 0, "tile columns must divide the workgroup");
        c = t % TC;
        j = t / TC + q * (NT / TC);
    }
}

// Ops whose stores are conditional expose keeps() (uniform: whether any row is
// skipped) and flag(i) (row i of the tile is written iff flag(i) != 0).  The
// last stage issues every flag load it needs together, before its
// butterflies, so that no store waits behind a flag load (a wait for
// outstanding vector memory operations would also wait for the stores already
// issued) and the loads overlap each other.
template <class Op, class = void>
struct has_keep : std::false_type {};
template <class Op>
struct has_keep<Op, std::void_t<decltype(std::declval<const Op &>().flag(0))>> : std::true_type {};

// Ops with load_r(q, r, i, c) supply the first stage's inputs from registers
// indexed by the thread's butterfly q and point r (constants once unrolled).
template <class Op, class = void>
struct has_load_r : std::false_type {};
template <class Op>
struct has_load_r<Op, std::void_t<decltype(std::declval<const Op &>().load_r(0, 0, 0, 0))>> : std::true_type {};

// Ops with SYNC_LAST = true store the last stage's outputs into the tile's own
// LDS: the stage then waits for every thread's reads before its stores.
template <class Op, class = void>
struct has_sync_last : std::false_type {};
template <class Op>
struct has_sync_last<Op, std::enable_if_t<Op::SYNC_LAST>> : std::true_type {};

// TM_J tiles whose stages all give a line the same number of butterflies, a
// divisor of 64 (512 = 8 8 8, 64 = 8 8): the threads of a line then lie in one
// wave in every stage, each line owns its LDS rows, and an ordering within the
// wave replaces the workgroup barrier between stages.
template <int L, int MODE>
constexpr bool lines_in_wave() {
    using PL = PlanM<L, MODE>;
    const int lr = L / PL::r[0];
    if (64 % lr != 0) return false;
    for (int s = 1; s < PL::n; ++s)
        if (L / PL::r[s] != lr) return false;
    return true;
}

__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int L, int MODE>
__device__ __forceinline__ void stage_sync() {
    if constexpr ((MODE & TM_BASE) == TM_J && lines_in_wave<L, MODE>()) wave_order();
    else __syncthreads();
}

// Ops that know their keep bits in advance (the same rows for every call on a
// tile) expose KBITS and kb: the bits of the last stage, one word per
// butterfly of this thread, as last_keep_bits computes them.
template <class Op, class = void>
struct has_kbits : std::false_type {};
template <class Op>
struct has_kbits<Op, std::enable_if_t<Op::KBITS>> : std::true_type {};

// Ops that take the last stage's outputs with the butterfly and row indices
// (q, r) of this thread, for values they fetched in advance, expose STORE_QR
// and store_qr(q, r, i, c, v).
template <class Op, class = void>
struct has_store_qr : std::false_type {};
template <class Op>
struct has_store_qr<Op, std::enable_if_t<Op::STORE_QR>> : std::true_type {};

// Shape of the last stage of a line transform.
template <typename T, int L, int MODE>
struct LastStage {
    using SH = Shape<T, L, MODE>;
    static constexpr int S = PlanM<L, MODE>::n - 1;
    static constexpr int R = PlanM<L, MODE>::r[S];
    static constexpr int NSV = stage_ns<L, MODE, S>();
    static constexpr int LR = L / R;
    static constexpr int NB = LR * SH::TC;
    static constexpr int PER = (NB + SH::NT - 1) / SH::NT;
};

// Keep bits of the last stage: bit r of word q is set iff row base + r NSV of
// butterfly q of this thread is written (op.flag of that row is nonzero).
template <typename T, int L, int MODE, class Op>
__device__ __forceinline__ void last_keep_bits(const Op &op, unsigned (&kbits)[LastStage<T, L, MODE>::PER]) {
    using LS = LastStage<T, L, MODE>;
    constexpr int R = LS::R, NSV = LS::NSV, LR = LS::LR, NB = LS::NB, PER = LS::PER;
    constexpr int NT = Shape<T, L, MODE>::NT, TC = Shape<T, L, MODE>::TC;
    static_assert(R <= 16, "keep flags are packed 16 per butterfly");
    if (op.keeps()) {
        int fl[PER][R];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = threadIdx.x + q * NT;
            int j, c;
            split_q<NT, MODE, LR, TC>(q, j, c);
            const int k = j & (NSV - 1);
            const int base = (NB % NT == 0 || b < NB) ? (j - k) * R + k : 0;
#pragma unroll
            for (int r = 0; r < R; ++r) fl[q][r] = op.flag(base + r * NSV);   // base + r NSV < L
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            kbits[q] = 0;
#pragma unroll
            for (int r = 0; r < R; ++r) kbits[q] |= fl[q][r] != 0 ? (1u << r) : 0u;
        }
    } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) kbits[q] = 0xffffu;
    }
}

// The cells this thread's last stage writes: fn(q, r, i, c) for butterfly q
// and output r (row i of column or line c), for the butterflies it owns.
template <typename T, int L, int MODE, class Fn>
__device__ __forceinline__ void last_stage_cells(Fn &&fn) {
    using LS = LastStage<T, L, MODE>;
    constexpr int R = LS::R, NSV = LS::NSV, LR = LS::LR, NB = LS::NB, PER = LS::PER;
    constexpr int NT = Shape<T, L, MODE>::NT, TC = Shape<T, L, MODE>::TC;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = threadIdx.x + q * NT;
        if (NB % NT == 0 || b < NB) {
            int j, c;
            split_q<NT, MODE, LR, TC>(q, j, c);
            const int k = j & (NSV - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) fn(q, r, base + r * NSV, c);
        }
    }
}

// Stage S reads src (LDS; global memory or registers for the first stage) and
// writes dst (LDS; global memory for the last stage).  SYNC: the stage places
// its own barriers (src == dst, in place); otherwise the caller orders the
// buffers.  PADX >= 0 overrides the tile's row padding.
template <typename T, int L, int MODE, int DIR, int S, bool STAGED, bool SYNC = true, int PADX = -1, class Op>
__device__ __forceinline__ void fft_stage(const cplx<T> *src, cplx<T> *dst, const cplx<T> *tw, Op &op) {
    using C = cplx<T>;
    using SH = Shape<T, L, MODE>;
    constexpr int NT = SH::NT, TC = SH::TC, PAD = PADX >= 0 ? PADX : SH::PAD;
    constexpr int R = PlanM<L, MODE>::r[S];
    constexpr int NSV = stage_ns<L, MODE, S>();
    constexpr bool FIRST = (S == 0) && !STAGED;   // first stage reads global memory
    constexpr bool LAST = (S == PlanM<L, MODE>::n - 1);
    constexpr int LR = L / R;
    constexpr int NB = LR * TC;
    constexpr int PER = (NB + NT - 1) / NT;
    constexpr int TWS = L / (NSV * R);
    static_assert((NSV & (NSV - 1)) == 0, "stages before the last have power-of-two spans");
    constexpr bool KEEP = LAST && has_keep<Op>::value;
    static_assert(!KEEP || R <= 16, "keep flags are packed 16 per butterfly");
    unsigned kbits[PER];
    if constexpr (KEEP) {
        static_assert(!KEEP || PER == LastStage<T, L, MODE>::PER, "last stage shape");
        if constexpr (has_kbits<Op>::value) {
#pragma unroll
            for (int q = 0; q < PER; ++q) kbits[q] = op.kb[q];
        } else {
            last_keep_bits<T, L, MODE>(op, kbits);
        }
    }
    C v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = threadIdx.x + q * NT;
        if (NB % NT == 0 || b < NB) {
            int j, c;
            split_q<NT, MODE, LR, TC>(q, j, c);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = j + r * LR;
                if constexpr (FIRST && has_load_r<Op>::value) v[q][r] = op.load_r(q, r, i, c);
                else if constexpr (FIRST) v[q][r] = op.load(i, c);
                else v[q][r] = src[lds_addr<MODE, L, TC, PAD>(i, c)];
            }
            if constexpr (NSV > 1) {
                const int k = j & (NSV - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[r * k * TWS];
                    if constexpr (DIR > 0) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dft<R, DIR>(v[q]);
        }
    }
    // in-place LDS stages wait for every read before any write; the last stage
    // writes global memory from registers, and every caller puts a barrier
    // between a tile's last stage and the next writes to the LDS tile (ops
    // that store into that tile wait here)
    if constexpr (SYNC && !FIRST && !LAST) stage_sync<L, MODE>();
    if constexpr (LAST && has_sync_last<Op>::value) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = threadIdx.x + q * NT;
        if (NB % NT == 0 || b < NB) {
            int j, c;
            split_q<NT, MODE, LR, TC>(q, j, c);
            const int k = j & (NSV - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int o = base + r * NSV;
                if constexpr (KEEP) {
                    if (kbits[q] & (1u << r)) op.store(o, c, v[q][r]);
                } else if constexpr (LAST && has_store_qr<Op>::value) {
                    op.store_qr(q, r, o, c, v[q][r]);
                } else if constexpr (LAST) {
                    op.store(o, c, v[q][r]);
                } else {
                    dst[lds_addr<MODE, L, TC, PAD>(o, c)] = v[q][r];
                }
            }
        }
    }
    if constexpr (SYNC && !LAST) stage_sync<L, MODE>();
}

// STAGED: the tile is first copied into LDS with a plain row loop (one load in
// flight per row instead of a whole radix-8 butterfly's worth of addresses),
// and the first stage reads LDS.  Used where the load does extra work.
template <typename T, int L, int MODE, int DIR, bool STAGED, class Op>
__device__ __forceinline__ void fft_line_tile(cplx<T> *lds, const cplx<T> *tw, Op &op) {
    constexpr bool ST = STAGED && (MODE & TM_BASE) != TM_J;   // staged loads are for column tiles
    if constexpr (ST) {
        using SH = Shape<T, L, MODE>;
        constexpr int NT = SH::NT, TC = SH::TC, PAD = SH::PAD;
        const int c = threadIdx.x % TC;
#pragma unroll 8
        for (int i = threadIdx.x / TC; i < L; i += NT / TC) lds[lds_addr<MODE, L, TC, PAD>(i, c)] = op.load(i, c);
        __syncthreads();
    }
    using PL = PlanM<L, MODE>;
    fft_stage<T, L, MODE, DIR, 0, ST>(lds, lds, tw, op);
    if constexpr (PL::n > 1) fft_stage<T, L, MODE, DIR, 1, ST>(lds, lds, tw, op);
    if constexpr (PL::n > 2) fft_stage<T, L, MODE, DIR, 2, ST>(lds, lds, tw, op);
    if constexpr (PL::n > 3) fft_stage<T, L, MODE, DIR, 3, ST>(lds, lds, tw, op);
}

// Ops with an active() member may skip a whole tile (same answer for every
// thread of the workgroup).
template <class Op, class = void>
struct has_active : std::false_type {};
template <class Op>
struct has_active<Op, std::void_t<decltype(std::declval<const Op &>().active())>> : std::true_type {};

// Ops with ROWF = true (and rowflag(i), wants_rowf()) read only the rows of a
// tile whose flag is set (the others are zero); the flags of the tile are
// staged in LDS once.
template <class Op, class = void>
struct has_rowf : std::false_type {};
template <class Op>
struct has_rowf<Op, std::enable_if_t<Op::ROWF>> : std::true_type {};

// One launch = one pass over one axis.  Op::iters() line transforms are run
// per tile (more than one when a tile is reused across several radii).
// Ops with PERSIST = true (and begin_at(tile, batch), a set-up that can be
// repeated) may run persistent: with items > 0 each workgroup takes the work
// items blockIdx.x, + gridDim.x, ... of items = tiles x batches, loading the
// twiddles once.
template <class Op, class = void>
struct has_persist : std::false_type {};
template <class Op>
struct has_persist<Op, std::enable_if_t<Op::PERSIST>> : std::true_type {};

template <typename T, int L, int MODE, int DIR, class Op>
__global__ __launch_bounds__((Shape<T, L, MODE>::NT), (Shape<T, L, MODE>::MINW)) void k_fft(Op op, int items,
                                                                                         int tiles) {
    using C = cplx<T>;
    using SH = Shape<T, L, MODE>;
    __shared__ C lds[SH::LDS];
    __shared__ C tw[L];
    __shared__ unsigned char rowf[has_rowf<Op>::value ? L : 1];
    const C *twg = reinterpret_cast<const C *>(op.tw);
    if constexpr (has_persist<Op>::value) {
        if (items > 0) {   // the same for every thread
            for (int t = threadIdx.x; t < L; t += SH::NT) tw[t] = twg[t];
            for (int item = blockIdx.x; item < items; item += gridDim.x) {
                op.template begin_at<SH::TC>(item % tiles, item / tiles);
                if constexpr (has_active<Op>::value) {
                    if (!op.active()) continue;   // the same for every thread
                }
                __syncthreads();   // twiddles in; the previous item is done with the LDS tile
                const int it_n = op.iters();
                for (int it = 0; it < it_n; ++it) {
                    op.set_iter(it);
                    fft_line_tile<T, L, MODE, DIR, Op::STAGED>(lds, tw, op);
                    if (it + 1 < it_n) __syncthreads();
                }
            }
            return;
        }
    }
    op.template begin<SH::TC>();
    if constexpr (has_active<Op>::value) {
        if (!op.active()) return;   // the same for every thread of the workgroup
    }
    for (int t = threadIdx.x; t < L; t += SH::NT) tw[t] = twg[t];
    if constexpr (has_rowf<Op>::value) {
        if (op.wants_rowf()) {   // the same for every thread
            for (int t = threadIdx.x; t < L; t += SH::NT) rowf[t] = op.rowflag(t);
            op.rowf = rowf;
        }
    }
    __syncthreads();
    const int it_n = op.iters();
    for (int it = 0; it < it_n; ++it) {
        op.set_iter(it);
        fft_line_tile<T, L, MODE, DIR, Op::STAGED>(lds, tw, op);
        if (it + 1 < it_n) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// tile geometry: element (i, c) of a tile lives at base + i * si + c * sc
// ---------------------------------------------------------------------------
struct Dims {
    int nx, ny, nz;
};

enum Axis { AX_Z = 0, AX_Y = 1, AX_X = 2 };

struct Tile {
    size_t base;
    int si, sc;
    int p0, p1;   // tile coordinates: Z: first row (x*ny + y); Y: (x, z0); X: (y, z0)
};

__device__ __forceinline__ Tile make_tile(int axis, const Dims &d, int t, int TC) {
    Tile g;
    if (axis == AX_Z) {
        g.p0 = t * TC;
        g.p1 = 0;
        g.base = (size_t)g.p0 * d.nz;
        g.si = 1;
        g.sc = d.nz;
    } else {
        const int per = d.nz / TC;
        const int a = t / per;
        const int z0 = (t - a * per) * TC;
        g.p0 = a;
        g.p1 = z0;
        g.si = (axis == AX_Y) ? d.nz : d.ny * d.nz;
        g.sc = 1;
        g.base = (axis == AX_Y) ? (size_t)a * d.ny * d.nz + z0 : (size_t)a * d.nz + z0;
    }
    return g;
}

// Offset of element (i, c) from the tile base; below 2^31 for every grid up to 2^30 cells.
__device__ __forceinline__ unsigned off(const Tile &g, int i, int c) {
    return (unsigned)i * (unsigned)g.si + (unsigned)c * (unsigned)g.sc;
}

// Octant folding of a frequency index: k and n - k share an entry.
__device__ __forceinline__ int fold(int k, int n) { return k <= n - k ? k : n - k; }

// ---------------------------------------------------------------------------
// Scale of the packed pair.  Two real fields share one complex transform as
// a + i s b.  Float rounding in a complex transform is relative to the size
// of the complex values, so the rounding of s b leaks into a's spectrum and
// maps, and the reverse.  In the estimator a is N = D - alpha R, whose sums
// cancel between cells, and b is the random field R, several times larger
// per cell and one-signed.  s is therefore a power of two (exact to apply and
// to undo) that brings the root mean square of s b to about a quarter of a's:
// a's rounding then stays within a few per cent of that of a transformed
// alone, and b's grows about fourfold on sums that do not cancel.  s is
// chosen on the device (no host synchronisation, graph-safe) from the sums
// of squares of both fields, added in a fixed order.  It is undone exactly:
// stored maps of b are multiplied by 1/s, sums of order p over maps of b by
// s^-p.
// ---------------------------------------------------------------------------
constexpr int PS_T = 256;

template <typename T, int PV>
__device__ __forceinline__ void pack_sums_body(const T *__restrict__ a, const T *__restrict__ b, size_t n,
                                               double *__restrict__ part);

template <typename T, int PV>
__global__ __launch_bounds__(PS_T) void k_pack_sums(const T *__restrict__ a, const T *__restrict__ b, size_t n,
                                                    double *__restrict__ part) {
    pack_sums_body<T, PV>(a, b, n, part);
}

template <typename T, int PV>
__device__ __forceinline__ void pack_sums_body(const T *__restrict__ a, const T *__restrict__ b, size_t n,
                                               double *__restrict__ part) {
    __shared__ double red[PS_T / 64][2];
    double sa = 0.0, sb = 0.0;
    const size_t nv = n / PV, stride = (size_t)gridDim.x * PS_T;
    for (size_t i = (size_t)blockIdx.x * PS_T + threadIdx.x; i < nv; i += stride) {
        if constexpr (PV == 1) {
            const double x = (double)a[i], y = (double)b[i];
            sa += x * x;
            sb += y * y;
        } else {
            using V = typename std::conditional<std::is_same<T, float>::value, float4, double2>::type;
            const V x = reinterpret_cast<const V *>(a)[i];
            const V y = reinterpret_cast<const V *>(b)[i];
            if constexpr (std::is_same<T, float>::value) {
                sa += (double)x.x * x.x + (double)x.y * x.y + (double)x.z * x.z + (double)x.w * x.w;
                sb += (double)y.x * y.x + (double)y.y * y.y + (double)y.z * y.z + (double)y.w * y.w;
            } else {
                sa += x.x * x.x + x.y * x.y;
                sb += y.x * y.x + y.y * y.y;
            }
        }
    }
    if (blockIdx.x == 0)   // the tail beyond whole vectors
        for (size_t i = nv * PV + threadIdx.x; i < n; i += PS_T) {
            const double x = (double)a[i], y = (double)b[i];
            sa += x * x;
            sb += y * y;
        }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o >= 1; o >>= 1) {
        sa += __shfl_xor(sa, o);
        sb += __shfl_xor(sb, o);
    }
    if (lane == 0) {
        red[wv][0] = sa;
        red[wv][1] = sb;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double v = 0.0;
        for (int w = 0; w < PS_T / 64; ++w) v += red[w][threadIdx.x];
        part[2 * blockIdx.x + threadIdx.x] = v;
    }
}

// One workgroup: the G partial pairs (sum a^2, sum b^2) in a fixed order, then s.  Fields that are
// zero or not finite leave s = 1.  |k| <= 60 keeps s b and its maps far from
// the float range limits.
constexpr int PSR_T = 1024;   // threads of the one workgroup that adds the partials

__global__ __launch_bounds__(PSR_T) void k_pack_scale(const double *__restrict__ part, int G, PackScale *out) {
    // one workgroup per pair (size classes: one per job, partials G apart)
    part += 2 * (size_t)blockIdx.x * G;
    out += blockIdx.x;
    __shared__ double red[2][PSR_T];
    double sa = 0.0, sb = 0.0;
    for (int g = threadIdx.x; g < G; g += PSR_T) {
        const double2 v = reinterpret_cast<const double2 *>(part)[g];
        sa += v.x;
        sb += v.y;
    }
    red[0][threadIdx.x] = sa;
    red[1][threadIdx.x] = sb;
    __syncthreads();
    for (int h = PSR_T / 2; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ta = red[0][0], tb = red[1][0];
        int k = 0;
        if (ta > 0.0 && tb > 0.0 && isfinite(ta) && isfinite(tb)) {
            // rms(s b) = rms(a) / 4:  k = log2(rms a / rms b) - 2
            const double e = 0.5 * (log2(ta) - log2(tb)) - 2.0;
            k = (int)rint(e);
            k = k < -60 ? -60 : (k > 60 ? 60 : k);
        }
        PackScale ps;
        ps.s = ldexp(1.0, k);
        ps.s_inv = ldexp(1.0, -k);
        ps.sf = (float)ps.s;
        ps.sf_inv = (float)ps.s_inv;
        ps.k = k;
        ps.pad = 0;
        *out = ps;
    }
}

template <typename T>
__device__ __forceinline__ T scale_of(const PackScale *ps) {
    if constexpr (std::is_same<T, float>::value) return ps->sf;
    else return ps->s;
}
template <typename T>
__device__ __forceinline__ T scale_inv_of(const PackScale *ps) {
    if constexpr (std::is_same<T, float>::value) return ps->sf_inv;
    else return ps->s_inv;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------
// With `mask` (line flags [nx * ny], both fields zero on lines without one):
// z-line tiles without a flagged line do nothing, and only flagged lines are
// written (the y pass then reads the others as zero).  TWO: b is given and
// multiplied by the pair's scale s (a separate instantiation, so that no
// branch on b sits between the loads of a tile and they all issue together).
template <typename T, bool TWO>
struct OpPack {
    static constexpr bool STAGED = false;   // z pass, forward: (a + i s b) -> spec
    using C = cplx<T>;
    const void *tw;
    Dims d;
    const T *a;
    const T *b;
    C *out;
    Tile g;
    const unsigned char *mask;
    int tcn;
    const PackScale *ps;
    T sb;
    template <int TC> __device__ void begin() {
        g = make_tile(AX_Z, d, blockIdx.x, TC);
        tcn = TC;
        a += g.base;
        if constexpr (TWO) {
            b += g.base;
            sb = scale_of<T>(ps);
        }
        out += g.base;
    }
    __device__ bool active() const {   // the same for every thread: any line of the tile flagged
        if (!mask) return true;
        int any = 0;
        for (int k = 0; k < tcn; ++k) any |= mask[(size_t)g.p0 + k];
        return any != 0;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const {
        const unsigned k = off(g, i, c);
        if constexpr (TWO) return C{a[k], b[k] * sb};
        else return C{a[k], (T)0};
    }
    __device__ void store(int i, int c, C v) const {
        if (mask && !mask[(size_t)g.p0 + c]) return;
        out[off(g, i, c)] = v;
    }
};

// z pass, forward, for every job of a size class (job = blockIdx.y): N_j + i s_j R_j -> spec[j].
struct OpPackJobs {
    static constexpr bool STAGED = false;
    using C = float2;
    const void *tw;
    Dims d;
    const ClassJob *tab;
    C *spec;
    size_t nc;
    const PackScale *scales;
    Tile g;
    const float *a, *b;
    C *out;
    float sb;
    template <int TC> __device__ void begin() {
        g = make_tile(AX_Z, d, blockIdx.x, TC);
        const ClassJob &j = tab[blockIdx.y];
        a = j.N + g.base;
        b = j.R + g.base;
        out = spec + (size_t)blockIdx.y * nc + g.base;
        sb = scales[blockIdx.y].sf;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const {
        const unsigned k = off(g, i, c);
        return C{a[k], b[k] * sb};
    }
    __device__ void store(int i, int c, C v) const { out[off(g, i, c)] = v; }
};

// With `xcount` and `mask` (y axis only): tiles of x-slabs without carrying
// lines do nothing, and only rows y of carrying lines (x, y) are written.
// RF: inputs known to be zero are not read: with `lmask` (y axis), rows y of
// lines (x, y) without a flag; with `lxcount` (x axis), rows x of slabs without
// a carrying line.
template <typename T, bool RF = false>
struct OpInplace {
    static constexpr bool STAGED = false;   // any axis, in place; blockIdx.y selects a grid of the batch
    static constexpr bool ROWF = RF;
    using C = cplx<T>;
    const void *tw;
    Dims d;
    int axis;
    C *buf;
    size_t nc;
    Tile g;
    C *p;
    const unsigned char *mask;
    const int *xcount;
    const unsigned char *lmask;
    const int *lxcount;
    const unsigned char *rowf = nullptr;   // LDS: the tile's row flags from lmask / lxcount
    // persistent launches (the inverse y pass): workgroups loop over tiles
    static constexpr bool PERSIST = !RF;
    bool persist = false;
    template <int TC> __device__ void begin() { begin_at<TC>(blockIdx.x, blockIdx.y); }
    template <int TC> __device__ void begin_at(int tile, int batch) {
        g = make_tile(axis, d, tile, TC);
        p = buf + (size_t)batch * nc + g.base;
    }
    __device__ bool active() const { return !xcount || xcount[g.p0] > 0; }
    __device__ bool wants_rowf() const { return lmask != nullptr || lxcount != nullptr; }
    __device__ unsigned char rowflag(int i) const {
        if (lmask) return lmask[(size_t)g.p0 * d.ny + i];
        return lxcount[i] > 0 ? 1 : 0;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const {
        if constexpr (RF) {
            if (rowf && !rowf[i]) return C{};
        }
        return p[off(g, i, c)];
    }
    __device__ bool keeps() const { return mask != nullptr; }
    __device__ int flag(int i) const { return mask[(size_t)g.p0 * d.ny + i]; }
    __device__ void store(int i, int c, C v) const { p[off(g, i, c)] = v; }   // rows with a flag
};


// x pass, inverse, for radii m0 .. m0+nb-1: spec * K_m -> tspec[m - m0].
// The kernel octant of radius m is stored [ky'][kz'][kx'] (x fastest), so the
// values a thread needs for its (ky, kz) column are one contiguous run.
// With loop = 0 each workgroup handles one (tile, radius) pair.  Workgroups are
// dispatched round-robin over the 8 XCDs; the nb radii of one tile get ids 8
// apart so that they run on one XCD back to back and re-read the tile of
// `spec` from that XCD's L2.  With loop = 1 each workgroup runs the nb radii of
// its tile one after the other.
template <typename T, bool STG>
struct OpMulK {
    static constexpr bool STAGED = STG;
    using C = cplx<T>;
    const void *tw;
    Dims d;
    const C *spec;
    const T *kspec;
    C *tspec;
    size_t nc;
    size_t kel;   // octant elements per radius
    int m0, nb, tiles, loop;
    Tile g;
    int m, col;
    const C *src;   // spec at this tile and this thread's column
    C *dst;
    const T *kcol;  // octant of radius m at this thread's (ky, kz) column
    // radius pairing (one real field): slot m multiplies by K_{2m} + i K_{2m+1}
    int pair, ns;
    const T *kcol_b;
    template <int TC> __device__ void begin() {
        const int w = blockIdx.x;
        int tile;
        if (loop) {
            tile = w;
            m = 0;
        } else if ((tiles & 7) == 0) {
            const int xcd = w & 7, slot = w >> 3;
            tile = (slot / nb) * 8 + xcd;
            m = slot % nb;
        } else {
            tile = w / nb;
            m = w % nb;
        }
        g = make_tile(AX_X, d, tile, TC);
        col = threadIdx.x % TC;
        src = spec + g.base + col;
        set_radius();
    }
    __device__ void set_radius() {
        const int oy = fold(g.p0, d.ny), oz = fold(g.p1 + col, d.nz);
        const size_t co = ((size_t)oy * (d.nz / 2 + 1) + oz) * (d.nx / 2 + 1);
        if (pair) {
            const int ra = 2 * (m0 + m), rb = ra + 1;
            kcol = kspec + (size_t)ra * kel + co;
            kcol_b = rb < ns ? kspec + (size_t)rb * kel + co : nullptr;
        } else {
            kcol = kspec + (size_t)(m0 + m) * kel + co;
        }
        dst = tspec + (size_t)m * nc + g.base + col;
    }
    __device__ int iters() const { return loop ? nb : 1; }
    __device__ void set_iter(int it) {
        if (loop) {
            m = it;
            set_radius();
        }
    }
    __device__ C load(int i, int) const {
        const int fi = fold(i, d.nx);
        const T kv = kcol[fi];
        const C s = src[(size_t)(unsigned)i * (unsigned)g.si];
        if (pair) {   // s (ka + i kb)
            const T kb = kcol_b ? kcol_b[fi] : (T)0;
            return C{s.x * kv - s.y * kb, s.y * kv + s.x * kb};
        }
        return C{s.x * kv, s.y * kv};
    }
    __device__ void store(int i, int, C v) const { dst[(size_t)(unsigned)i * (unsigned)g.si] = v; }
};

// z pass, inverse: tspec[m] -> real parts to maps_a[m0+m], imaginary to maps_b[m0+m].
// With `pair` (one real field, radii paired): slot j holds C_{2j} + i C_{2j+1};
// the real part goes to maps_a[2 (m0 + j)], the imaginary part to the next row
// of maps_a when that radius exists.
template <typename T>
struct OpUnpack {
    static constexpr bool STAGED = false;
    using C = cplx<T>;
    const void *tw;
    Dims d;
    const C *tspec;
    T *ma;
    T *mb;
    size_t nc;
    int m0;
    Tile g;
    const C *src;
    int pair, ns;
    const unsigned char *mask;   // NULL, or line flags [nx * ny]: only lines with a flag are written
    int tcn;
    const PackScale *ps;         // two packed fields: the maps of b are stored times 1/s
    T sbi;
    template <int TC> __device__ void begin() {
        g = make_tile(AX_Z, d, blockIdx.x, TC);
        tcn = TC;
        sbi = ps ? scale_inv_of<T>(ps) : (T)1;
        src = tspec + (size_t)blockIdx.y * nc + g.base;
        if (pair) {
            const int ra = 2 * (m0 + blockIdx.y);
            mb = ra + 1 < ns ? ma + (size_t)(ra + 1) * nc + g.base : nullptr;
            ma += (size_t)ra * nc + g.base;
            return;
        }
        const size_t o = (size_t)(m0 + blockIdx.y) * nc + g.base;
        ma += o;
        if (mb) mb += o;
    }
    __device__ bool active() const {   // the same for every thread: any line of the tile flagged
        if (!mask) return true;
        int any = 0;
        for (int k = 0; k < tcn; ++k) any |= mask[(size_t)g.p0 + k];
        return any != 0;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const { return src[off(g, i, c)]; }
    __device__ void store(int i, int c, C v) const {
        if (mask && !mask[(size_t)g.p0 + c]) return;
        const unsigned k = off(g, i, c);
        ma[k] = v.x;
        if (mb) mb[k] = v.y * sbi;
    }
};

// z pass, inverse, for every job of a size class: blockIdx.y = job * nb + slot;
// tspec[job][slot] -> rows m0 + slot of the job's maps (R's times 1 / s_j).
struct OpUnpackJobs {
    static constexpr bool STAGED = false;
    using C = float2;
    const void *tw;
    Dims d;
    const float2 *tspec;
    const ClassJob *tab;
    const PackScale *scales;
    size_t nc;
    int m0, nb;
    Tile g;
    const C *src;
    float *ma, *mb;
    float sbi;
    template <int TC> __device__ void begin() {
        g = make_tile(AX_Z, d, blockIdx.x, TC);
        const int job = blockIdx.y / nb, slot = blockIdx.y - job * nb;
        const ClassJob &j = tab[job];
        src = tspec + (size_t)blockIdx.y * nc + g.base;
        const size_t o = (size_t)(m0 + slot) * nc + g.base;
        ma = j.mapsN + o;
        mb = j.mapsR + o;
        sbi = scales[job].sf_inv;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const { return src[off(g, i, c)]; }
    __device__ void store(int i, int c, C v) const {
        const unsigned k = off(g, i, c);
        ma[k] = v.x;
        mb[k] = v.y * sbi;
    }
};

// z pass, forward, of two shell indicators generated on the fly:
// real part = [lo_a <= |delta|^2 < hi_a], imaginary part likewise for b,
// with delta the minimum-image offset of the cell from cell (0, 0, 0).
struct OpShellFill {
    static constexpr bool STAGED = false;
    using C = double2;
    const void *tw;
    Dims d;
    double lo_a, hi_a, lo_b, hi_b;
    C *out;
    Tile g;
    template <int TC> __device__ void begin() { g = make_tile(AX_Z, d, blockIdx.x, TC); }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const {
        const int row = g.p0 + c;
        const int x = row / d.ny, y = row - (row / d.ny) * d.ny, z = i;
        const int dx = 2 * x <= d.nx ? x : x - d.nx;
        const int dy = 2 * y <= d.ny ? y : y - d.ny;
        const int dz = 2 * z <= d.nz ? z : z - d.nz;
        const double d2 = (double)(dx * dx + dy * dy + dz * dz);
        return C{(d2 >= lo_a && d2 < hi_a) ? 1.0 : 0.0, (d2 >= lo_b && d2 < hi_b) ? 1.0 : 0.0};
    }
    __device__ void store(int i, int c, C v) const { out[g.base + off(g, i, c)] = v; }
};

// x pass, forward, of the packed shell pair: keep the octant, x fastest,
// scaled by 1/N_c: kspec[m][ky][kz][kx] for kx <= nx/2, ky <= ny/2, kz <= nz/2.
template <typename K>
struct OpExtract {
    static constexpr bool STAGED = false;
    using C = double2;
    const void *tw;
    Dims d;
    const C *buf;
    K *kspec;
    size_t kel;
    int ma, mb;
    double scale;
    Tile g;
    template <int TC> __device__ void begin() { g = make_tile(AX_X, d, blockIdx.x, TC); }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const { return buf[g.base + off(g, i, c)]; }
    __device__ void store(int i, int c, C v) const {
        const int ky = g.p0, kz = g.p1 + c, kx = i;
        if (2 * kx > d.nx || 2 * ky > d.ny || 2 * kz > d.nz) return;
        const size_t ko = ((size_t)ky * (d.nz / 2 + 1) + kz) * (d.nx / 2 + 1) + kx;
        kspec[(size_t)ma * kel + ko] = (K)(v.x * scale);
        if (mb >= 0) kspec[(size_t)mb * kel + ko] = (K)(v.y * scale);
    }
};

// ---------------------------------------------------------------------------
// x pass, inverse, with the kernel multiply, for a batch of radii, keeping the
// spectrum tile resident: the tile (all kx of one ky and TC columns kz) is
// read from HBM once per batch instead of once per radius, each thread
// holding in registers the points its first-stage butterflies take (the same
// for every radius).  For each radius the kernel octant values of the tile's
// columns (one contiguous run per column, x fastest) are staged into LDS with
// coalesced reads, prefetched into registers while the previous radius is
// transformed.
// ---------------------------------------------------------------------------
// Row stride (values) of the staged kernel values of one tile column.  The
// first stage's lanes read TC columns x 64/TC consecutive rows; a stride of
// 64/TC modulo 32 banks puts those 64 reads on distinct banks (two rounds of
// 32) instead of bank (column + row) mod 32.
template <int L, int TC>
constexpr int kt_stride() {
    constexpr int nxh = L / 2 + 1, want = (64 / TC) % 32;
    return nxh + (((want - nxh) % 32) + 32) % 32;
}

template <typename T, int L, int TC, int PER0, bool PAIR = false>
struct OpResident {
    static constexpr bool STAGED = false;
    static constexpr bool KBITS = true;
    using C = cplx<T>;
    const C (*sreg)[8];   // registers: this thread's first-stage inputs [PER0][8]
    const T *kt;          // LDS: kernel values [TC][L/2 + 1]; with PAIR a second such block (radius b)
    C *out;               // global: output tile base
    unsigned si;
    const unsigned char *xf;   // LDS: x-slab carries field (row written), or NULL: every row
    const unsigned *kb;        // registers: the last stage's keep bits, taken once per tile
    __device__ C load_r(int q, int r, int i, int c) const {
        const C s = sreg[q][r];
        const int e = c * kt_stride<L, TC>() + (i <= L - i ? i : L - i);
        const T k = kt[e];
        if constexpr (PAIR) {   // s (K_a + i K_b)
            const T kb = kt[TC * kt_stride<L, TC>() + e];
            return C{s.x * k - s.y * kb, s.y * k + s.x * kb};
        }
        return C{s.x * k, s.y * k};
    }
    __device__ bool keeps() const { return xf != nullptr; }
    __device__ int flag(int i) const { return xf[i]; }
    __device__ void store(int i, int c, C v) const { out[(unsigned)i * si + (unsigned)c] = v; }   // rows with a flag
};

template <typename T, int L, bool PAIR = false>
constexpr bool resident_fits() {
    using SH = Shape<T, L, TM_R>;
    return Plan<L>::r[0] == 8 &&
           (size_t)SH::LDS * sizeof(cplx<T>) + (size_t)L * sizeof(cplx<T>) +
                   (PAIR ? 2 : 1) * (size_t)SH::TC * kt_stride<L, SH::TC>() * sizeof(T) + (size_t)L <=
               160 * 1024;
}

// Two exchange buffers (rows padded by one value) in place of one: the three
// stages of a line then alternate buffers and need one barrier each between
// them, two per radius instead of five.
template <typename T, int L>
constexpr bool pingpong_fits() {
    using SH = Shape<T, L, TM_R>;
    return Plan<L>::n == 3 &&
           2 * (size_t)L * (SH::TC + 1) * sizeof(cplx<T>) + (size_t)L * sizeof(cplx<T>) +
                   (size_t)SH::TC * kt_stride<L, SH::TC>() * sizeof(T) + (size_t)L <=
               160 * 1024;
}

// PAIR (one real field, radii paired): slot m is multiplied by K_{2j} + i K_{2j+1}
// with j = m0 + m (K_{2j} alone when 2j + 1 = pair_ns), so one transform gives
// the maps of two radii; the two kernel rows are staged side by side.
template <typename T, int L, bool PPW, bool PAIR>
__global__ __launch_bounds__((Shape<T, L, TM_R>::NT), (Shape<T, L, TM_R>::MINW)) void k_xmul_resident(
    const cplx<T> *__restrict__ spec, const T *__restrict__ kspec, cplx<T> *__restrict__ tspec,
    const cplx<T> *__restrict__ twg, Dims d, size_t nc, size_t kel, int m0, int nb, const int *__restrict__ xcount,
    int pair_ns) {
    using C = cplx<T>;
    using SH = Shape<T, L, TM_R>;
    constexpr int TC = SH::TC, NT = SH::NT, NXH = L / 2 + 1;
    constexpr int KR = PAIR ? 2 : 1;                     // kernel rows per slot
    // size classes: job blockIdx.y has its spectrum at spec + job nc and its
    // nb slots at tspec + job nb nc (one job otherwise)
    spec += (size_t)blockIdx.y * nc;
    tspec += (size_t)blockIdx.y * nb * nc;
    constexpr int KPT = (KR * TC * NXH + NT - 1) / NT;   // kernel values staged per thread
    constexpr bool PP = PPW && !PAIR && pingpong_fits<T, L>();
    constexpr int PADR = PP ? 1 : SH::PAD, LDSN = L * (TC + PADR);
    __shared__ C lds[PP ? 2 * LDSN : LDSN];
    __shared__ C tw[L];
    constexpr int KS = kt_stride<L, TC>();
    __shared__ T kt[KR * TC * KS];   // [KR][TC][KS]: rows of NXH values, padded
    __shared__ unsigned char xf[L];   // x-slabs carrying field (when xcount is given)
    // Tiles (ky, kz-block) and (ny - ky, kz-block) read the same kernel values,
    // and where a tile's rows are narrower than 128 bytes (TC complex values)
    // the ZG z-blocks of one 128-byte run share every cache line they read and
    // write.  Workgroups are dispatched round-robin over the 8 XCDs; ids w,
    // w + 8, ..., w + 8 (2 ZG - 1) (same XCD, consecutive) take such a group of
    // 2 ZG tiles, so the other reads of each kernel block and line hit that
    // XCD's L2 and its partial-line writes merge there.  Pair k = 0 holds the
    // two self-mirrored rows ky = 0 and ky = ny/2.
    const int nzb = d.nz / TC;
    constexpr int RUN = TC * (int)sizeof(C);
    constexpr int ZG = RUN >= 128 ? 1 : 128 / RUN, GM = 2 * ZG;
    int tile = blockIdx.x;
    const int nzg = nzb / ZG;
    if (nzb % ZG == 0 && (((d.ny / 2) * nzg) & 7) == 0) {
        const int xcd = blockIdx.x & 7, s8 = blockIdx.x >> 3;
        const int p = (s8 / GM) * 8 + xcd, member = s8 % GM;
        const int k = p / nzg, zb = (p - k * nzg) * ZG + member % ZG;
        const int ky = member / ZG == 0 ? k : (k == 0 ? d.ny / 2 : d.ny - k);
        tile = ky * nzb + zb;
    }
    const Tile g = make_tile(AX_X, d, tile, TC);
    for (int t = threadIdx.x; t < L; t += NT) {
        tw[t] = twg[t];
        if (xcount) xf[t] = xcount[t] > 0 ? 1 : 0;
    }
    // this thread's first-stage points (radix 8, butterflies q of the first stage)
    constexpr int LR0 = L / 8, NB0 = LR0 * TC, PER0 = (NB0 + NT - 1) / NT;
    C sreg[PER0][8];
#pragma unroll
    for (int q = 0; q < PER0; ++q) {
        const int b = threadIdx.x + q * NT;
        int j, c;
        split_q<NT, TM_R, LR0, TC>(q, j, c);
#pragma unroll
        for (int r = 0; r < 8; ++r)
            sreg[q][r] = (NB0 % NT == 0 || b < NB0)
                             ? spec[g.base + (size_t)(unsigned)(j + r * LR0) * (unsigned)g.si + c]
                             : C{};
    }
    const int oy = fold(g.p0, d.ny);
    const int nzh = d.nz / 2 + 1;
    auto kload = [&](int m, T (&kv)[KPT]) {
        const int ra = PAIR ? 2 * (m0 + m) : m0 + m;
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < KR * TC * NXH) {
                const int h = e / (TC * NXH), el = e - h * (TC * NXH);   // h = 1: radius b of the pair
                const int c = el / NXH, ox = el - (el / NXH) * NXH;
                const int rr = ra + h;
                kv[q] = (!PAIR || rr < pair_ns)
                            ? kspec[(size_t)rr * kel + ((size_t)oy * nzh + fold(g.p1 + c, d.nz)) * NXH + ox]
                            : (T)0;
            }
        }
    };
    auto kstage = [&](const T (&kv)[KPT]) {
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
            const int e = threadIdx.x + q * NT;
            if (e < KR * TC * NXH) {
                const int hc = e / NXH, ox = e - hc * NXH;   // (h, c) row, then ox
                kt[hc * KS + ox] = kv[q];
            }
        }
    };
    // the last stage's keep bits: the same rows for every radius of the tile
    __syncthreads();   // xf written
    unsigned kmask[LastStage<T, L, TM_R>::PER];
    {
        const OpResident<T, L, TC, PER0, PAIR> op0{sreg, kt, tspec + g.base, (unsigned)g.si, xcount ? xf : nullptr,
                                                   nullptr};
        last_keep_bits<T, L, TM_R>(op0, kmask);
    }
    T kv[KPT];
    kload(0, kv);
    if constexpr (PP) {
        // Stage 0 writes buffer A, stage 1 reads A and writes B, stage 2 reads
        // B.  Each write follows the last read of the same buffer across a
        // barrier: A's reads end before the barrier after stage 1, B's before
        // the barrier after the next radius's stage 0.  The kernel values of
        // radius m + 1 are written during stage 1 of radius m, after every
        // stage-0 read of radius m's values and before the barrier that
        // precedes their first read.
        kstage(kv);
        if (nb > 1) kload(1, kv);
        __syncthreads();
        C *const la = lds, *const lb = lds + LDSN;
        for (int m = 0; m < nb; ++m) {
            OpResident<T, L, TC, PER0, PAIR> op{sreg, kt, tspec + (size_t)m * nc + g.base, (unsigned)g.si,
                                                xcount ? xf : nullptr, kmask};
            fft_stage<T, L, TM_R, +1, 0, false, false, PADR>(la, la, tw, op);
            __syncthreads();
            fft_stage<T, L, TM_R, +1, 1, false, false, PADR>(la, lb, tw, op);
            if (m + 1 < nb) {
                kstage(kv);
                if (m + 2 < nb) kload(m + 2, kv);
            }
            __syncthreads();
            fft_stage<T, L, TM_R, +1, 2, false, false, PADR>(lb, lb, tw, op);
        }
    } else {
        for (int m = 0; m < nb; ++m) {
            kstage(kv);
            __syncthreads();
            if (m + 1 < nb) kload(m + 1, kv);
            OpResident<T, L, TC, PER0, PAIR> op{sreg, kt, tspec + (size_t)m * nc + g.base, (unsigned)g.si,
                                                xcount ? xf : nullptr, kmask};
            fft_line_tile<T, L, TM_R, +1, false>(lds, tw, op);
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// z pass, inverse, with the equidistant summation of Eq. ksinDiag in place of
// the map stores: for the radii of one batch (blockIdx.y) and both packed
// fields, sum F(x) C_m(x)^p for p = 1 .. P over every cell.  Each workgroup
// runs a strided set of z-line tiles, accumulating in FP64 per thread, and
// writes one partial row per (radius, workgroup); rows are reduced in a fixed
// order afterwards.
// ---------------------------------------------------------------------------
template <typename T, int P, int PER, int R>
struct OpDiag {
    static constexpr bool STAGED = false;
    static constexpr bool STORE_QR = true;
    using C = cplx<T>;
    static constexpr unsigned NONE = 0xffffffffu;
    const C *src;
    const T *fa;
    const T *fb;
    const unsigned *row;   // LDS: first cell of each line of the tile, NONE for no line
    double acc[2][P];
    // F of both fields at this thread's last-stage cells, loaded when the tile
    // starts so that the loads are in flight during its transform (0 where
    // the tile has no line)
    T va[PER][R], vb[PER][R];
    __device__ C load(int i, int c) const {
        const unsigned r = row[c];
        if (r == NONE) return C{(T)0, (T)0};
        return src[r + (unsigned)i];
    }
    template <int L, int MODE>
    __device__ void prefetch() {
        last_stage_cells<T, L, MODE>([&](int q, int r, int i, int c) {
            const unsigned rw = row[c];
            const bool ok = rw != NONE;
            const unsigned k = ok ? rw + (unsigned)i : 0u;
            va[q][r] = ok ? fa[k] : (T)0;
            vb[q][r] = (ok && fb) ? fb[k] : (T)0;
        });
    }
    // a cell outside every line adds F = 0: nothing
    __device__ void store_qr(int q, int r, int, int, C v) {
        const T a = va[q][r];
        T pw = v.x;
        acc[0][0] += (double)(a * pw);
#pragma unroll
        for (int p = 1; p < P; ++p) {
            pw *= v.x;
            acc[0][p] += (double)(a * pw);
        }
        if (fb) {
            const T b = vb[q][r];
            pw = v.y;
            acc[1][0] += (double)(b * pw);
#pragma unroll
            for (int p = 1; p < P; ++p) {
                pw *= v.y;
                acc[1][p] += (double)(b * pw);
            }
        }
    }
};

template <typename T, int L, int P>
__global__ __launch_bounds__((Shape<T, L, TM_J>::NT), (Shape<T, L, TM_J>::MINW)) void k_zinv_diag(
    const cplx<T> *__restrict__ tspec, const T *__restrict__ fa, const T *__restrict__ fb,
    const cplx<T> *__restrict__ twg, Dims d, size_t nc, int tiles, double *__restrict__ part,
    const int *__restrict__ list, const int *__restrict__ count) {
    using C = cplx<T>;
    using SH = Shape<T, L, TM_J>;
    constexpr int NT = SH::NT, NW = NT / 64, TC = SH::TC;
    __shared__ C lds[SH::LDS];
    __shared__ C tw[L];
    __shared__ double red[NW][2 * P];
    __shared__ unsigned row[TC];
    for (int t = threadIdx.x; t < L; t += NT) tw[t] = twg[t];
    using LS = LastStage<T, L, TM_J>;
    OpDiag<T, P, LS::PER, LS::R> op;
#pragma unroll
    for (int p = 0; p < P; ++p) op.acc[0][p] = op.acc[1][p] = 0.0;
    op.row = row;
    op.src = tspec + (size_t)blockIdx.y * nc;
    op.fa = fa;
    op.fb = fb;
    // with a list: tiles of TC listed lines (the lines carrying field; the
    // others add nothing), else tiles of TC consecutive lines
    const int nlist = list ? *count : 0;
    const int ntiles = list ? (nlist + TC - 1) / TC : tiles;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();   // the previous tile is done with row (and the twiddles are in)
        for (int c = threadIdx.x; c < TC; c += NT) {
            const int k = tile * TC + c;
            row[c] = list ? (k < nlist ? (unsigned)list[k] * (unsigned)d.nz : decltype(op)::NONE)
                          : (unsigned)k * (unsigned)d.nz;
        }
        __syncthreads();
        op.template prefetch<L, TM_J>();
        fft_line_tile<T, L, TM_J, +1, false>(lds, tw, op);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int p = 0; p < P; ++p) {
            double v = op.acc[f][p];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0) red[wv][f * P + p] = v;
        }
    __syncthreads();
    if (threadIdx.x < 2 * P) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) v += red[w][threadIdx.x];
        part[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (2 * P) + threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------------------
// Size classes, n = 3, at most 16 radii: the inverse z pass and the summation
// in one kernel, so that no map is written to memory (Eq. ksin_delta needs
// only the sums).  A tile holds LPT = TC / 16 consecutive z-lines of one job
// for 16 radius slots (tile column c = slot LPT + line).  Its transform
// leaves C_m on the tile's cells in LDS (both packed fields; R's times
// 1 / s_j), and the workgroup then sums F(x) C_a(x) C_b(x) over those cells
// on the matrix cores, as k_mm3s does from stored maps: one 16 x 16 tile per
// field, lane (r, h) = (lane % 16, lane / 16) holding cells 8 h .. 8 h + 7 of
// a 32-cell chunk for radius r; split bfloat16 (32 cells per instruction) or
// float32 (v_mfma_f32_16x16x4f32, cell 8 h + e of each lane group in the
// e-th instruction: no operand splitting on the vector units).
// Slots from n_radii on transform zeros.  Workgroups of job blockIdx.y take
// tiles blockIdx.x, + gridDim.x, ...; each writes float64 partial tiles (the
// 32 x 32 layout of the summation, zeros beyond 16 x 16) for N and R of its
// job, which the summation's reduction adds in a fixed order.
// ---------------------------------------------------------------------------
template <int L>
struct ZMM {
    using SH = Shape<float, L, TM_J>;
    static constexpr int RS = 16;                  // radius slots
    static constexpr int TC = SH::TC;
    static constexpr int LPT = TC / RS;            // grid lines per tile
    static constexpr int CELLS = LPT * L;          // cells per tile
    static constexpr int P = CELLS + 4;            // LDS row of one slot (floats), padded
    static constexpr bool OK = TC >= RS && SH::NT == 256 && CELLS % 32 == 0;
};

template <int L>
struct OpZinvMM {
    static constexpr bool STAGED = false;
    static constexpr bool SYNC_LAST = true;   // the maps take the transform tile's LDS
    using C = float2;
    static constexpr int LPT = ZMM<L>::LPT, P = ZMM<L>::P, RS = ZMM<L>::RS;
    const float2 *src;   // slot 0 of the job's spectra, at the tile's first cell
    size_t nc;
    int ns;
    float *maps;         // LDS [2][RS][P]
    float sbi;
    __device__ C load(int i, int c) const {
        const int sl = c / LPT, l = c - sl * LPT;
        if (sl >= ns) return C{0.f, 0.f};
        return src[(size_t)sl * nc + (unsigned)(l * L + i)];
    }
    __device__ void store(int i, int c, C v) const {
        const int sl = c / LPT, l = c - sl * LPT;
        const int o = sl * P + l * L + i;
        maps[o] = v.x;
        maps[RS * P + o] = v.y * sbi;
    }
};

template <int L, int MODE, int PREC>
__global__ __launch_bounds__(256, 4) void k_zinv_mm3_jobs(const float2 *__restrict__ tspec,
                                                         const ClassJob *__restrict__ tab,
                                                         const PackScale *__restrict__ scales,
                                                         const float2 *__restrict__ twg, Dims d, size_t nc, int ns,
                                                         double *__restrict__ partial) {
    using Z = ZMM<L>;
    using SH = typename Z::SH;
    constexpr int NT = 256, NWV = NT / 64, CELLS = Z::CELLS, P = Z::P, NCH = CELLS / 32;
    constexpr int FPT = (2 * CELLS + NT - 1) / NT;   // field values staged per thread
    static_assert(Z::OK, "tile shape");
    static_assert(2 * 16 * P * sizeof(float) >= NWV * 8 * 64 * sizeof(double), "combine area");
    // the maps of a tile (both fields, 16 slots) and its field values take the
    // LDS of the transform tile once its last stage has read it
    static_assert((2 * 16 * P + 2 * CELLS) * sizeof(float) <= SH::LDS * sizeof(float2), "maps in the tile's LDS");
    __shared__ __align__(16) float2 lds[SH::LDS];
    __shared__ float2 tw[L];
    float *const maps = reinterpret_cast<float *>(lds);
    float *const fl = maps + 2 * 16 * P;
    const int job = blockIdx.y;
    const ClassJob &jb = tab[job];
    for (int t = threadIdx.x; t < L; t += NT) tw[t] = twg[t];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r = lane & 15, h = lane >> 4;
    const bool hm = r < ns;
    floatx4_t acc0 = floatx4_t{0}, acc1 = floatx4_t{0};
    double accd[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    OpZinvMM<L> op;
    op.nc = nc;
    op.ns = ns;
    op.maps = maps;
    op.sbi = scales[job].sf_inv;
    const float2 *jspec = tspec + (size_t)job * ns * nc;
    const long ntiles = (long)d.nx * d.ny / Z::LPT;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const size_t cell0 = (size_t)tile * CELLS;   // the tile's lines are consecutive
        float fv[FPT];
#pragma unroll
        for (int k = 0; k < FPT; ++k) {   // both fields on the tile's cells, loaded before the transform
            const int idx = threadIdx.x + k * NT;
            fv[k] = idx < CELLS ? jb.N[cell0 + idx] : (idx < 2 * CELLS ? jb.R[cell0 + idx - CELLS] : 0.f);
        }
        op.src = jspec + cell0;
        __syncthreads();   // the previous tile is done with maps, fl and lds (twiddles in)
        fft_line_tile<float, L, MODE, +1, false>(lds, tw, op);
#pragma unroll
        for (int k = 0; k < FPT; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < 2 * CELLS) fl[idx] = fv[k];
        }
        __syncthreads();
        for (int q = w; q < 2 * NCH; q += NWV) {   // (field, 32-cell chunk), the same for the whole wave
            const int f = q >= NCH ? 1 : 0;
            const int x0 = (q - f * NCH) * 32 + 8 * h;
            const float *mp = maps + (f * 16 + r) * P + x0;
            const float *fp = fl + f * CELLS + x0;
            float a[8], b[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                b[e] = hm ? mp[e] : 0.f;
                a[e] = fp[e] * b[e];
            }
            floatx4_t &acc = f == 0 ? acc0 : acc1;
            if constexpr (PREC == CONKER_MM_F32) {   // float32 products: four cells per instruction
#pragma unroll
                for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], acc, 0, 0, 0);
            } else {
                mma16_split3(acc, a, b);
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {   // float64 after every tile (at most 2 NCH / NWV chunks of 32 cells)
            accd[0][v] += (double)acc0[v];
            accd[1][v] += (double)acc1[v];
        }
        acc0 = floatx4_t{0};
        acc1 = floatx4_t{0};
    }
    __syncthreads();
    double *red = reinterpret_cast<double *>(maps);
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[((w * 2 + f) * 4 + v) * 64 + lane] = accd[f][v];
    __syncthreads();
    for (int f = 0; f < 2; ++f) {
        double *out = partial + ((size_t)(job * 2 + f) * gridDim.x + blockIdx.x) * 1024;
        for (int e = threadIdx.x; e < 1024; e += NT) {   // element (i, j): lane j + 16 (i / 4), register i % 4
            const int i = e >> 5, j = e & 31;
            double sum = 0.0;
            if (i < 16 && j < 16) {
                const int l = j + 16 * (i >> 2), v = i & 3;
#pragma unroll
                for (int q = 0; q < NWV; ++q) sum += red[((q * 2 + f) * 4 + v) * 64 + l];
            }
            out[e] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <typename T, int L>
int tc_of_mode(int mode) {
    switch (mode) {
        case TM_J: return Shape<T, L, TM_J>::TC;
        case TM_C: return Shape<T, L, TM_C>::TC;
        default: return Shape<T, L, TM_W>::TC;
    }
}

template <typename T>
int tc_of(int L, int mode) {
    switch (L) {
        case 96: return tc_of_mode<T, 96>(mode);
        case 192: return tc_of_mode<T, 192>(mode);
        case 384: return tc_of_mode<T, 384>(mode);
        case 32: return tc_of_mode<T, 32>(mode);
        case 64: return tc_of_mode<T, 64>(mode);
        case 128: return tc_of_mode<T, 128>(mode);
        case 256: return tc_of_mode<T, 256>(mode);
        case 512: return tc_of_mode<T, 512>(mode);
        default: return tc_of_mode<T, 1024>(mode);
    }
}

int env_flag(const char *name, int dflt) {
    const char *e = std::getenv(name);
    return e ? (e[0] == '0' ? 0 : 1) : dflt;
}

// Column tiles of the x- and y-axis passes: the context's setting (1 narrow,
// 2 wide), else CONKER_X_WIDE / CONKER_Y_WIDE, else wide (256-byte runs).  A
// wide tile needs at least as many z columns as it holds.
template <typename T>
int col_mode_for(const conker_ctx *ctx, const Dims &d, int axis) {
    static const int x_wide = env_flag("CONKER_X_WIDE", 1);
    static const int y_wide = env_flag("CONKER_Y_WIDE", 1);
    const int t = axis == AX_X ? ctx->tune.x_tile : ctx->tune.y_tile;
    const bool wide = t ? t == 2 : (axis == AX_X ? x_wide : y_wide) != 0;
    const int L = axis == AX_X ? d.nx : d.ny;
    return (wide && d.nz >= tc_of<T>(L, TM_W)) ? (int)TM_W : (int)TM_C;
}

// Whether the float32 passes of length L take the other radix schedule: the
// context's radix setting (1 the usual schedules, 2 the other one where a
// length has it), else CONKER_RADIX16=1, else the usual ones.
bool radix_alt(const conker_ctx *ctx, int L) {
    static const int env = env_flag("CONKER_RADIX16", 0);
    const int r = ctx->tune.radix;
    const bool want = r ? r == 2 : env != 0;
    return want && (L == 64 || L == 128 || L == 256 || L == 1024);
}

template <typename T, int MODE, int DIR, class Op>
int launch_len_mode(conker_ctx *ctx, int L, int axis, const Dims &d, dim3 gy, Op op) {
    auto go = [&](auto Lc) -> int {
        constexpr int LL = decltype(Lc)::value;
        // the other schedule where the length has one (float only), else the usual one
        constexpr int MM = ((MODE & TM_ALT) && PlanAlt<LL>::has && std::is_same<T, float>::value) ? MODE
                                                                                                  : (MODE & TM_BASE);
        using SH = Shape<T, LL, MM>;
        long tiles;
        if (axis == AX_Z) tiles = (long)d.nx * d.ny / SH::TC;
        else if (axis == AX_Y) tiles = (long)d.nx * d.nz / SH::TC;
        else tiles = (long)d.ny * d.nz / SH::TC;
        dim3 grid((unsigned)(tiles * gy.z), gy.y, 1);
        int items = 0;
        if constexpr (has_persist<Op>::value) {
            if (op.persist && gy.z == 1) {   // one workgroup per CU loops over tiles x batches
                items = (int)(tiles * gy.y);
                grid = dim3((unsigned)std::min<long>(items, cu_count(ctx)), 1, 1);
            }
        }
        hipLaunchKernelGGL((k_fft<T, LL, MM, DIR, Op>), grid, dim3(SH::NT), 0, ctx->stream, op, items, (int)tiles);
        CK_LAUNCH(ctx);
        return CONKER_OK;
    };
    switch (L) {
        case 32: return go(std::integral_constant<int, 32>());
        case 64: return go(std::integral_constant<int, 64>());
        case 96: return go(std::integral_constant<int, 96>());
        case 128: return go(std::integral_constant<int, 128>());
        case 192: return go(std::integral_constant<int, 192>());
        case 256: return go(std::integral_constant<int, 256>());
        case 384: return go(std::integral_constant<int, 384>());
        case 512: return go(std::integral_constant<int, 512>());
        case 1024: return go(std::integral_constant<int, 1024>());
        default: return fail(ctx, CONKER_EUNSUPPORTED, "FFT length %d", L);
    }
}

template <typename T, int DIR, class Op>
int launch_len(conker_ctx *ctx, int kind, int mode, int L, int axis, const Dims &d, dim3 gy, Op op) {
    ProfScope ps(ctx, kind);
    if (std::is_same<T, float>::value && radix_alt(ctx, L)) {
        if (mode == TM_J) return launch_len_mode<T, TM_J | TM_ALT, DIR>(ctx, L, axis, d, gy, op);
        if (mode == TM_C) return launch_len_mode<T, TM_C | TM_ALT, DIR>(ctx, L, axis, d, gy, op);
        return launch_len_mode<T, TM_W | TM_ALT, DIR>(ctx, L, axis, d, gy, op);
    }
    if (mode == TM_J) return launch_len_mode<T, TM_J, DIR>(ctx, L, axis, d, gy, op);
    if (mode == TM_C) return launch_len_mode<T, TM_C, DIR>(ctx, L, axis, d, gy, op);
    return launch_len_mode<T, TM_W, DIR>(ctx, L, axis, d, gy, op);
}

// Sums of squares of a and b, then the pair's scale into the context's PackScale.
template <typename T>
int pack_scale_t(conker_ctx *ctx, size_t n, const T *a, const T *b) {
    constexpr int PV = 16 / (int)sizeof(T);
    const bool vec = (((uintptr_t)a | (uintptr_t)b) & 15) == 0;
    const size_t units = vec ? n / PV : n;
    const int G = (int)std::max<size_t>(1, std::min<size_t>({(size_t)SCAL_MAX_PART, (size_t)4 * cu_count(ctx),
                                                            (units + PS_T - 1) / PS_T}));
    double *part = (double *)((char *)ctx->scal.p + SCAL_PART_OFF);
    ProfScope ps(ctx, PK_PACK_SCALE);
    if (vec)
        hipLaunchKernelGGL((k_pack_sums<T, PV>), dim3(G), dim3(PS_T), 0, ctx->stream, a, b, n, part);
    else
        hipLaunchKernelGGL((k_pack_sums<T, 1>), dim3(G), dim3(PS_T), 0, ctx->stream, a, b, n, part);
    CK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_pack_scale, dim3(1), dim3(PSR_T), 0, ctx->stream, (const double *)part, G,
                       (PackScale *)ctx->scal.p);
    CK_LAUNCH(ctx);
    return CONKER_OK;
}

template <typename T>
int forward_pair_t(conker_ctx *ctx, const conker_grid *g, const void *a, const void *b, void *spec,
                   const Support *sup) {
    using C = cplx<T>;
    const bool f64 = std::is_same<T, double>::value;
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, f64, &twz));
    CK_OK(twiddles(ctx, d.ny, f64, &twy));
    CK_OK(twiddles(ctx, d.nx, f64, &twx));
    const size_t nc = ncells(g);
    // with the fields' support: the z pass writes carrying lines, the y pass
    // reads them in carrying slabs only, the x pass reads carrying slabs
    const unsigned char *mask = sup ? sup->mask : nullptr;
    const int *xcount = sup ? sup->xcount : nullptr;
    if (b) {
        if (sup && sup->sums) {   // sums of squares taken with the support: only their reduction
            ProfScope ps(ctx, PK_PACK_SCALE_REDUCE);
            hipLaunchKernelGGL(k_pack_scale, dim3(1), dim3(PSR_T), 0, ctx->stream, sup->sums, sup->sums_n,
                               (PackScale *)ctx->scal.p);
            CK_LAUNCH(ctx);
        } else {
            CK_OK(pack_scale_t<T>(ctx, nc, (const T *)a, (const T *)b));
        }
    }
    if (b) {
        OpPack<T, true> pz{twz, d, (const T *)a, (const T *)b, (C *)spec, {}, mask, 0, pack_scale_dev(ctx), (T)1};
        CK_OK((launch_len<T, -1>(ctx, PK_FFT_FWD_Z, TM_J, d.nz, AX_Z, d, dim3(1, 1), pz)));
    } else {
        OpPack<T, false> pz{twz, d, (const T *)a, nullptr, (C *)spec, {}, mask, 0, nullptr, (T)1};
        CK_OK((launch_len<T, -1>(ctx, PK_FFT_FWD_Z, TM_J, d.nz, AX_Z, d, dim3(1, 1), pz)));
    }
    OpInplace<T, true> py{twy, d, AX_Y, (C *)spec, nc, {}, nullptr, nullptr, xcount, mask, nullptr};
    CK_OK((launch_len<T, -1>(ctx, PK_FFT_FWD_Y, col_mode_for<T>(ctx, d, AX_Y), d.ny, AX_Y, d, dim3(1, 1), py)));
    OpInplace<T, true> px{twx, d, AX_X, (C *)spec, nc, {}, nullptr, nullptr, nullptr, nullptr, xcount};
    CK_OK((launch_len<T, -1>(ctx, PK_FFT_FWD_X, col_mode_for<T>(ctx, d, AX_X), d.nx, AX_X, d, dim3(1, 1), px)));
    return CONKER_OK;
}

template <typename T>
int inverse_batch_t(conker_ctx *ctx, const conker_grid *g, const void *spec, const void *kspec, int m0,
                    int nb, void *tspec, void *maps_a, void *maps_b, const Support *sup, int pair_ns,
                    bool sup_maps) {
    const int pair = pair_ns > 0 ? 1 : 0;
    const bool use_sup = sup && (!maps_a || sup_maps);
    const int *xcount = use_sup ? sup->xcount : nullptr;
    const unsigned char *mask = use_sup ? sup->mask : nullptr;
    using C = cplx<T>;
    const bool f64 = std::is_same<T, double>::value;
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, f64, &twz));
    CK_OK(twiddles(ctx, d.ny, f64, &twy));
    CK_OK(twiddles(ctx, d.nx, f64, &twx));
    const size_t nc = ncells(g);
    const size_t kel = (size_t)(d.nx / 2 + 1) * (d.ny / 2 + 1) * (d.nz / 2 + 1);
    static const int loop = [] {
        const char *e = std::getenv("CONKER_XMUL_LOOP");
        return (e && e[0] == '1') ? 1 : 0;
    }();
    const int xm = col_mode_for<T>(ctx, d, AX_X);
    static const int staged = [] {
        const char *e = std::getenv("CONKER_XMUL_STAGED");
        return (e && e[0] == '0') ? 0 : 1;
    }();
    const int tiles = (int)((long)d.ny * d.nz / tc_of<T>(d.nx, xm));
    const dim3 gxm(1, 1, loop ? 1u : (unsigned)nb);
    static const int resident_env = env_flag("CONKER_XMUL_RESIDENT", 1);
    const int resident = ctx->tune.x_resident ? ctx->tune.x_resident >= 2 : resident_env;
    // two exchange buffers pay where most rows are skipped (the pass is bound by
    // its arithmetic and barriers); with every row stored, one buffer measures faster
    const bool one_buffer = ctx->tune.x_resident == 3 || (ctx->tune.x_resident == 0 && !xcount);
    static const bool persist_y = env_flag("CONKER_Y_PERSIST", 1) != 0;
    bool done = false;
    if (resident) {
        auto go = [&](auto Lc) -> int {
            constexpr int LL = decltype(Lc)::value;
            auto run = [&](auto kern) {
                using SH = Shape<T, LL, TM_R>;
                ProfScope ps(ctx, PK_FFT_INV_X_MUL);
                const unsigned nt = (unsigned)((long)d.ny * d.nz / SH::TC);
                hipLaunchKernelGGL(kern, dim3(nt), dim3(SH::NT), 0, ctx->stream, (const C *)spec, (const T *)kspec,
                                   (C *)tspec, (const C *)twx, d, nc, kel, m0, nb, xcount, pair_ns);
            };
            if (d.nz % Shape<T, LL, TM_R>::TC) return CONKER_OK;
            if (pair) {   // one exchange buffer (the second kernel row takes the room of the other)
                if constexpr (resident_fits<T, LL, true>()) {
                    run(k_xmul_resident<T, LL, false, true>);
                    CK_LAUNCH(ctx);
                    done = true;
                }
            } else if constexpr (resident_fits<T, LL>()) {
                if (one_buffer) run(k_xmul_resident<T, LL, false, false>);
                else run(k_xmul_resident<T, LL, true, false>);
                CK_LAUNCH(ctx);
                done = true;
            }
            return CONKER_OK;
        };
        int st = CONKER_OK;
        switch (d.nx) {
            case 96: st = go(std::integral_constant<int, 96>()); break;
            case 192: st = go(std::integral_constant<int, 192>()); break;
            case 384: st = go(std::integral_constant<int, 384>()); break;
            case 32: st = go(std::integral_constant<int, 32>()); break;
            case 64: st = go(std::integral_constant<int, 64>()); break;
            case 128: st = go(std::integral_constant<int, 128>()); break;
            case 256: st = go(std::integral_constant<int, 256>()); break;
            case 512: st = go(std::integral_constant<int, 512>()); break;
            case 1024: st = go(std::integral_constant<int, 1024>()); break;
            default: break;
        }
        CK_OK(st);
    }
    if (done) {
    } else if (staged) {
        OpMulK<T, true> px{twx, d, (const C *)spec, (const T *)kspec, (C *)tspec, nc, kel, m0, nb, tiles, loop,
                           {}, 0, 0, nullptr, nullptr, nullptr, pair, pair_ns, nullptr};
        CK_OK((launch_len<T, +1>(ctx, PK_FFT_INV_X_MUL, xm, d.nx, AX_X, d, gxm, px)));
    } else {
        OpMulK<T, false> px{twx, d, (const C *)spec, (const T *)kspec, (C *)tspec, nc, kel, m0, nb, tiles, loop,
                            {}, 0, 0, nullptr, nullptr, nullptr, pair, pair_ns, nullptr};
        CK_OK((launch_len<T, +1>(ctx, PK_FFT_INV_X_MUL, xm, d.nx, AX_X, d, gxm, px)));
    }
    OpInplace<T> py{twy, d, AX_Y, (C *)tspec, nc, {}, nullptr, mask, xcount};
    py.persist = persist_y && xcount != nullptr;   // pays where many slabs are skipped
    CK_OK((launch_len<T, +1>(ctx, PK_FFT_INV_Y, col_mode_for<T>(ctx, d, AX_Y), d.ny, AX_Y, d,
                                 dim3(1, (unsigned)nb), py)));
    if (!maps_a) return CONKER_OK;   // x and y passes only
    OpUnpack<T> pz{twz, d, (const C *)tspec, (T *)maps_a, (T *)maps_b, nc, m0, {}, nullptr, pair, pair_ns, mask, 0,
                   (maps_b && !pair) ? pack_scale_dev(ctx) : nullptr, (T)1};
    CK_OK((launch_len<T, +1>(ctx, PK_FFT_INV_Z, TM_J, d.nz, AX_Z, d, dim3(1, (unsigned)nb), pz)));
    return CONKER_OK;
}

template <typename T, int P>
int zinv_diag_t(conker_ctx *ctx, const conker_grid *g, const void *tspec, int nb, const void *fa, const void *fb,
                int blocks, void *part, const int *list, const int *count) {
    using C = cplx<T>;
    const bool f64 = std::is_same<T, double>::value;
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz;
    CK_OK(twiddles(ctx, d.nz, f64, &twz));
    const size_t nc = ncells(g);
    auto go = [&](auto Lc) -> int {
        constexpr int LL = decltype(Lc)::value;
        using SH = Shape<T, LL, TM_J>;
        const int tiles = (int)((long)d.nx * d.ny / SH::TC);
        if (blocks > tiles) return fail(ctx, CONKER_EINVAL, "more partial rows than z tiles");
        ProfScope ps(ctx, PK_DIAG_Z);
        hipLaunchKernelGGL((k_zinv_diag<T, LL, P>), dim3((unsigned)blocks, (unsigned)nb), dim3(SH::NT), 0,
                           ctx->stream, (const C *)tspec, (const T *)fa, (const T *)fb, (const C *)twz, d, nc,
                           tiles, (double *)part, list, count);
        CK_LAUNCH(ctx);
        return CONKER_OK;
    };
    switch (d.nz) {
        case 32: return go(std::integral_constant<int, 32>());
        case 64: return go(std::integral_constant<int, 64>());
        case 96: return go(std::integral_constant<int, 96>());
        case 128: return go(std::integral_constant<int, 128>());
        case 192: return go(std::integral_constant<int, 192>());
        case 256: return go(std::integral_constant<int, 256>());
        case 384: return go(std::integral_constant<int, 384>());
        case 512: return go(std::integral_constant<int, 512>());
        case 1024: return go(std::integral_constant<int, 1024>());
        default: return fail(ctx, CONKER_EUNSUPPORTED, "FFT length %d", d.nz);
    }
}

template <typename T>
int zinv_diag_p(conker_ctx *ctx, const conker_grid *g, const void *tspec, int nb, const void *fa, const void *fb,
                int pmax, int blocks, void *part, const int *list, const int *count) {
    switch (pmax) {
        case 1: return zinv_diag_t<T, 1>(ctx, g, tspec, nb, fa, fb, blocks, part, list, count);
        case 2: return zinv_diag_t<T, 2>(ctx, g, tspec, nb, fa, fb, blocks, part, list, count);
        case 3: return zinv_diag_t<T, 3>(ctx, g, tspec, nb, fa, fb, blocks, part, list, count);
        case 4: return zinv_diag_t<T, 4>(ctx, g, tspec, nb, fa, fb, blocks, part, list, count);
        default: return fail(ctx, CONKER_EINVAL, "power %d outside 1..4", pmax);
    }
}

// Resident first inverse pass over M jobs of a size class (grid y = job).
int xmul_resident_jobs(conker_ctx *ctx, const Dims &d, int M, const float2 *spec, const float *kspec,
                       float2 *tspec, const void *twx, size_t nc, size_t kel, int m0, int nb, bool *done) {
    *done = false;
    auto go = [&](auto Lc) -> int {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (resident_fits<float, LL>()) {
            using SH = Shape<float, LL, TM_R>;
            if (d.nz % SH::TC) return CONKER_OK;
            ProfScope ps(ctx, PK_FFT_INV_X_MUL);
            const dim3 grid((unsigned)((long)d.ny * d.nz / SH::TC), (unsigned)M);
            hipLaunchKernelGGL((k_xmul_resident<float, LL, false, false>), grid, dim3(SH::NT), 0, ctx->stream,
                               spec, kspec, tspec, (const float2 *)twx, d, nc, kel, m0, nb, (const int *)nullptr, 0);
            CK_LAUNCH(ctx);
            *done = true;
        }
        return CONKER_OK;
    };
    switch (d.nx) {
        case 96: return go(std::integral_constant<int, 96>());
        case 192: return go(std::integral_constant<int, 192>());
        case 384: return go(std::integral_constant<int, 384>());
        case 32: return go(std::integral_constant<int, 32>());
        case 64: return go(std::integral_constant<int, 64>());
        case 128: return go(std::integral_constant<int, 128>());
        case 256: return go(std::integral_constant<int, 256>());
        case 512: return go(std::integral_constant<int, 512>());
        case 1024: return go(std::integral_constant<int, 1024>());
        default: return CONKER_OK;
    }
}

}  // namespace

namespace conker {

int fft_inverse_z_diag(conker_ctx *ctx, const conker_grid *g, bool f64, const void *tspec, int nb,
                       const void *fa, const void *fb, int pmax, int blocks, void *part,
                       const Support *sup) {
    const int *list = sup ? sup->list : nullptr, *count = sup ? sup->count : nullptr;
    return f64 ? zinv_diag_p<double>(ctx, g, tspec, nb, fa, fb, pmax, blocks, part, list, count)
               : zinv_diag_p<float>(ctx, g, tspec, nb, fa, fb, pmax, blocks, part, list, count);
}

int fft_z_tiles(const conker_grid *g, bool f64) {
    const int tc = f64 ? tc_of<double>(g->dims[2], TM_J) : tc_of<float>(g->dims[2], TM_J);
    return (int)((long)g->dims[0] * g->dims[1] / tc);
}

int fft_forward_pair(conker_ctx *ctx, const conker_grid *g, bool f64, const void *a, const void *b,
                     void *spec, const Support *sup) {
    return f64 ? forward_pair_t<double>(ctx, g, a, b, spec, sup) : forward_pair_t<float>(ctx, g, a, b, spec, sup);
}

int fft_inverse_batch(conker_ctx *ctx, const conker_grid *g, bool f64, const void *spec,
                      const void *kspec, int m0, int nb, void *tspec, void *maps_a, void *maps_b,
                      const Support *sup, int pair_ns, bool sup_maps) {
    return f64 ? inverse_batch_t<double>(ctx, g, spec, kspec, m0, nb, tspec, maps_a, maps_b, sup, pair_ns, sup_maps)
               : inverse_batch_t<float>(ctx, g, spec, kspec, m0, nb, tspec, maps_a, maps_b, sup, pair_ns, sup_maps);
}

bool fft_jobs_ok(const conker_grid *g) {
    const Dims d{g->dims[0], g->dims[1], g->dims[2]};
    bool ok = false;
    auto go = [&](auto Lc) {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (resident_fits<float, LL>()) ok = d.nz % Shape<float, LL, TM_R>::TC == 0;
    };
    switch (d.nx) {
        case 96: go(std::integral_constant<int, 96>()); break;
        case 192: go(std::integral_constant<int, 192>()); break;
        case 384: go(std::integral_constant<int, 384>()); break;
        case 32: go(std::integral_constant<int, 32>()); break;
        case 64: go(std::integral_constant<int, 64>()); break;
        case 128: go(std::integral_constant<int, 128>()); break;
        case 256: go(std::integral_constant<int, 256>()); break;
        case 512: go(std::integral_constant<int, 512>()); break;
        case 1024: go(std::integral_constant<int, 1024>()); break;
        default: break;
    }
    return ok;
}

int fft_forward_jobs(conker_ctx *ctx, const conker_grid *g, int M, const ClassJob *tab, void *spec,
                     PackScale *scales, const double *part, int sums_G) {
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, false, &twz));
    CK_OK(twiddles(ctx, d.ny, false, &twy));
    CK_OK(twiddles(ctx, d.nx, false, &twx));
    const size_t nc = ncells(g);
    {
        ProfScope ps(ctx, PK_PACK_SCALE_REDUCE);
        hipLaunchKernelGGL(k_pack_scale, dim3((unsigned)M), dim3(PSR_T), 0, ctx->stream, part, sums_G, scales);
        CK_LAUNCH(ctx);
    }
    OpPackJobs pz{twz, d, tab, (float2 *)spec, nc, scales, {}, nullptr, nullptr, nullptr, 1.f};
    CK_OK((launch_len<float, -1>(ctx, PK_FFT_FWD_Z, TM_J, d.nz, AX_Z, d, dim3(1, (unsigned)M), pz)));
    OpInplace<float> py{twy, d, AX_Y, (float2 *)spec, nc, {}, nullptr, nullptr, nullptr};
    CK_OK((launch_len<float, -1>(ctx, PK_FFT_FWD_Y, col_mode_for<float>(ctx, d, AX_Y), d.ny, AX_Y, d,
                                 dim3(1, (unsigned)M), py)));
    OpInplace<float> px{twx, d, AX_X, (float2 *)spec, nc, {}, nullptr, nullptr, nullptr};
    CK_OK((launch_len<float, -1>(ctx, PK_FFT_FWD_X, col_mode_for<float>(ctx, d, AX_X), d.nx, AX_X, d,
                                 dim3(1, (unsigned)M), px)));
    return CONKER_OK;
}

bool fft_mm3_jobs_ok(const conker_grid *g, int ns) {
    if (ns < 1 || ns > 16) return false;
    bool ok = false;
    auto go = [&](auto Lc) {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (ZMM<LL>::OK) ok = ((long)g->dims[0] * g->dims[1]) % ZMM<LL>::LPT == 0;
    };
    switch (g->dims[2]) {
        case 32: go(std::integral_constant<int, 32>()); break;
        case 64: go(std::integral_constant<int, 64>()); break;
        case 96: go(std::integral_constant<int, 96>()); break;
        case 128: go(std::integral_constant<int, 128>()); break;
        case 192: go(std::integral_constant<int, 192>()); break;
        case 256: go(std::integral_constant<int, 256>()); break;
        default: break;
    }
    return ok && fft_jobs_ok(g);
}

int fft_mm3_jobs_blocks(conker_ctx *ctx, int M) { return std::max(1, 4 * cu_count(ctx) / M); }   // four workgroups per CU

int fft_inverse_mm3_jobs(conker_ctx *ctx, const conker_grid *g, int M, const ClassJob *tab, const void *kspec, int ns,
                         const void *spec, void *tspec, const PackScale *scales, double *partial, conker_mmprec prec) {
    if (prec != CONKER_MM_SPLIT_BF16 && prec != CONKER_MM_F32)
        return fail(ctx, CONKER_EINVAL, "size class: fused summation in split bfloat16 or float32 only");
    if (!fft_mm3_jobs_ok(g, ns)) return fail(ctx, CONKER_EUNSUPPORTED, "size class: no fused summation for this grid");
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, false, &twz));
    CK_OK(twiddles(ctx, d.ny, false, &twy));
    CK_OK(twiddles(ctx, d.nx, false, &twx));
    const size_t nc = ncells(g);
    const size_t kel = (size_t)(d.nx / 2 + 1) * (d.ny / 2 + 1) * (d.nz / 2 + 1);
    bool done = false;
    CK_OK(xmul_resident_jobs(ctx, d, M, (const float2 *)spec, (const float *)kspec, (float2 *)tspec, twx, nc, kel, 0,
                             ns, &done));
    if (!done) return fail(ctx, CONKER_EUNSUPPORTED, "size class: no resident first inverse pass for this grid");
    OpInplace<float> py{twy, d, AX_Y, (float2 *)tspec, nc, {}, nullptr, nullptr, nullptr};
    CK_OK((launch_len<float, +1>(ctx, PK_FFT_INV_Y, col_mode_for<float>(ctx, d, AX_Y), d.ny, AX_Y, d,
                                 dim3(1, (unsigned)(M * ns)), py)));
    const int G = fft_mm3_jobs_blocks(ctx, M);
    ProfScope ps(ctx, PK_FUSED_ZC);
    const bool alt = radix_alt(ctx, d.nz);
    auto go = [&](auto Lc) {
        constexpr int LL = decltype(Lc)::value;
        if constexpr (ZMM<LL>::OK) {
            auto run = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3((unsigned)G, (unsigned)M), dim3(256), 0, ctx->stream,
                                   (const float2 *)tspec, tab, scales, (const float2 *)twz, d, nc, ns, partial);
            };
            const bool f32 = prec == CONKER_MM_F32;
            if (alt && PlanAlt<LL>::has) {
                if (f32) run(k_zinv_mm3_jobs<LL, TM_J | TM_ALT, CONKER_MM_F32>);
                else run(k_zinv_mm3_jobs<LL, TM_J | TM_ALT, CONKER_MM_SPLIT_BF16>);
            } else {
                if (f32) run(k_zinv_mm3_jobs<LL, TM_J, CONKER_MM_F32>);
                else run(k_zinv_mm3_jobs<LL, TM_J, CONKER_MM_SPLIT_BF16>);
            }
        }
    };
    switch (d.nz) {
        case 32: go(std::integral_constant<int, 32>()); break;
        case 64: go(std::integral_constant<int, 64>()); break;
        case 96: go(std::integral_constant<int, 96>()); break;
        case 128: go(std::integral_constant<int, 128>()); break;
        case 192: go(std::integral_constant<int, 192>()); break;
        case 256: go(std::integral_constant<int, 256>()); break;
        default: break;
    }
    CK_LAUNCH(ctx);
    return CONKER_OK;
}

int fft_inverse_jobs(conker_ctx *ctx, const conker_grid *g, int M, const ClassJob *tab, const void *kspec, int m0,
                     int nb, const void *spec, void *tspec, const PackScale *scales) {
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, false, &twz));
    CK_OK(twiddles(ctx, d.ny, false, &twy));
    CK_OK(twiddles(ctx, d.nx, false, &twx));
    const size_t nc = ncells(g);
    const size_t kel = (size_t)(d.nx / 2 + 1) * (d.ny / 2 + 1) * (d.nz / 2 + 1);
    bool done = false;
    CK_OK(xmul_resident_jobs(ctx, d, M, (const float2 *)spec, (const float *)kspec, (float2 *)tspec, twx, nc, kel,
                             m0, nb, &done));
    if (!done) return fail(ctx, CONKER_EUNSUPPORTED, "size class: no resident first inverse pass for this grid");
    OpInplace<float> py{twy, d, AX_Y, (float2 *)tspec, nc, {}, nullptr, nullptr, nullptr};
    CK_OK((launch_len<float, +1>(ctx, PK_FFT_INV_Y, col_mode_for<float>(ctx, d, AX_Y), d.ny, AX_Y, d,
                                 dim3(1, (unsigned)(M * nb)), py)));
    OpUnpackJobs pz{twz, d, (const float2 *)tspec, tab, scales, nc, m0, nb, {}, nullptr, nullptr, nullptr, 1.f};
    CK_OK((launch_len<float, +1>(ctx, PK_FFT_INV_Z, TM_J, d.nz, AX_Z, d, dim3(1, (unsigned)(M * nb)), pz)));
    return CONKER_OK;
}

int fft_shell_pair(conker_ctx *ctx, const conker_grid *g, double lo_a, double hi_a, double lo_b,
                   double hi_b, void *work, void *kspec, bool out_f64, int ma, int mb) {
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, true, &twz));
    CK_OK(twiddles(ctx, d.ny, true, &twy));
    CK_OK(twiddles(ctx, d.nx, true, &twx));
    const size_t nc = ncells(g);
    const size_t kel = (size_t)(d.nx / 2 + 1) * (d.ny / 2 + 1) * (d.nz / 2 + 1);
    OpShellFill pz{twz, d, lo_a, hi_a, lo_b, hi_b, (double2 *)work, {}};
    CK_OK((launch_len<double, -1>(ctx, PK_BANK_Z, TM_J, d.nz, AX_Z, d, dim3(1, 1), pz)));
    OpInplace<double> py{twy, d, AX_Y, (double2 *)work, nc, {}, nullptr};
    CK_OK((launch_len<double, -1>(ctx, PK_BANK_Y, TM_C, d.ny, AX_Y, d, dim3(1, 1), py)));
    const double scale = 1.0 / (double)nc;
    if (out_f64) {
        OpExtract<double> px{twx, d, (const double2 *)work, (double *)kspec, kel, ma, mb, scale, {}};
        CK_OK((launch_len<double, -1>(ctx, PK_BANK_X, TM_C, d.nx, AX_X, d, dim3(1, 1), px)));
    } else {
        OpExtract<float> px{twx, d, (const double2 *)work, (float *)kspec, kel, ma, mb, scale, {}};
        CK_OK((launch_len<double, -1>(ctx, PK_BANK_X, TM_C, d.nx, AX_X, d, dim3(1, 1), px)));
    }
    return CONKER_OK;
}

}  // namespace conker
