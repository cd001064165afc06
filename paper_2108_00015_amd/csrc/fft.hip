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
#include <type_traits>

#include "common.h"

using namespace conker;

namespace {

template <typename T>
using cplx = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * (DIR i)
template <int DIR, typename C>
__device__ __forceinline__ C mul_di(C a) {
    if constexpr (DIR > 0) return C{-a.y, a.x};
    else return C{a.y, -a.x};
}

// X_k = sum_r v_r exp(DIR 2 pi i r k / R), in place.
template <int R, int DIR, typename C>
__device__ __forceinline__ void dft(C *v) {
    if constexpr (R == 2) {
        C a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    } else if constexpr (R == 4) {
        C a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
        C a2 = cadd(v[1], v[3]), a3 = mul_di<DIR>(csub(v[1], v[3]));
        v[0] = cadd(a0, a2);
        v[2] = csub(a0, a2);
        v[1] = cadd(a1, a3);
        v[3] = csub(a1, a3);
    } else {
        static_assert(R == 8, "radix");
        using T = decltype(v[0].x);
        C e[4] = {v[0], v[2], v[4], v[6]};
        C o[4] = {v[1], v[3], v[5], v[7]};
        dft<4, DIR>(e);
        dft<4, DIR>(o);
        const T h = (T)0.70710678118654752440;   // 1/sqrt(2)
        const T d = (T)DIR;
        // o_k *= exp(DIR 2 pi i k / 8)
        o[1] = C{(o[1].x - d * o[1].y) * h, (o[1].y + d * o[1].x) * h};
        o[2] = mul_di<DIR>(o[2]);
        o[3] = C{(-o[3].x - d * o[3].y) * h, (d * o[3].x - o[3].y) * h};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
}

// Radix schedule per line length (product of the stage radices).
template <int L>
struct Plan;
template <> struct Plan<32>   { static constexpr int n = 2; static constexpr int r[4] = {8, 4, 1, 1}; };
template <> struct Plan<64>   { static constexpr int n = 2; static constexpr int r[4] = {8, 8, 1, 1}; };
template <> struct Plan<128>  { static constexpr int n = 3; static constexpr int r[4] = {8, 4, 4, 1}; };
template <> struct Plan<256>  { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 4, 1}; };
template <> struct Plan<512>  { static constexpr int n = 3; static constexpr int r[4] = {8, 8, 8, 1}; };
template <> struct Plan<1024> { static constexpr int n = 4; static constexpr int r[4] = {8, 8, 4, 4}; };

template <int L, int S>
constexpr int stage_ns() {   // product of radices before stage S
    int p = 1;
    for (int s = 0; s < S; ++s) p *= Plan<L>::r[s];
    return p;
}

// Tile shapes.  MAPJ: lanes run along a line (z-axis tiles of whole lines);
// MAPC: lanes run across the TC columns of a tile (y and x axes).
template <typename T, int L>
struct Shape {
    static constexpr bool f64 = std::is_same<T, double>::value;
    // columns per tile for strided (y, x) passes: runs of TC complex values
    static constexpr int TC_C = f64 ? (L >= 1024 ? 4 : 8) : (L >= 1024 ? 8 : 16);
    static constexpr int PAD_C = f64 ? 0 : (L >= 1024 ? 0 : 2);
    // lines per tile for contiguous (z) passes
    static constexpr int TC_J = (f64 ? 2048 : 4096) / L;
    static constexpr int PADSH_J = 3;   // one pad element every 8
};

template <bool MAPJ, int L, int TC, int PAD>
__device__ __forceinline__ int lds_addr(int i, int c) {
    if constexpr (MAPJ) return c * (L + (L >> 3)) + i + (i >> 3);
    else return i * (TC + PAD) + c;
}

// Butterfly q of this thread -> (j = butterfly index within a line, c = column).
// MAPC: the column is fixed per thread (NT is a multiple of TC), j steps by NT/TC.
// MAPJ: lanes run along j; the line index steps by NT/LR (or j by NT when LR > NT).
template <int NT, bool MAPJ, int LR, int TC>
__device__ __forceinline__ void split_q(int q, int &j, int &c) {
    const int t = threadIdx.x;
    if constexpr (MAPJ) {
        if constexpr (NT % LR == 0) { j = t % LR; c = t / LR + q * (NT / LR); }
        else { const int b = t + q * NT; j = b % LR; c = b / LR; }
    } else {
        static_assert(NT % TC == 0, "tile columns must divide the workgroup");
        c = t % TC;
        j = t / TC + q * (NT / TC);
    }
}

template <typename T, int L, int TC, int PAD, bool MAPJ, int DIR, int NT, int S, class Op>
__device__ __forceinline__ void fft_stage(cplx<T> *lds, const cplx<T> *tw, Op &op) {
    using C = cplx<T>;
    constexpr int R = Plan<L>::r[S];
    constexpr int NSV = stage_ns<L, S>();
    constexpr bool FIRST = (S == 0);
    constexpr bool LAST = (S == Plan<L>::n - 1);
    constexpr int LR = L / R;
    constexpr int NB = LR * TC;
    constexpr int PER = (NB + NT - 1) / NT;
    constexpr int TWS = L / (NSV * R);
    C v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = threadIdx.x + q * NT;
        if (NB % NT == 0 || b < NB) {
            int j, c;
            split_q<NT, MAPJ, LR, TC>(q, j, c);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = j + r * LR;
                if constexpr (FIRST) v[q][r] = op.load(i, c);
                else v[q][r] = lds[lds_addr<MAPJ, L, TC, PAD>(i, c)];
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
    if constexpr (!FIRST) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int b = threadIdx.x + q * NT;
        if (NB % NT == 0 || b < NB) {
            int j, c;
            split_q<NT, MAPJ, LR, TC>(q, j, c);
            const int k = j & (NSV - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int o = base + r * NSV;
                if constexpr (LAST) op.store(o, c, v[q][r]);
                else lds[lds_addr<MAPJ, L, TC, PAD>(o, c)] = v[q][r];
            }
        }
    }
    if constexpr (!LAST) __syncthreads();
}

template <typename T, int L, int TC, int PAD, bool MAPJ, int DIR, int NT, class Op>
__device__ __forceinline__ void fft_line_tile(cplx<T> *lds, const cplx<T> *tw, Op &op) {
    fft_stage<T, L, TC, PAD, MAPJ, DIR, NT, 0>(lds, tw, op);
    if constexpr (Plan<L>::n > 1) fft_stage<T, L, TC, PAD, MAPJ, DIR, NT, 1>(lds, tw, op);
    if constexpr (Plan<L>::n > 2) fft_stage<T, L, TC, PAD, MAPJ, DIR, NT, 2>(lds, tw, op);
    if constexpr (Plan<L>::n > 3) fft_stage<T, L, TC, PAD, MAPJ, DIR, NT, 3>(lds, tw, op);
}

// Threads per workgroup: 512 when a tile holds at least 512 first-stage
// butterflies (keeps each thread to one or two radix-8 butterflies per stage,
// so that the strided passes fit in ~128 registers), else 256.
template <typename T, int L, bool MAPJ>
constexpr int threads_of() {
    using S = Shape<T, L>;
    constexpr int tc = MAPJ ? S::TC_J : S::TC_C;
    return (!MAPJ && (L / 8) * tc >= 512) ? 512 : 256;
}

template <typename T, int L, bool MAPJ>
constexpr int lds_elems() {
    using S = Shape<T, L>;
    if constexpr (MAPJ) return S::TC_J * (L + (L >> 3));
    else return L * (S::TC_C + S::PAD_C);
}

// One launch = one pass over one axis.  Op::iters() line transforms are run
// per tile (more than one when a tile is reused across several radii).
template <typename T, int L, bool MAPJ, int DIR, class Op>
__global__ __launch_bounds__((threads_of<T, L, MAPJ>()), (threads_of<T, L, MAPJ>() == 512 ? 4 : 2)) void k_fft(
    Op op) {
    using C = cplx<T>;
    using S = Shape<T, L>;
    constexpr int NT = threads_of<T, L, MAPJ>();
    constexpr int TC = MAPJ ? S::TC_J : S::TC_C;
    constexpr int PAD = MAPJ ? 0 : S::PAD_C;
    __shared__ C lds[lds_elems<T, L, MAPJ>()];
    __shared__ C tw[L];
    const C *twg = reinterpret_cast<const C *>(op.tw);
    for (int t = threadIdx.x; t < L; t += NT) tw[t] = twg[t];
    op.begin(TC);
    __syncthreads();
    const int it_n = op.iters();
    for (int it = 0; it < it_n; ++it) {
        op.set_iter(it);
        fft_line_tile<T, L, TC, PAD, MAPJ, DIR, NT>(lds, tw, op);
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

__device__ __forceinline__ size_t at(const Tile &g, int i, int c) {
    return g.base + (size_t)i * g.si + (size_t)c * g.sc;
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------
template <typename T>
struct OpPack {   // z pass, forward: (a + i b) -> spec
    using C = cplx<T>;
    const void *tw;
    Dims d;
    const T *a;
    const T *b;
    C *out;
    Tile g;
    __device__ void begin(int TC) { g = make_tile(AX_Z, d, blockIdx.x, TC); }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const {
        const size_t k = at(g, i, c);
        return C{a[k], b ? b[k] : (T)0};
    }
    __device__ void store(int i, int c, C v) const { out[at(g, i, c)] = v; }
};

template <typename T>
struct OpInplace {   // any axis, in place; blockIdx.y selects a grid of the batch
    using C = cplx<T>;
    const void *tw;
    Dims d;
    int axis;
    C *buf;
    size_t nc;
    Tile g;
    C *p;
    __device__ void begin(int TC) {
        g = make_tile(axis, d, blockIdx.x, TC);
        p = buf + (size_t)blockIdx.y * nc;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const { return p[at(g, i, c)]; }
    __device__ void store(int i, int c, C v) const { p[at(g, i, c)] = v; }
};

// x pass, inverse, for radii m0 .. m0+nb-1: spec * K_m -> tspec[m - m0].
// K_m is stored as its octant [nx/2+1][ny/2+1][nz/2+1]; k and n - k share an entry.
// One radius per workgroup.  Workgroups are dispatched round-robin over the 8
// XCDs; the nb radii of one tile are given ids 8 apart so that they run on the
// same XCD back to back and re-read the tile of `spec` from that XCD's L2.
template <typename T>
struct OpMulK {
    using C = cplx<T>;
    const void *tw;
    Dims d;
    const C *spec;
    const T *kspec;
    C *tspec;
    size_t nc;
    size_t kel;   // octant elements per radius
    int m0, nb, tiles;
    Tile g;
    int m;
    const C *src;   // spec at this tile and this thread's column
    C *dst;
    const T *kcol;  // kspec of radius m at this thread's (ky, kz) column
    int kplane;     // octant elements per kx
    __device__ void begin(int TC) {
        const int w = blockIdx.x;
        int tile;
        if ((tiles & 7) == 0) {
            const int xcd = w & 7, slot = w >> 3;
            tile = (slot / nb) * 8 + xcd;
            m = slot % nb;
        } else {
            tile = w / nb;
            m = w % nb;
        }
        g = make_tile(AX_X, d, tile, TC);
        const int c = threadIdx.x % TC;
        const int ky = g.p0, kz = g.p1 + c;
        const int oy = ky <= d.ny - ky ? ky : d.ny - ky;
        const int oz = kz <= d.nz - kz ? kz : d.nz - kz;
        kplane = (d.ny / 2 + 1) * (d.nz / 2 + 1);
        kcol = kspec + (size_t)(m0 + m) * kel + (size_t)oy * (d.nz / 2 + 1) + oz;
        src = spec + g.base + c;
        dst = tspec + (size_t)m * nc + g.base + c;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int) const {
        const int ox = i <= d.nx - i ? i : d.nx - i;
        const T kv = kcol[(unsigned)(ox * kplane)];
        const C s = src[(size_t)(unsigned)i * (unsigned)g.si];
        return C{s.x * kv, s.y * kv};
    }
    __device__ void store(int i, int, C v) const { dst[(size_t)(unsigned)i * (unsigned)g.si] = v; }
};

// z pass, inverse: tspec[m] -> real parts to maps_a[m0+m], imaginary to maps_b[m0+m].
template <typename T>
struct OpUnpack {
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
    size_t off;
    __device__ void begin(int TC) {
        g = make_tile(AX_Z, d, blockIdx.x, TC);
        src = tspec + (size_t)blockIdx.y * nc;
        off = (size_t)(m0 + blockIdx.y) * nc;
    }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const { return src[at(g, i, c)]; }
    __device__ void store(int i, int c, C v) const {
        const size_t k = off + at(g, i, c);
        ma[k] = v.x;
        if (mb) mb[k] = v.y;
    }
};

// z pass, forward, of two shell indicators generated on the fly:
// real part = [lo_a <= |delta|^2 < hi_a], imaginary part likewise for b,
// with delta the minimum-image offset of the cell from cell (0, 0, 0).
struct OpShellFill {
    using C = double2;
    const void *tw;
    Dims d;
    double lo_a, hi_a, lo_b, hi_b;
    C *out;
    Tile g;
    __device__ void begin(int TC) { g = make_tile(AX_Z, d, blockIdx.x, TC); }
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
    __device__ void store(int i, int c, C v) const { out[at(g, i, c)] = v; }
};

// x pass, forward, of the packed shell pair: keep the octant, scale by 1/N_c.
template <typename K>
struct OpExtract {
    using C = double2;
    const void *tw;
    Dims d;
    const C *buf;
    K *kspec;
    size_t kel;
    int ma, mb;
    double scale;
    Tile g;
    __device__ void begin(int TC) { g = make_tile(AX_X, d, blockIdx.x, TC); }
    __device__ int iters() const { return 1; }
    __device__ void set_iter(int) {}
    __device__ C load(int i, int c) const { return buf[at(g, i, c)]; }
    __device__ void store(int i, int c, C v) const {
        const int ky = g.p0, kz = g.p1 + c, kx = i;
        if (2 * kx > d.nx || 2 * ky > d.ny || 2 * kz > d.nz) return;
        const size_t ko = ((size_t)kx * (d.ny / 2 + 1) + ky) * (d.nz / 2 + 1) + kz;
        kspec[(size_t)ma * kel + ko] = (K)(v.x * scale);
        if (mb >= 0) kspec[(size_t)mb * kel + ko] = (K)(v.y * scale);
    }
};

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <typename T, int L>
constexpr int tc_of(bool mapj) {
    return mapj ? Shape<T, L>::TC_J : Shape<T, L>::TC_C;
}

template <typename T>
int tc_of(int L, bool mapj) {
    switch (L) {
        case 32: return tc_of<T, 32>(mapj);
        case 64: return tc_of<T, 64>(mapj);
        case 128: return tc_of<T, 128>(mapj);
        case 256: return tc_of<T, 256>(mapj);
        case 512: return tc_of<T, 512>(mapj);
        default: return tc_of<T, 1024>(mapj);
    }
}

template <typename T, bool MAPJ, int DIR, class Op>
int launch_len(conker_ctx *ctx, int kind, int L, int axis, const Dims &d, dim3 gy, Op op) {
    ProfScope ps(ctx, kind);
    auto go = [&](auto Lc) -> int {
        constexpr int LL = decltype(Lc)::value;
        const int TC = tc_of<T, LL>(MAPJ);
        long tiles;
        if (axis == AX_Z) tiles = (long)d.nx * d.ny / TC;
        else if (axis == AX_Y) tiles = (long)d.nx * d.nz / TC;
        else tiles = (long)d.ny * d.nz / TC;
        dim3 grid((unsigned)(tiles * gy.z), gy.y, 1);
        hipLaunchKernelGGL((k_fft<T, LL, MAPJ, DIR, Op>), grid, dim3(threads_of<T, LL, MAPJ>()), 0, ctx->stream,
                           op);
        CK_LAUNCH(ctx);
        return CONKER_OK;
    };
    switch (L) {
        case 32: return go(std::integral_constant<int, 32>());
        case 64: return go(std::integral_constant<int, 64>());
        case 128: return go(std::integral_constant<int, 128>());
        case 256: return go(std::integral_constant<int, 256>());
        case 512: return go(std::integral_constant<int, 512>());
        case 1024: return go(std::integral_constant<int, 1024>());
        default: return fail(ctx, CONKER_EUNSUPPORTED, "FFT length %d", L);
    }
}

template <typename T>
int forward_pair_t(conker_ctx *ctx, const conker_grid *g, const void *a, const void *b, void *spec) {
    using C = cplx<T>;
    const bool f64 = std::is_same<T, double>::value;
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, f64, &twz));
    CK_OK(twiddles(ctx, d.ny, f64, &twy));
    CK_OK(twiddles(ctx, d.nx, f64, &twx));
    const size_t nc = ncells(g);
    OpPack<T> pz{twz, d, (const T *)a, (const T *)b, (C *)spec, {}};
    CK_OK((launch_len<T, true, -1>(ctx, PK_FFT_FWD_Z, d.nz, AX_Z, d, dim3(1, 1), pz)));
    OpInplace<T> py{twy, d, AX_Y, (C *)spec, nc, {}, nullptr};
    CK_OK((launch_len<T, false, -1>(ctx, PK_FFT_FWD_Y, d.ny, AX_Y, d, dim3(1, 1), py)));
    OpInplace<T> px{twx, d, AX_X, (C *)spec, nc, {}, nullptr};
    CK_OK((launch_len<T, false, -1>(ctx, PK_FFT_FWD_X, d.nx, AX_X, d, dim3(1, 1), px)));
    return CONKER_OK;
}

template <typename T>
int inverse_batch_t(conker_ctx *ctx, const conker_grid *g, const void *spec, const void *kspec,
                    int m0, int nb, void *tspec, void *maps_a, void *maps_b) {
    using C = cplx<T>;
    const bool f64 = std::is_same<T, double>::value;
    Dims d{g->dims[0], g->dims[1], g->dims[2]};
    const void *twz, *twy, *twx;
    CK_OK(twiddles(ctx, d.nz, f64, &twz));
    CK_OK(twiddles(ctx, d.ny, f64, &twy));
    CK_OK(twiddles(ctx, d.nx, f64, &twx));
    const size_t nc = ncells(g);
    const size_t kel = (size_t)(d.nx / 2 + 1) * (d.ny / 2 + 1) * (d.nz / 2 + 1);
    OpMulK<T> px{twx, d, (const C *)spec, (const T *)kspec, (C *)tspec, nc, kel, m0, nb, 0, {}, 0,
                 nullptr, nullptr, nullptr, 0};
    px.tiles = (int)((long)d.ny * d.nz / tc_of<T>(d.nx, false));
    CK_OK((launch_len<T, false, +1>(ctx, PK_FFT_INV_X_MUL, d.nx, AX_X, d, dim3(1, 1, (unsigned)nb), px)));
    OpInplace<T> py{twy, d, AX_Y, (C *)tspec, nc, {}, nullptr};
    CK_OK((launch_len<T, false, +1>(ctx, PK_FFT_INV_Y, d.ny, AX_Y, d, dim3(1, (unsigned)nb), py)));
    OpUnpack<T> pz{twz, d, (const C *)tspec, (T *)maps_a, (T *)maps_b, nc, m0, {}, nullptr, 0};
    CK_OK((launch_len<T, true, +1>(ctx, PK_FFT_INV_Z, d.nz, AX_Z, d, dim3(1, (unsigned)nb), pz)));
    return CONKER_OK;
}

}  // namespace

namespace conker {

int fft_forward_pair(conker_ctx *ctx, const conker_grid *g, bool f64, const void *a, const void *b,
                     void *spec) {
    return f64 ? forward_pair_t<double>(ctx, g, a, b, spec) : forward_pair_t<float>(ctx, g, a, b, spec);
}

int fft_inverse_batch(conker_ctx *ctx, const conker_grid *g, bool f64, const void *spec,
                      const void *kspec, int m0, int nb, void *tspec, void *maps_a, void *maps_b) {
    return f64 ? inverse_batch_t<double>(ctx, g, spec, kspec, m0, nb, tspec, maps_a, maps_b)
               : inverse_batch_t<float>(ctx, g, spec, kspec, m0, nb, tspec, maps_a, maps_b);
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
    CK_OK((launch_len<double, true, -1>(ctx, PK_BANK_Z, d.nz, AX_Z, d, dim3(1, 1), pz)));
    OpInplace<double> py{twy, d, AX_Y, (double2 *)work, nc, {}, nullptr};
    CK_OK((launch_len<double, false, -1>(ctx, PK_BANK_Y, d.ny, AX_Y, d, dim3(1, 1), py)));
    const double scale = 1.0 / (double)nc;
    if (out_f64) {
        OpExtract<double> px{twx, d, (const double2 *)work, (double *)kspec, kel, ma, mb, scale, {}};
        CK_OK((launch_len<double, false, -1>(ctx, PK_BANK_X, d.nx, AX_X, d, dim3(1, 1), px)));
    } else {
        OpExtract<float> px{twx, d, (const double2 *)work, (float *)kspec, kel, ma, mb, scale, {}};
        CK_OK((launch_len<double, false, -1>(ctx, PK_BANK_X, d.nx, AX_X, d, dim3(1, 1), px)));
    }
    return CONKER_OK;
}

}  // namespace conker
