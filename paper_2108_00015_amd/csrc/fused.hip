// Convolution and summation in one pass for orders n = 2 and 3 (Sec. 2.4 and
// Sec. 2.5, Eqs. countconv, randconv, ksin_delta, ksi2_delta, ksi3), without
// writing the per-radius maps to memory.
//
// After the forward transform and the inverse x and y passes of every radius
// (fft.hip), each z-line of the batch spectra still has to be transformed back
// along z.  Here one workgroup takes one line (x, y) at a time: its eight
// waves inverse-transform the line of every radius m (512 points, three
// radix-8 stages within a wave, exchanging through a per-wave LDS scratch) and
// leave C_m(x, y, z) for all m and z in LDS, field a in the real part and
// field b in the imaginary part.  The line's cells are then contracted on the
// matrix cores:
//   W3[a][b] += sum_z F(z) C_a(z) C_b(z)     (32 x 32 output tile)
//   W2[a]    += sum_z F(z) C_a(z)            (column 31, where C is replaced by 1)
// for both fields, exactly as conker_contract_npt does from stored maps.
// float32 accumulators are flushed into float64 every two lines; workgroups
// are persistent over lines and write float64 partials that a second kernel
// sums in a fixed order.
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "split3.h"
#include "fft_math.h"

using namespace conker;
using namespace conker::fftm;

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int NZ = 512;           // line length (z axis)
constexpr int NW = 8;             // waves per workgroup
constexpr int NT = NW * 64;
constexpr int MAXR = 30;          // radii held in LDS at once
constexpr int MROW = NZ + 4;      // padded row (floats) of the map store
constexpr int FLUSH_LINES = 2;
constexpr int PART = 2 * 1024;   // per-workgroup partial: W3a, W3b (W2 in column 31)

// Bank-conflict-free placement of the 512-point scratch for the three
// exchange patterns of the radix-8 stages (a bijection on 0..511).
__device__ __forceinline__ int swz(int e) { return e ^ ((e >> 3) & 31); }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// acc += A^T B over the 16 cells of one chunk: lane (row r, half h) holds the
// values of cells 8h .. 8h+7 of its row.
template <int PREC>
__device__ __forceinline__ void mma_chunk(floatx16 &acc, const float (&a)[8], const float (&b)[8]) {
    if constexpr (PREC == CONKER_MM_SPLIT_BF16) {
        bf16x8 ah, am, al, bh, bm, bl;
        split3(a, ah, am, al);
        split3(b, bh, bm, bl);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bm, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(am, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bm, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], acc, 0, 0, 0);
    }
}

// Lines: lines[0 .. *count) when `lines` is given (the lines carrying field;
// the others add nothing), else every line 0 .. nlines - 1.
template <int PREC>
__global__ __launch_bounds__(NT, 1) void k_zinv_contract(const float2 *__restrict__ tspec, int ns, size_t nc,
                                                         int nlines, const int *__restrict__ lines,
                                                         const int *__restrict__ count,
                                                         const float *__restrict__ Fa,
                                                         const float *__restrict__ Fb,
                                                         const float2 *__restrict__ twg,
                                                         double *__restrict__ partial) {
    const int nact = lines ? *count : nlines;
    // maps of the current line, one plane per field: Mf[field][radius][z]
    __shared__ __align__(16) float Mf[2 * MAXR * MROW];
    __shared__ float2 S[NW * NZ];
    __shared__ float2 tw[NZ];
    __shared__ unsigned long long zb[2][NW];   // per field and 64-cell block: bit c set iff F(c) != 0
    __shared__ unsigned char clist[NW][8];     // per wave: the line's non-empty 16-cell chunks it sums
    static_assert(NT == NZ, "one cell of the line per thread");
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 31, h = lane >> 5;
    // contraction split: waves 0..3 sum field a, waves 4..7 field b, 128 cells each
    const int fld = w >> 2, part = w & 3;
    const bool active = fld == 0 || Fb != nullptr;
    const float *F = fld == 0 ? Fa : Fb;
    const float *Mrow = Mf + (fld * MAXR + (r < ns ? r : 0)) * MROW;
    for (int t = threadIdx.x; t < NZ; t += NT) {
        const float2 v = twg[t];
        tw[t] = float2{v.x, -v.y};   // inverse transform: exp(+2 pi i t / NZ)
    }
    float2 *Sw = S + w * NZ;
    floatx16 acc = floatx16{0};
    double dacc[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) dacc[v] = 0.0;
    int since = 0;
    auto line_of = [&](int idx) -> int { return lines ? lines[idx] : idx; };
    float2 nxt[8];   // this wave's next (line, radius) item, loaded one item ahead
    if (w < ns && (int)blockIdx.x < nact) {
        const float2 *src = tspec + (size_t)w * nc + (size_t)line_of(blockIdx.x) * NZ;
#pragma unroll
        for (int q = 0; q < 8; ++q) nxt[q] = src[lane + 64 * q];
    }
    __syncthreads();
    // this lane's second- and third-stage twiddles, read once (strided LDS
    // reads conflict: the second stage's eight addresses for one q lie 64 q
    // bytes apart)
    float2 w2[7], w3[7];
#pragma unroll
    for (int q = 1; q < 8; ++q) {
        w2[q - 1] = tw[q * (lane & 7) * 8];
        w3[q - 1] = tw[q * lane];
    }

    for (int idx = blockIdx.x; idx < nact; idx += gridDim.x) {
        const size_t base = (size_t)line_of(idx) * NZ;
        // this line's F, one cell per thread, for the chunk lists below
        const float fza = Fa[base + threadIdx.x];
        const float fzb = Fb ? Fb[base + threadIdx.x] : 0.f;
        // ---- inverse z transform of every radius of this line --------------
        for (int m = w; m < ns; m += NW) {
            float2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = nxt[q];
            {   // prefetch the next (line, radius) item of this wave
                int mn = m + NW;
                int in = idx;
                if (mn >= ns) {
                    mn = w;
                    in = idx + gridDim.x;
                }
                if (mn < ns && in < nact) {
                    const float2 *src = tspec + (size_t)mn * nc + (size_t)line_of(in) * NZ;
#pragma unroll
                    for (int q = 0; q < 8; ++q) nxt[q] = src[lane + 64 * q];
                }
            }
            dft<8, +1>(v);                                   // stage 1: no twiddles
#pragma unroll
            for (int q = 0; q < 8; ++q) Sw[swz(8 * lane + q)] = v[q];
            wave_sync();
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = Sw[swz(lane + 64 * q)];
            {
                const int k = lane & 7;                      // stage 2: Ns = 8
#pragma unroll
                for (int q = 1; q < 8; ++q) v[q] = cmul(v[q], w2[q - 1]);
                dft<8, +1>(v);
                wave_sync();
                const int b2 = (lane - k) * 8 + k;
#pragma unroll
                for (int q = 0; q < 8; ++q) Sw[swz(b2 + 8 * q)] = v[q];
            }
            wave_sync();
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = Sw[swz(lane + 64 * q)];
#pragma unroll
            for (int q = 1; q < 8; ++q) v[q] = cmul(v[q], w3[q - 1]);   // stage 3: Ns = 64
            dft<8, +1>(v);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                Mf[m * MROW + lane + 64 * q] = v[q].x;
                Mf[(MAXR + m) * MROW + lane + 64 * q] = v[q].y;
            }
            wave_sync();
        }
        {   // cells outside the survey (F = 0 of either sign) add exactly nothing
            const unsigned long long ba = __ballot((__float_as_uint(fza) << 1) != 0);
            const unsigned long long bb = __ballot((__float_as_uint(fzb) << 1) != 0);
            if (lane == 0) {
                zb[0][w] = ba;
                zb[1][w] = bb;
            }
        }
        __syncthreads();
        // ---- contraction: the non-empty 16-cell chunks of this wave's field,
        // dealt round-robin to the field's four waves -------------------------
        if (active) {
            int nq;
            {
                const int k = lane & 31;   // chunk k: cells 16k .. 16k + 15
                const bool on = lane < 32 && ((zb[fld][k >> 2] >> ((k & 3) * 16)) & 0xffffull) != 0;
                const unsigned mk = (unsigned)__ballot(on);
                const int pos = __popc(mk & ((1u << k) - 1u)), cnt = __popc(mk);
                if (on && (pos & 3) == part) clist[w][pos >> 2] = (unsigned char)k;
                nq = cnt > part ? (cnt - part + 3) >> 2 : 0;
                wave_sync();
            }
#pragma unroll 2
            for (int j = 0; j < nq; ++j) {
                const int c0 = (int)clist[w][j] * 16 + 8 * h;
                float x[8], f[8], p[8];
                {
                    const float4 *mp = reinterpret_cast<const float4 *>(Mrow + c0);
                    const float4 t0 = mp[0], t1 = mp[1];
                    // rows below ns: the maps; row 31: the constant 1, so that column 31 of the
                    // product accumulates sum F C_a (the n = 2 sums); other rows: 0
                    const bool ok = r < ns;
                    const float pad = r == 31 ? 1.f : 0.f;
                    x[0] = ok ? t0.x : pad; x[1] = ok ? t0.y : pad; x[2] = ok ? t0.z : pad; x[3] = ok ? t0.w : pad;
                    x[4] = ok ? t1.x : pad; x[5] = ok ? t1.y : pad; x[6] = ok ? t1.z : pad; x[7] = ok ? t1.w : pad;
                }
                {
                    const float4 *fp = reinterpret_cast<const float4 *>(F + base + c0);
                    const float4 f0 = fp[0], f1 = fp[1];
                    f[0] = f0.x; f[1] = f0.y; f[2] = f0.z; f[3] = f0.w;
                    f[4] = f1.x; f[5] = f1.y; f[6] = f1.z; f[7] = f1.w;
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) p[e] = f[e] * x[e];
                mma_chunk<PREC>(acc, p, x);
            }
            if (++since == FLUSH_LINES) {
                since = 0;
#pragma unroll
                for (int v = 0; v < 16; ++v) dacc[v] += (double)acc[v];
                acc = floatx16{0};
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) dacc[v] += (double)acc[v];
    // ---- combine the four waves of each field and write the partial -------
    double *scr = reinterpret_cast<double *>(Mf);   // NW * 16 * 64 doubles = 64 KiB
    double *out = partial + (size_t)blockIdx.x * PART;
#pragma unroll
    for (int v = 0; v < 16; ++v) scr[(w * 16 + v) * 64 + lane] = dacc[v];
    __syncthreads();
    for (int e = threadIdx.x; e < 2048; e += NT) {
        const int f = e >> 10, i = (e >> 5) & 31, j = e & 31;   // field, row i (radius a), column j (radius b)
        const int l = j + 32 * ((i >> 2) & 1), v = (i & 3) + 4 * (i >> 3);
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += scr[((4 * f + k) * 16 + v) * 64 + l];
        out[e] = s;
    }
}

// Sums the workgroup partials in order and gathers the tuples:
//   n = 3: W[(a, b)], a <= b, lexicographic;  n = 2: W[a].
// Field b was transformed times the pair's scale s: its sums carry s^(n-1).
__global__ void k_fused_finish(const double *__restrict__ partial, int G, int ns, int n, double *Wa,
                               double *Wb, const PackScale *ps) {
    const int cnt = n == 3 ? ns * (ns + 1) / 2 : ns;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * cnt) return;
    const int f = t / cnt, k = t - f * cnt;
    double *W = f == 0 ? Wa : Wb;
    if (!W) return;
    int e;
    if (n == 3) {
        int a = 0, rem = k;
        while (rem >= ns - a) { rem -= ns - a; ++a; }
        const int b = a + rem;
        e = f * 1024 + a * 32 + b;
    } else {
        e = f * 1024 + k * 32 + 31;   // column 31 = the constant 1
    }
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += partial[(size_t)g * PART + e];
    if (f == 1)
        for (int p = 1; p < n; ++p) s *= ps->s_inv;   // a power of two: exact
    W[k] = s;
}

}  // namespace

// Every other order, precision and grid: the maps go to the context's
// workspace, but only on the z-lines carrying centre field -- the x pass
// writes carrying x-slabs, the y pass carrying lines, the z pass the maps of
// carrying lines -- since every term of every sum carries the centre field
// (the other cells of the maps are never read).  The sums are then those of
// conker_contract_npt, over the 64-cell blocks where the centre field is
// non-zero, all of which lie on carrying lines.
static int convolve_contract_maps(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa,
                                  const void *fb, const void *ca, const void *cb, const void *kspec, int ns, int n,
                                  conker_mmprec prec, double *Wa, double *Wb) {
    if (n < 2 || n > 5) return fail(c, CONKER_EINVAL, "order n=%d outside 2..5", n);
    if (ns < 1 || ns > 64) return fail(c, CONKER_EINVAL, "n_radii=%d outside 1..64", ns);
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (prec == CONKER_MM_F64 ? dt != CONKER_F64 : dt != CONKER_F32)
        return fail(c, CONKER_EINVAL, "float64 summation needs float64 fields, the others float32");
    if (prec != CONKER_MM_F64 && prec != CONKER_MM_F32 && prec != CONKER_MM_SPLIT_BF16 && prec != CONKER_MM_SPLIT_F16)
        return fail(c, CONKER_EINVAL, "bad precision");
    const bool f64 = dt == CONKER_F64;
    CK_HIP(c, hipSetDevice(c->device));
    Support sup;
    bool have_sup = false;
    {   // axis order of the transforms (cubic grids): the passes run on permuted copies
        const void *in[4] = {fa, fb, ca, cb}, *out[4];
        CK_OK(order_fields(c, g, f64, ns, in, 4, out, &sup, &have_sup));
        fa = out[0]; fb = out[1]; ca = out[2]; cb = out[3];
    }
    const size_t nc = ncells(g);
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    const size_t cbytes = 2 * nc * esz;
    const size_t mbytes = (size_t)ns * nc * esz;
    CK_OK(ws_reserve(c, c->maps, (fb ? 2 : 1) * mbytes));
    const int B = batch_radii(c, cbytes, ns, cbytes);
    CK_OK(ws_reserve(c, c->spec, cbytes));
    CK_OK(ws_reserve(c, c->tspec, (size_t)B * cbytes));
    if (!have_sup) CK_OK(support_lines(c, g, f64, ca, cb, &sup));
    void *ma = c->maps.p;
    void *mb = fb ? (void *)((char *)c->maps.p + mbytes) : nullptr;
    // the convolved fields are the centre fields (auto-correlation): their
    // support also prunes the forward transform
    CK_OK(fft_forward_pair(c, g, f64, fa, fb, c->spec.p, (fa == ca && fb == cb) ? &sup : nullptr));
    for (int m0 = 0; m0 < ns; m0 += B) {
        const int nb = (m0 + B <= ns) ? B : ns - m0;
        CK_OK(fft_inverse_batch(c, g, f64, c->spec.p, kspec, m0, nb, c->tspec.p, ma, mb, &sup, 0, true));
    }
    CK_OK(conker_contract_npt(c, g, dt, ca, ma, ns, n, prec, Wa));
    if (fb) CK_OK(conker_contract_npt(c, g, dt, cb, mb, ns, n, prec, Wb));
    return CONKER_OK;
}

// Maps from fa (fb), summed against the centre fields ca (cb) of vertex 0.
static int convolve_contract(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa, const void *fb,
                             const void *ca, const void *cb, const void *kspec, int ns, int n, conker_mmprec prec,
                             double *Wa, double *Wb) {
    CK_OK(check_grid(c, g, true));
    if (!fa || !ca || !kspec || !Wa) return fail(c, CONKER_EINVAL, "NULL pointer");
    if ((fb == nullptr) != (Wb == nullptr) || (fb == nullptr) != (cb == nullptr))
        return fail(c, CONKER_EINVAL, "field_b, its centre field and W_b must all be given or all be NULL");
    // the fused kernel: float32 with f32 or split-bf16 products, n = 2, 3,
    // z-lines of 512 cells, at most 30 radii (the maps of one line in LDS)
    if ((n != 2 && n != 3) || dt != CONKER_F32 || (prec != CONKER_MM_F32 && prec != CONKER_MM_SPLIT_BF16) ||
        g->dims[2] != NZ || ns < 1 || ns > MAXR)
        return convolve_contract_maps(c, g, dt, fa, fb, ca, cb, kspec, ns, n, prec, Wa, Wb);
    CK_HIP(c, hipSetDevice(c->device));
    Support sup;
    bool have_sup = false;
    {   // axis order of the transforms (cubic grids): the passes run on permuted copies
        const void *in[4] = {fa, fb, ca, cb}, *out[4];
        CK_OK(order_fields(c, g, false, ns, in, 4, out, &sup, &have_sup));
        fa = out[0]; fb = out[1]; ca = out[2]; cb = out[3];
    }
    const size_t nc = ncells(g);
    const size_t cbytes = nc * sizeof(float2);
    CK_OK(ws_reserve(c, c->spec, cbytes));
    CK_OK(ws_reserve(c, c->tspec, (size_t)ns * cbytes));
    if (!have_sup) CK_OK(support_lines(c, g, false, ca, cb, &sup));
    CK_OK(fft_forward_pair(c, g, false, fa, fb, c->spec.p, (fa == ca && fb == cb) ? &sup : nullptr));
    CK_OK(fft_inverse_batch(c, g, false, c->spec.p, kspec, 0, ns, c->tspec.p, nullptr, nullptr, &sup));
    const void *twz;
    CK_OK(twiddles(c, NZ, false, &twz));
    const int nlines = g->dims[0] * g->dims[1];
    const int G = std::min(nlines, cu_count(c));
    CK_OK(ws_reserve(c, c->partial, (size_t)G * PART * sizeof(double)));
    {
        ProfScope ps(c, PK_FUSED_ZC);
        if (prec == CONKER_MM_SPLIT_BF16)
            hipLaunchKernelGGL(k_zinv_contract<CONKER_MM_SPLIT_BF16>, dim3(G), dim3(NT), 0, c->stream,
                               (const float2 *)c->tspec.p, ns, nc, nlines, sup.list, sup.count, (const float *)ca,
                               (const float *)cb,
                               (const float2 *)twz, (double *)c->partial.p);
        else
            hipLaunchKernelGGL(k_zinv_contract<CONKER_MM_F32>, dim3(G), dim3(NT), 0, c->stream,
                               (const float2 *)c->tspec.p, ns, nc, nlines, sup.list, sup.count, (const float *)ca,
                               (const float *)cb,
                               (const float2 *)twz, (double *)c->partial.p);
        CK_LAUNCH(c);
    }
    ProfScope ps(c, PK_CONTRACT_REDUCE);
    const int cnt = n == 3 ? ns * (ns + 1) / 2 : ns;
    hipLaunchKernelGGL(k_fused_finish, dim3((2 * cnt + 127) / 128), dim3(128), 0, c->stream,
                       (const double *)c->partial.p, G, ns, n, Wa, Wb, pack_scale_dev(c));
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_convolve_contract(conker_ctx *c, const conker_grid *g, conker_dtype dt, const void *fa,
                                        const void *fb, const void *kspec, int ns, int n, conker_mmprec prec,
                                        double *Wa, double *Wb) {
    return convolve_contract(c, g, dt, fa, fb, fa, fb, kspec, ns, n, prec, Wa, Wb);
}

extern "C" int conker_convolve_contract_cross(conker_ctx *c, const conker_grid *g, conker_dtype dt,
                                              const void *fa, const void *fb, const void *ca, const void *cb,
                                              const void *kspec, int ns, int n, conker_mmprec prec, double *Wa,
                                              double *Wb) {
    return convolve_contract(c, g, dt, fa, fb, ca, cb, kspec, ns, n, prec, Wa, Wb);
}
