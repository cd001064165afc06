// Survey front end (Sec. 2.2): sky coordinates and redshifts to comoving
// Cartesian positions (Eqs. hubbleint, cartesianx, cartesiany, cartesianz), and
// the expected random count per cell from factorizable angular and redshift
// selection functions (Eq. factorizablility).
//
// r(z) = c/H0 int_0^z dz'/E(z'), E = sqrt(Om (1+z)^3 + Ok (1+z)^2 + OL), is
// tabulated on TAB equal intervals of [0, z_max]: each interval integrated
// with 8-point Gauss-Legendre (nodes from Newton's method on the Legendre
// polynomial, computed on the host), the intervals summed in order by one
// workgroup.  Between nodes r is the cubic Hermite interpolant of r and
// dr/dz = c/(H0 E); its error is far below float32 resolution.  z(r) inverts
// the same interpolant (bisection over the table, then Newton steps).
#include <cmath>

#include "common.h"

using namespace conker;

namespace {

constexpr int TAB = 8192;   // table intervals
constexpr int GL = 8;       // Gauss-Legendre points per interval

struct GaussLegendre {
    double x[GL], w[GL];
};

struct Cosmo {
    double Om, Ok, OL, c_h0, z_max, h;   // c_h0 = c / H0, h = z_max / TAB
};

__device__ __forceinline__ double e_of_z(const Cosmo &q, double z) {
    const double zp = 1.0 + z;
    return sqrt(q.Om * zp * zp * zp + q.Ok * zp * zp + q.OL);
}

// seg[i] = int over interval i of dz / E(z)
__global__ void k_intervals(Cosmo q, GaussLegendre gl, double *__restrict__ seg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= TAB) return;
    const double a = i * q.h, half = 0.5 * q.h;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < GL; ++k) s += gl.w[k] / e_of_z(q, a + half * (1.0 + gl.x[k]));
    seg[i] = s * half;
}

// r[0] = 0, r[i + 1] = r[i] + c/H0 seg[i], in order: 1024 threads x 8 intervals
__global__ __launch_bounds__(1024) void k_prefix(Cosmo q, const double *__restrict__ seg, double *__restrict__ r) {
    __shared__ double part[1024];
    constexpr int PER = TAB / 1024;
    const int t = threadIdx.x;
    double s = 0.0;
    for (int k = 0; k < PER; ++k) s += seg[t * PER + k];
    part[t] = s;
    __syncthreads();
    if (t == 0) {   // the 1024 partial sums, serially, for a fixed order
        double acc = 0.0;
        for (int k = 0; k < 1024; ++k) {
            const double v = part[k];
            part[k] = acc;
            acc += v;
        }
        r[TAB] = acc * q.c_h0;
    }
    __syncthreads();
    double acc = part[t];
    for (int k = 0; k < PER; ++k) {
        r[t * PER + k] = acc * q.c_h0;
        acc += seg[t * PER + k];
    }
}

// Hermite interpolant on interval i at local coordinate u in [0, 1]
__device__ __forceinline__ double hermite(const Cosmo &q, const double *r, int i, double u, double *drdz) {
    const double z0 = i * q.h, z1 = (i + 1) * q.h;
    const double d0 = q.c_h0 / e_of_z(q, z0), d1 = q.c_h0 / e_of_z(q, z1);
    const double u2 = u * u, u3 = u2 * u;
    const double h00 = 2 * u3 - 3 * u2 + 1, h10 = u3 - 2 * u2 + u, h01 = -2 * u3 + 3 * u2, h11 = u3 - u2;
    if (drdz) {
        const double g00 = 6 * u2 - 6 * u, g10 = 3 * u2 - 4 * u + 1, g01 = -6 * u2 + 6 * u, g11 = 3 * u2 - 2 * u;
        *drdz = (g00 * r[i] + g01 * r[i + 1]) / q.h + g10 * d0 + g11 * d1;
    }
    return h00 * r[i] + h10 * q.h * d0 + h01 * r[i + 1] + h11 * q.h * d1;
}

__device__ __forceinline__ double r_of_z(const Cosmo &q, const double *r, double z) {
    int i = (int)floor(z / q.h);
    if (i >= TAB) i = TAB - 1;
    if (i < 0) i = 0;
    return hermite(q, r, i, z / q.h - i, nullptr);
}

// z(r) for 0 <= rr <= r[TAB]
__device__ double z_of_r(const Cosmo &q, const double *r, double rr) {
    int lo = 0, hi = TAB;   // r[lo] <= rr <= r[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (r[mid] <= rr) lo = mid;
        else hi = mid;
    }
    double u = (rr - r[lo]) / (r[lo + 1] - r[lo]);
    for (int it = 0; it < 4; ++it) {
        double d;
        const double f = hermite(q, r, lo, u, &d) - rr;
        u -= f / (d * q.h);
        u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
    }
    return (lo + u) * q.h;
}

__global__ __launch_bounds__(256) void k_sky_to_xyz(Cosmo q, const double *__restrict__ rt,
                                                    const double *__restrict__ ra, const double *__restrict__ dec,
                                                    const double *__restrict__ z, int64_t n, float *__restrict__ pos) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double zi = z[i];
        float x = NAN, y = NAN, w = NAN;
        if (zi >= 0.0 && zi <= q.z_max) {
            const double r = r_of_z(q, rt, zi);
            const double a = ra[i] * (M_PI / 180.0), d = dec[i] * (M_PI / 180.0);
            const double cd = cos(d);
            x = (float)(r * cd * cos(a));
            y = (float)(r * cd * sin(a));
            w = (float)(r * sin(d));
        }
        pos[3 * i + 0] = x;
        pos[3 * i + 1] = y;
        pos[3 * i + 2] = w;
    }
}

struct GridGeomC {
    double ox, oy, oz, cell;
    int nx, ny, nz;
};

struct Tables {
    const double *p_ang;
    int n_dec, n_ra;
    double ra0, ra1, dec0, dec1;
    const double *p_z;
    int n_z;
    double z0, z1;
};

template <typename T>
__global__ __launch_bounds__(256) void k_analytic_randoms(Cosmo q, const double *__restrict__ rt, Tables tb,
                                                          GridGeomC g, double n_tot, T *__restrict__ out) {
    const size_t nc = (size_t)g.nx * g.ny * g.nz;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
        const int iz = (int)(c % g.nz), iy = (int)((c / g.nz) % g.ny), ix = (int)(c / ((size_t)g.nz * g.ny));
        const double X = g.ox + (ix + 0.5) * g.cell, Y = g.oy + (iy + 0.5) * g.cell, Z = g.oz + (iz + 0.5) * g.cell;
        const double r = sqrt(X * X + Y * Y + Z * Z);
        double v = 0.0;
        if (r > 0.0 && r <= rt[TAB]) {
            const double dec = asin(Z / r) * (180.0 / M_PI);
            double ra = atan2(Y, X) * (180.0 / M_PI);
            ra = fmod(ra, 360.0);
            if (ra < 0.0) ra += 360.0;
            const double zz = z_of_r(q, rt, r);
            const int ia = (int)floor((ra - tb.ra0) / (tb.ra1 - tb.ra0) * tb.n_ra);
            const int id = (int)floor((dec - tb.dec0) / (tb.dec1 - tb.dec0) * tb.n_dec);
            const int ib = (int)floor((zz - tb.z0) / (tb.z1 - tb.z0) * tb.n_z);
            if (ia >= 0 && ia < tb.n_ra && id >= 0 && id < tb.n_dec && ib >= 0 && ib < tb.n_z) {
                const double drdz = q.c_h0 / e_of_z(q, zz);
                v = n_tot * tb.p_ang[(size_t)id * tb.n_ra + ia] * tb.p_z[ib] / (r * r * drdz) * g.cell * g.cell *
                    g.cell;
            }
        }
        out[c] = (T)v;
    }
}

// Gauss-Legendre nodes and weights on [-1, 1]: roots of P_n by Newton's method.
GaussLegendre gauss_legendre() {
    GaussLegendre gl;
    const int n = GL;
    for (int i = 0; i < n; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;   // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);   // P_n'(x)
            const double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        gl.x[i] = x;
        gl.w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return gl;
}

int check_cosmo(conker_ctx *c, const conker_cosmology *cm) {
    if (!cm) return fail(c, CONKER_EINVAL, "NULL cosmology");
    if (!(cm->h0 > 0.0) || !(cm->c > 0.0) || !(cm->z_max > 0.0))
        return fail(c, CONKER_EINVAL, "need H0 > 0, c > 0 and z_max > 0");
    // E(z)^2 must stay positive on [0, z_max]: check at the ends and the stationary point of the cubic
    auto e2 = [&](double z) {
        const double zp = 1.0 + z;
        return cm->omega_m * zp * zp * zp + cm->omega_k * zp * zp + cm->omega_lambda;
    };
    if (!(e2(0.0) > 0.0) || !(e2(cm->z_max) > 0.0)) return fail(c, CONKER_EINVAL, "E(z)^2 <= 0 in [0, z_max]");
    if (cm->omega_m != 0.0) {
        const double zs = -2.0 * cm->omega_k / (3.0 * cm->omega_m) - 1.0;
        if (zs > 0.0 && zs < cm->z_max && !(e2(zs) > 0.0)) return fail(c, CONKER_EINVAL, "E(z)^2 <= 0 in [0, z_max]");
    }
    return CONKER_OK;
}

// Table of r at the TAB + 1 nodes, in the context's workspace.
int build_table(conker_ctx *c, const conker_cosmology *cm, Cosmo &q, const double **table) {
    q = Cosmo{cm->omega_m, cm->omega_k, cm->omega_lambda, cm->c / cm->h0, cm->z_max, cm->z_max / TAB};
    CK_OK(ws_reserve(c, c->cosmo, (2 * TAB + 8) * sizeof(double)));
    double *seg = (double *)c->cosmo.p;
    double *r = seg + TAB;
    static const GaussLegendre gl = gauss_legendre();
    hipLaunchKernelGGL(k_intervals, dim3(TAB / 256), dim3(256), 0, c->stream, q, gl, seg);
    CK_LAUNCH(c);
    hipLaunchKernelGGL(k_prefix, dim3(1), dim3(1024), 0, c->stream, q, (const double *)seg, r);
    CK_LAUNCH(c);
    *table = r;
    return CONKER_OK;
}

}  // namespace

extern "C" int conker_sky_to_cartesian(conker_ctx *c, const conker_cosmology *cm, const double *ra,
                                       const double *dec, const double *z, int64_t n, float *pos) {
    if (!c) return CONKER_EINVAL;
    CK_OK(check_cosmo(c, cm));
    if (n < 0) return fail(c, CONKER_EINVAL, "negative count");
    if (n > 0 && (!ra || !dec || !z || !pos)) return fail(c, CONKER_EINVAL, "NULL pointer");
    CK_HIP(c, hipSetDevice(c->device));
    ProfScope ps(c, PK_SURVEY);
    Cosmo q;
    const double *rt;
    CK_OK(build_table(c, cm, q, &rt));
    if (n == 0) return CONKER_OK;
    const int threads = 256;
    const int64_t want = (n + threads - 1) / threads;
    const int blocks = (int)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(k_sky_to_xyz, dim3(blocks), dim3(threads), 0, c->stream, q, rt, ra, dec, z, n, pos);
    CK_LAUNCH(c);
    return CONKER_OK;
}

extern "C" int conker_analytic_randoms(conker_ctx *c, const conker_grid *g, conker_dtype dt,
                                       const conker_cosmology *cm, double n_tot, const double *p_ang, int n_dec,
                                       int n_ra, const double *ra_range, const double *dec_range, const double *p_z,
                                       int n_z, const double *z_range, void *R) {
    CK_OK(check_grid(c, g, false));
    CK_OK(check_cosmo(c, cm));
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (!p_ang || !p_z || !ra_range || !dec_range || !z_range || !R) return fail(c, CONKER_EINVAL, "NULL pointer");
    if (n_dec < 1 || n_ra < 1 || n_z < 1) return fail(c, CONKER_EINVAL, "empty selection table");
    if (!(ra_range[1] > ra_range[0]) || !(dec_range[1] > dec_range[0]) || !(z_range[1] > z_range[0]))
        return fail(c, CONKER_EINVAL, "table ranges must be increasing");
    if (z_range[0] < 0.0 || z_range[1] > cm->z_max)
        return fail(c, CONKER_EINVAL, "the redshift table must lie inside [0, z_max]");
    CK_HIP(c, hipSetDevice(c->device));
    ProfScope ps(c, PK_SURVEY);
    Cosmo q;
    const double *rt;
    CK_OK(build_table(c, cm, q, &rt));
    Tables tb{p_ang, n_dec, n_ra, ra_range[0], ra_range[1], dec_range[0], dec_range[1], p_z, n_z, z_range[0],
              z_range[1]};
    GridGeomC gg{g->origin[0], g->origin[1], g->origin[2], g->cell, g->dims[0], g->dims[1], g->dims[2]};
    const size_t nc = ncells(g);
    const int threads = 256;
    const size_t want = (nc + threads - 1) / threads;
    const int blocks = (int)(want < 8192 ? want : 8192);
    if (dt == CONKER_F32)
        hipLaunchKernelGGL(k_analytic_randoms<float>, dim3(blocks), dim3(threads), 0, c->stream, q, rt, tb, gg, n_tot,
                           (float *)R);
    else
        hipLaunchKernelGGL(k_analytic_randoms<double>, dim3(blocks), dim3(threads), 0, c->stream, q, rt, tb, gg,
                           n_tot, (double *)R);
    CK_LAUNCH(c);
    return CONKER_OK;
}
