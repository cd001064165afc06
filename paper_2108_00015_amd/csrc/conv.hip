// Shell-kernel bank (Sec. 2.3) and shell convolutions (Sec. 2.4).
#include <cmath>
#include <cstdlib>

#include "common.h"

using namespace conker;

namespace conker {

// Radii convolved per inverse batch: one read of the forward spectrum serves
// this many kernel multiplies and inverse x-axis transforms.  Default: every
// radius, as long as the batch spectra take at most half of the device memory
// that is free or already held for them (so that the choice is the same from
// call to call and the buffer is not regrown).  A context setting
// (conker_set_tune, conker_batch_autotune) or CONKER_RADIUS_BATCH replaces it.
int batch_radii(conker_ctx *c, size_t per_radius_bytes, int n_radii, size_t fixed_bytes) {
    int b = n_radii;
    if (c->capturing) {   // inside a graph capture: use the batch buffer as planned
        const size_t fit = per_radius_bytes ? c->tspec.bytes / per_radius_bytes : (size_t)n_radii;
        b = (int)(fit < 1 ? 1 : (fit < (size_t)n_radii ? fit : (size_t)n_radii));
        if (c->tune.radius_batch && c->tune.radius_batch < b) b = c->tune.radius_batch;
        return b;
    }
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
        const size_t budget = (fr + c->tspec.bytes) / 2;
        const size_t fit = per_radius_bytes ? budget / per_radius_bytes : (size_t)n_radii;
        if ((size_t)b > fit) b = (int)(fit < 1 ? 1 : fit);
    }
    if (c->tune.radius_batch) {
        b = c->tune.radius_batch;
    } else if (const char *e = std::getenv("CONKER_RADIUS_BATCH")) {
        int v = std::atoi(e);
        if (v >= 1 && v <= 64) b = v;
    }
    if (b > n_radii) b = n_radii;
    if (c->ws_cap) {
        while (b > 1 && c->ws_bytes - c->tspec.bytes - c->spec.bytes + fixed_bytes +
                                (size_t)b * per_radius_bytes > c->ws_cap)
            --b;
    }
    return b < 1 ? 1 : b;
}

}  // namespace conker


extern "C" int conker_make_shell_kernels(conker_ctx *c, const conker_grid *g, const double *h_radii,
                                         int n_radii, conker_dtype dt, void *d_kspec,
                                         int64_t *h_sizes) {
    CK_OK(check_grid(c, g, true));
    if (n_radii <= 0 || !h_radii || !d_kspec) return fail(c, CONKER_EINVAL, "bad radii or NULL pointer");
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    std::vector<double> r(n_radii);
    for (int m = 0; m < n_radii; ++m) {
        r[m] = h_radii[m] / g->cell;
        CK_OK(check_shell(c, g, r[m]));
    }
    CK_HIP(c, hipSetDevice(c->device));
    const size_t nc = ncells(g);
    CK_OK(ws_reserve(c, c->spec, nc * sizeof(double2)));
    for (int m = 0; m < n_radii; m += 2) {
        const double ra = r[m];
        const double rb = (m + 1 < n_radii) ? r[m + 1] : ra;
        CK_OK(fft_shell_pair(c, g, (ra - 0.5) * (ra - 0.5), (ra + 0.5) * (ra + 0.5),
                             (rb - 0.5) * (rb - 0.5), (rb + 0.5) * (rb + 0.5), c->spec.p, d_kspec,
                             dt == CONKER_F64, m, (m + 1 < n_radii) ? m + 1 : -1));
    }
    if (h_sizes)
        for (int m = 0; m < n_radii; ++m) CK_OK(conker_shell_size(r[m], &h_sizes[m]));
    return CONKER_OK;
}

extern "C" int conker_convolve_shells(conker_ctx *c, const conker_grid *g, conker_dtype dt,
                                      const void *fa, const void *fb, const void *kspec,
                                      int n_radii, void *ma, void *mb) {
    CK_OK(check_grid(c, g, true));
    if (dt != CONKER_F32 && dt != CONKER_F64) return fail(c, CONKER_EINVAL, "bad dtype");
    if (!fa || !kspec || !ma) return fail(c, CONKER_EINVAL, "NULL pointer");
    if ((fb == nullptr) != (mb == nullptr))
        return fail(c, CONKER_EINVAL, "field_b and maps_b must both be given or both be NULL");
    if (n_radii <= 0) return fail(c, CONKER_EINVAL, "n_radii must be positive");
    CK_HIP(c, hipSetDevice(c->device));
    const bool f64 = dt == CONKER_F64;
    const size_t nc = ncells(g);
    const size_t cbytes = nc * (f64 ? sizeof(double2) : sizeof(float2));
    // one field: pair the radii instead (slot j carries C_{2j} + i C_{2j+1})
    const bool pair = fb == nullptr && n_radii > 1;
    const int slots = pair ? (n_radii + 1) / 2 : n_radii;
    const int B = batch_radii(c, cbytes, slots, cbytes);
    CK_OK(ws_reserve(c, c->spec, cbytes));
    CK_OK(ws_reserve(c, c->tspec, (size_t)B * cbytes));
    CK_OK(fft_forward_pair(c, g, f64, fa, fb, c->spec.p));
    for (int m0 = 0; m0 < slots; m0 += B) {
        const int nb = (m0 + B <= slots) ? B : slots - m0;
        CK_OK(fft_inverse_batch(c, g, f64, c->spec.p, kspec, m0, nb, c->tspec.p, ma, mb, nullptr,
                                pair ? n_radii : 0));
    }
    return CONKER_OK;
}
