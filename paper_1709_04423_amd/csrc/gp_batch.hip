// Batched form: many independent 2D problems advanced together.
#include "gp_internal.h"

extern "C" {

gp_status gp_batch_create(gp_batch **out, int count, const int64_t *n, const double *dx, const double *dt,
                          gp_mode mode, const double *omega, const double *g, gp_prec prec)
{
    (void)mode; (void)prec;
    if (!out || count < 1 || !n || !dx || !dt || !omega || !g) return gp::set_error("bad argument"), GP_EINVAL;
    *out = nullptr;
    gp::set_error("batch form not built yet");
    return GP_EUNSUPPORTED;
}

gp_status gp_batch_destroy(gp_batch *batch) { (void)batch; return GP_OK; }

gp_status gp_batch_step(gp_batch *batch, void *const *psis, int64_t nsteps, void *stream)
{
    (void)stream;
    if (!batch || !psis || nsteps < 0) return gp::set_error("bad argument"), GP_EINVAL;
    return GP_EUNSUPPORTED;
}

gp_status gp_batch_autotune(gp_batch *batch, const char *cache_path, void *stream)
{
    (void)batch; (void)cache_path; (void)stream;
    return GP_EUNSUPPORTED;
}

gp_status gp_batch_observables(gp_batch *batch, int k, const void *psi, gp_obs *out, void *stream)
{
    (void)batch; (void)k; (void)psi; (void)out; (void)stream;
    return GP_EUNSUPPORTED;
}

}
