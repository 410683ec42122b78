// pp_server_hip.cpp -- the serving loop's device backend: one pp_handle per
// case on its own HIP stream, plus the case's resident pressure.
//
// A case's last pressure stays on the device between its requests and is the
// initial guess of its next solve (warm start); the result is copied out to the
// request's p_out on the case's stream.
#include "../../include/pp.h"
#include "../../include/pp_server.h"

#include <hip/hip_runtime.h>

namespace {

struct HipCase {
    pp_handle h = nullptr;
    hipStream_t stream = nullptr;
    double* p = nullptr;
    size_t n = 0;
};

size_t hip_footprint(void*, const pp_config* cfg)
{
    size_t b = pp_footprint_bytes(cfg);
    if (b == 0) return 0;
    return b + (size_t)cfg->nx * cfg->ny * cfg->nz * sizeof(double) + 4096;
}

int hip_open(void*, const pp_config* cfg, void** out)
{
    auto* c = new HipCase;
    c->n = (size_t)cfg->nx * cfg->ny * cfg->nz;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return PP_ERR_HIP;
    }
    if (hipMalloc((void**)&c->p, c->n * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamDestroy(c->stream);
        delete c;
        return PP_ERR_OOM;
    }
    if (hipMemsetAsync(c->p, 0, c->n * sizeof(double), c->stream) != hipSuccess) {
        (void)hipFree(c->p);
        (void)hipStreamDestroy(c->stream);
        delete c;
        return PP_ERR_HIP;
    }
    int rc = pp_create(cfg, c->stream, &c->h);
    if (rc != PP_OK) {
        (void)hipFree(c->p);
        (void)hipStreamDestroy(c->stream);
        delete c;
        return rc;
    }
    *out = c;
    return PP_OK;
}

int hip_set_density(void*, void* cs, const double* rho) { return pp_set_density(static_cast<HipCase*>(cs)->h, rho); }

int hip_solve(void*, void* cs, const double* rhs, double* p_out, pp_stats* st)
{
    auto* c = static_cast<HipCase*>(cs);
    int rc = pp_solve(c->h, rhs, c->p, st);
    if (p_out && (rc == PP_OK || rc == PP_ERR_NOT_CONVERGED)) {
        if (hipMemcpyAsync(p_out, c->p, c->n * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return PP_ERR_HIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return PP_ERR_HIP;
    }
    return rc;
}

void hip_close(void*, void* cs)
{
    auto* c = static_cast<HipCase*>(cs);
    if (!c) return;
    pp_destroy(c->h);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->p) (void)hipFree(c->p);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* hip_error(void*, void* cs) { return cs ? pp_last_error(static_cast<HipCase*>(cs)->h) : pp_last_error(nullptr); }

}  // namespace

pp_backend ppsrv_hip_backend()
{
    return pp_backend{nullptr, hip_footprint, hip_open, hip_set_density, hip_solve, hip_close, hip_error};
}
