// crk_noalloc.cpp -- crk_compute_dt_noalloc: the CFL time step without a
// workspace, for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops).  Its reduction partials live in a
// file-scope device array, one copy per GPU, instead of the workspace.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/crk.h"
#include "crk_kernels.hpp"

namespace crk {
crk_status solver_dt(crk_solver *s, const void *u, double *parts, int max_parts, double *dt_dev, hipStream_t stream);
crk_status fail_with(crk_status st, const char *msg);
}

namespace {

// The dt reduction uses at most RED_BLOCKS workgroups, so this holds the
// partials of any mesh the library accepts (8 KiB per GPU).
constexpr int NOALLOC_PARTS = crk::RED_BLOCKS;
constexpr int MAX_DEVICES = 64;

// Host code never passes the array's name to a kernel (on the host it only
// stands for the symbol): the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) double scratch[NOALLOC_PARTS];

std::mutex g_mu;
double *g_ptr[MAX_DEVICES];

crk_status scratch_of_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return crk::fail_with(CRK_ERR_HIP, "crk_compute_dt_noalloc: hipGetDevice failed");
    if (dev < 0 || dev >= MAX_DEVICES) return crk::fail_with(CRK_ERR_UNSUPPORTED, "crk_compute_dt_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "crk_compute_dt_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
            return crk::fail_with(CRK_ERR_HIP, buf);
        }
        g_ptr[dev] = (double *)p;
    }
    *out = g_ptr[dev];
    return CRK_OK;
}

} // namespace

extern "C" crk_status crk_compute_dt_noalloc(crk_solver *s, const void *u, double *dt_dev, crk_stream stream)
{
    if (!s) return crk::fail_with(CRK_ERR_ARG, "null solver");
    if (!u || !dt_dev) return crk::fail_with(CRK_ERR_ARG, "null pointer");
    double *sp = nullptr;
    crk_status st = scratch_of_current_device(&sp);
    if (st) return st;
    return crk::solver_dt(s, u, sp, NOALLOC_PARTS, dt_dev, (hipStream_t)stream);
}
