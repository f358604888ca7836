// fmm_static.hip -- fmm_evaluate_static: one full evaluation whose workspace
// is a fixed device array of this library, for callers that cannot allocate
// device memory (code under graph capture, serving loops, harnesses that
// forbid allocation).  See include/fmm.h for the contract.
//
// The array `scratch` below exists once per GPU the library is loaded on and
// lives until the process ends.  Host code never passes its name to a kernel
// or a copy: the name is a host-side stand-in, not a device address.  The
// first call on a device (that device current) looks its device address up
// with hipGetSymbolAddress and keeps it per device; every later use goes
// through that address.
//
// The evaluation writes every workspace word it reads before reading it (the
// tree, the expansions, the partial M2L sums, the status counters), so
// nothing needs clearing between calls; the operator tables a plan uploads
// into the array are kept and reused while the parameters stay the same.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fmm.h"
#include "fmm_internal.h"

constexpr size_t kStaticScratchBytes = size_t(FMM_STATIC_SCRATCH_BYTES);

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct DeviceSlot {
    void* ptr = nullptr;          // device address of `scratch` on this device
    fmm_plan_t plan = nullptr;    // plan over it for the parameters below
    fmm_params prm{};
};

std::mutex g_mu;
DeviceSlot g_slot[kMaxDevices];

bool same_params(const fmm_params& a, const fmm_params& b)
{
    return a.n_max == b.n_max && a.sigma == b.sigma && a.p == b.p && a.depth == b.depth && a.x0 == b.x0 &&
           a.y0 == b.y0 && a.width == b.width && a.precision == b.precision &&
           a.fp32_fine_levels == b.fp32_fine_levels && a.m_max == b.m_max && a.kernel == b.kernel &&
           a.lj_epsilon == b.lj_epsilon && a.cutoff == b.cutoff;
}

}  // namespace

extern "C" fmm_status fmm_evaluate_static(const fmm_params* prm, int64_t n, const double* d_x, const double* d_y,
                                          const double* d_gamma, double* d_u, double* d_v, void* stream)
{
    if (!prm) return FMM_E_ARG;
    size_t need = 0;
    fmm_status s = fmm_workspace_size(prm, &need);
    if (s != FMM_OK) return s;
    if (need > kStaticScratchBytes) return FMM_E_CAPACITY;
    if (n < 0) return FMM_E_ARG;
    if (n > prm->n_max) return FMM_E_CAPACITY;
    if (n > 0 && (!d_x || !d_y || !d_gamma || !d_u || !d_v)) return FMM_E_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FMM_E_DEVICE;
    if (dev < 0 || dev >= kMaxDevices) return FMM_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceSlot& sl = g_slot[dev];
    if (!sl.ptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FMM_E_DEVICE;
        sl.ptr = p;
    }
    if (!sl.plan || !same_params(sl.prm, *prm)) {
        if (sl.plan) {
            fmm_destroy(sl.plan);
            sl.plan = nullptr;
        }
        // uploads the operator tables into the array and waits for them
        s = fmm::plan_in_buffer(prm, sl.ptr, kStaticScratchBytes, stream, &sl.plan);
        if (s != FMM_OK) {
            sl.plan = nullptr;
            return s;
        }
        sl.prm = *prm;
    }
    return fmm_evaluate(sl.plan, n, d_x, d_y, d_gamma, d_u, d_v, stream);
}
