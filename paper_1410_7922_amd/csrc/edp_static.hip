// edp_solve_static: the EDP solve of edp_solve with its workspace in a static device array, for
// callers that cannot allocate device memory (code under stream capture, serving loops, harnesses
// that forbid allocation).  The array is a file-scope __device__ object: every GPU the library runs
// on holds its own copy, at its own address, until the process ends.  Its name is not a device
// address in host code; the address comes from hipGetSymbolAddress, looked up once per device with
// that device current and kept in a table, and only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/edp.h"

namespace {

__device__ __align__(256) unsigned char scratch[EDP_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices];   // device address of this device's scratch, or null before the lookup
std::mutex g_mu;

// Device address of the calling thread's current device's scratch array (looked up on first use).
edp_status scratch_of(int dev, void** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return EDP_E_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return EDP_OK;
}

}  // namespace

extern "C" edp_status edp_solve_static(const edp_problem* prob, const edp_tuning* tuning, const void* d_cost,
                                       int32_t* d_labels, int64_t* d_energy, int32_t* d_status, void* stream) {
    size_t need = 0;
    edp_status st = edp_workspace_size(prob, EDP_OP_EDP, tuning, &need);
    if (st != EDP_OK) return st;
    if (need > (size_t)EDP_STATIC_SCRATCH_BYTES) return EDP_E_WORKSPACE;
    if (!d_cost || !d_labels) return EDP_E_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EDP_E_HIP;
    if (stream) {
        // the scratch looked up is the current device's: the stream must run on that device
        int sdev = -1;
        if (hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess) return EDP_E_HIP;
        if (sdev != dev) return EDP_E_INVALID;
    }
    void* ws = nullptr;
    st = scratch_of(dev, &ws);
    if (st != EDP_OK) return st;
    // edp_solve clears the control words it needs at zero with a fill kernel on every call; the sum
    // arrays are written before they are read, so the previous call's contents do not matter
    return edp_solve(prob, tuning, d_cost, d_labels, d_energy, d_status, ws, (size_t)EDP_STATIC_SCRATCH_BYTES, stream);
}
