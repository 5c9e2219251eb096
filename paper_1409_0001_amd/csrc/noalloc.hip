// cgd_deposit_noalloc: the particle centroid deposit of cgd_deposit on hex
// meshes, with every temporary buffer in one file-scope device array instead
// of the mesh's workspace, so that the call allocates nothing (for callers
// that cannot call hipMalloc: code under stream capture, tight serving
// loops).  The kernels are cgd_deposit's tiled path, given addresses inside
// that array.
//
// The array lives once per GPU for the life of the process.  Host code never
// uses its name as an address: the library looks up each device's copy with
// hipGetSymbolAddress on the first call on that device (with the device
// current) and passes that pointer to the kernels.
#include <algorithm>
#include <mutex>
#include <string>

#include "cgd_internal.h"

namespace cgd {
namespace {

// Scratch of the no-allocation deposit: the deposit counters (DepositInfo)
// in the first kInfoBytes, the tiled deposit's buffers after them.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr size_t kInfoBytes = 4096;
static_assert(sizeof(DepositInfo) <= kInfoBytes, "deposit counters fit the head of the scratch");

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (looked up once, with the device current).
cgd_status scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("cgd_deposit_noalloc: device index out of range");
        return CGD_E_INVALID;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error(std::string("cgd_deposit_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
            return CGD_E_HIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CGD_OK;
}

// n = 0: the field (and accumulators) are zero.
__global__ void k_zero_outputs(float* __restrict__ field, long long* __restrict__ acc, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        field[i] = 0.f;
        if (acc) acc[i] = 0;
    }
}

}  // namespace
}  // namespace cgd

using namespace cgd;

extern "C" cgd_status cgd_deposit_noalloc(cgd_mesh m, int64_t n, const float* pos, int32_t F, const float* values,
                                          float* field, int64_t* acc, void* stream) {
    if (!m || F < 1 || F > CGD_MAX_FIELDS || n < 0 || (n > 0 && (!pos || !values)) || !field) {
        set_error("cgd_deposit_noalloc: need a mesh, 1 <= F <= CGD_MAX_FIELDS, n >= 0, pos / values (n > 0) "
                  "and field");
        return CGD_E_INVALID;
    }
    if (m->kind != 0) {
        set_error("cgd_deposit_noalloc: uniform hex meshes only");
        return CGD_E_UNSUPPORTED;
    }
    if (reinterpret_cast<uintptr_t>(acc) % 8 || reinterpret_cast<uintptr_t>(pos) % 4 ||
        reinterpret_cast<uintptr_t>(values) % 4 || reinterpret_cast<uintptr_t>(field) % 4) {
        set_error("cgd_deposit_noalloc: misaligned pointer");
        return CGD_E_INVALID;
    }
    const size_t temp = n > 0 ? deposit_hex_temp_bytes(m, n, F) : 0;
    if (n > 0 && (temp == 0 || temp > kNoAllocBytes - kInfoBytes)) {
        set_error("cgd_deposit_noalloc: " + std::to_string(n) + " particles x " + std::to_string(F) +
                  " fields need " + (temp ? std::to_string(temp) + " bytes of scratch" : std::string("the direct path")) +
                  "; the limit is " + std::to_string(kNoAllocBytes - kInfoBytes) +
                  " bytes (12 bytes per particle at F = 1, 20 at F = 2 or 3, 20 + 4 (F - 3) above) on grids of "
                  "at most 16384 tiles");
        return CGD_E_INVALID;
    }
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cgd_deposit_noalloc: no HIP device");
        return CGD_E_HIP;
    }
    if (prev != m->device && hipSetDevice(m->device) != hipSuccess) {
        (void)hipGetLastError();
        set_error("cgd_deposit_noalloc: cannot make the mesh's device current");
        return CGD_E_HIP;
    }
    void* base = nullptr;
    cgd_status rc = scratch_ptr(m->device, &base);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rc == CGD_OK) {
        if (n == 0) {
            const int64_t total = (int64_t)F * m->cells;
            const int blocks = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (total + 255) / 256));
            hipLaunchKernelGGL(k_zero_outputs, dim3(blocks), dim3(256), 0, s, field,
                               reinterpret_cast<long long*>(acc), total);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) {
                set_error(std::string("cgd_deposit_noalloc: ") + hipGetErrorString(e));
                rc = CGD_E_HIP;
            }
        } else {
            ScaleForce fs;
            for (int f = 0; f < CGD_MAX_FIELDS; ++f) fs.s[f] = -1;
            DepositInfo* info = static_cast<DepositInfo*>(base);
            void* tmp = static_cast<unsigned char*>(base) + kInfoBytes;
            rc = deposit_hex(m, n, pos, F, values, field, acc, info, tmp, fs, nullptr, s);
        }
    }
    if (prev != m->device) (void)hipSetDevice(prev);
    return rc;
}
