// dg_invariants_noalloc: the invariants of dg_invariants_dev without a
// workspace, for callers that cannot allocate device memory.  The kernel's
// reduction scratch (per-block partial sums and the last-block ticket) lives
// in a file-scope device array of fixed size; each device holds its own copy
// for the life of the process.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abi_types.h"
#include "dg_launch.h"

using namespace dgk;

namespace {

// The pointwise reductions launch at most pointwise_block_cap() blocks, each
// publishing up to 4 doubles; the ticket counters (every kind's set, as in a
// workspace) come first, rounded up to 256 bytes.
constexpr int kScratchBlocks = 1024;
constexpr size_t kScratchCounterBytes = (kCntBytes + 255) / 256 * 256;
constexpr size_t kScratchBytes =
    kScratchCounterBytes + (size_t)kScratchBlocks * 4 * sizeof(double);
static_assert(kCntBytes <= kScratchCounterBytes, "ticket counters must fit their slot");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

__global__ void k_clear_counters(unsigned* c, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) c[i] = 0u;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch` on each device

// Device address of this device's scratch array; the first call on a device
// looks it up (the array's name is only a host-side handle) and clears the
// ticket counters on `s`.
int scratch_on(int dev, hipStream_t s, void** out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(DG_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        hipLaunchKernelGGL(k_clear_counters, dim3(1), dim3(256), 0, s, (unsigned*)p,
                           (int)(kCntBytes / sizeof(unsigned)));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "scratch counter clear launch");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return DG_OK;
}

}  // namespace

extern "C" {

int dg_invariants_noalloc(const dg_grid* g, const double* omega, const double* psi,
                          double* out_dev3, void* stream) {
    if (!g || !omega || !psi || !out_dev3) return fail(DG_E_INVAL, "NULL argument");
    if (pointwise_block_cap() > kScratchBlocks)
        return fail(DG_E_INVAL, "reduction needs %d blocks, the static scratch holds %d",
                    pointwise_block_cap(), kScratchBlocks);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(DG_E_INVAL, "device %d beyond the %d the static scratch supports",
                    dev, kMaxDevices);
    const hipStream_t s = (hipStream_t)stream;
    void* p = nullptr;
    const int rc = scratch_on(dev, s, &p);
    if (rc != DG_OK) return rc;
    DevScratch d{};
    d.counters = (unsigned*)p;
    d.partials = (double*)((char*)p + kScratchCounterBytes);
    d.max_blocks = kScratchBlocks;
    e = launch_invariants(g->geom, g->k64, omega, psi, out_dev3, d, s);
    if (e != hipSuccess) return hip_fail(e, "invariants launch");
    return DG_OK;
}

}  // extern "C"
