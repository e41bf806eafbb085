// Operator application that allocates nothing: the contribution slots that
// nnmg_vmult keeps in the level's own buffer live here in one statically
// sized device array per GPU instead.  For callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc).
//
// The array is a file-scope __device__ object: every GPU the library runs on
// holds its own copy, at its own address, from the loading of the code object
// until the process ends.  Host code never passes the array's name to a
// kernel (on the host it names a stand-in, not device memory); it asks the
// runtime for the device address once per device, at context creation with
// that device current, and uses that address from then on.
//
// Every call on one GPU shares that GPU's array, which keeps the last call's
// contents.  The operator kernel writes every slot the gather reads (each
// unconstrained, unmerged (cell, node) pair owns exactly one slot), so nothing
// has to start at zero.  Calls that overlap on one GPU (different streams or
// threads without ordering) race on the array.
#include <mutex>

#include "../internal.hpp"
#include "common.hpp"

namespace nnmg {

static __device__ __align__(256) double scratch[kNoallocScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_ptr[kMaxDevices] = {};
}  // namespace

void* noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) fail(NNMG_ERR_UNSUPPORTED, "device index too large for the static scratch table");
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[device]) {
        int cur = -1;
        NNMG_HIP(hipGetDevice(&cur));
        if (cur != device) fail(NNMG_ERR_INVALID_ARG, "static scratch: the device must be current");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(NNMG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[device] = p;
    }
    return g_ptr[device];
}

void vmult_noalloc(const Level& L, int prec, const void* src, void* dst, void* scratch_dev, hipStream_t s) {
    if (!scratch_dev) fail(NNMG_ERR_INVALID_ARG, "static scratch not initialised for this device");
    const size_t word = prec == NNMG_FP64 ? 8 : 4;
    const size_t need = L.contrib_len * (size_t)L.ncomp * word;
    if (need > kNoallocScratchBytes)
        fail(NNMG_ERR_UNSUPPORTED, "nnmg_vmult_noalloc: the level needs " + std::to_string(need) +
                                       " bytes of contribution slots in this precision; the static scratch holds " +
                                       std::to_string(kNoallocScratchBytes) + " (use nnmg_vmult)");
    // the same kernels as nnmg_vmult's slot path, with the slots in the static
    // array: cell kernel, gather into dst (every unconstrained value has
    // slots, so it writes all of them), identity on constrained rows
    launch_vmult_contrib(L, prec, src, scratch_dev, s, 1);
    launch_gather(L, prec, scratch_dev, dst, false, s, 1);
    launch_copy_constrained(L.d_constrained.ptr, L.constrained_idx.size(), src, dst, prec, s, 1);
}

}  // namespace nnmg
