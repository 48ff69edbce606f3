// Allocation-free observables: lll_observables_noalloc.
//
// The same two kernels as lll_observables (per-block fp64 partials, then one
// block that reduces them in block order), with everything they need besides
// the caller's state and output held in one file-scope device array: the
// replica descriptor, the block-to-replica table and the partials.  The
// array's device address is looked up once per device with
// hipGetSymbolAddress; host code never passes the array's name itself.  No
// hipMalloc, hipFree, hipMemset or host-to-device copy is issued, so the call
// can be captured into a HIP graph: the descriptor and the table are written
// by a small kernel that takes the descriptor as a by-value argument.
#include <mutex>

#include "../../include/lll.h"
#include "lll_internal.hpp"

namespace lll {

// Layout of the scratch array (byte offsets, each 256-aligned).
constexpr int kNoallocMaxBlocks = 2048;  // the observables pass uses at most this many blocks
constexpr size_t kNoallocRepOff = 0;
constexpr size_t kNoallocTabOff = 256;
constexpr size_t kNoallocPartOff = kNoallocTabOff + sizeof(int32_t) * kNoallocMaxBlocks;
constexpr size_t kNoallocBytes = kNoallocPartOff + sizeof(double) * 8 * kNoallocMaxBlocks;
static_assert(sizeof(RepDev) <= kNoallocTabOff, "descriptor slot");
static_assert(kNoallocPartOff % 256 == 0, "partials alignment");

// 139,520 bytes per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

__global__ void __launch_bounds__(256) noalloc_setup_kernel(RepDev R, unsigned char* base, int nob) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<RepDev*>(base + kNoallocRepOff) = R;
    int32_t* tab = reinterpret_cast<int32_t*>(base + kNoallocTabOff);
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nob; b += gridDim.x * blockDim.x)
        tab[b] = 0;
}

}  // namespace lll

using namespace lll;

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array (looked up once
// per device, with that device current).
hipError_t scratch_of_current_device(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return hipSuccess;
}

}  // namespace

// Shared with lll_api.hip: parameter checks and the replica descriptor.
lll_status noalloc_describe(int32_t Lx, int32_t Ly, int32_t Lz, lll_bc bc, const lll_params* p,
                            RepDev* R, int* anis);
lll_status noalloc_error(lll_status s, const char* msg, int code);

extern "C" lll_status lll_observables_noalloc(int32_t Lx, int32_t Ly, int32_t Lz, lll_bc bc,
                                              lll_precision prec, const lll_params* params,
                                              const void* sx, const void* sy, const void* sz,
                                              double* out_dev, void* hip_stream) {
    if (!sx || !sy || !sz || !out_dev)
        return noalloc_error(LLL_EINVAL, "NULL state or output pointer", 0);
    if (prec != LLL_FP64 && prec != LLL_FP32) return noalloc_error(LLL_EINVAL, "bad precision", 0);
    RepDev R;
    int anis = 0;
    lll_status s = noalloc_describe(Lx, Ly, Lz, bc, params, &R, &anis);
    if (s != LLL_OK) return s;
    const int64_t items = obs_item_count(Lx, Ly, Lz);
    const int nob = (int)(items < kNoallocMaxBlocks ? items : kNoallocMaxBlocks);
    if (nob < 1 || nob > kNoallocMaxBlocks)
        return noalloc_error(LLL_EINVAL, "observables blocks exceed the scratch array", nob);
    R.off = 0;
    R.ob0 = 0;
    R.nob = nob;
    unsigned char* base = nullptr;
    hipError_t e = scratch_of_current_device(&base);
    if (e != hipSuccess) return noalloc_error(LLL_EDEVICE, "hipGetSymbolAddress(scratch)", (int)e);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(noalloc_setup_kernel, dim3((nob + 255) / 256), dim3(256), 0, st, R, base, nob);
    if ((e = hipGetLastError()) != hipSuccess)
        return noalloc_error(LLL_EDEVICE, "setup launch", (int)e);
    const RepDev* reps = reinterpret_cast<const RepDev*>(base + kNoallocRepOff);
    const int32_t* tab = reinterpret_cast<const int32_t*>(base + kNoallocTabOff);
    double* part = reinterpret_cast<double*>(base + kNoallocPartOff);
    State S{const_cast<void*>(sx), const_cast<void*>(sy), const_cast<void*>(sz)};
    e = launch_obs(prec == LLL_FP64 ? 0 : 1, anis, reps, tab, nob, 1, S, part, out_dev, nullptr, 0,
                   st);
    if (e != hipSuccess) return noalloc_error(LLL_EDEVICE, "observables launch", (int)e);
    return LLL_OK;
}
