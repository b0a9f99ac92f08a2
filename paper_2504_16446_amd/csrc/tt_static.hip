// Library-owned scratch for tt_loss_grad_noalloc: one fixed-size device
// array per GPU, reserved when the library's code object is loaded there and
// held until the process ends.  Host code never passes `scratch` itself to a
// kernel (in host code the name denotes a host-side stand-in); it uses the
// device address looked up once per device with hipGetSymbolAddress.
#include <mutex>

#include "tt_device.h"
#include "tt_internal.h"

namespace tt {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;  // the caller makes `device` current
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        g_err[device] = e;
        g_done[device] = true;
    }
    return g_err[device];
}

void *static_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_done[device] ? g_ptr[device] : nullptr;
}

// p[0 .. n4) = 0 (a fill kernel rather than a memset node, so that a caller
// may capture the entry point in a graph)
__global__ __launch_bounds__(256) void k_zero4(float4 *__restrict__ p, long long n4)
{
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n4; i += (long long)gridDim.x * 256)
        p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st)
{
    if (bytes % 16 || reinterpret_cast<uintptr_t>(p) % 16) return hipErrorInvalidValue;
    const long long n4 = (long long)(bytes / 16);
    if (n4 == 0) return hipSuccess;
    const int grid = (int)std::min<long long>((n4 + 255) / 256, 8192);
    hipLaunchKernelGGL(k_zero4, dim3(grid), dim3(256), 0, st, reinterpret_cast<float4 *>(p), n4);
    return hipGetLastError();
}

}  // namespace tt
