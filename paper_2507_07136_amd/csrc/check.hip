// Optional validation of the code indices (the LS2_CHECK mode).
//
// By default the compositing kernels take a code index modulo L (L is a power
// of two), so an index outside [0, L) can never address memory outside the
// pixel's L accumulators, but it silently lands on another atom.  With the
// environment variable LS2_CHECK=1 (or ls2_set_check(1)) every entry point
// that reads topk_idx first scans it on the device and returns LS2_ERR_ARG if
// any index lies outside [0, L).  The scan synchronises the stream once, so
// the mode is for debugging and cannot be used under stream capture.
#include <atomic>
#include <cstdlib>
#include <mutex>

#include "ls2_internal.h"

namespace ls2 {

// One flag word per device; every checking call on a device shares it, so
// concurrent checking calls on one device race (the mode is for debugging).
static __device__ __align__(256) unsigned g_bad_index[1];

namespace {

std::atomic<int> g_check{-1};  // -1: not read from the environment yet

constexpr int kMaxDevices = 64;
unsigned* g_flag_ptr[kMaxDevices] = {};
std::mutex g_flag_mu;

unsigned* flag_ptr() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_flag_mu);
    if (!g_flag_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_bad_index)) != hipSuccess) return nullptr;
        g_flag_ptr[dev] = static_cast<unsigned*>(p);
    }
    return g_flag_ptr[dev];
}

}  // namespace

__global__ __launch_bounds__(64) void k_check_clear(unsigned* flag) {
    if (threadIdx.x == 0) flag[0] = 0u;
}

__global__ __launch_bounds__(256) void k_check_indices(long long count, int L, const int* __restrict__ idx,
                                                       unsigned* __restrict__ flag) {
    bool bad = false;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x)
        bad |= idx[i] < 0 || idx[i] >= L;
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

bool check_mode() {
    int v = g_check.load(std::memory_order_relaxed);
    if (v < 0) {
        const char* e = std::getenv("LS2_CHECK");
        v = (e && e[0] && !(e[0] == '0' && e[1] == 0)) ? 1 : 0;
        int expected = -1;
        g_check.compare_exchange_strong(expected, v);
        v = g_check.load(std::memory_order_relaxed);
    }
    return v == 1;
}

int check_code_indices(long long count, int L, const int32_t* topk_idx, hipStream_t stream) {
    if (!check_mode() || count <= 0) return LS2_OK;
    unsigned* flag = flag_ptr();
    if (!flag) return LS2_ERR_DEVICE;
    hipLaunchKernelGGL(k_check_clear, dim3(1), dim3(64), 0, stream, flag);
    LS2_LAUNCH_CHECK();
    const long long want = (count + 255) / 256;
    const unsigned grid = (unsigned)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_check_indices, dim3(grid), dim3(256), 0, stream, count, L, topk_idx, flag);
    LS2_LAUNCH_CHECK();
    unsigned host = 0;
    if (hipMemcpyAsync(&host, flag, sizeof(unsigned), hipMemcpyDeviceToHost, stream) != hipSuccess)
        return LS2_ERR_DEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return LS2_ERR_DEVICE;
    return host ? LS2_ERR_ARG : LS2_OK;
}

}  // namespace ls2

extern "C" int ls2_set_check(int enabled) {
    const int prev = ls2::check_mode() ? 1 : 0;
    ls2::g_check.store(enabled ? 1 : 0);
    return prev;
}
