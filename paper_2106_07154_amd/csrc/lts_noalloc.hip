// The surrogate's weight-gradient product P = A^T D on device buffers with
// no allocation: the per-block partials of the ordered reduction live in one
// fixed device array of this file instead of memory the library allocates.
// The kernels are the ones lts_nn_gemm_tn_bf16 runs (lts_mpnn.hip), with the
// same row partition, so both entry points produce the same bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lts_mpnn.h"
#include "lts_surrogate.h"

namespace {

// Capacity of the partial buffer.  Each GPU the library runs on holds its own
// copy until the process ends.
constexpr size_t kScratchBytes = size_t(1) << 24;

static __device__ __align__(256) float scratch[kScratchBytes / sizeof(float)];

// Device address of `scratch` per device, looked up once per device with that
// device current.  In host code the array's name is not a device address.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_scratch[kMaxDevices] = {};

lts_status scratch_for_current_device(float** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LTS_EDEVICE;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LTS_EDEVICE;
        g_scratch[dev] = static_cast<float*>(p);
    }
    *out = g_scratch[dev];
    return LTS_OK;
}

// P = 0 for an empty product (a kernel, not a memset node, so the call can be
// recorded into a graph).
__global__ void k_zero(float* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

}  // namespace

extern "C" {

long long lts_nn_gemm_tn_noalloc_max_rows(int K) {
    if (K < 16 || K > 128 || K % 16) return 0;
    const long long parts = (long long)(kScratchBytes / ((size_t)K * 64 * sizeof(float)));
    return parts * lts::nn::kReduceRows;
}

lts_status lts_nn_gemm_tn_bf16_device_noalloc(const uint16_t* A, int N, int K, const uint16_t* D,
                                              float* P, void* stream) {
    if (N < 0 || K < 16 || K > 128 || K % 16 || !P) return LTS_EINVAL;
    if (N > 0 && (!A || !D)) return LTS_EINVAL;
    if ((long long)N > lts_nn_gemm_tn_noalloc_max_rows(K)) return LTS_EINVAL;
    float* part = nullptr;
    lts_status st = scratch_for_current_device(&part);
    if (st != LTS_OK) return st;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    if (N == 0) {
        hipLaunchKernelGGL(k_zero, dim3((K * 64 + 255) / 256), dim3(256), 0, s, P, K * 64);
    } else {
        // every partial the reduction reads is written first by the product
        lts::nn::gemm_tn(A, K, N, K, D, lts::nn::kReduceRows, part, P, s);
    }
    return hipGetLastError() == hipSuccess ? LTS_OK : LTS_EDEVICE;
}

}  // extern "C"
