// Device peak probe: sustained vector fused multiply-add rate, FP64 or FP32 (unpacked), the
// figure against which the pair kernels' arithmetic rates are read.  No SPH state involved.
#include <cstdint>

#include <hip/hip_runtime.h>

#include "../../include/sph.h"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_CHAINS = 8;  // independent chains per thread hide the FMA latency

template <typename T>
__global__ void __launch_bounds__(PROBE_THREADS) k_fma_chains(double* __restrict__ out, int iters) {
    const int64_t i = (int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x;
    T a[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = (T)(1e-3 * (c + 1) + 1e-9 * (double)threadIdx.x);
    const T m = (T)0.9999999, b = (T)1e-7;
#pragma unroll 4
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = fma(a[c], m, b);
    }
    T s = a[0];
#pragma unroll
    for (int c = 1; c < PROBE_CHAINS; ++c) s += a[c];
    out[i] = (double)s;  // keeps every chain live
}

}  // namespace

extern "C" sph_status sph_peak_probe(int32_t kind, double* out_dev, int64_t n_threads, int32_t iters, void* stream) {
    if ((kind != 0 && kind != 1) || !out_dev || n_threads <= 0 || n_threads % PROBE_THREADS != 0 || iters <= 0 ||
        n_threads / PROBE_THREADS > INT32_MAX)
        return SPH_E_ARG;
    const dim3 grid((unsigned)(n_threads / PROBE_THREADS)), block(PROBE_THREADS);
    hipStream_t s = (hipStream_t)stream;
    if (kind == 0) hipLaunchKernelGGL(k_fma_chains<double>, grid, block, 0, s, out_dev, (int)iters);
    else hipLaunchKernelGGL(k_fma_chains<float>, grid, block, 0, s, out_dev, (int)iters);
    return hipGetLastError() == hipSuccess ? SPH_OK : SPH_E_DEVICE;
}
