// Map arithmetic after the contraction, and the content hash of device inputs.
//
//   eels_map_mean   the frozen-phonon map: the mean of the maps of several thermal
//                   configurations (the Results' nanoparticle discussion counts one frozen-
//                   phonon pass per configuration; the map is their average), summed in FP64
//                   in configuration order, so it does not depend on the launch shape;
//   eels_map_ratio  the BF-corrected map: the EELS map divided by the incoherent bright-field
//                   image of the EELS detector's angles (Results, nanoparticle discussion);
//   device_hash64   a 64-bit hash of a device buffer (the serving layer's residency key).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "eels.h"
#include "internal.h"

namespace eels {

namespace {

__global__ void k_map_mean(double* __restrict__ out, const double* __restrict__ maps, int n_maps, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < n_maps; ++c) s += maps[(int64_t)c * n + i];
    out[i] = s / (double)n_maps;
}

__global__ void k_map_ratio(double* __restrict__ out, const double* __restrict__ num, const double* __restrict__ den,
                            int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = den[i];
    out[i] = d > 0.0 ? num[i] / d : 0.0;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {   // the splitmix64 finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// sum over 32-bit words w_i of mix64(i * golden + w_i) (mod 2^64): order-independent, so the
// block sums can be added in any order and the result is the same every time
__global__ __launch_bounds__(256) void k_hash64(unsigned long long* __restrict__ out, const uint32_t* __restrict__ w,
                                                int64_t n) {
    __shared__ unsigned long long red[256];
    unsigned long long s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s += mix64((uint64_t)i * 0x9E3779B97F4A7C15ull + w[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, red[0]);
}

__global__ void k_zero64(unsigned long long* p) { *p = 0ull; }

}  // namespace

eels_status device_hash64(const void* d_ptr, size_t bytes, uint64_t* d_scratch, uint64_t* out, hipStream_t st) {
    if (!d_scratch || !out) return EELS_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_zero64, dim3(1), dim3(1), 0, st, (unsigned long long*)d_scratch);
    const int64_t n = (int64_t)(bytes / 4);
    if (n > 0 && d_ptr)
        hipLaunchKernelGGL(k_hash64, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, st,
                           (unsigned long long*)d_scratch, (const uint32_t*)d_ptr, n);
    if (hipMemcpyAsync(out, d_scratch, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("device hash failed");
        return EELS_ERR_DEVICE;
    }
    *out ^= (uint64_t)bytes * 0xD6E8FEB86659FD93ull;
    return EELS_OK;
}

}  // namespace eels

extern "C" {

eels_status eels_map_mean(double* d_out, const double* d_maps, int n_maps, int64_t n, void* stream) {
    if (!d_out || !d_maps || n_maps < 1 || n < 0) return EELS_ERR_INVALID_ARG;
    if (n == 0) return EELS_OK;
    hipLaunchKernelGGL(eels::k_map_mean, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, d_out,
                       d_maps, n_maps, n);
    if (hipGetLastError() != hipSuccess) {
        eels::set_error("map mean launch failed");
        return EELS_ERR_DEVICE;
    }
    return EELS_OK;
}

eels_status eels_map_ratio(double* d_out, const double* d_num, const double* d_den, int64_t n, void* stream) {
    if (!d_out || !d_num || !d_den || n < 0) return EELS_ERR_INVALID_ARG;
    if (n == 0) return EELS_OK;
    hipLaunchKernelGGL(eels::k_map_ratio, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       d_out, d_num, d_den, n);
    if (hipGetLastError() != hipSuccess) {
        eels::set_error("map ratio launch failed");
        return EELS_ERR_DEVICE;
    }
    return EELS_OK;
}

}  // extern "C"
