// Streaming stores for outputs written once and read again only after they have left the
// caches (window captures, window transposes): the nontemporal hint keeps them from
// displacing the lines that the same kernel reads.  (The sweeps' own state, and the GEMM
// outputs, measured no faster with it.)  Nontemporal loads for inputs read once (the windows
// the transposes read, the grids of the raster DFTs); the sweeps' state loads measured slower
// with it.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace eels {

__device__ __forceinline__ void st_stream(float2* p, float2 v) {
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), (unsigned long long*)p);
}
__device__ __forceinline__ void st_stream(uint32_t* p, uint32_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(float4* p, float4 v) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(__builtin_bit_cast(v4u, v), (v4u*)p);
}
template <typename V>
__device__ __forceinline__ void st_stream_vec(V* p, V v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ float2 ld_stream(const float2* p) {
    return __builtin_bit_cast(float2, __builtin_nontemporal_load((const unsigned long long*)p));
}

}  // namespace eels
