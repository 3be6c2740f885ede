// Device-side load/store of FP32 or BF16 storage (oat_dtype 0 / 1).
#ifndef OAT_DTYPE_HPP
#define OAT_DTYPE_HPP

#include <hip/hip_runtime.h>

namespace oat {

__device__ __forceinline__ float load_val(const void *p, size_t i, int dt)
{
    if (dt == 0) return ((const float *)p)[i];
    return __uint_as_float(((unsigned)((const unsigned short *)p)[i]) << 16);
}

// Round-to-nearest-even FP32 -> BF16 (values here are finite).
__device__ __forceinline__ unsigned short to_bf16(float v)
{
    unsigned u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ void store_val(void *p, size_t i, int dt, float v)
{
    if (dt == 0)
        ((float *)p)[i] = v;
    else
        ((unsigned short *)p)[i] = to_bf16(v);
}

}  // namespace oat

#endif  // OAT_DTYPE_HPP
