// Achievable-bandwidth calibration: a plain device copy (STREAM "copy") with
// 16-byte accesses.  Its rate is the practical ceiling the hopping kernel is
// compared against, next to the 8 TB/s nominal HBM figure.
#include "bsm_internal.h"

namespace bsm {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                     size_t n) {
    size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        if constexpr (NT) {
            f32x4 v = __builtin_nontemporal_load(src + i);
            __builtin_nontemporal_store(v, dst + i);
        } else {
            dst[i] = src[i];
        }
    }
}

}  // namespace bsm

using namespace bsm;

extern "C" bsm_status bsm_stream_copy(const void *src, void *dst, size_t bytes, int32_t nontemporal,
                                      int32_t blocks, void *stream) {
    if (!src || !dst || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15))
        return fail(BSM_ERR_ARG, "stream_copy needs 16-byte aligned buffers and size");
    if (blocks <= 0) blocks = 256 * 8;
    size_t n = bytes / 16;
    if (nontemporal)
        k_stream_copy<true><<<blocks, 256, 0, (hipStream_t)stream>>>((const f32x4 *)src, (f32x4 *)dst, n);
    else
        k_stream_copy<false><<<blocks, 256, 0, (hipStream_t)stream>>>((const f32x4 *)src, (f32x4 *)dst, n);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}
