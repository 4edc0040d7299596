// Achievable-bandwidth calibration: a plain device copy (STREAM "copy") and
// a read-only sweep with 16-byte accesses.  Their rates are the practical
// ceilings the hopping kernel is compared against (it is ~90 % reads), next
// to the 8 TB/s nominal HBM figure.
#include "bsm_internal.h"

namespace bsm {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Workgroup b sweeps its own contiguous chunk of the buffer (its 256
// threads on consecutive 16-byte elements), each thread keeping kCopyUnroll
// loads in flight before it stores: all workgroups streaming through one
// buffer-wide stride pattern in lockstep was measured slower.
constexpr int kCopyUnroll = 4;

__device__ inline void chunk_of(size_t n, size_t &lo, size_t &hi) {
    const size_t per = (n + gridDim.x - 1) / gridDim.x;
    lo = (size_t)blockIdx.x * per;
    hi = lo + per < n ? lo + per : n;
}

template <bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(const f32x4 *__restrict__ src, f32x4 *__restrict__ dst,
                                                     size_t n) {
    size_t lo, hi;
    chunk_of(n, lo, hi);
    size_t i = lo + threadIdx.x;
    for (; i + (kCopyUnroll - 1) * 256 < hi; i += kCopyUnroll * 256) {
        f32x4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++)
            v[u] = NT ? __builtin_nontemporal_load(src + i + u * 256) : src[i + u * 256];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) {
            if constexpr (NT) __builtin_nontemporal_store(v[u], dst + i + u * 256);
            else dst[i + u * 256] = v[u];
        }
    }
    for (; i < hi; i += 256) dst[i] = src[i];
}

// STREAM-style read: every 16-byte element is loaded once and folded into a
// per-workgroup value (written to out[blockIdx.x] so the loads are kept).
// With as many workgroups as 256-element chunks each thread loads one
// element, the shape that reads fastest on this GPU (measured: 6.6 TB/s
// with ordinary loads, 6.9 with streaming ones, against 6.0 for a few
// thousand workgroups looping over long chunks).
template <bool NT>
__global__ __launch_bounds__(256) void k_stream_read(const f32x4 *__restrict__ src, size_t n, float *out) {
    size_t lo, hi;
    chunk_of(n, lo, hi);
    size_t i = lo + threadIdx.x;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (; i + (kCopyUnroll - 1) * 256 < hi; i += kCopyUnroll * 256) {
        f32x4 v[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) v[u] = NT ? __builtin_nontemporal_load(src + i + u * 256) : src[i + u * 256];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) acc += v[u];
    }
    for (; i < hi; i += 256) acc += NT ? __builtin_nontemporal_load(src + i) : src[i];
    float s = acc[0] + acc[1] + acc[2] + acc[3];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __shared__ float ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
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

extern "C" bsm_status bsm_stream_read(const void *src, size_t bytes, int32_t nontemporal, int32_t blocks, float *out,
                                      void *stream) {
    if (!src || !out || (bytes & 15) || ((uintptr_t)src & 15))
        return fail(BSM_ERR_ARG, "stream_read needs a 16-byte aligned buffer and size");
    if (blocks <= 0) blocks = 256 * 8;
    if (nontemporal)
        k_stream_read<true><<<blocks, 256, 0, (hipStream_t)stream>>>((const f32x4 *)src, bytes / 16, out);
    else
        k_stream_read<false><<<blocks, 256, 0, (hipStream_t)stream>>>((const f32x4 *)src, bytes / 16, out);
    BSM_HIP(hipGetLastError());
    return BSM_OK;
}
