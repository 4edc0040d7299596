// Spin projection and reconstruction of the 16-RHS block hops, shared by the
// FP32 and FP16 block kernels: one lane holds one RHS (column of the matrix
// core tile) and four colour rows of the result.
#pragma once
#include "bsm_internal.h"

namespace bsm {

typedef float f4 __attribute__((ext_vector_type(4)));

template <int MU>
__device__ inline void project_c(const float2 (&s)[4], float sg, float2 &h0, float2 &h1) {
    const float2 s0 = s[0], s1 = s[1], s2 = s[2], s3 = s[3];
    if constexpr (MU == 0) {
        h0 = make_float2(fmaf(-sg, s2.x, s0.x), fmaf(-sg, s2.y, s0.y));
        h1 = make_float2(fmaf(-sg, s3.x, s1.x), fmaf(-sg, s3.y, s1.y));
    } else if constexpr (MU == 1) {
        h0 = make_float2(fmaf(-sg, s3.y, s0.x), fmaf(sg, s3.x, s0.y));
        h1 = make_float2(fmaf(-sg, s2.y, s1.x), fmaf(sg, s2.x, s1.y));
    } else if constexpr (MU == 2) {
        h0 = make_float2(fmaf(sg, s3.x, s0.x), fmaf(sg, s3.y, s0.y));
        h1 = make_float2(fmaf(-sg, s2.x, s1.x), fmaf(-sg, s2.y, s1.y));
    } else {
        h0 = make_float2(fmaf(-sg, s2.y, s0.x), fmaf(sg, s2.x, s0.y));
        h1 = make_float2(fmaf(sg, s3.y, s1.x), fmaf(-sg, s3.x, s1.y));
    }
}

// acc[spin][re/im] (rows 4q+v of colour) += hop contribution from G = U h
template <int MU>
__device__ inline void reconstruct_c(f4 (&acc)[4][2], float sg, float w, f4 g0r, f4 g0i, f4 g1r, f4 g1i) {
    const float v = -sg * w;
    acc[0][0] += w * g0r; acc[0][1] += w * g0i;
    acc[1][0] += w * g1r; acc[1][1] += w * g1i;
    if constexpr (MU == 0) {          // A^dag g = (g0, g1)
        acc[2][0] += v * g0r; acc[2][1] += v * g0i;
        acc[3][0] += v * g1r; acc[3][1] += v * g1i;
    } else if constexpr (MU == 1) {   // (i g1, i g0)
        acc[2][0] -= v * g1i; acc[2][1] += v * g1r;
        acc[3][0] -= v * g0i; acc[3][1] += v * g0r;
    } else if constexpr (MU == 2) {   // (g1, -g0)
        acc[2][0] += v * g1r; acc[2][1] += v * g1i;
        acc[3][0] -= v * g0r; acc[3][1] -= v * g0i;
    } else {                          // (i g0, -i g1)
        acc[2][0] -= v * g0i; acc[2][1] += v * g0r;
        acc[3][0] += v * g1i; acc[3][1] -= v * g1r;
    }
}

}  // namespace bsm
