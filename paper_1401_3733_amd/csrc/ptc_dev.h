// Device helpers shared by the network kernels: the transport T_p of one
// F32 spinor along a path p in {stay, +mu (1..4), -mu (5..8)}.
#pragma once
#include "dispatch.h"
#include "spinor_io.h"

namespace bsm {

typedef float f4v __attribute__((ext_vector_type(4)));

// t = (T_p v)(x) for the site (p_x, h) with coordinates c
template <int D>
__device__ inline void transport(const Geom &g, const char *U, size_t lblk, const char *v_full, size_t pblk,
                                 int px, uint32_t h, const Coords &c, int path, cx<float> (&t)[4 * D]) {
    if (path == 0) {
        load_spinor<BSM_F32, D, float>(v_full + px * pblk, g.Vh_pad, h, t);
        return;
    }
    const int mu = (path - 1) & 3;
    const bool back = path > 4;
    float w;
    uint32_t hn;
    switch (mu) {
    case 0: hn = neighbour<0>(g, c, back, w); break;
    case 1: hn = neighbour<1>(g, c, back, w); break;
    case 2: hn = neighbour<2>(g, c, back, w); break;
    default: hn = neighbour<3>(g, c, back, w); break;
    }
    cx<float> s[4 * D];
    load_spinor<BSM_F32, D, float>(v_full + (1 - px) * pblk, g.Vh_pad, hn, s);
    const char *blk = U + (size_t)((back ? 1 - px : px) * 4 + mu) * lblk;
    const uint32_t hl = back ? hn : h;
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int i = 0; i < D; i++) t[a * D + i] = mk<float>(0.f, 0.f);
#pragma unroll
    for (int i = 0; i < D; i++)
#pragma unroll
        for (int j = 0; j < D; j++) {
            const cx<float> u = load_link<BSM_F32, false, float>(blk, g.Vh_pad, i * D + j, hl);
#pragma unroll
            for (int a = 0; a < 4; a++) {
                if (!back) t[a * D + i] = cfma(u, s[a * D + j], t[a * D + i]);
                else t[a * D + j] = cfma_conj(u, s[a * D + i], t[a * D + j]);
            }
        }
#pragma unroll
    for (int k = 0; k < 4 * D; k++) t[k] = w * t[k];
}

// geometry of path p >= 1 at site (px, h): source half index, boundary
// factor, link block and the half index of the link
struct PathSite {
    uint32_t hn, hl;
    float w;
    const char *blk;
    bool back;
};

__device__ inline PathSite path_site(const Geom &g, const char *U, size_t lblk, int px, uint32_t h,
                                     const Coords &c, int path) {
    PathSite ps;
    const int mu = (path - 1) & 3;
    ps.back = path > 4;
    switch (mu) {
    case 0: ps.hn = neighbour<0>(g, c, ps.back, ps.w); break;
    case 1: ps.hn = neighbour<1>(g, c, ps.back, ps.w); break;
    case 2: ps.hn = neighbour<2>(g, c, ps.back, ps.w); break;
    default: ps.hn = neighbour<3>(g, c, ps.back, ps.w); break;
    }
    ps.blk = U + (size_t)((ps.back ? 1 - px : px) * 4 + mu) * lblk;
    ps.hl = ps.back ? ps.hn : h;
    return ps;
}

}  // namespace bsm
