// The full-lattice Wilson operator out = a in + b H in (both parities) in one
// pass that reads most links once.
//
// Applied parity by parity, every link U_mu(x) is read twice: as the forward
// link of x and as the backward link of x + mu, in the other pass.  Here one
// thread owns the sites of an (x, y, z) column over TC consecutive time
// slices (both parities, one slice after the other), and the lanes of a
// wavefront cover R = 64 / LX whole x-rows of the same z and time slice:
//   t: the thread's own U_t(x, t) serves the forward hop of (x, t) and, with
//      the projected spinor of (x, t), gives the backward term of (x, t+1),
//      carried in registers to the next slice; psi(x, t+1) is loaded once and
//      is the own spinor of the next slice;
//   x: lane x forms P psi(x) for the forward hop of x - 1 and U_x(x)^dag
//      P psi(x) for the backward hop of x + 1; both travel by cross-lane
//      shuffle, so U_x and the x-neighbour spinors are read once;
//   y: the same between the rows of a wavefront; the first row loads its
//      backward neighbour and link, the last row its forward neighbour;
//   z: both neighbours and the backward link are loaded (the general hop).
// Links read per site: t 1, x 1, y 1 + 1/R, z 2 (against 8).
#include "dphi.h"
#include "hop.h"

namespace bsm {

template <class T>
__device__ inline cx<T> shfl_cx(cx<T> v, int src) {
    return mk<T>(__shfl(v.re, src, 64), __shfl(v.im, src, 64));
}

template <int D, class T>
__device__ inline void shfl_half(const cx<T> (&a0)[D], const cx<T> (&a1)[D], int src, cx<T> (&b0)[D],
                                 cx<T> (&b1)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) {
        b0[i] = shfl_cx(a0[i], src);
        b1[i] = shfl_cx(a1[i], src);
    }
}

template <int D, class T>
__device__ inline void select_half(bool take_a, const cx<T> (&a0)[D], const cx<T> (&a1)[D], cx<T> (&b0)[D],
                                   cx<T> (&b1)[D]) {
#pragma unroll
    for (int i = 0; i < D; i++) {
        b0[i] = take_a ? a0[i] : b0[i];
        b1[i] = take_a ? a1[i] : b1[i];
    }
}

__device__ inline uint32_t half_index(const Geom &g, int t, int z, int y, int x) {
    return (((uint32_t)t * g.L[3] + z) * g.L[2] + y) * g.LXh + (x >> 1);
}

template <int D, bool REAL, int SP, int LP>
__global__ __launch_bounds__(256) void k_dphi(Geom g, DphiArgs a) {
    using T = typename Compute<SP>::T;
    // streamed links (measured: 228 us per SU(3) FP32 application against
    // 239 us with cached loads, although the y and z links are read twice)
    constexpr bool NT = (BSM_LINK_NT >> SP) & 1;
    using Links = LinkRegs<D, REAL, LP, NT, T>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wpg = blockDim.x >> 6;
    const int LX = g.L[1], R = 64 / LX;
    const int x = lane % LX, r = lane / LX;
    // workgroup -> (y block, z, t chunk)
    const int nyb = g.L[2] / (R * wpg), nzb = g.L[3];
    uint32_t b = blockIdx.x;
    const int yb = b % nyb; b /= nyb;
    const int z = b % nzb;
    const int t0 = (int)(b / nzb) * a.tc;
    const int y = (yb * wpg + wave) * R + r;
    const size_t sblk = spinor_block_bytes(SP, D, g.Vh_pad);
    const size_t lblk = link_block_bytes(LP, REAL, D, g.Vh_pad);
    const char *U = (const char *)a.U;
    const char *in = (const char *)a.in;
    char *out = (char *)a.out;
    const T eta = a.dagger ? (T)-1 : (T)1;
    const int LT = g.L[0], LY = g.L[2];
    // boundary factors of this lane's x and y hops (the antiperiodic sign of a wrapping hop)
    const T wxf = (x == LX - 1 && ((g.apbc >> 1) & 1)) ? (T)-1 : (T)1;
    const T wxb = (x == 0 && ((g.apbc >> 1) & 1)) ? (T)-1 : (T)1;
    const T wyf = (y == LY - 1 && ((g.apbc >> 2) & 1)) ? (T)-1 : (T)1;
    const T wyb = (y == 0 && ((g.apbc >> 2) & 1)) ? (T)-1 : (T)1;
    const int xf_lane = r * LX + (x == LX - 1 ? 0 : x + 1);
    const int xb_lane = r * LX + (x == 0 ? LX - 1 : x - 1);
    const bool y_up_in = r + 1 < R, y_dn_in = r >= 1;
    const int yu_lane = y_up_in ? lane + LX : lane, yd_lane = y_dn_in ? lane - LX : lane;
    // the one y-neighbour a lane may load: below for the first row, above otherwise
    const int ye = r == 0 ? (y == 0 ? LY - 1 : y - 1) : (y == LY - 1 ? 0 : y + 1);

    // own spinor of the first slice, and the carried backward t term from t0 - 1
    int t = t0;
    int p = (t + z + y + x) & 1;
    uint32_t h = half_index(g, t, z, y, x);
    cx<T> s_cur[4 * D];
    load_spinor<SP, D, T>(in + p * sblk, g.Vh_pad, h, s_cur);
    cx<T> cb0[D], cb1[D];
    T wcb;
    {
        const int tp = t == 0 ? LT - 1 : t - 1;
        wcb = (t == 0 && (g.apbc & 1)) ? (T)-1 : (T)1;
        const uint32_t hp = half_index(g, tp, z, y, x);
        cx<T> sp[4 * D];
        load_spinor<SP, D, T>(in + (1 - p) * sblk, g.Vh_pad, hp, sp);
        Links Lp;
        const char *blk = U + (size_t)((1 - p) * 4 + 0) * lblk;
        Lp.load(blk, g.Vh_pad, hp);
        cx<T> h0[D], h1[D];
        project<0, D, T>(sp, -eta, h0, h1);
        link_mul<D, REAL, LP, true, NT, T>(Lp, blk, g.Vh_pad, hp, h0, h1, cb0, cb1);
    }
#pragma unroll 1
    for (int k = 0; k < a.tc; k++, t++) {
        p = (t + z + y + x) & 1;
        h = half_index(g, t, z, y, x);
        const char *inp = in + (1 - p) * sblk;   // neighbours are of the other parity
        cx<T> acc[4 * D];
#pragma unroll
        for (int i = 0; i < 4 * D; i++) acc[i] = mk<T>(0, 0);
        // ---- t: forward with the next slice's own spinor, backward carried
        const int tn = t == LT - 1 ? 0 : t + 1;
        const T wtf = (t == LT - 1 && (g.apbc & 1)) ? (T)-1 : (T)1;
        const uint32_t hn = half_index(g, tn, z, y, x);
        cx<T> s_next[4 * D];
        load_spinor<SP, D, T>(inp, g.Vh_pad, hn, s_next);
        const char *blk_t = U + (size_t)(p * 4 + 0) * lblk;
        Links Lt;
        Lt.load(blk_t, g.Vh_pad, h);
        const char *blk_x = U + (size_t)(p * 4 + 1) * lblk;
        Links Lx;
        Lx.load(blk_x, g.Vh_pad, h);
        const char *blk_y = U + (size_t)(p * 4 + 2) * lblk;
        Links Ly;
        Ly.load(blk_y, g.Vh_pad, h);
        // the y neighbour outside the wavefront, and for the first row its link
        const uint32_t he = half_index(g, t, z, ye, x);
        cx<T> s_e[4 * D];
        load_spinor<SP, D, T>(inp, g.Vh_pad, he, s_e);
        const char *blk_e = r == 0 ? U + (size_t)((1 - p) * 4 + 2) * lblk : blk_y;
        const uint32_t hl_e = r == 0 ? he : h;
        Links Le;
        Le.load(blk_e, g.Vh_pad, hl_e);
        {
            cx<T> h0[D], h1[D], g0[D], g1[D];
            project<0, D, T>(s_next, eta, h0, h1);
            link_mul<D, REAL, LP, false, NT, T>(Lt, blk_t, g.Vh_pad, h, h0, h1, g0, g1);
            reconstruct<0, D, T>(acc, eta, wtf, g0, g1);
            reconstruct<0, D, T>(acc, -eta, wcb, cb0, cb1);
            // carried to the next slice: U_t(x, t)^dag P psi(x, t)
            project<0, D, T>(s_cur, -eta, h0, h1);
            link_mul<D, REAL, LP, true, NT, T>(Lt, blk_t, g.Vh_pad, h, h0, h1, cb0, cb1);
            wcb = wtf;
        }
        // ---- x: both neighbours inside the row
        {
            cx<T> h0[D], h1[D], n0[D], n1[D], g0[D], g1[D];
            project<1, D, T>(s_cur, eta, h0, h1);           // for the forward hop of x - 1
            shfl_half<D, T>(h0, h1, xf_lane, n0, n1);
            link_mul<D, REAL, LP, false, NT, T>(Lx, blk_x, g.Vh_pad, h, n0, n1, g0, g1);
            reconstruct<1, D, T>(acc, eta, wxf, g0, g1);
            project<1, D, T>(s_cur, -eta, h0, h1);          // backward term of x + 1
            link_mul<D, REAL, LP, true, NT, T>(Lx, blk_x, g.Vh_pad, h, h0, h1, g0, g1);
            shfl_half<D, T>(g0, g1, xb_lane, n0, n1);
            reconstruct<1, D, T>(acc, -eta, wxb, n0, n1);
        }
        // ---- y: neighbours in the wavefront's other rows, else loaded
        {
            cx<T> h0[D], h1[D], n0[D], n1[D], e0[D], e1[D], g0[D], g1[D];
            // forward: P psi(y + 1) from the row above, or from the loaded spinor
            project<2, D, T>(s_cur, eta, h0, h1);
            shfl_half<D, T>(h0, h1, yu_lane, n0, n1);
            project<2, D, T>(s_e, eta, e0, e1);
            select_half<D, T>(!y_up_in, e0, e1, n0, n1);
            link_mul<D, REAL, LP, false, NT, T>(Ly, blk_y, g.Vh_pad, h, n0, n1, g0, g1);
            reconstruct<2, D, T>(acc, eta, wyf, g0, g1);
            // backward: U_y(y - 1)^dag P psi(y - 1) from the row below, or formed here
            project<2, D, T>(s_cur, -eta, h0, h1);
            link_mul<D, REAL, LP, true, NT, T>(Ly, blk_y, g.Vh_pad, h, h0, h1, g0, g1);
            shfl_half<D, T>(g0, g1, yd_lane, n0, n1);
            project<2, D, T>(s_e, -eta, e0, e1);
            link_mul<D, REAL, LP, true, NT, T>(Le, blk_e, g.Vh_pad, hl_e, e0, e1, g0, g1);
            select_half<D, T>(!y_dn_in, g0, g1, n0, n1);
            reconstruct<2, D, T>(acc, -eta, wyb, n0, n1);
        }
        // ---- z: both neighbours and the backward link loaded
#pragma unroll
        for (int dir = 0; dir < 2; dir++) {
            const bool back = dir == 1;
            const int zn = back ? (z == 0 ? g.L[3] - 1 : z - 1) : (z == g.L[3] - 1 ? 0 : z + 1);
            const bool wrap = back ? z == 0 : z == g.L[3] - 1;
            const T wz = (wrap && ((g.apbc >> 3) & 1)) ? (T)-1 : (T)1;
            const uint32_t hz = half_index(g, t, zn, y, x);
            cx<T> sz[4 * D];
            load_spinor<SP, D, T>(inp, g.Vh_pad, hz, sz);
            const char *blk_z = U + (size_t)((back ? 1 - p : p) * 4 + 3) * lblk;
            const uint32_t hl = back ? hz : h;
            Links Lz;
            Lz.load(blk_z, g.Vh_pad, hl);
            const T sg = back ? -eta : eta;
            cx<T> h0[D], h1[D], g0[D], g1[D];
            project<3, D, T>(sz, sg, h0, h1);
            if (!back) link_mul<D, REAL, LP, false, NT, T>(Lz, blk_z, g.Vh_pad, hl, h0, h1, g0, g1);
            else link_mul<D, REAL, LP, true, NT, T>(Lz, blk_z, g.Vh_pad, hl, h0, h1, g0, g1);
            if (!back) reconstruct<3, D, T>(acc, sg, wz, g0, g1);
            else reconstruct<3, D, T>(acc, sg, wz, g0, g1);
        }
        // ---- out = a psi + b H psi
        cx<T> res[4 * D];
#pragma unroll
        for (int i = 0; i < 4 * D; i++)
            res[i] = mk<T>(fma((T)a.b, acc[i].re, (T)a.a * s_cur[i].re), fma((T)a.b, acc[i].im, (T)a.a * s_cur[i].im));
        store_spinor_nt<SP, D, T>(out + p * sblk, g.Vh_pad, h, res);
#pragma unroll
        for (int i = 0; i < 4 * D; i++) s_cur[i] = s_next[i];
    }
}


bool dphi_fits(const Geom &g) {
    const int LX = g.L[1];
    if (LX < 2 || LX > 32 || 64 % LX != 0) return false;   // whole rows, at least two per wavefront
    const int R = 64 / LX;
    return g.L[2] % R == 0;
}

static int dphi_waves(const Geom &g) {
    const int rows = g.L[2] / (64 / g.L[1]);
    return rows % 4 == 0 ? 4 : rows % 2 == 0 ? 2 : 1;
}

// Time slices each thread marches over: the longer the march, the fewer
// chunk starts (each reloads the backward t term), but the grid must keep
// two workgroups per CU; 32^3 x 64 SU(3) FP32: 16 slices 228 us, 4 slices
// 235 us, 32 slices 227 us (SU(2): 126, 133 and 147 us).
int dphi_tchunk(const Geom &g) {
    if (!dphi_fits(g)) return 1;
    const int64_t cols = (int64_t)(g.L[2] / ((64 / g.L[1]) * dphi_waves(g))) * g.L[3];
    for (int tc : {16, 8})
        if (g.L[0] % tc == 0 && cols * (g.L[0] / tc) >= 2 * 256) return tc;
    for (int tc : {4, 2, 1})
        if (g.L[0] % tc == 0) return tc;
    return 1;
}

template <int SP, int LP>
struct DphiSel {
    template <int D>
    struct ByD {
        static bsm_status run(const Geom &g, bool real, const DphiArgs &a, hipStream_t st) {
            if constexpr (dphi_compiled(SP, D)) {
                const int wpg = dphi_waves(g);
                const int R = 64 / g.L[1];
                const unsigned grid = (unsigned)(g.L[2] / (R * wpg) * g.L[3] * (g.L[0] / a.tc));
                if (real) k_dphi<D, true, SP, LP><<<grid, 64 * wpg, 0, st>>>(g, a);
                else k_dphi<D, false, SP, LP><<<grid, 64 * wpg, 0, st>>>(g, a);
                BSM_HIP(hipGetLastError());
                return BSM_OK;
            }
            return fail(BSM_ERR_UNSUPPORTED, "one-pass D_W not compiled for this d_R and precision");
        }
    };
};

bsm_status launch_dphi(const Geom &g, int d, bool real, int prec, int link_prec, const DphiArgs &a,
                       hipStream_t st) {
    if (!dphi_fits(g) || a.tc < 1 || g.L[0] % a.tc) return fail(BSM_ERR_ARG, "one-pass D_W: lattice does not fit");
    if (prec == BSM_F32 && link_prec == BSM_F32)
        return dispatch_d<DphiSel<BSM_F32, BSM_F32>::ByD>(d, g, real, a, st);
    return fail(BSM_ERR_UNSUPPORTED, "one-pass D_W: F32 fields and links only");
}

}  // namespace bsm
