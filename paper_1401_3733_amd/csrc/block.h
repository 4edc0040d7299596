// Multi-RHS ("block") fields for the batched solver: up to kNR right-hand
// sides stored together so each link load serves all of them.
//
// Block spinor, one parity block: [h][c < d][spin 4][rhs kNR] complex float,
// site stride d * 4 * kNR complex.  A full block field is the even block
// followed by the odd one.  RHS slots beyond n_rhs hold zeros.
// Block links (real adjoint links only): [q][mu][h][i * d + j] float.
#pragma once
#include "bsm_internal.h"

namespace bsm {

constexpr int kNR = 16;   // RHS per block = the N width of one MFMA tile

inline size_t block_site_bytes(int d) { return (size_t)d * 4 * kNR * 8; }
inline size_t block_parity_bytes(const Geom &g, int d) { return block_site_bytes(d) * g.Vh_pad; }
inline size_t block_link_bytes(const Geom &g, int d) { return (size_t)8 * g.Vh_pad * d * d * 4; }

// Site order of the block hops.  Logical site s walks tiles of tt x tz x ty
// lattice rows (full x extent), rows y-fastest inside a tile, tiles in
// (t, z, y) order, so all eight neighbours of a site lie within a few
// hundred sites of it in the walk (a plain half-index walk puts the z and t
// neighbours 2 LX/2 LY and LX/2 LY LZ sites away, beyond what is in flight,
// and re-fetches their 16-RHS blocks).  tt = 0: the plain walk.
struct BlockTile { int tt = 0, tz = 0, ty = 0; };
// largest extents from {6, 4, 3, 2} (t) and {4, 2} (z, y) dividing the
// lattice; tt = 0 when no tiling fits
BlockTile block_tile_for(const Geom &g);
__device__ inline uint32_t block_site(const Geom &g, const BlockTile &b, uint32_t s) {
    if (b.tt == 0) return s;
    const uint32_t row = g.div_xh.div(s), xh = s - row * g.LXh;
    uint32_t r = row;
    const uint32_t yi = r % b.ty; r /= b.ty;
    const uint32_t zi = r % b.tz; r /= b.tz;
    const uint32_t ti = r % b.tt; r /= b.tt;
    const uint32_t nyb = g.L[2] / b.ty, nzb = g.L[3] / b.tz;
    const uint32_t yb = r % nyb; r /= nyb;
    const uint32_t zb = r % nzb, tb = r / nzb;
    const uint32_t t = tb * b.tt + ti, z = zb * b.tz + zi, y = yb * b.ty + yi;
    return ((t * g.L[3] + z) * g.L[2] + y) * g.LXh + xh;
}

struct BlockHopArgs {
    const float *U;          // block links
    const float2 *in[2];     // in[p]: parity block read for output parity p
    const float2 *x[2];
    float2 *out[2];
    float a[kNR], b[kNR];    // out_r = a_r x_r + b_r H in_r
    int use_x;
    int dagger;
    int p0, np;
    double *norm_partials;   // [workgroup][kNR]
    int spw = 1, wpb = 4;    // plan: sites per wavefront, wavefronts per workgroup
    BlockTile tile;          // plan: site order
    int xchunk = 0;          // plan: workgroup run length per XCD (xcd_chunk_remap)
};

bsm_status launch_hop_block(const Geom &g, int d, const BlockHopArgs &a, hipStream_t st);
// a tuned plan into the launch arguments
void apply_block_plan(const Geom &g, const BlockPlan &p, BlockHopArgs &a);
// workgroups (= norm partials) of a launch under its plan
int hop_block_grid(const Geom &g, const BlockHopArgs &a);
// largest partial count of any plan (one site per workgroup), per parity
inline int hop_block_grid_max(const Geom &g) { return g.Vh; }
// time every plan on scratch block fields with the given links and keep the
// fastest in ctx->block_plans[d]
bsm_status block_autotune(bsm_ctx ctx, int d, const float *U_block, float2 *scratch_in, float2 *scratch_out,
                          hipStream_t st);

// FP16 block fields (the batched solver's inner recurrence in F16S): per
// parity block the codes [h][c < d][rhs][spin] half2 (16 bytes per colour and
// RHS: the four spin components), then one float scale per site and RHS
// [h][rhs].  A value is code * scale; scale = max |re|, |im| over the 4 d
// components of that site and RHS, codes = rne_f16(v * (1 / scale)) (the
// per-site F16S quantisation of the single-RHS fields, per RHS).
__host__ __device__ inline size_t blockh_site_bytes(int d) { return (size_t)d * kNR * 16; }
__host__ __device__ inline size_t blockh_scale_off(const Geom &g, int d) { return blockh_site_bytes(d) * g.Vh_pad; }
__host__ __device__ inline size_t blockh_parity_bytes(const Geom &g, int d) { return (blockh_site_bytes(d) + kNR * 4) * g.Vh_pad; }
// FP16 block links: row-major d x kpad halves (kpad = d rounded up to 4,
// zero padded) per (parity, mu, site), in two orientations: [0] U, [1] U^T,
// so that the matrix-core operand of the forward and of the backward hop is
// one 8-byte load of a row either way.  [o][q * 4 + mu][h][i][k], one link
// every blockh_link_halves(d) halves: links of 128 bytes or more start on a
// 128-byte cache line (d = 15: 480 -> 512 bytes), so a streamed link never
// shares a line with the next one.
constexpr int blockh_kpad(int d) { return (d + 3) & ~3; }
__host__ __device__ constexpr int blockh_link_halves(int d) {
    return d * blockh_kpad(d) * 2 < 128 ? d * blockh_kpad(d) : (d * blockh_kpad(d) * 2 + 127) / 128 * 64;
}
inline size_t blockh_link_bytes(const Geom &g, int d) {
    return (size_t)2 * 8 * g.Vh_pad * blockh_link_halves(d) * 2;
}

struct BlockHopHArgs {
    const __half *U;         // FP16 block links
    const char *in[2];       // FP16 parity blocks
    const char *x[2];
    char *out[2];
    float a[kNR], b[kNR];    // out_r = a_r x_r + b_r H in_r
    int use_x;
    int dagger;
    int p0, np;
    double *norm_partials;   // [workgroup][kNR]: |out_r|^2 of the stored (rounded) values
    int wpb = 4;             // plan: wavefronts (= sites) per workgroup
    BlockTile tile;          // plan: site order
    int xchunk = 0;          // plan: workgroup run length per XCD (xcd_chunk_remap)
};
bsm_status launch_hop_blockh(const Geom &g, int d, const BlockHopHArgs &a, hipStream_t st);
int hop_blockh_grid(const Geom &g, const BlockHopHArgs &a);
void apply_blockh_plan(const Geom &g, const BlockPlan &p, BlockHopHArgs &a);
bsm_status blockh_autotune(bsm_ctx ctx, int d, const __half *U_blockh, char *scratch_in, char *scratch_out,
                           hipStream_t st);
// represented links (LP F64 or F32) -> FP16 block links
bsm_status launch_gauge_to_blockh(const Geom &g, int d, int link_prec, const void *U_rep, __half *U_blockh,
                                  hipStream_t st);
// canonical complex128 [n_rhs][V][4][d] <-> FP16 block field (both parities)
bsm_status launch_pack_blockh(const Geom &g, int d, int n_rhs, const void *canon, void *block, bool unpack,
                              hipStream_t st);
// per-RHS vector kernels of the F16S inner recurrence (one parity block):
// p16 = r32 + beta p16 ;  x32 += alpha p16, r32 -= alpha q16 with |r32|^2
// partials [workgroup][kNR] (blockh_blas_grid workgroups)
int blockh_blas_grid(const Geom &g);
bsm_status blockh_xpay(const Geom &g, int d, char *p, const float2 *r, const double *beta, hipStream_t st);
bsm_status blockh_update(const Geom &g, int d, float2 *x, const char *p, float2 *r, const char *q,
                         const double *alpha, double *partials, hipStream_t st);

// FP64 block fields (the batched solver's reliable updates): [h][c][spin][rhs]
// double2, links [q][mu][h][i*d + j] double
inline size_t block64_parity_bytes(const Geom &g, int d) { return (size_t)d * 4 * kNR * 16 * g.Vh_pad; }
inline size_t block64_link_bytes(const Geom &g, int d) { return (size_t)8 * g.Vh_pad * d * d * 8; }

struct BlockHop64Args {
    const double *U;
    const double2 *in[2];
    const double2 *x[2];
    const double2 *y[2];
    double2 *out[2];
    double a[kNR], b[kNR], c[kNR];   // out_r = a_r x_r + b_r H in_r (+ c_r y_r with use_y)
    int use_x, use_y;
    int dagger;
    int p0, np;
    BlockTile tile;          // site order (block_tile_for)
    int xchunk = 0;          // workgroup run length per XCD (xcd_chunk_remap)
};
bsm_status launch_hop_block64(const Geom &g, int d, const BlockHop64Args &a, hipStream_t st);
bsm_status launch_gauge_to_block64(const Geom &g, int d, const void *U_rep64, double *U_block, hipStream_t st);
// mode 0: block = the parity block at std_off of the n_rhs F64 fields (stride std_stride), zero slots beyond;
// mode 1: block32 = (float) block for the RHS selected in sel;
// mode 2: the parity block at std_off of the RHS selected in sel = block (std64 is written)
bsm_status launch_block64_io(const Geom &g, int d, int n_rhs, unsigned sel, const char *std64, size_t std_stride,
                             size_t std_off, double2 *block, float2 *block32, int mode, hipStream_t st);
// per-RHS |v|^2 into dst[16] (device), partials: block64_norm_parts * 16 doubles
bsm_status block64_norms(const Geom &g, int d, const double2 *v, double *partials, double *dst, hipStream_t st);
int block64_norm_parts(const Geom &g, int d);

// layout conversions
bsm_status launch_gauge_to_block(const Geom &g, int d, int link_prec, const void *U_rep, float *U_block,
                                 hipStream_t st);
// canonical complex128 [n_rhs][V][4][d] <-> block (both parities)
bsm_status launch_pack_block(const Geom &g, int d, int n_rhs, const void *canon, void *block, bool unpack,
                             hipStream_t st);
// n_rhs standard F64 fields (per-RHS field stride std_stride, parity block at
// offset std_off) <-> one parity block of a block field, for the RHS whose
// bit is set in sel:
//   mode 0: block = std (RHS slots >= n_rhs are zeroed) ;  mode 1: std += block
bsm_status launch_std_block(const Geom &g, int d, int n_rhs, unsigned sel, char *std64, size_t std_stride,
                            size_t std_off, float2 *block, int mode, hipStream_t st);
// the same for an FP64 block: mode 0 block = std, mode 2 std = block (sites < Vh)
bsm_status launch_block64_std(const Geom &g, int d, int n_rhs, unsigned sel, char *std64, size_t std_stride,
                              size_t std_off, double2 *block, int mode, hipStream_t st);

// per-RHS vector kernels on nblk parity blocks of block fields (F32)
// partials layout [workgroup][kNR]; returns the workgroup count
int block_blas_grid(const Geom &g, int d, int nblk);
bsm_status block_update(const Geom &g, int d, int nblk, float2 *x, const float2 *p, float2 *r,
                        const float2 *q, const double *alpha, double *partials, hipStream_t st);
bsm_status block_xpay(const Geom &g, int d, int nblk, float2 *p, const float2 *r, const double *beta,
                      hipStream_t st);
bsm_status block_norm(const Geom &g, int d, int nblk, const float2 *v, double *partials, hipStream_t st);
// per-RHS scalars: op 0: pAp -> alpha ; op 1: rr_new -> beta, rr, hist ; op 2: rr, hist
// alpha/beta are zero for RHS whose mask entry is 0
// (long partial lists are first summed in parallel into presum, which holds
// kBlockPresum * kNR doubles; nullable)
constexpr int kBlockPresum = 1024;
bsm_status block_scalars(const double *partials, int nparts, double *scal, const int *mask, int op,
                         int hist_slot, double *presum, hipStream_t st);

// device scalar layout for the batched solver (kNR doubles each)
enum { B_RR = 0, B_PAP = 1, B_ALPHA = 2, B_BETA = 3, B_HIST = 4 };
constexpr int kBlockHist = 64;   // history slots (iterations per graph replay)
inline size_t block_scal_doubles() { return (size_t)(B_HIST + kBlockHist) * kNR; }

}  // namespace bsm
