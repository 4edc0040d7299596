// C ABI: context, validation, sizes, layout conversion, representation and
// the Wilson-Dirac operator.  Every entry point validates its arguments
// before launching anything.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "blas.h"
#include "block.h"
#include "dispatch.h"
#include "dphi.h"

namespace bsm {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

bsm_status fail(bsm_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

bsm_status hip_check(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return BSM_ERR_HIP;
}

bsm_status ctx_work_slot(bsm_ctx ctx, int slot, size_t bytes, void **out) {
    if (slot < 0 || slot > 2) return fail(BSM_ERR_ARG, "scratch slot");
    void *&w = ctx->work[slot];
    size_t &wb = ctx->work_bytes[slot];
    if (bytes > wb) {
        if (w) BSM_HIP(hipFree(w));
        w = nullptr;
        wb = 0;
        hipError_t e = hipMalloc(&w, bytes);
        if (e != hipSuccess) return fail(BSM_ERR_NOMEM, "scratch allocation failed");
        // padding sites of internal fields are never written by the operator
        // kernels and must read as zero in the vector reductions.  The fill
        // runs on the null stream and may still be in flight when hipMemset
        // returns; solvers use their own streams, so wait for it here.
        BSM_HIP(hipMemset(w, 0, bytes));
        BSM_HIP(hipDeviceSynchronize());
        wb = bytes;
    }
    *out = w;
    return BSM_OK;
}

bsm_status ctx_work(bsm_ctx ctx, size_t bytes, void **out) { return ctx_work_slot(ctx, 0, bytes, out); }

bsm_status ctx_pinned(bsm_ctx ctx, size_t bytes, void **out) {
    if (bytes > ctx->pinned_bytes) {
        if (ctx->pinned) BSM_HIP(hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
        if (hipHostMalloc(&ctx->pinned, bytes, hipHostMallocDefault) != hipSuccess)
            return fail(BSM_ERR_NOMEM, "pinned host scratch");
        ctx->pinned_bytes = bytes;
    }
    *out = ctx->pinned;
    return BSM_OK;
}

bsm_status ctx_solver_stream(bsm_ctx ctx, hipStream_t *out) {
    if (!ctx->solver_stream) BSM_HIP(hipStreamCreateWithFlags(&ctx->solver_stream, hipStreamNonBlocking));
    *out = ctx->solver_stream;
    return BSM_OK;
}

int hop_blocks(const Geom &g) { return (g.Vh + 255) / 256; }

static bool plan_fits(const Geom &g, const HopPlan &p, int d, bool /*otf*/ = false) {
    if (p.order == 0 || p.order == 2) return true;
    if (p.order == 3 && d > kColMaxD) return false;
    int64_t S3 = (int64_t)g.Vh / g.L[0];
    if (p.order == 4) return S3 % (256 * kXcds) == 0;
    return p.tchunk >= 1 && S3 % 256 == 0 && g.L[0] % p.tchunk == 0;
}

static int plan_lp(int link_prec) { return link_base(link_prec) % 3 + (link_is_otf(link_prec) ? 3 : 0); }

static HopPlan &plan_slot(bsm_ctx ctx, int d, bool real, int prec, int link_prec) {
    const bool adj = real || (link_rn(link_prec) >> 4) == BSM_REP_ADJ;
    return ctx->plans[d & 15][adj ? 1 : 0][prec % 3][plan_lp(link_prec)];
}

void apply_plan(bsm_ctx ctx, int d, bool real, int prec, int link_prec, HopArgs &a) {
    const bool otf = link_is_otf(link_prec);
    HopPlan p = plan_slot(ctx, d, real, prec, link_prec);
    if (!plan_fits(ctx->g, p, d, otf)) p = HopPlan{};
    a.order = p.order;
    a.tchunk = p.tchunk;
    a.wide = otf ? 0 : hop_wide_of(d, prec);
}

// on-the-fly instances (hop_otf.hip)
static bsm_status launch_hop_otf(const Geom &g, int rn, int prec, int lp, const HopArgs &a, hipStream_t st) {
#define BSM_OTF_CASE(SP, LP, REP, N)                                              \
    if (prec == SP && lp == LP && rn == otf_rn(REP, N))                            \
        return hop_run_otf<SP, LP, otf_rn(REP, N)>(g, a, st);
#define BSM_OTF_CASES_LOWP(REP, N)             \
    BSM_OTF_CASE(BSM_F32, BSM_F32, REP, N)      \
    BSM_OTF_CASE(BSM_F16S, BSM_F32, REP, N)     \
    BSM_OTF_CASE(BSM_F16S, BSM_F16S, REP, N)
    BSM_OTF_CASES_LOWP(BSM_REP_SYM, 2)
    BSM_OTF_CASES_LOWP(BSM_REP_SYM, 3)
    BSM_OTF_CASES_LOWP(BSM_REP_SYM, 4)
    BSM_OTF_CASES_LOWP(BSM_REP_ASYM, 3)
    BSM_OTF_CASES_LOWP(BSM_REP_ASYM, 4)
    BSM_OTF_CASES_LOWP(BSM_REP_ADJ, 2)
    BSM_OTF_CASES_LOWP(BSM_REP_ADJ, 3)
    BSM_OTF_CASES_LOWP(BSM_REP_ADJ, 4)
    BSM_OTF_CASE(BSM_F64, BSM_F64, BSM_REP_SYM, 2)
    BSM_OTF_CASE(BSM_F64, BSM_F64, BSM_REP_SYM, 3)
    BSM_OTF_CASE(BSM_F64, BSM_F64, BSM_REP_ASYM, 3)
    BSM_OTF_CASE(BSM_F64, BSM_F64, BSM_REP_ASYM, 4)
    BSM_OTF_CASE(BSM_F64, BSM_F64, BSM_REP_ADJ, 2)
#undef BSM_OTF_CASES_LOWP
#undef BSM_OTF_CASE
    return fail(BSM_ERR_UNSUPPORTED, "no on-the-fly operator for this representation, N and precision pair");
}

template <int SP, int LP>
struct HopSel {
    template <int D>
    struct ByD {
        static bsm_status run(const Geom &g, bool real, const HopArgs &a, hipStream_t st) {
            return hop_run<SP, LP, D>(g, real, a, st);
        }
    };
};

bsm_status launch_hop(const Geom &g, int d, bool real, int prec, int link_prec, const HopArgs &a_in,
                      hipStream_t st) {
    // Without fused norms the kernel choice is invisible to the caller, so the
    // colour split is used wherever it applies; with norms the caller sized
    // the partials for a.wide (apply_plan and hop_grid) and that is kept.
    HopArgs a = a_in;
    if (link_is_otf(link_prec)) {
        a.wide = 0;
        return launch_hop_otf(g, link_rn(link_prec), prec, link_base(link_prec), a, st);
    }
    if (!a.norm_partials) a.wide = hop_wide_of(d, prec);
    if (prec == BSM_F64 && link_prec == BSM_F64)
        return dispatch_d<HopSel<BSM_F64, BSM_F64>::ByD>(d, g, real, a, st);
    if (prec == BSM_F32 && link_prec == BSM_F32)
        return dispatch_d<HopSel<BSM_F32, BSM_F32>::ByD>(d, g, real, a, st);
    if (prec == BSM_F16S && link_prec == BSM_F32)
        return dispatch_d<HopSel<BSM_F16S, BSM_F32>::ByD>(d, g, real, a, st);
    if (prec == BSM_F16S && link_prec == BSM_F16S)
        return dispatch_d<HopSel<BSM_F16S, BSM_F16S>::ByD>(d, g, real, a, st);
    return fail(BSM_ERR_UNSUPPORTED,
                "no operator for spinor precision " + std::to_string(prec) + " with link precision " +
                    std::to_string(link_prec));
}

}  // namespace bsm

using namespace bsm;

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

static bsm_status check_ctx(bsm_ctx ctx) {
    if (!ctx) return fail(BSM_ERR_ARG, "null context");
    return BSM_OK;
}

static bsm_status check_desc(const bsm_field_desc *d) {
    if (!d) return fail(BSM_ERR_ARG, "null field descriptor");
    if (d->N < 2) return fail(BSM_ERR_ARG, "N must be >= 2");
    if (d->rep < 0 || d->rep > 3) return fail(BSM_ERR_ARG, "unknown representation");
    int dim = bsm_rep_dim(d->N, d->rep);
    if (dim != d->d_R)
        return fail(BSM_ERR_ARG, "d_R = " + std::to_string(d->d_R) + " does not match dim(N=" +
                                     std::to_string(d->N) + ", rep) = " + std::to_string(dim));
    if (d->d_R < 2 || d->d_R > 15) return fail(BSM_ERR_ARG, "d_R must be in [2, 15]");
    if (d->prec < 0 || d->prec > 2) return fail(BSM_ERR_ARG, "bad spinor precision");
    const int lb = d->link_prec & ~BSM_LINKS_FUNDAMENTAL;
    if (lb < 0 || lb > 2) return fail(BSM_ERR_ARG, "bad link precision");
    return BSM_OK;
}

// calls that need links stored in the representation
static bsm_status check_stored_links(const bsm_field_desc *d) {
    if (link_is_otf(link_code(d)))
        return fail(BSM_ERR_ARG, "this call needs links stored in the representation (no BSM_LINKS_FUNDAMENTAL)");
    return BSM_OK;
}

#define CHECK(x)                         \
    do {                                 \
        bsm_status _s = (x);             \
        if (_s != BSM_OK) return _s;     \
    } while (0)

extern "C" {

const char *bsm_last_error(void) { return g_err.c_str(); }

int32_t bsm_rep_dim(int32_t N, int32_t rep) {
    if (N < 1) return -1;
    switch (rep) {
    case BSM_REP_FUND: return N;
    case BSM_REP_ADJ: return N * N - 1;
    case BSM_REP_SYM: return N * (N + 1) / 2;
    case BSM_REP_ASYM: return N * (N - 1) / 2;
    }
    return -1;
}

static bsm_status geom_of(const bsm_lattice *lat, Geom &g) {
    if (!lat) return fail(BSM_ERR_ARG, "null lattice");
    int64_t V = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (lat->L[mu] <= 0 || (lat->L[mu] & 1))
            return fail(BSM_ERR_ARG, "lattice extents must be positive and even (L[" +
                                         std::to_string(mu) + "] = " + std::to_string(lat->L[mu]) + ")");
        if (lat->bc[mu] != 1 && lat->bc[mu] != -1) return fail(BSM_ERR_ARG, "bc must be +1 or -1");
        V *= lat->L[mu];
    }
    if (V / 2 > (1 << 30)) return fail(BSM_ERR_ARG, "lattice too large");
    g = Geom{};
    for (int mu = 0; mu < 4; mu++) g.L[mu] = lat->L[mu];
    g.LXh = lat->L[1] / 2;
    g.Vh = (int32_t)(V / 2);
    // Planes of a length that is a multiple of 1024 sites would all start at
    // the same offset modulo 16 KB (a multiple of 16 MB apart at 32^3 x 64),
    // and streaming several of them at once was measured up to 26 % slower
    // (FP64 vector update); 256 extra sites stagger them.  Padding sites are
    // never written by the operators and are skipped by every reduction.
    g.Vh_pad = (g.Vh + 63) / 64 * 64;
    if (g.Vh_pad % 1024 == 0) g.Vh_pad += 256;
    g.apbc = 0;
    for (int mu = 0; mu < 4; mu++)
        if (lat->bc[mu] < 0) g.apbc |= 1 << mu;
    g.div_xh = FastDiv(g.LXh);
    g.div_y = FastDiv(g.L[2]);
    g.div_z = FastDiv(g.L[3]);
    return BSM_OK;
}

bsm_status bsm_ctx_create(const bsm_lattice *lat, bsm_ctx *out) {
    if (!lat || !out) return fail(BSM_ERR_ARG, "null argument");
    Geom g0;
    CHECK(geom_of(lat, g0));
    bsm_ctx c = new bsm_ctx_s();   // value-initialised: zeros, then the plans' defaults
    c->lat = *lat;
    Geom &g = c->g;
    g = g0;
    c->n_partials = reduction_slots(g.Vh);
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc(&c->partials, sizeof(double) * c->n_partials);
    if (e == hipSuccess) e = hipMalloc(&c->scal, sizeof(double) * kScalars);
    if (e == hipSuccess) e = hipMemset(c->scal, 0, sizeof(double) * kScalars);
    if (e == hipSuccess) e = hipHostMalloc(&c->host_scal, sizeof(double) * kScalars, hipHostMallocDefault);
    if (e != hipSuccess) {
        bsm_ctx_destroy(c);
        return hip_check(e, "bsm_ctx_create");
    }
    bsm_status ns = noalloc_scratch_init(c->device);
    if (ns != BSM_OK) {
        bsm_ctx_destroy(c);
        return ns;
    }
    *out = c;
    return BSM_OK;
}

int64_t bsm_reduction_slots(const bsm_lattice *lat) {
    Geom g;
    if (geom_of(lat, g) != BSM_OK) return -1;
    return reduction_slots(g.Vh);
}

int64_t bsm_hop_norm_slots(const bsm_lattice *lat, const bsm_field_desc *desc) {
    Geom g;
    if (geom_of(lat, g) != BSM_OK || check_desc(desc) != BSM_OK) return -1;
    HopArgs a{};
    a.np = 2;
    a.wide = hop_wide_of(desc->d_R, desc->prec);
    int64_t most = 0;
    // every traversal plan a context may pick for this operator
    for (int order = 0; order <= 4; order++) {
        a.order = order;
        a.tchunk = 1;
        if (order == 3 && (g.Vh / g.L[0]) % 256 != 0) continue;
        most = std::max<int64_t>(most, hop_grid(g, a));
    }
    return most;
}

void bsm_ctx_destroy(bsm_ctx c) {
    if (!c) return;
    if (c->partials) (void)hipFree(c->partials);
    if (c->scal) (void)hipFree(c->scal);
    if (c->host_scal) (void)hipHostFree(c->host_scal);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->solver_stream) (void)hipStreamDestroy(c->solver_stream);
    for (void *w : c->work)
        if (w) (void)hipFree(w);
    delete c;
}

size_t bsm_gauge_bytes(bsm_ctx ctx, const bsm_field_desc *desc) {
    if (check_ctx(ctx) != BSM_OK || check_desc(desc) != BSM_OK) return 0;
    return 8 * link_block_bytes(link_base(desc->link_prec), link_real(desc), link_dim(desc), ctx->g.Vh_pad);
}

size_t bsm_spinor_bytes(bsm_ctx ctx, const bsm_field_desc *desc, int32_t nparity, int32_t n_rhs) {
    if (check_ctx(ctx) != BSM_OK || check_desc(desc) != BSM_OK) return 0;
    if ((nparity != 1 && nparity != 2) || n_rhs < 1) {
        fail(BSM_ERR_ARG, "nparity must be 1 or 2 and n_rhs >= 1");
        return 0;
    }
    return (size_t)nparity * n_rhs * spinor_block_bytes(desc->prec, desc->d_R, ctx->g.Vh_pad);
}

static bsm_status pack_common(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs,
                              const void *canon, void *internal, void *stream, bool unpack) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (!canon || !internal) return fail(BSM_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > 65535) return fail(BSM_ERR_ARG, "n_rhs out of range");
    if (!aligned16(canon) || !aligned16(internal)) return fail(BSM_ERR_ARG, "fields must be 16-byte aligned");
    return launch_pack_spinor(ctx->g, desc->d_R, desc->prec, n_rhs, canon, internal,
                              (hipStream_t)stream, unpack);
}

bsm_status bsm_pack_spinor(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs, const void *canon,
                           void *internal, void *stream) {
    return pack_common(ctx, desc, n_rhs, canon, internal, stream, false);
}

bsm_status bsm_unpack_spinor(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs,
                             const void *internal, void *canon, void *stream) {
    return pack_common(ctx, desc, n_rhs, canon, const_cast<void *>(internal), stream, true);
}

bsm_status bsm_gauge_represent(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_fund,
                               void *U_rep, void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (!U_fund || !U_rep) return fail(BSM_ERR_ARG, "null field pointer");
    if (!aligned16(U_fund) || !aligned16(U_rep)) return fail(BSM_ERR_ARG, "fields must be 16-byte aligned");
    if (desc->rep != BSM_REP_FUND && desc->N > 6)
        return fail(BSM_ERR_ARG, "two-index and adjoint representations need N <= 6 for d_R <= 15");
    if (link_is_otf(link_code(desc)))   // fundamental storage: U itself
        return launch_represent(ctx->g, desc->N, BSM_REP_FUND, desc->N, link_base(desc->link_prec), U_fund,
                                U_rep, (hipStream_t)stream);
    return launch_represent(ctx->g, desc->N, desc->rep, desc->d_R, link_base(desc->link_prec), U_fund, U_rep,
                            (hipStream_t)stream);
}

bsm_status bsm_unpack_gauge(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, void *canon,
                            void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (!U_rep || !canon) return fail(BSM_ERR_ARG, "null field pointer");
    return launch_unpack_gauge(ctx->g, link_dim(desc), link_real(desc), link_base(desc->link_prec), U_rep,
                               canon, (hipStream_t)stream);
}

bsm_status bsm_dslash_apply(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, double kappa,
                            int32_t dagger, const void *in, void *out, void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (!U_rep || !in || !out) return fail(BSM_ERR_ARG, "null field pointer");
    if (!aligned16(in) || !aligned16(out) || !aligned16(U_rep)) return fail(BSM_ERR_ARG, "fields must be 16-byte aligned");
    if (in == out) return fail(BSM_ERR_ARG, "in and out must not overlap");
    if (!(kappa >= 0) || !std::isfinite(kappa)) return fail(BSM_ERR_ARG, "kappa must be finite and >= 0");
    size_t bb = spinor_block_bytes(desc->prec, desc->d_R, ctx->g.Vh_pad);
    const char *ip = (const char *)in;
    char *op = (char *)out;
    if (op < ip + 2 * bb && ip < op + 2 * bb) return fail(BSM_ERR_ARG, "in and out must not overlap");
    // one pass over both parities with most links read once, where the
    // lattice and the precision allow; otherwise both parities in one launch
    // of the even-odd hop
    const int lc = link_code(desc);
    if (!link_is_otf(lc) && desc->prec == lc && (lc == BSM_F32 || lc == BSM_F64) &&
        dphi_compiled(desc->prec, desc->d_R) && dphi_fits(ctx->g)) {
        DphiArgs d{};
        d.U = U_rep;
        d.in = in;
        d.out = out;
        d.a = 1.0;
        d.b = -kappa;
        d.dagger = dagger ? 1 : 0;
        d.tc = dphi_tchunk(ctx->g);
        return launch_dphi(ctx->g, desc->d_R, link_real(desc), desc->prec, lc, d, (hipStream_t)stream);
    }
    HopArgs a{};
    a.U = U_rep;
    a.in[0] = ip + bb;    // even output reads odd sites
    a.in[1] = ip;
    a.x[0] = ip;
    a.x[1] = ip + bb;
    a.out[0] = op;
    a.out[1] = op + bb;
    a.a = 1.0;
    a.b = -kappa;
    a.dagger = dagger ? 1 : 0;
    a.p0 = 0;
    a.np = 2;
    a.norm_partials = nullptr;
    apply_plan(ctx, desc->d_R, link_real(desc), desc->prec, link_code(desc), a);
    return launch_hop(ctx->g, desc->d_R, link_real(desc), desc->prec, link_code(desc), a,
                      (hipStream_t)stream);
}

bsm_status bsm_dslash_eo(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t out_parity,
                         int32_t dagger, double a, const void *x, double b, const void *in, void *out,
                         void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (out_parity != 0 && out_parity != 1) return fail(BSM_ERR_ARG, "out_parity must be 0 or 1");
    if (!U_rep || !in || !out) return fail(BSM_ERR_ARG, "null field pointer");
    if (a != 0.0 && !x) return fail(BSM_ERR_ARG, "x is null but a != 0");
    if (!aligned16(in) || !aligned16(out) || (x && !aligned16(x))) return fail(BSM_ERR_ARG, "fields must be 16-byte aligned");
    size_t bb = spinor_block_bytes(desc->prec, desc->d_R, ctx->g.Vh_pad);
    const char *ip = (const char *)in;
    char *op = (char *)out;
    if (op < ip + bb && ip < op + bb) return fail(BSM_ERR_ARG, "in and out must not overlap");
    HopArgs h{};
    h.U = U_rep;
    h.in[out_parity] = in;
    h.x[out_parity] = x;
    h.out[out_parity] = out;
    h.a = a;
    h.b = b;
    h.dagger = dagger ? 1 : 0;
    h.p0 = out_parity;
    h.np = 1;
    h.norm_partials = nullptr;
    apply_plan(ctx, desc->d_R, link_real(desc), desc->prec, link_code(desc), h);
    return launch_hop(ctx->g, desc->d_R, link_real(desc), desc->prec, link_code(desc), h,
                      (hipStream_t)stream);
}

bsm_status bsm_vec_axpby(bsm_ctx ctx, const bsm_field_desc *desc, int32_t nparity, double a,
                         const void *x, double b, const void *y, int32_t prec_out, void *out,
                         void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (nparity != 1 && nparity != 2) return fail(BSM_ERR_ARG, "nparity must be 1 or 2");
    if (!x || !out || (b != 0.0 && !y)) return fail(BSM_ERR_ARG, "null field pointer");
    if (prec_out < 0 || prec_out > 2) return fail(BSM_ERR_ARG, "bad output precision");
    if (y && prec_out != desc->prec) return fail(BSM_ERR_UNSUPPORTED, "conversion takes no y");
    Vec O{out, prec_out}, X{const_cast<void *>(x), desc->prec},
        Y{b != 0.0 ? const_cast<void *>(y) : nullptr, desc->prec};
    return blas_axpby(ctx->g, desc->d_R, nparity, O, a, X, b, Y, nullptr, (hipStream_t)stream);
}

bsm_status bsm_vec_dot(bsm_ctx ctx, const bsm_field_desc *desc, int32_t nparity, const void *x,
                       const void *y, double *result, void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (nparity != 1 && nparity != 2) return fail(BSM_ERR_ARG, "nparity must be 1 or 2");
    if (!x || !result) return fail(BSM_ERR_ARG, "null pointer");
    hipStream_t st = (hipStream_t)stream;
    Vec X{const_cast<void *>(x), desc->prec}, Y{const_cast<void *>(y), desc->prec};
    CHECK(blas_dot(ctx->g, desc->d_R, nparity, X, Y, ctx->partials, st));
    CHECK(reduce_into(ctx->partials, blas_blocks(ctx->g, nparity), ctx->scal + S_TMP, st));
    BSM_HIP(hipMemcpyAsync(ctx->host_scal + S_TMP, ctx->scal + S_TMP, sizeof(double),
                           hipMemcpyDeviceToHost, st));
    BSM_HIP(hipStreamSynchronize(st));
    *result = ctx->host_scal[S_TMP];
    return BSM_OK;
}

static bsm_status check_block(bsm_ctx ctx, const bsm_field_desc *desc) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    CHECK(check_stored_links(desc));
    if (desc->rep != BSM_REP_ADJ) return fail(BSM_ERR_UNSUPPORTED, "block fields need real (adjoint) links");
    return BSM_OK;
}

// FP16 block fields and links for an F16S descriptor, FP32 ones otherwise
static bool block_half(const bsm_field_desc *desc) { return desc->prec == BSM_F16S; }

static size_t block_parity_bytes_of(const Geom &g, const bsm_field_desc *desc) {
    return block_half(desc) ? blockh_parity_bytes(g, desc->d_R) : block_parity_bytes(g, desc->d_R);
}

size_t bsm_block_bytes(bsm_ctx ctx, const bsm_field_desc *desc) {
    if (check_block(ctx, desc) != BSM_OK) return 0;
    return 2 * block_parity_bytes_of(ctx->g, desc);
}

size_t bsm_block_gauge_bytes(bsm_ctx ctx, const bsm_field_desc *desc) {
    if (check_block(ctx, desc) != BSM_OK) return 0;
    return block_half(desc) ? blockh_link_bytes(ctx->g, desc->d_R) : block_link_bytes(ctx->g, desc->d_R);
}

bsm_status bsm_pack_block(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs, const void *canon,
                          void *block, void *stream) {
    CHECK(check_block(ctx, desc));
    if (!canon || !block) return fail(BSM_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > kNR) return fail(BSM_ERR_ARG, "n_rhs must be in [1, 16]");
    if (block_half(desc))
        return launch_pack_blockh(ctx->g, desc->d_R, n_rhs, canon, block, false, (hipStream_t)stream);
    return launch_pack_block(ctx->g, desc->d_R, n_rhs, canon, block, false, (hipStream_t)stream);
}

bsm_status bsm_unpack_block(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs, const void *block,
                            void *canon, void *stream) {
    CHECK(check_block(ctx, desc));
    if (!canon || !block) return fail(BSM_ERR_ARG, "null field pointer");
    if (n_rhs < 1 || n_rhs > kNR) return fail(BSM_ERR_ARG, "n_rhs must be in [1, 16]");
    if (block_half(desc))
        return launch_pack_blockh(ctx->g, desc->d_R, n_rhs, canon, const_cast<void *>(block), true,
                                  (hipStream_t)stream);
    return launch_pack_block(ctx->g, desc->d_R, n_rhs, canon, const_cast<void *>(block), true,
                             (hipStream_t)stream);
}

bsm_status bsm_gauge_to_block(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, void *U_block,
                              void *stream) {
    CHECK(check_block(ctx, desc));
    if (!U_rep || !U_block) return fail(BSM_ERR_ARG, "null field pointer");
    if (block_half(desc))
        return launch_gauge_to_blockh(ctx->g, desc->d_R, desc->link_prec, U_rep, (__half *)U_block,
                                      (hipStream_t)stream);
    return launch_gauge_to_block(ctx->g, desc->d_R, desc->link_prec, U_rep, (float *)U_block,
                                 (hipStream_t)stream);
}

bsm_status bsm_dslash_eo_block(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_block,
                               int32_t out_parity, int32_t dagger, const double *a, const void *x,
                               const double *b, const void *in, void *out, void *stream) {
    CHECK(check_block(ctx, desc));
    if (out_parity != 0 && out_parity != 1) return fail(BSM_ERR_ARG, "out_parity must be 0 or 1");
    if (!U_block || !in || !out || !b) return fail(BSM_ERR_ARG, "null pointer");
    if (a && !x) return fail(BSM_ERR_ARG, "x is null but a is given");
    const size_t bb = block_parity_bytes_of(ctx->g, desc);
    const char *ip = (const char *)in;
    char *op = (char *)out;
    if (op < ip + bb && ip < op + bb) return fail(BSM_ERR_ARG, "in and out must not overlap");
    const BlockPlan &plan = ctx->block_plans[desc->d_R][block_half(desc) ? 1 : 0];
    if (block_half(desc)) {
        BlockHopHArgs h{};
        h.U = (const __half *)U_block;
        h.in[out_parity] = ip;
        h.x[out_parity] = (const char *)x;
        h.out[out_parity] = op;
        h.use_x = a ? 1 : 0;
        for (int r = 0; r < kNR; r++) {
            h.a[r] = a ? (float)a[r] : 0.f;
            h.b[r] = (float)b[r];
        }
        h.dagger = dagger ? 1 : 0;
        h.p0 = out_parity;
        h.np = 1;
        apply_blockh_plan(ctx->g, plan, h);
        return launch_hop_blockh(ctx->g, desc->d_R, h, (hipStream_t)stream);
    }
    BlockHopArgs h{};
    h.U = (const float *)U_block;
    h.in[out_parity] = (const float2 *)in;
    h.x[out_parity] = (const float2 *)x;
    h.out[out_parity] = (float2 *)out;
    h.use_x = a ? 1 : 0;
    for (int r = 0; r < kNR; r++) {
        h.a[r] = a ? (float)a[r] : 0.f;
        h.b[r] = (float)b[r];
    }
    h.dagger = dagger ? 1 : 0;
    h.p0 = out_parity;
    h.np = 1;
    apply_block_plan(ctx->g, plan, h);
    return launch_hop_block(ctx->g, desc->d_R, h, (hipStream_t)stream);
}

bsm_status bsm_block_autotune(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_block, void *stream) {
    CHECK(check_block(ctx, desc));
    if (!U_block) return fail(BSM_ERR_ARG, "null pointer");
    const size_t bb = block_parity_bytes_of(ctx->g, desc);
    void *w = nullptr;
    CHECK(ctx_work(ctx, 2 * bb + 256, &w));
    char *in = (char *)w;
    char *out = (char *)w + (bb + 255) / 256 * 256;
    if (block_half(desc))
        return blockh_autotune(ctx, desc->d_R, (const __half *)U_block, in, out, (hipStream_t)stream);
    return block_autotune(ctx, desc->d_R, (const float *)U_block, (float2 *)in, (float2 *)out,
                          (hipStream_t)stream);
}

bsm_status bsm_set_block_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t sites_per_wave,
                              int32_t waves_per_group, int32_t tiled, int32_t xcd_chunk) {
    CHECK(check_block(ctx, desc));
    if (sites_per_wave != 1 && sites_per_wave != 2) return fail(BSM_ERR_ARG, "sites_per_wave must be 1 or 2");
    if (sites_per_wave != 1 && block_half(desc))
        return fail(BSM_ERR_ARG, "the FP16 block hop runs one site per wavefront");
    if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
        return fail(BSM_ERR_ARG, "waves_per_group must be 1, 2 or 4");
    if (tiled != 0 && tiled != 1) return fail(BSM_ERR_ARG, "tiled must be 0 or 1");
    if (tiled && block_tile_for(ctx->g).tt == 0)
        return fail(BSM_ERR_ARG, "tiled order needs T divisible by 2 or 3 and LY, LZ even");
    if (xcd_chunk < 0 || xcd_chunk > 4096) return fail(BSM_ERR_ARG, "xcd_chunk must be in 0..4096");
    BlockPlan &b = ctx->block_plans[desc->d_R][block_half(desc) ? 1 : 0];
    b.spw = sites_per_wave;
    b.wpb = waves_per_group;
    b.tiled = tiled;
    b.xchunk = xcd_chunk;
    b.us = -1.f;   // set by hand: not tuned, and the batched solver keeps it
    return BSM_OK;
}

bsm_status bsm_get_block_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t *sites_per_wave,
                              int32_t *waves_per_group, int32_t *tiled, int32_t *xcd_chunk, float *us) {
    CHECK(check_block(ctx, desc));
    const BlockPlan &b = ctx->block_plans[desc->d_R][block_half(desc) ? 1 : 0];
    if (sites_per_wave) *sites_per_wave = b.spw;
    if (waves_per_group) *waves_per_group = b.wpb;
    if (tiled) *tiled = b.tiled;
    if (xcd_chunk) *xcd_chunk = b.xchunk;
    if (us) *us = b.us;
    return BSM_OK;
}

bsm_status bsm_set_hop_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t order, int32_t tchunk) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    HopPlan p;
    p.order = order;
    p.tchunk = tchunk;
    if (order < 0 || order > 4) return fail(BSM_ERR_ARG, "order must be 0 ... 4");
    if (!plan_fits(ctx->g, p, desc->d_R, link_is_otf(link_code(desc))))
        return fail(BSM_ERR_ARG, "plan does not tile this lattice (or needs links stored in the representation)");
    plan_slot(ctx, desc->d_R, link_real(desc), desc->prec, link_code(desc)) = p;
    return BSM_OK;
}

bsm_status bsm_autotune(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, void *stream) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    if (!U_rep) return fail(BSM_ERR_ARG, "null gauge field");
    hipStream_t st = (hipStream_t)stream;
    const Geom &g = ctx->g;
    const bool real = link_real(desc);
    const int lc = link_code(desc);
    const bool otf = link_is_otf(lc);
    size_t bb = spinor_block_bytes(desc->prec, desc->d_R, g.Vh_pad);
    void *work = nullptr;
    CHECK(ctx_work(ctx, 2 * bb, &work));
    BSM_HIP(hipMemsetAsync(work, 0, 2 * bb, st));
    std::vector<HopPlan> cand;
    {
        HopPlan p;
        cand.push_back(p);
        p.order = 4;
        p.tchunk = 1;
        if (plan_fits(g, p, desc->d_R, otf)) cand.push_back(p);
        for (int order : {1, 3})
            for (int tc : {2, 4, 8, 16, 32}) {
                p.order = order;
                p.tchunk = tc;
                if (plan_fits(g, p, desc->d_R, otf)) cand.push_back(p);
            }
    }
    hipEvent_t e0, e1;
    BSM_HIP(hipEventCreate(&e0));
    BSM_HIP(hipEventCreate(&e1));
    HopPlan best;
    float best_us = 1e30f;
    const int reps = 10;
    for (const HopPlan &p : cand) {
        HopArgs a{};
        a.U = U_rep;
        a.a = 0.0;
        a.b = 1.0;
        a.np = 1;
        a.order = p.order;
        a.tchunk = p.tchunk;
        float ms = 0.f;
        for (int rep = -2; rep < reps; rep++) {
            int par = rep & 1;
            a.p0 = par;
            a.in[par] = (char *)work + (1 - par) * bb;
            a.out[par] = (char *)work + par * bb;
            if (rep == 0) BSM_HIP(hipEventRecord(e0, st));
            CHECK(launch_hop(g, desc->d_R, real, desc->prec, lc, a, st));
        }
        BSM_HIP(hipEventRecord(e1, st));
        BSM_HIP(hipEventSynchronize(e1));
        BSM_HIP(hipEventElapsedTime(&ms, e0, e1));
        float us = 1000.f * ms / reps;
        if (us < best_us) {
            best_us = us;
            best = p;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    best.us = best_us;
    plan_slot(ctx, desc->d_R, real, desc->prec, lc) = best;
    return BSM_OK;
}

bsm_status bsm_get_hop_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t *order, int32_t *tchunk,
                            float *us) {
    CHECK(check_ctx(ctx));
    CHECK(check_desc(desc));
    const HopPlan &p = plan_slot(ctx, desc->d_R, link_real(desc), desc->prec, link_code(desc));
    if (order) *order = p.order;
    if (tchunk) *tchunk = p.tchunk;
    if (us) *us = p.us;
    return BSM_OK;
}

}  // extern "C"
