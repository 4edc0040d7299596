/*
 * bsm.h - C ABI of libbsm, the MI355X (gfx950) Wilson-Dirac library.
 *
 * The operation (paper, Section II.B): a sparse nearest-neighbour Dirac
 * operator that couples the fermion vectors of neighbouring lattice sites
 * through the gauge links, applied to a fermion field and inverted by a
 * conjugate-gradient solve.  Here it is the Wilson form with hopping
 * parameter kappa:
 *
 *   (D psi)(x) = psi(x) - kappa * H psi(x)
 *   (H psi)(x) = sum_mu  s+ (1 - g_mu) U_mu(x) psi(x+mu)
 *                      + s- (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)
 *
 * with g_mu Euclidean chiral gamma matrices (g_0 = [[0,1],[1,0]],
 * g_k = [[0,-i s_k],[i s_k,0]]), s+- = bc[mu] on hops that wrap around the
 * lattice and 1 otherwise.  D^dag is the same stencil with g_mu -> -g_mu.
 * Section II.A fixes the fields: an N x N complex link on every link of an
 * L^3 x T periodic hypercubic lattice, and a colour vector of dimension
 * d_R >= N in a representation of SU(N) at every site (here times 4 spin
 * components, one flavour).
 *
 * Conventions
 *   Lattice   L[0] = T (mu = 0 is time), L[1..3] = LX, LY, LZ; all even.
 *             bc[mu] = +1 periodic, -1 antiperiodic.
 *   Canonical (user-facing) layout, complex128 interleaved (re, im):
 *             site s = ((t*LZ + z)*LY + y)*LX + x;
 *             spinor [V][4 spin][d], block of n RHS [n][V][4][d];
 *             links  [V][4 mu][N][N] (U_mu(x) at [s][mu]).
 *   Internal  even-odd checkerboarded structure-of-arrays, private to the
 *             library; reach it only through pack/unpack and size it only
 *             through the *_bytes queries.  Parity 0 = even (t+x+y+z even).
 *             A "full" field is the even block followed by the odd block; a
 *             "parity" field is one block.
 *
 * Ownership: every buffer is allocated and owned by the caller (device
 * memory unless stated).  The library never frees caller memory.  A context
 * owns only its own scratch and autotune cache.
 * Streams: hipStream_t passed as void* (NULL = default stream).  Every call
 * is asynchronous on that stream except bsm_cg_solve, bsm_batched_solve and
 * bsm_fgcr_solve, which return after the solve has finished.
 * Errors: arguments are validated before any launch; a non-OK status leaves
 * outputs untouched unless stated, and bsm_last_error() (thread-local)
 * describes it.
 */
#ifndef BSM_H
#define BSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BSM_OK = 0,
    BSM_ERR_ARG = 1,            /* bad pointer, size, extent, kappa or (N, rep, d_R) */
    BSM_ERR_UNSUPPORTED = 2,    /* valid request with no compiled kernel */
    BSM_ERR_HIP = 3,            /* HIP runtime failure; message in bsm_last_error */
    BSM_ERR_NOMEM = 4,          /* scratch allocation failed */
    BSM_ERR_NOT_CONVERGED = 5,  /* max_iter reached; best iterate and stats returned */
    BSM_ERR_NONFINITE = 6       /* NaN/Inf met in a reduction; best iterate returned */
} bsm_status;

typedef enum { BSM_REP_FUND = 0, BSM_REP_ADJ = 1, BSM_REP_SYM = 2, BSM_REP_ASYM = 3 } bsm_rep;

/* storage precision.  Spinors: F64, F32, or F16S = binary16 with one float32
 * scale per site (s = max |component| over the 8 d reals, codes =
 * rne_f16(float32(v * float32(1/s)))).  Links: F64, F32 or F16S meaning plain
 * binary16 (entries of a unitary matrix are bounded by 1, no scale). */
typedef enum { BSM_F64 = 0, BSM_F32 = 1, BSM_F16S = 2 } bsm_prec;

/* Flag ORed into bsm_field_desc.link_prec: the gauge field holds the
 * fundamental N x N links U (the field content of Section II.A, 2 N^2 reals
 * per link) instead of R(U), and every operator forms the representation on
 * the fly inside the hop, applying R(U) (or R(U)^dag) to the projected half
 * spinor without building the d_R x d_R matrix: two-index S -> V S V^T, adjoint
 * X -> V X V^dag (V = U or U^dag).  bsm_gauge_represent then stores U itself
 * (in the precision of the low bits), bsm_gauge_bytes sizes it and
 * bsm_unpack_gauge returns [V][4][N][N].  Operators with these links:
 * sym N = 2, 3, 4; asym N = 3, 4; adj N = 2, 3, 4 with F32 spinors and F32
 * links or F16S spinors and F32 or F16S links; F64 spinors and F64 links for
 * d_R <= 6 (BSM_ERR_UNSUPPORTED otherwise).  Accepted by bsm_dslash_apply,
 * bsm_dslash_eo, the plan and autotune calls and bsm_cg_solve (PLAIN and
 * MIXED; U_rep64 then holds F64 fundamental links too); refused
 * (BSM_ERR_ARG) by the block, network, batched and benchmark-task calls.
 * For fundamental fermions the flag changes nothing. */
#define BSM_LINKS_FUNDAMENTAL 16

typedef struct {
    int32_t L[4];
    int32_t bc[4];
} bsm_lattice;

/* A field's gauge group SU(N), fermion representation and dimension d_R
 * (must equal dim(N, rep), 2 <= d_R <= 15), spinor precision and link
 * precision.  Adjoint links are real and stored as real d x d matrices. */
typedef struct {
    int32_t N;
    int32_t rep;        /* bsm_rep */
    int32_t d_R;
    int32_t prec;       /* bsm_prec of spinors */
    int32_t link_prec;  /* bsm_prec of links */
} bsm_field_desc;

typedef struct bsm_ctx_s *bsm_ctx;

/* Create a context for one lattice on the current HIP device.  Fails with
 * BSM_ERR_ARG for odd or non-positive extents or bc not +-1. */
bsm_status bsm_ctx_create(const bsm_lattice *lat, bsm_ctx *out);
void bsm_ctx_destroy(bsm_ctx ctx);

/* FP64 reduction slots (one partial sum per workgroup) that a context for
 * this lattice allocates: enough for every fused-norm launch of the solvers
 * on it, whatever the representation, precision and traversal plan.  Host
 * only, no device access; -1 for an invalid lattice. */
int64_t bsm_reduction_slots(const bsm_lattice *lat);
/* Workgroups of the largest fused-norm hop launch (both parities, any
 * traversal plan) for this operator type on this lattice, i.e. the
 * reduction slots such a launch writes.  A hop whose grid exceeds the
 * context's slots is refused with BSM_ERR_ARG before any launch.  Host only;
 * -1 for an invalid lattice or descriptor. */
int64_t bsm_hop_norm_slots(const bsm_lattice *lat, const bsm_field_desc *desc);

/* Message for the last non-OK status returned on this thread. */
const char *bsm_last_error(void);

/* Dimension of the representation (N, rep), or -1. */
int32_t bsm_rep_dim(int32_t N, int32_t rep);

/* Bytes of an internal gauge field (all 4 V links in desc->link_prec). */
size_t bsm_gauge_bytes(bsm_ctx ctx, const bsm_field_desc *desc);
/* Bytes of an internal spinor field: nparity = 1 (one parity block) or 2
 * (full lattice), times n_rhs consecutive fields. */
size_t bsm_spinor_bytes(bsm_ctx ctx, const bsm_field_desc *desc, int32_t nparity, int32_t n_rhs);

/* Canonical complex128 spinor(s) -> internal full field(s), in desc->prec.
 * canon: device [n_rhs][V][4][d]; internal: device, bsm_spinor_bytes(2, n_rhs). */
bsm_status bsm_pack_spinor(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs,
                           const void *canon, void *internal, void *stream);
/* Internal full field(s) -> canonical complex128 (dequantised for F16S). */
bsm_status bsm_unpack_spinor(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs,
                             const void *internal, void *canon, void *stream);

/* Links in the fermion representation (Section II.A: the fermion vectors
 * transform under a representation R of SU(N)):
 *   fund R(U) = U;  adj R_ab = 2 Tr(T_a U T_b U^dag) with T_a the generalised
 *   Gell-Mann matrices / 2 (for each pair j<k the symmetric then the
 *   antisymmetric one, then the N-1 diagonal ones);  sym / asym
 *   R_AB = Tr(e_A^dag U e_B U^T) with e_(aa) = E_aa, e_(ab) = (E_ab +- E_ba)/sqrt2,
 *   pairs a <= b (sym) or a < b (asym) in lexicographic order.
 * Computed in FP64, stored in desc->link_prec.
 * U_fund: device canonical complex128 [V][4][N][N]; U_rep: device,
 * bsm_gauge_bytes(desc). */
bsm_status bsm_gauge_represent(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_fund,
                               void *U_rep, void *stream);
/* Internal represented links -> canonical complex128 [V][4][d][d] (tests). */
bsm_status bsm_unpack_gauge(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                            void *canon, void *stream);

/* out = D in (dagger = 0) or D^dag in (dagger = 1) on full internal fields
 * in desc->prec (F64 or F32; F16S uses links in desc->link_prec).
 * in and out must not overlap. */
bsm_status bsm_dslash_apply(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                            double kappa, int32_t dagger, const void *in, void *out,
                            void *stream);

/* Even-odd hopping block: out = a * x + b * H_{p, 1-p} in, where p =
 * out_parity, in is a parity field of parity 1-p, x (nullable when a = 0) and
 * out are parity fields of parity p.  dagger selects the blocks of D^dag.
 * in must not overlap out; x may alias out. */
bsm_status bsm_dslash_eo(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                         int32_t out_parity, int32_t dagger, double a, const void *x, double b,
                         const void *in, void *out, void *stream);

/* Traversal plan of the hopping kernels for one operator type (d_R, link
 * type, spinor and link precision) in this context.
 *   order 0: one thread per output site, workgroups over consecutive sites,
 *            regrouped so each XCD (own L2) walks one contiguous range;
 *   order 1: 256-site spatial tiles, workgroups walk (t-chunk, tile, t) with
 *            t fastest over chunks of tchunk time slices;
 *   order 2: as order 0 without the per-XCD regrouping;
 *   order 3: column sweep: one thread per spatial site over tchunk
 *            consecutive time slices, time neighbours reused from registers
 *            (d_R <= 6; stored or fundamental links);
 *   order 4: XCD bands: each of the 8 XCDs owns 1/8 of the 256-site tiles
 *            of every time slice and walks its band t-major, so time
 *            neighbours are re-read from its own L2 (tchunk ignored).
 * Orders 1 and 3 need LX*LY*LZ/2 to be a multiple of 256 and T a multiple
 * of tchunk, order 4 LX*LY*LZ/2 a multiple of 2048; BSM_ERR_ARG otherwise.  Links are always streamed with
 * non-temporal loads. */
bsm_status bsm_set_hop_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t order, int32_t tchunk);
/* us: measured time per hop of the chosen plan (0 if never tuned) */
bsm_status bsm_get_hop_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t *order, int32_t *tchunk,
                            float *us);
/* Time every plan that fits this lattice on the given links (scratch
 * spinors owned by the context) and keep the fastest for this operator type.
 * Synchronous. */
bsm_status bsm_autotune(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, void *stream);

/* Plain device copy of bytes (multiple of 16, 16-byte aligned) with 16-byte
 * accesses on `blocks` workgroups (<= 0: 2048); nontemporal selects streaming
 * loads and stores.  Calibrates the achievable HBM bandwidth. */
bsm_status bsm_stream_copy(const void *src, void *dst, size_t bytes, int32_t nontemporal,
                           int32_t blocks, void *stream);
/* Read-only sweep of bytes (multiple of 16, 16-byte aligned) on `blocks`
 * workgroups (<= 0: 2048), each over its own contiguous chunk, with
 * streaming loads when nontemporal; out (device, >= blocks floats) receives
 * one sum per workgroup so the loads are kept.  Calibrates the achievable
 * read bandwidth. */
bsm_status bsm_stream_read(const void *src, size_t bytes, int32_t nontemporal, int32_t blocks, float *out,
                           void *stream);

/* ------------------------------------------------------------- vector ops
 * The Krylov linear algebra of the solvers (paper, Section II.B: CG repeats
 * the operator plus vector updates), on internal fields of nparity (1 or 2)
 * parity blocks.  Sums accumulate in FP64 in a fixed order (bitwise
 * reproducible).  Supported precision mixes: all operands in desc->prec, or
 * out in prec_out with x (and no y) in desc->prec (a conversion). */
/* out = a * x + b * y (y nullable when b == 0); out may alias x or y */
bsm_status bsm_vec_axpby(bsm_ctx ctx, const bsm_field_desc *desc, int32_t nparity, double a,
                         const void *x, double b, const void *y, int32_t prec_out, void *out,
                         void *stream);
/* *result = Re <x, y> (|x|^2 when y is null); synchronous, result on the host */
bsm_status bsm_vec_dot(bsm_ctx ctx, const bsm_field_desc *desc, int32_t nparity, const void *x,
                       const void *y, double *result, void *stream);

/* ---------------------------------------------------------------- solvers */
typedef enum {
    BSM_SOLVER_PLAIN = 0,       /* CG in FP64 (full D^dag D, or Schur if schur=1) */
    BSM_SOLVER_MIXED = 1,       /* reliable-update CG, inner precision desc->prec */
    BSM_SOLVER_BATCHED = 2,     /* n_rhs right-hand sides with their own kappas (bsm_batched_solve) */
    BSM_SOLVER_FGCR_NET = 3,    /* flexible GCR with the network preconditioner (bsm_fgcr_solve) */
    BSM_SOLVER_SHIFTED = 4,     /* one source, n_rhs kappas in one Krylov space (bsm_shifted_solve) */
} bsm_solver_variant;

typedef struct {
    int32_t variant;       /* bsm_solver_variant */
    int32_t schur;         /* 1: even-odd Schur complement, 0: full lattice */
    double kappa;
    double tol;            /* target true relative residual ||b - D x|| / ||b|| */
    int32_t max_iter;
    double delta;          /* reliable update threshold (MIXED), e.g. 0.1 */
    int32_t check_every;   /* iterations between host convergence checks (<= 0: the solver's default) */
    int32_t restart;       /* FGCR: Krylov vectors per cycle (e.g. 16) */
    int32_t precond_layers; /* FGCR: 0 applies the network as one collapsed operator
                               (bsm_precond_apply_collapsed) where d_R <= 3; 1 always
                               applies it layer by layer in FP32 (bsm_precond_apply) */
    int32_t n_rhs;         /* BATCHED, SHIFTED: number of right-hand sides / kappas */
    const double *kappas;  /* BATCHED, SHIFTED: host array of n_rhs kappas (kappa is then ignored) */
    int32_t channels;      /* FGCR_NET: network channels */
    const void *net;       /* FGCR_NET: network weights (device, bsm_net_bytes), NULL: M = 1 */
} bsm_solver_params;

typedef struct {
    int32_t iters;
    int32_t reliable_updates;
    int32_t restarts;
    int32_t converged;
    double true_rel_res;
    double seconds;
    int32_t fell_back;     /* FGCR: finished by the plain CG fallback */
    int32_t precond_applies;
} bsm_solver_stats;

/* Solve D x = b (Section II.B: the operator is inverted by conjugate
 * gradients; here CG on the normal equations).  params->variant BATCHED,
 * SHIFTED and FGCR_NET forward to bsm_batched_solve and bsm_shifted_solve
 * (n_rhs, kappas from params; stats an array of n_rhs) and bsm_fgcr_solve
 * (channels, net from params), with the arguments and behaviour documented
 * there; the rest of this comment is about PLAIN and MIXED.  b and x are full internal
 * fields in F64 (desc->prec is the inner precision for MIXED and must be F64
 * for PLAIN); U_rep holds links in desc->link_prec for the inner operator and
 * U_rep64 the FP64 links used for every true residual (may equal U_rep when
 * that is F64).  x is overwritten (start x = 0).  Stopping: the normal
 * residual only triggers a check; the FP64 full-lattice true residual must be
 * <= tol, otherwise iteration continues with the trigger tightened by 0.3.
 * Both run check_every iterations between host checks (check_every <= 0:
 * 8); MIXED decides its reliable updates there, from the |r|^2 of every
 * iteration of the chunk, keeps the chunk's search directions (at most 48
 * iterations per chunk; check_every + 1 inner-precision fields of scratch)
 * and adds them to its low-precision solution once per chunk.
 * Synchronous: returns when done, with stats filled in even on failure. */
bsm_status bsm_cg_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                        const void *U_rep64, const bsm_solver_params *params, const void *b,
                        void *x, bsm_solver_stats *stats, void *stream);

/* ------------------------------------------------- learned preconditioner
 * A gauge-covariant network of parallel-transport convolution (PTC) layers:
 *   out_i(x) = sum_j sum_p W_p^{ij} (T_p v_j)(x),  p in {stay, +mu, -mu} (9 paths)
 *   T_{+mu} v(x) = s+ U_mu(x) v(x+mu),  T_{-mu} v(x) = s- U_mu(x-mu)^dag v(x-mu)
 * W_p^{ij} complex 4 x 4 spin matrices, complex float [cout][cin][9][4][4].
 * The preconditioner is M(r) = L2(L1(r)) with L1: 1 -> C channels and
 * L2: C -> 1 (weights W1 then W2, consecutive: bsm_net_bytes).  Channel fields
 * are consecutive F32 full internal fields.  desc: spinor F32, link F32,
 * complex links (d_R <= 6). */
size_t bsm_net_bytes(int32_t channels);
bsm_status bsm_ptc_layer(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t cin,
                         int32_t cout, const void *W, const void *in, void *out, void *stream);
/* the adjoint layer: in has cout channels, out cin channels */
bsm_status bsm_ptc_layer_adjoint(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t cin,
                                 int32_t cout, const void *W, const void *in, void *out, void *stream);
/* dW = dL/dRe W + i dL/dIm W for a layer with input v (cin channels) and
 * output gradient G = dL/dRe out + i dL/dIm out (cout channels):
 * dW_p^{ij}[a][b] = sum_x sum_c G_i(x)[a][c] conj((T_p v_j)(x)[b][c]).  FP64 sums. */
bsm_status bsm_ptc_weight_grad(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t cin,
                               int32_t cout, const void *G, const void *v, void *dW, void *stream);
/* z = M(r) for F32 full fields r, z */
bsm_status bsm_precond_apply(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t channels,
                             const void *net, const void *r, void *z, void *stream);
/* Backward pass of z = M(r) = L2(L1(r)) for one field r, the gradients that
 * training the network needs: with the output gradient
 * dz = dL/dRe z + i dL/dIm z of a real loss L,
 *   dr       = M^dag dz = L1^dag (L2^dag dz)        (skipped when dr is NULL),
 *   dweights = [dW1, dW2] in the layout of net (bsm_net_bytes(channels)),
 *              dW2_p^{0j} = sum_x dz(x) conj((T_p h_j)(x))^T with h = L1 r,
 *              dW1_p^{j0} = sum_x (L2^dag dz)_j(x) conj((T_p r)(x))^T
 * (each entry as in bsm_ptc_weight_grad: dL/dRe W + i dL/dIm W, FP64 sums).
 * desc as for bsm_precond_apply; r, dz, dr: F32 full fields (dr must not
 * overlap r or dz); dweights is overwritten.  Scratch from the context.
 * Asynchronous on stream. */
bsm_status bsm_precond_backward(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t channels,
                                const void *net, const void *r, const void *dz, void *dr, void *dweights,
                                void *stream);
/* z = M(r) with the two layers collapsed into one operator, which both
 * layers being linear allows (spin matrices commute with the transports):
 *   z = sum_p T_p G_p,  G_p(y) = sum_q C_pq (T_q r)(y),  C_pq = sum_j W2_p^{0j} W1_q^{j0}.
 * Transports in FP32; the 36 x 36 complex mixing runs on FP16 matrix cores
 * with FP32 accumulation on per-site scaled fields, and the nine mixed fields
 * are kept in FP16 with that scale, so z agrees with bsm_precond_apply to a
 * relative O(1e-3) (norm-wise).  Non-finite components of r give non-finite
 * components of z.  d_R <= 3 (BSM_ERR_UNSUPPORTED otherwise); scratch from
 * the context.  desc->link_prec may be BSM_F16S here (U_rep then holds FP16
 * links, e.g. from bsm_gauge_represent with link_prec F16S), which FGCR uses
 * for its network.  Asynchronous on stream. */
bsm_status bsm_precond_apply_collapsed(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                                       int32_t channels, const void *net, const void *r, void *z, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and result as bsm_precond_apply_collapsed, but its
 * scratch (the nine FP16 mixed fields, their per-site scales and the
 * collapsed mixing matrix: 144 d_R + 4 bytes per lattice site plus
 * 13 KB) lives in a static device array of 64 MiB that the library holds on
 * every device it runs on until the process ends, never in memory it
 * allocates.  The call itself allocates nothing; the context (created
 * beforehand) must belong to the current device.  BSM_ERR_ARG, before any
 * launch, when the lattice needs more than 64 MiB of scratch (d_R = 3: up to
 * about 77 000 sites per parity, e.g. 16^3 x 32).  Every call on a device
 * shares that device's array and leaves its contents behind: calls that
 * overlap on one device (other streams, other threads) race and must be
 * ordered by the caller.  Asynchronous on stream. */
bsm_status bsm_precond_apply_collapsed_noalloc(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep,
                                               int32_t channels, const void *net, const void *r, void *z,
                                               void *stream);

typedef struct {
    float lr, beta1, beta2, eps;   /* Adam (e.g. 1e-3, 0.9, 0.999, 1e-8) */
    int32_t batch;                 /* pairs per step */
    int32_t steps;
    uint64_t seed;                 /* batch selection (splitmix64 counter stream) */
    int32_t step0;                 /* Adam steps already taken with adam_state (0 at first) */
} bsm_train_params;
/* Adam steps on loss = mean over a batch of |M(r) - e|^2 / |e|^2 with
 * gradients from the adjoint layers and the weight-gradient kernel.
 * r_pairs, e_pairs: n_pairs consecutive F32 full fields each.  adam_state:
 * device, 2 * bsm_net_bytes(channels) bytes, zero before the first call.
 * losses: host array of steps (batch loss before each update).  Synchronous. */
bsm_status bsm_precond_train(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, int32_t channels,
                             void *net, void *adam_state, const void *r_pairs, const void *e_pairs,
                             int32_t n_pairs, const bsm_train_params *params, float *losses, void *stream);
/* Training pairs from plain FP64 Schur CG on D x = b with b = D x*_s for
 * each of n_solves solutions x*_s (F64 full fields): after k = iters[q]
 * iterations from x_0 = 0 (q < n_snap; k = 0 gives e = x*), e = x* - x_k
 * and r = D e, stored as F32 full fields at r_out / e_out [s * n_snap + q].
 * U_rep64: FP64 links.  Synchronous. */
bsm_status bsm_precond_pairs(bsm_ctx ctx, const bsm_field_desc *desc64, const void *U_rep64, double kappa,
                             int32_t n_solves, const void *x_star, int32_t n_snap, const int32_t *iters,
                             void *r_out, void *e_out, void *stream);
/* Flexible GCR(params->restart) on D x = b with z = M(r) from the network
 * (net nullable: M = 1; params->precond_layers picks the collapsed FP16 or
 * the layered FP32 form of M).  Each restart cycle solves the correction equation
 * D e = r in FP32 (directions, D, Gram-Schmidt; sums in FP64), then
 * x += e in FP64 and r = b - D x is recomputed in FP64 (the deciding residual).  A cycle
 * that reduces |r| by less than a factor 2, or meets a non-finite value,
 * hands over to plain FP64 Schur CG from the current x (from x = 0 after a
 * non-finite value).  desc/U_rep: F32 spinors and F32 links (the inner
 * operator and the network); U_rep64: FP64 links.  b, x: F64 full fields;
 * padding sites of b must be zero (as pack leaves them).  Synchronous. */
bsm_status bsm_fgcr_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, const void *U_rep64,
                          const bsm_solver_params *params, int32_t channels, const void *net, const void *b,
                          void *x, bsm_solver_stats *stats, void *stream);

/* ------------------------------------------------------- many right-hand sides
 * Block fields hold up to 16 right-hand sides together (layout private) so
 * that one link load serves all of them; available for real (adjoint)
 * links, where the hop of 16 RHS at a site is a dense product of the d x d
 * link with a d x 64 block of projected half spinors, done on matrix cores.
 * desc->rep must be BSM_REP_ADJ for the block calls below.  desc->prec
 * selects the block precision: BSM_F16S gives FP16 block fields (a float
 * scale per site and RHS, the codes rounded as the F16S spinors are) and
 * FP16 block links (d_R 3, 8, 15), with FP16 matrix-core products
 * accumulated in FP32; any other precision gives FP32 fields and links on
 * FP32 matrix cores.  desc->link_prec is the precision of the represented
 * links given to bsm_gauge_to_block (F64 or F32). */
/* bytes of one full block field (both parities, 16 RHS slots) */
size_t bsm_block_bytes(bsm_ctx ctx, const bsm_field_desc *desc);
/* bytes of the links in block layout */
size_t bsm_block_gauge_bytes(bsm_ctx ctx, const bsm_field_desc *desc);
/* canonical complex128 [n_rhs][V][4][d] (n_rhs <= 16) <-> block field;
 * pack zeroes the unused RHS slots */
bsm_status bsm_pack_block(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs, const void *canon,
                          void *block, void *stream);
bsm_status bsm_unpack_block(bsm_ctx ctx, const bsm_field_desc *desc, int32_t n_rhs, const void *block,
                            void *canon, void *stream);
/* represented links (internal layout, link_prec F64 or F32) -> block layout */
bsm_status bsm_gauge_to_block(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, void *U_block,
                              void *stream);
/* Even-odd hop of every RHS slot: out_r = a_r x_r + b_r H_{p,1-p} in_r, with
 * a, b host arrays of 16 (a nullable: x is not read), in / x / out one parity
 * block of block fields (in must not overlap out; x may be out). */
bsm_status bsm_dslash_eo_block(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_block,
                               int32_t out_parity, int32_t dagger, const double *a, const void *x,
                               const double *b, const void *in, void *out, void *stream);
/* Block hop launch plan per d_R: sites per wavefront (1, or 2 processed
 * interleaved with half the register budget per wavefront), wavefronts
 * per workgroup (1, 2, 4), the site order (tiled = 1: tiles of a few
 * lattice rows in t, z and y, so the neighbours of a site are visited close
 * together and their 16-RHS blocks are fetched fewer times; needs T
 * divisible by 2 or 3 and LY, LZ even, else BSM_ERR_ARG) and the order of
 * workgroups over the 8 XCDs (xcd_chunk = 0: each XCD takes one contiguous
 * eighth of the sites; c in 1..4096: each XCD takes runs of c consecutive
 * workgroups in turn, so the XCDs sweep nearby sites together and share the
 * memory-side cache).  FP16 and FP32 block hops keep separate plans; the
 * FP16 one runs one site per wavefront (sites_per_wave must be 1).
 * bsm_block_autotune times every plan on the
 * given block links (scratch fields owned by the context) and keeps the
 * fastest; the batched solver tunes once per d_R, precision and context
 * unless a plan was set by hand.  us: time per hop of the tuned plan (0: default plan,
 * -1: set by hand).  Synchronous. */
bsm_status bsm_block_autotune(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_block, void *stream);
bsm_status bsm_set_block_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t sites_per_wave,
                              int32_t waves_per_group, int32_t tiled, int32_t xcd_chunk);
bsm_status bsm_get_block_plan(bsm_ctx ctx, const bsm_field_desc *desc, int32_t *sites_per_wave,
                              int32_t *waves_per_group, int32_t *tiled, int32_t *xcd_chunk, float *us);
/* Solve D(kappa_r) x_r = b_r for n_rhs right-hand sides with their own
 * kappa_r (Section II.B's inversion, for a family of masses).  b and x are
 * n_rhs consecutive full internal FP64 fields; U_rep64 are FP64 links.
 * Adjoint links: 16 RHS at a time share every link load on matrix cores
 * (inner recurrence captured as a HIP graph of check_every iterations, or
 * with check_every <= 0 of 8 (FP32) or 4 (F16S) iterations, FP64
 * reliable updates with threshold delta, each RHS retired once its FP64
 * true residual <= tol); desc->prec = BSM_F16S runs the inner recurrence
 * on FP16 block fields and links (x and r in FP32), any other precision on
 * FP32 ones.  Other representations: one mixed-precision solve
 * per RHS at inner precision desc->prec.  stats: host array of n_rhs.
 * Synchronous. */
bsm_status bsm_batched_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep64,
                             const bsm_solver_params *params, int32_t n_rhs, const double *kappas,
                             const void *b, void *x, bsm_solver_stats *stats, void *stream);

/* Solve D(kappa_i) x_i = b for n_kappa (1 ... 32) kappas and ONE source b
 * (Section II.B's inversion for a family of masses) in one Krylov space:
 * D(kappa) = kappa (1/kappa - H), so the systems differ by multiples of the
 * identity.  The seed is the largest kappa; BiCG with the gamma5 shadow
 * sequence (valid since D^dag = gamma5 D gamma5; one operator application
 * per iteration, real coefficients) carries every shifted member along with
 * colinear residuals; a member retires when its residual estimate is below
 * params->delta * tol (delta <= 0: 0.3), then its FP64 full-lattice true
 * residual decides, and a member that misses tol (or a breakdown) is
 * finished by plain FP64 Schur CG (stats.fell_back; max_iter bounds the
 * shared iteration and each fallback solve).  desc: F64 spinors, F64 links (stored, or fundamental
 * with BSM_LINKS_FUNDAMENTAL); b: full FP64 field; x: n_kappa consecutive
 * full FP64 fields, overwritten; stats: host array of n_kappa (iters =
 * shared iterations until the member retired, plus fallback iterations).
 * The members' solutions and directions are formed from the kept seed
 * residuals every 16 iterations (and at the end) rather than each iteration.
 * Scratch: the context's, (20 + n_kappa) full FP64 fields (fewer residuals
 * are kept, down to (5 + n_kappa) fields, when that much device memory is
 * not available; BSM_ERR_NOMEM below that).  Synchronous. */
bsm_status bsm_shifted_solve(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep64,
                             const bsm_solver_params *params, int32_t n_kappa, const double *kappas,
                             const void *b, void *x, bsm_solver_stats *stats, void *stream);

/* -------------------------------------------------------- benchmark tasks
 * Section III's benchmark: three tasks (an elementary vector operation, a
 * matrix-vector operation, then the full Dirac operator) are each repeated
 * on fixed random fields, the number of repetitions between two readings of
 * the clock doubling after every reading, and rated as
 * repetitions x flops per repetition / elapsed time.  The paper does not
 * define the two elementary operations or the flop counts; here:
 *   BSM_TASK_VECTOR  out = 0.5 in + 0.5 out                 (bsm_vec_axpby)
 *   BSM_TASK_MATVEC  out = sum_mu U_mu(x) in(x), each spin  (bsm_link_matvec)
 *   BSM_TASK_DPHI    out = D in with the given kappa        (bsm_dslash_apply)
 * Fields are full internal fields (both parities). */
typedef enum { BSM_TASK_VECTOR = 0, BSM_TASK_MATVEC = 1, BSM_TASK_DPHI = 2 } bsm_task;

/* Link x spinor at every site, no neighbour access:
 *   out(x)_s = sum_mu U_mu(x) in(x)_s   for spin s = 0..3,
 * U_mu(x) the forward link of site x in the fermion representation.  in and
 * out are full internal fields in desc->prec, U_rep in desc->link_prec
 * (precision pairs as for bsm_dslash_apply); they must not overlap.
 * Asynchronous. */
bsm_status bsm_link_matvec(bsm_ctx ctx, const bsm_field_desc *desc, const void *U_rep, const void *in, void *out,
                           void *stream);

/* Flop count and algorithmic bytes of one repetition of task on the whole
 * lattice (host only, no device access).  Flops per site: vector 24 d;
 * mat-vec 128 d^2 - 8 d (real links 64 d^2 - 8 d); Dphi 128 d^2 + 72 d (real
 * 64 d^2 + 72 d).  Bytes count every element touched once: vector 3 spinor
 * fields, mat-vec and Dphi the 4 V links plus 2 spinor fields.
 * BSM_ERR_ARG for odd or non-positive extents, a bad descriptor or task. */
bsm_status bsm_task_cost(const bsm_lattice *lat, const bsm_field_desc *desc, int32_t task, double *flops,
                         double *bytes);

/* The timed loop: one untimed call (which validates the arguments), then
 * rounds of 1, 2, 4, ... repetitions on `stream`, the elapsed time read with
 * HIP events after each round, until it reaches min_seconds (0 <
 * min_seconds <= 3600).  iterations (host) receives the total repetitions,
 * seconds (host) the elapsed time.  kappa is used by BSM_TASK_DPHI only,
 * U_rep is ignored by BSM_TASK_VECTOR.  Synchronous. */
bsm_status bsm_task_run(bsm_ctx ctx, const bsm_field_desc *desc, int32_t task, const void *U_rep, double kappa,
                        const void *in, void *out, double min_seconds, void *stream, int64_t *iterations,
                        double *seconds);

#ifdef __cplusplus
}
#endif
#endif /* BSM_H */
