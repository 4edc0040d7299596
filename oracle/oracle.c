/*
 * FP64 CPU oracle for the Wilson-Dirac hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or constant with the GPU library: gamma matrices, representation
 * bases and the stencil are all written out here again from their
 * definitions.
 *
 * What it computes (paper, Section II.A-B: a sparse nearest-neighbour Dirac
 * operator on N x N gauge links acting on colour vectors in a representation
 * of SU(N), inverted by conjugate gradients):
 *
 *   (D psi)(x) = psi(x) - kappa * sum_mu [ s+_mu(x) (1 - g_mu) U_mu(x) psi(x+mu)
 *                                        + s-_mu(x) (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
 *
 * (Wilson form, r = 1, hopping-parameter normalisation, one flavour), with
 * s+- the boundary sign for hops that wrap around the lattice (bc[mu], -1 in
 * time for the antiperiodic workloads).  The adjoint operator is the same
 * stencil with g_mu -> -g_mu.  Everything is plain loops in double complex,
 * parallel over sites with OpenMP only.
 *
 * Canonical layouts (all arrays complex interleaved):
 *   site s = ((t*LZ + z)*LY + y)*LX + x with L[0]=T, L[1]=LX, L[2]=LY, L[3]=LZ
 *   spinor [V][4][d], links [V][4][d][d] (U_mu(x) at [s][mu]).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------ */
/* geometry                                                            */
/* ------------------------------------------------------------------ */

static void site_coords(const int L[4], long s, int c[4])
{
    c[1] = (int)(s % L[1]); s /= L[1];
    c[2] = (int)(s % L[2]); s /= L[2];
    c[3] = (int)(s % L[3]); s /= L[3];
    c[0] = (int)s;
}

static long site_index(const int L[4], const int c[4])
{
    return (((long)c[0] * L[3] + c[3]) * L[2] + c[2]) * L[1] + c[1];
}

static long volume(const int L[4]) { return (long)L[0] * L[1] * L[2] * L[3]; }

/* neighbour of s one step along +mu (dir=+1) or -mu (dir=-1); *sign gets the
 * boundary factor when the step wraps around the lattice */
static long neighbour(const int L[4], const int bc[4], long s, int mu, int dir, double *sign)
{
    int c[4];
    site_coords(L, s, c);
    *sign = 1.0;
    c[mu] += dir;
    if (c[mu] == L[mu]) { c[mu] = 0; *sign = bc[mu]; }
    if (c[mu] < 0) { c[mu] = L[mu] - 1; *sign = bc[mu]; }
    return site_index(L, c);
}

int orc_parity(const int L[4], long s)
{
    int c[4];
    site_coords(L, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

/* ------------------------------------------------------------------ */
/* gamma matrices: Euclidean chiral basis                              */
/*   g_0 = [[0, 1], [1, 0]],  g_k = [[0, -i s_k], [i s_k, 0]]  (2x2 blocks) */
/* ------------------------------------------------------------------ */

static cplx G[4][4][4];   /* G[mu][row][col] */
static int gamma_ready = 0;

static void build_gammas(void)
{
    if (gamma_ready) return;
    cplx sig[4][2][2];
    memset(sig, 0, sizeof sig);
    sig[0][0][0] = 1; sig[0][1][1] = 1;            /* identity */
    sig[1][0][1] = 1; sig[1][1][0] = 1;            /* sigma_1 */
    sig[2][0][1] = -I; sig[2][1][0] = I;           /* sigma_2 */
    sig[3][0][0] = 1; sig[3][1][1] = -1;           /* sigma_3 */
    memset(G, 0, sizeof G);
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) {
            G[0][a][2 + b] = sig[0][a][b];
            G[0][2 + a][b] = sig[0][a][b];
            for (int k = 1; k <= 3; k++) {
                G[k][a][2 + b] = -I * sig[k][a][b];
                G[k][2 + a][b] = I * sig[k][a][b];
            }
        }
    gamma_ready = 1;
}

/* copy gamma_mu out (tests check the Clifford algebra on it) */
void orc_gamma(int mu, double *out /* 4x4 complex */)
{
    build_gammas();
    memcpy(out, G[mu], sizeof(cplx) * 16);
}

/* ------------------------------------------------------------------ */
/* representations (Section II.A: fermions in a representation of SU(N))
 *   fund : R(U) = U
 *   adj  : R_ab = 2 Tr(T_a U T_b U^dag), T_a generalised Gell-Mann / 2
 *          (for each pair j<k: symmetric, then antisymmetric; then the
 *          N-1 diagonal ones), Tr T_a T_b = delta_ab / 2
 *   sym  : R_AB = Tr(e_A^dag U e_B U^T), e_(aa) = E_aa,
 *          e_(ab) = (E_ab + E_ba)/sqrt2 for a<b, pairs a<=b lexicographic
 *   asym : same with e_(ab) = (E_ab - E_ba)/sqrt2, pairs a<b
 * rep codes: 0 fund, 1 adj, 2 sym, 3 asym                              */
/* ------------------------------------------------------------------ */

int orc_rep_dim(int N, int rep)
{
    switch (rep) {
    case 0: return N;
    case 1: return N * N - 1;
    case 2: return N * (N + 1) / 2;
    case 3: return N * (N - 1) / 2;
    }
    return -1;
}

/* basis matrices of the representation space: nb matrices of N x N */
static cplx *rep_basis(int N, int rep, int *nb)
{
    int d = orc_rep_dim(N, rep);
    cplx *B = calloc((size_t)d * N * N, sizeof(cplx));
    int A = 0;
#define E(A_, i_, j_) B[((size_t)(A_) * N + (i_)) * N + (j_)]
    if (rep == 1) {
        for (int j = 0; j < N; j++)
            for (int k = j + 1; k < N; k++) {
                E(A, j, k) = 0.5; E(A, k, j) = 0.5; A++;
                E(A, j, k) = -0.5 * I; E(A, k, j) = 0.5 * I; A++;
            }
        for (int l = 1; l < N; l++) {
            double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
            for (int m = 0; m < l; m++) E(A, m, m) = nrm;
            E(A, l, l) = -l * nrm;
            A++;
        }
    } else if (rep == 2 || rep == 3) {
        double sg = rep == 2 ? 1.0 : -1.0;
        for (int a = 0; a < N; a++)
            for (int b = a; b < N; b++) {
                if (a == b) {
                    if (rep == 3) continue;
                    E(A, a, a) = 1.0;
                } else {
                    E(A, a, b) = 1.0 / sqrt(2.0);
                    E(A, b, a) = sg / sqrt(2.0);
                }
                A++;
            }
    }
#undef E
    *nb = d;
    return B;
}

static void matmul(int N, const cplx *A, const cplx *B, cplx *C)
{
    for (int i = 0; i < N; i++)
        for (int j = 0; j < N; j++) {
            cplx s = 0;
            for (int k = 0; k < N; k++) s += A[i * N + k] * B[k * N + j];
            C[i * N + j] = s;
        }
}

/* R: nlinks x d x d.  Returns d, or -1 for an unknown (N, rep). */
int orc_represent(int N, int rep, long nlinks, const double *Uin, double *Rout)
{
    int d = orc_rep_dim(N, rep);
    if (d < 1) return -1;
    const cplx *U = (const cplx *)Uin;
    cplx *R = (cplx *)Rout;
    if (rep == 0) {
        memcpy(R, U, sizeof(cplx) * (size_t)nlinks * N * N);
        return d;
    }
    int nb;
    cplx *B = rep_basis(N, rep, &nb);
#pragma omp parallel
    {
        cplx *Ud = malloc(sizeof(cplx) * N * N);    /* U^dag or U^T */
        cplx *X = malloc(sizeof(cplx) * N * N);
        cplx *Y = malloc(sizeof(cplx) * N * N);
#pragma omp for schedule(static)
        for (long l = 0; l < nlinks; l++) {
            const cplx *u = U + (size_t)l * N * N;
            cplx *r = R + (size_t)l * d * d;
            for (int i = 0; i < N; i++)
                for (int j = 0; j < N; j++)
                    Ud[i * N + j] = rep == 1 ? conj(u[j * N + i]) : u[j * N + i];
            for (int b = 0; b < d; b++) {
                /* X = U e_b U^dag (adj) or U e_b U^T (sym/asym) */
                matmul(N, u, B + (size_t)b * N * N, Y);
                matmul(N, Y, Ud, X);
                for (int a = 0; a < d; a++) {
                    const cplx *ea = B + (size_t)a * N * N;
                    cplx s = 0;
                    /* adj: 2 Tr(T_a X); sym/asym: Tr(e_a^dag X) */
                    for (int i = 0; i < N; i++)
                        for (int j = 0; j < N; j++)
                            s += (rep == 1 ? 2.0 * ea[j * N + i] : conj(ea[i * N + j])) * X[i * N + j];
                    r[a * d + b] = s;
                }
            }
        }
        free(Ud); free(X); free(Y);
    }
    free(B);
    return d;
}

/* ------------------------------------------------------------------ */
/* hopping term and Wilson-Dirac operator                              */
/* ------------------------------------------------------------------ */

/* out(x) = sum over the 8 hops of x (only sites with mask(x) set):
 *   s+ (1 -+ g_mu) U_mu(x) in(x+mu) + s- (1 +- g_mu) U_mu(x-mu)^dag in(x-mu)
 * the lower sign in the projectors is used for the adjoint (dagger = 1). */
static void hop_site(const int L[4], const int bc[4], int d, const cplx *U, int dagger,
                     const cplx *in, long s, cplx *o /* 4*d */)
{
    cplx v[4][16], w;
    double eta = dagger ? -1.0 : 1.0;
    for (int k = 0; k < 4 * d; k++) o[k] = 0;
    for (int mu = 0; mu < 4; mu++) {
        for (int dir = -1; dir <= 1; dir += 2) {
            double sign;
            long y = neighbour(L, bc, s, mu, dir, &sign);
            const cplx *link = dir > 0 ? U + ((size_t)s * 4 + mu) * d * d
                                       : U + ((size_t)y * 4 + mu) * d * d;
            const cplx *p = in + (size_t)y * 4 * d;
            /* v = U psi(x+mu)  or  U^dag psi(x-mu), per spin component */
            for (int a = 0; a < 4; a++)
                for (int i = 0; i < d; i++) {
                    cplx acc = 0;
                    for (int j = 0; j < d; j++)
                        acc += dir > 0 ? link[i * d + j] * p[a * d + j]
                                       : conj(link[j * d + i]) * p[a * d + j];
                    v[a][i] = acc;
                }
            /* (1 - dir*eta*g_mu) v, times the boundary sign */
            for (int a = 0; a < 4; a++)
                for (int i = 0; i < d; i++) {
                    w = v[a][i];
                    for (int b = 0; b < 4; b++)
                        w -= dir * eta * G[mu][a][b] * v[b][i];
                    o[a * d + i] += sign * w;
                }
        }
    }
}

/* Full-lattice hopping operator H (D = 1 - kappa H); when parity >= 0 only
 * sites of that parity are computed (others set to zero): this is the even-odd
 * block H_{p, 1-p}, which reads only sites of the opposite parity. */
void orc_hop(const int L[4], const int bc[4], int d, const double *Uin, int dagger,
             int parity, const double *in, double *out)
{
    build_gammas();
    long V = volume(L);
    const cplx *U = (const cplx *)Uin;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx *o = (cplx *)out + (size_t)s * 4 * d;
        if (parity >= 0 && orc_parity(L, s) != parity) {
            for (int k = 0; k < 4 * d; k++) o[k] = 0;
            continue;
        }
        hop_site(L, bc, d, U, dagger, (const cplx *)in, s, o);
    }
}

/* out = in - kappa * H in  (dagger: the adjoint operator) */
void orc_dslash(const int L[4], const int bc[4], int d, const double *Uin, double kappa,
                int dagger, const double *in, double *out)
{
    build_gammas();
    long V = volume(L);
    const cplx *U = (const cplx *)Uin;
    const cplx *pin = (const cplx *)in;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx *o = (cplx *)out + (size_t)s * 4 * d;
        hop_site(L, bc, d, U, dagger, pin, s, o);
        for (int k = 0; k < 4 * d; k++) o[k] = pin[(size_t)s * 4 * d + k] - kappa * o[k];
    }
}

/* D psi evaluated at a list of sites only (for spot checks on big lattices):
 * out[k] = (D in)(sites[k]) */
void orc_dslash_sites(const int L[4], const int bc[4], int d, const double *Uin, double kappa,
                      int dagger, const double *in, long nsites, const long *sites, double *out)
{
    build_gammas();
    const cplx *U = (const cplx *)Uin;
    const cplx *pin = (const cplx *)in;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsites; k++) {
        cplx *o = (cplx *)out + (size_t)k * 4 * d;
        long s = sites[k];
        hop_site(L, bc, d, U, dagger, pin, s, o);
        for (int c = 0; c < 4 * d; c++) o[c] = pin[(size_t)s * 4 * d + c] - kappa * o[c];
    }
}

/* ------------------------------------------------------------------ */
/* vectors                                                             */
/* ------------------------------------------------------------------ */

static double vnorm2(long n, const cplx *a)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static double vdot_re(long n, const cplx *a, const cplx *b)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < n; i++) s += creal(conj(a[i]) * b[i]);
    return s;
}

/* ------------------------------------------------------------------ */
/* operators M used by the solvers                                     */
/*   kind 0: full D on the whole lattice                              */
/*   kind 1: Schur complement Dhat = 1 - kappa^2 H_eo H_oe on even sites */
/* ------------------------------------------------------------------ */

typedef struct {
    int kind, d;
    int L[4], bc[4];
    const double *U;
    double kappa;
    long V;
    cplx *tmp;   /* full-lattice work vector */
} op_t;

static void op_apply(op_t *op, int dagger, const cplx *in, cplx *out)
{
    long n = op->V * 4 * op->d;
    if (op->kind == 0) {
        orc_dslash(op->L, op->bc, op->d, op->U, op->kappa, dagger, (const double *)in, (double *)out);
        return;
    }
    /* tmp_o = H_oe in_e ; out_e = in_e - kappa^2 H_eo tmp_o ; odd sites of out = 0 */
    orc_hop(op->L, op->bc, op->d, op->U, dagger, 1, (const double *)in, (double *)op->tmp);
    orc_hop(op->L, op->bc, op->d, op->U, dagger, 0, (const double *)op->tmp, (double *)out);
    double k2 = op->kappa * op->kappa;
    int d = op->d;
#pragma omp parallel for schedule(static)
    for (long s = 0; s < op->V; s++) {
        int even = orc_parity(op->L, s) == 0;
        for (int c = 0; c < 4 * d; c++) {
            size_t i = (size_t)s * 4 * d + c;
            out[i] = even ? in[i] - k2 * out[i] : 0;
        }
    }
    (void)n;
}

/* CG on the normal equations M^dag M x = M^dag b (Hestenes-Stiefel),
 * starting from the x passed in.  Stops when |r|^2 <= tol2 * |M^dag b|^2 or
 * after maxit iterations.  Returns iterations done. */
static int cgnr(op_t *op, const cplx *b, cplx *x, double tol, int maxit, double *rel_normal)
{
    long n = op->V * 4 * op->d;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n);
    cplx *Ap = malloc(sizeof(cplx) * n), *t = malloc(sizeof(cplx) * n);
    cplx *rhs = malloc(sizeof(cplx) * n);
    op_apply(op, 1, b, rhs);                         /* M^dag b */
    double bn = vnorm2(n, rhs);
    op_apply(op, 0, x, t);                           /* r = M^dag (b - M x) */
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) t[i] = b[i] - t[i];
    op_apply(op, 1, t, r);
    memcpy(p, r, sizeof(cplx) * n);
    double rr = vnorm2(n, r);
    int it = 0;
    while (it < maxit && rr > tol * tol * bn) {
        op_apply(op, 0, p, t);
        op_apply(op, 1, t, Ap);
        double pAp = vdot_re(n, p, Ap);
        double alpha = rr / pAp;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
        double rr_new = vnorm2(n, r);
        double beta = rr_new / rr;
        rr = rr_new;
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
        it++;
    }
    if (rel_normal) *rel_normal = bn > 0 ? sqrt(rr / bn) : 0;
    free(r); free(p); free(Ap); free(t); free(rhs);
    return it;
}

/* || b - D x || / || b || on the full lattice */
double orc_true_residual(const int L[4], const int bc[4], int d, const double *U, double kappa,
                         const double *b, const double *x)
{
    long n = volume(L) * 4 * d;
    cplx *t = malloc(sizeof(cplx) * n);
    orc_dslash(L, bc, d, U, kappa, 0, x, (double *)t);
    const cplx *bb = (const cplx *)b;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) t[i] = bb[i] - t[i];
    double bn = vnorm2(n, bb), rn = vnorm2(n, t);
    free(t);
    return bn > 0 ? sqrt(rn / bn) : sqrt(rn);
}

/* Solve D x = b to a true relative residual <= tol.
 * schur = 0: CG on D^dag D over the whole lattice.
 * schur = 1: even-odd preconditioned: bhat_e = b_e + kappa H_eo b_o, CG on
 *            Dhat^dag Dhat for x_e, then x_o = b_o + kappa H_oe x_e.
 * The normal-equation residual only triggers the stop; the full-lattice true
 * residual decides, and if it is above tol the solve continues from the
 * current x with the trigger tightened by 0.3.
 * info[0] = iterations, info[1] = true relative residual, info[2] = restarts.
 * Returns 0 when converged, 1 otherwise. */
int orc_solve(const int L[4], const int bc[4], int d, const double *U, double kappa, int schur,
              const double *bin, double *xout, double tol, int maxit, double *info)
{
    build_gammas();
    op_t op;
    memcpy(op.L, L, sizeof op.L);
    memcpy(op.bc, bc, sizeof op.bc);
    op.d = d; op.U = U; op.kappa = kappa; op.V = volume(L); op.kind = schur ? 1 : 0;
    long n = op.V * 4 * d;
    op.tmp = malloc(sizeof(cplx) * n);
    const cplx *b = (const cplx *)bin;
    cplx *x = (cplx *)xout;
    cplx *bh = malloc(sizeof(cplx) * n);
    memset(x, 0, sizeof(cplx) * n);
    if (schur) {
        /* bh_e = b_e + kappa H_eo b_o ; odd entries zero */
        orc_hop(L, bc, d, U, 0, 0, bin, (double *)bh);
#pragma omp parallel for schedule(static)
        for (long s = 0; s < op.V; s++) {
            int even = orc_parity(L, s) == 0;
            for (int c = 0; c < 4 * d; c++) {
                size_t i = (size_t)s * 4 * d + c;
                bh[i] = even ? b[i] + kappa * bh[i] : 0;
            }
        }
    } else {
        memcpy(bh, b, sizeof(cplx) * n);
    }
    double trig = tol, res = INFINITY;
    int iters = 0, restarts = 0, ok = 0;
    for (;;) {
        iters += cgnr(&op, bh, x, trig, maxit - iters, NULL);
        if (schur) {
            /* x_o = b_o + kappa H_oe x_e */
            orc_hop(L, bc, d, U, 0, 1, (const double *)x, (double *)op.tmp);
#pragma omp parallel for schedule(static)
            for (long s = 0; s < op.V; s++) {
                if (orc_parity(L, s) == 0) continue;
                for (int c = 0; c < 4 * d; c++) {
                    size_t i = (size_t)s * 4 * d + c;
                    x[i] = b[i] + kappa * op.tmp[i];
                }
            }
        }
        res = orc_true_residual(L, bc, d, U, kappa, bin, xout);
        if (res <= tol) { ok = 1; break; }
        if (iters >= maxit) break;
        trig *= 0.3;
        restarts++;
        if (schur) {
            /* drop the odd part again: the Schur iteration lives on even sites */
#pragma omp parallel for schedule(static)
            for (long s = 0; s < op.V; s++)
                if (orc_parity(L, s) == 1)
                    for (int c = 0; c < 4 * d; c++) x[(size_t)s * 4 * d + c] = 0;
        }
    }
    info[0] = iters; info[1] = res; info[2] = restarts;
    free(op.tmp); free(bh);
    return ok ? 0 : 1;
}

/* plain CG on the normal equations of D (kind 0) or of the Schur complement
 * (kind 1) to a normal-residual target only, returning the iterate after
 * exactly the iterations it took; used by tests that count iterations. */
int orc_cgnr_raw(const int L[4], const int bc[4], int d, const double *U, double kappa, int kind,
                 const double *b, double *x, double tol, int maxit, double *rel_normal)
{
    build_gammas();
    op_t op;
    memcpy(op.L, L, sizeof op.L);
    memcpy(op.bc, bc, sizeof op.bc);
    op.d = d; op.U = U; op.kappa = kappa; op.V = volume(L); op.kind = kind;
    op.tmp = malloc(sizeof(cplx) * op.V * 4 * d);
    int it = cgnr(&op, (const cplx *)b, (cplx *)x, tol, maxit, rel_normal);
    free(op.tmp);
    return it;
}

/* Schur operator (kind 1) or D (kind 0) applied once, exposed for tests */
void orc_op_apply(const int L[4], const int bc[4], int d, const double *U, double kappa, int kind,
                  int dagger, const double *in, double *out)
{
    build_gammas();
    op_t op;
    memcpy(op.L, L, sizeof op.L);
    memcpy(op.bc, bc, sizeof op.bc);
    op.d = d; op.U = U; op.kappa = kappa; op.V = volume(L); op.kind = kind;
    op.tmp = malloc(sizeof(cplx) * op.V * 4 * d);
    op_apply(&op, dagger, (const cplx *)in, (cplx *)out);
    free(op.tmp);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* parallel-transport convolution (PTC) layer                          */
/*   out_i(x) = sum_j sum_p W_p^{ij} (T_p in_j)(x)                      */
/* paths p: 0 = stay, 1 + mu = hop from x + mu, 5 + mu = hop from x - mu */
/*   T_0 in(x) = in(x)                                                 */
/*   T_{1+mu} in(x) = s+ U_mu(x) in(x + mu)                            */
/*   T_{5+mu} in(x) = s- U_mu(x - mu)^dag in(x - mu)                   */
/* W_p^{ij} is a complex 4 x 4 spin matrix; W layout                   */
/* [cout][cin][9][4][4]; channel fields [c][V][4][d].                  */
/* ------------------------------------------------------------------ */

/* t[a][i] = (T_p f)(s) for spinor field f */
static void transport(const int L[4], const int bc[4], int d, const cplx *U, int p, const cplx *f, long s,
                      cplx *t)
{
    if (p == 0) {
        for (int k = 0; k < 4 * d; k++) t[k] = f[(size_t)s * 4 * d + k];
        return;
    }
    int mu = (p - 1) % 4;
    int dir = p <= 4 ? +1 : -1;
    double sign;
    long y = neighbour(L, bc, s, mu, dir, &sign);
    const cplx *link = dir > 0 ? U + ((size_t)s * 4 + mu) * d * d : U + ((size_t)y * 4 + mu) * d * d;
    const cplx *v = f + (size_t)y * 4 * d;
    for (int a = 0; a < 4; a++)
        for (int i = 0; i < d; i++) {
            cplx acc = 0;
            for (int j = 0; j < d; j++)
                acc += dir > 0 ? link[i * d + j] * v[a * d + j] : conj(link[j * d + i]) * v[a * d + j];
            t[a * d + i] = sign * acc;
        }
}

static int reverse_path(int p) { return p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4); }

void orc_ptc_layer(const int L[4], const int bc[4], int d, const double *Uin, int cin, int cout,
                   const double *Win, const double *in, double *out)
{
    const cplx *U = (const cplx *)Uin, *W = (const cplx *)Win, *f = (const cplx *)in;
    cplx *o = (cplx *)out;
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx t[4 * 16];
        for (int i = 0; i < cout; i++)
            for (int k = 0; k < 4 * d; k++) o[((size_t)i * V + s) * 4 * d + k] = 0;
        for (int j = 0; j < cin; j++)
            for (int p = 0; p < 9; p++) {
                transport(L, bc, d, U, p, f + (size_t)j * V * 4 * d, s, t);
                for (int i = 0; i < cout; i++) {
                    const cplx *w = W + (((size_t)i * cin + j) * 9 + p) * 16;
                    cplx *oi = o + ((size_t)i * V + s) * 4 * d;
                    for (int a = 0; a < 4; a++)
                        for (int b = 0; b < 4; b++)
                            for (int c = 0; c < d; c++) oi[a * d + c] += w[a * 4 + b] * t[b * d + c];
                }
            }
    }
}

/* the adjoint layer: out_j = sum_i sum_p (W_p^{ij})^dag (T_{rev p} in_i),
 * in: [cout][V][4][d] -> out: [cin][V][4][d] (T_p^dag = T_{rev p}) */
void orc_ptc_layer_adjoint(const int L[4], const int bc[4], int d, const double *Uin, int cin, int cout,
                           const double *Win, const double *in, double *out)
{
    const cplx *U = (const cplx *)Uin, *W = (const cplx *)Win, *f = (const cplx *)in;
    cplx *o = (cplx *)out;
    long V = volume(L);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < V; s++) {
        cplx t[4 * 16];
        for (int j = 0; j < cin; j++)
            for (int k = 0; k < 4 * d; k++) o[((size_t)j * V + s) * 4 * d + k] = 0;
        for (int i = 0; i < cout; i++)
            for (int p = 0; p < 9; p++) {
                transport(L, bc, d, U, reverse_path(p), f + (size_t)i * V * 4 * d, s, t);
                for (int j = 0; j < cin; j++) {
                    const cplx *w = W + (((size_t)i * cin + j) * 9 + p) * 16;
                    cplx *oj = o + ((size_t)j * V + s) * 4 * d;
                    for (int a = 0; a < 4; a++)
                        for (int b = 0; b < 4; b++)
                            for (int c = 0; c < d; c++) oj[b * d + c] += conj(w[a * 4 + b]) * t[a * d + c];
                }
            }
    }
}

/* gradient of a real loss with respect to W (Wirtinger convention
 * dL/dRe W + i dL/dIm W) given G = dL/dRe out + i dL/dIm out and the layer
 * input v:  dW_p^{ij}[a][b] = sum_x sum_c G_i(x)[a][c] conj((T_p v_j)(x)[b][c]) */
void orc_ptc_weight_grad(const int L[4], const int bc[4], int d, const double *Uin, int cin, int cout,
                         const double *Gin, const double *vin, double *dWout)
{
    const cplx *U = (const cplx *)Uin, *G = (const cplx *)Gin, *v = (const cplx *)vin;
    cplx *dW = (cplx *)dWout;
    long V = volume(L);
    size_t nw = (size_t)cout * cin * 9 * 16;
    for (size_t k = 0; k < nw; k++) dW[k] = 0;
#pragma omp parallel
    {
        cplx *loc = calloc(nw, sizeof(cplx));
        cplx t[4 * 16];
#pragma omp for schedule(static)
        for (long s = 0; s < V; s++)
            for (int j = 0; j < cin; j++)
                for (int p = 0; p < 9; p++) {
                    transport(L, bc, d, U, p, v + (size_t)j * V * 4 * d, s, t);
                    for (int i = 0; i < cout; i++) {
                        const cplx *g = G + ((size_t)i * V + s) * 4 * d;
                        cplx *w = loc + (((size_t)i * cin + j) * 9 + p) * 16;
                        for (int a = 0; a < 4; a++)
                            for (int b = 0; b < 4; b++)
                                for (int c = 0; c < d; c++) w[a * 4 + b] += g[a * d + c] * conj(t[b * d + c]);
                    }
                }
#pragma omp critical
        for (size_t k = 0; k < nw; k++) dW[k] += loc[k];
        free(loc);
    }
}
