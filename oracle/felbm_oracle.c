/*
 * Plain FP64 CPU oracle of the finite-element lattice Boltzmann method for
 * binary fluids (Matin, Misztal, Hernandez-Garcia, Mathiesen, arXiv
 * 1608.01906).  TEST INFRASTRUCTURE ONLY: the product path never calls,
 * links or loads this file; the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.
 *
 * It is written to be checked against the paper by eye: scalar loops over
 * elements and nodes, no blocking, no fusion, no assembled sparse matrix.
 * Every operator is applied element by element from the element volume and
 * the constant gradients of the linear shape functions.  The only
 * concurrency is across populations in the streaming stage (OpenMP, one
 * population per thread at a time), which leaves every population's
 * arithmetic and its order unchanged.
 *
 *  - Streaming (Section 2.2.1, Taylor expansion and Galerkin weak form):
 *      M (psi^{n+1} - psi^n) = -(dt C_a + dt^2 D_a) psi^n
 *    with M = int N N^T, C_a = int N c_ar d_r N^T,
 *    D_a = 1/2 int d_s N c_as c_ar d_r N^T.
 *    Consistent mass: M is inverted by conjugate gradients preconditioned
 *    with diag(M), iterated to round-off.  Lumped mass (the paper's choice
 *    at the end of Section 2.2.1): M is replaced by its row sums.
 *  - Discrete derivatives (Section 2.3): element-constant gradients of the
 *    linearly interpolated nodal field, averaged at each node with the
 *    element volumes as weights.
 *  - Collision and forcing (Sections 2.1 and 2.2): BGK operator, potential
 *    form F for the order parameter, stress form G for the
 *    pressure-momentum distribution, exact-difference body force, the
 *    post-streaming collision with factor 2 tau / (2 tau + 1) and the
 *    pre-streaming collision for the next step, done literally as two
 *    stages from the same nodal fields.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *  - 2-D runs use D2Q9 with the same formulas (the paper is 3-D, D3Q19);
 *    lattice weights are the standard ones, cs^2 = 1/3.
 *  - The moments (density, momentum, pressure) are taken from the streamed
 *    populations and used for both collision stages of a step.
 *  - The body force is 1/2 [g_eq(rho, u + g dt) - g_eq(rho, u)], whose
 *    momentum (dt/2) rho g matches the momentum moment of Section 2.2.
 *  - The Laplacian of rho is the recovered divergence of the recovered
 *    gradient; the stress term recovers the derivatives of the nodal
 *    products |grad rho|^2 and d_i rho d_j rho.
 *  - tau uses the composition clamped to [0, 1].
 *  - Walls: natural boundary in the weak form; after streaming, each
 *    population at a wall node pointing into the fluid takes the value of
 *    its opposite (nodal bounce-back).  A direction points into the fluid
 *    when e.n > 1e-12 for the wall's inward unit normal n: on a curved wall a
 *    direction tangential to the wall (e.n = 0) evaluates to a rounding-size
 *    number of either sign, and is left alone.
 *  - Initial state: equilibrium of the given rho, u, p plus the forcing of
 *    a pre-streaming collision (whose BGK part vanishes there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ESTATE -4
#define ORC_ENOTCONV -5

/* ---- velocity sets (standard weights; cs^2 = 1/3) ---------------------- */

static const int Q9E[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double Q9W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                              1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const int Q19E[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double Q19W[19] = {
    1.0 / 3,
    1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const double CS2 = 1.0 / 3.0;

typedef struct {
    int Q, dim;
    double e[19][3];
    double w[19];
    int opp[19];
} lattice_t;

static int make_lattice(int Q, lattice_t *L) {
    if (Q != 9 && Q != 19) return ORC_EINVAL;
    L->Q = Q;
    L->dim = (Q == 9) ? 2 : 3;
    for (int a = 0; a < Q; a++) {
        for (int r = 0; r < 3; r++) L->e[a][r] = (Q == 9) ? Q9E[a][r] : Q19E[a][r];
        L->w[a] = (Q == 9) ? Q9W[a] : Q19W[a];
    }
    for (int a = 0; a < Q; a++) {
        L->opp[a] = -1;
        for (int b = 0; b < Q; b++)
            if (L->e[b][0] == -L->e[a][0] && L->e[b][1] == -L->e[a][1] && L->e[b][2] == -L->e[a][2])
                L->opp[a] = b;
    }
    return ORC_OK;
}

/* ---- oracle state ------------------------------------------------------ */

typedef struct orc {
    lattice_t L;
    int dim, nv;               /* nv = dim + 1 vertices per element */
    int64_t N, E;
    int32_t *conn;             /* [E][nv] */
    double *vol;               /* [E] element volume */
    double *grad;              /* [E][nv][dim] gradient of each shape function */
    double *mlump;             /* [N] row sums of M = sum over elements of V/(d+1) */
    double *mdiag;             /* [N] diagonal of M */
    uint8_t *wall;             /* [N] */
    double *wnormal;           /* [N][dim] */
    /* physics */
    double rho_l, rho_v, tau_l, tau_v, sigma, xi, dt, grav[3];
    double beta, kappa;
    int have_phys;
    /* options */
    int mass_mode;             /* 0 consistent, 1 lumped */
    int lap_mode;              /* 0 recovered divergence of recovered gradient, 1 weak form */
    double cg_tol;
    int cg_maxit;
    /* state */
    int have_state;
    double *psibar;            /* [2Q][N]: f_0..f_{Q-1}, g_0..g_{Q-1} (pre-streaming collided) */
    /* last fields */
    double *rho, *u, *p;       /* [N], [N][dim], [N] */
    double *gradrho, *lap, *S, *mu, *gradmu;  /* diagnostics of the last step */
    double *delta;             /* [2Q][N] streaming increments of the last step */
    int last_cg_iters;
    double last_cg_relres;
    int threads;               /* threads over populations (0 = the OpenMP default) */
} orc;

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

void orc_destroy(orc *o) {
    if (!o) return;
    free(o->conn); free(o->vol); free(o->grad); free(o->mlump); free(o->mdiag);
    free(o->wall); free(o->wnormal); free(o->psibar); free(o->rho); free(o->u); free(o->p);
    free(o->gradrho); free(o->lap); free(o->S); free(o->mu); free(o->gradmu); free(o->delta);
    free(o);
}

/* Element geometry from the unwrapped vertex positions. */
static int element_geometry(int dim, const double X[4][3], double *vol, double g[4][3]) {
    if (dim == 2) {
        double j00 = X[1][0] - X[0][0], j01 = X[2][0] - X[0][0];
        double j10 = X[1][1] - X[0][1], j11 = X[2][1] - X[0][1];
        double det = j00 * j11 - j01 * j10;
        if (!(det > 0.0)) return ORC_EINVAL;
        *vol = det / 2.0;
        /* rows of J^{-1} are the gradients of the barycentric coordinates 1, 2 */
        g[1][0] = j11 / det;  g[1][1] = -j01 / det;
        g[2][0] = -j10 / det; g[2][1] = j00 / det;
        g[0][0] = -g[1][0] - g[2][0];
        g[0][1] = -g[1][1] - g[2][1];
        return ORC_OK;
    }
    double J[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) J[r][c] = X[c + 1][r] - X[0][r];
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0)) return ORC_EINVAL;
    *vol = det / 6.0;
    /* inverse by cofactors: Jinv[r][c] = cof[c][r] / det */
    double inv[3][3];
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int a = 1; a <= 3; a++)
        for (int r = 0; r < 3; r++) g[a][r] = inv[a - 1][r];
    for (int r = 0; r < 3; r++) g[0][r] = -(g[1][r] + g[2][r] + g[3][r]);
    return ORC_OK;
}

orc *orc_create(int Q, int dim, int64_t n_nodes, const double *xyz, int64_t n_elems,
                const int32_t *conn, const int8_t *shift, const double *box,
                const uint8_t *wall, const double *wall_normal, int *err) {
    *err = ORC_EINVAL;
    lattice_t L;
    if (make_lattice(Q, &L) != ORC_OK || L.dim != dim || n_nodes <= 0 || n_elems <= 0)
        return NULL;
    orc *o = (orc *)xcalloc(1, sizeof(orc));
    if (!o) { *err = ORC_ENOMEM; return NULL; }
    o->L = L;
    o->dim = dim;
    o->nv = dim + 1;
    o->N = n_nodes;
    o->E = n_elems;
    o->mass_mode = 0;
    o->cg_tol = 1e-15;
    o->cg_maxit = 500;
    int nv = o->nv;
    o->conn = (int32_t *)xcalloc((size_t)n_elems * nv, sizeof(int32_t));
    o->vol = (double *)xcalloc((size_t)n_elems, sizeof(double));
    o->grad = (double *)xcalloc((size_t)n_elems * nv * dim, sizeof(double));
    o->mlump = (double *)xcalloc((size_t)n_nodes, sizeof(double));
    o->mdiag = (double *)xcalloc((size_t)n_nodes, sizeof(double));
    o->wall = (uint8_t *)xcalloc((size_t)n_nodes, 1);
    o->wnormal = (double *)xcalloc((size_t)n_nodes * dim, sizeof(double));
    if (!o->conn || !o->vol || !o->grad || !o->mlump || !o->mdiag || !o->wall || !o->wnormal) {
        orc_destroy(o);
        *err = ORC_ENOMEM;
        return NULL;
    }
    memcpy(o->conn, conn, (size_t)n_elems * nv * sizeof(int32_t));
    if (wall) memcpy(o->wall, wall, (size_t)n_nodes);
    if (wall_normal) memcpy(o->wnormal, wall_normal, (size_t)n_nodes * dim * sizeof(double));
    for (int64_t e = 0; e < n_elems; e++) {
        double X[4][3] = {{0}};
        for (int a = 0; a < nv; a++) {
            int32_t k = conn[e * nv + a];
            if (k < 0 || k >= n_nodes) { orc_destroy(o); return NULL; }
            for (int r = 0; r < dim; r++) {
                double s = shift ? (double)shift[(e * nv + a) * dim + r] : 0.0;
                X[a][r] = xyz[k * dim + r] + s * (box ? box[r] : 0.0);
            }
        }
        double g[4][3];
        if (element_geometry(dim, X, &o->vol[e], g) != ORC_OK) { orc_destroy(o); return NULL; }
        for (int a = 0; a < nv; a++)
            for (int r = 0; r < dim; r++) o->grad[(e * nv + a) * dim + r] = g[a][r];
        /* M_T[a][b] = V (1 + delta_ab) / ((d+1)(d+2)) */
        double V = o->vol[e];
        for (int a = 0; a < nv; a++) {
            int32_t k = conn[e * nv + a];
            o->mlump[k] += V / nv;
            o->mdiag[k] += 2.0 * V / (nv * (nv + 1));
        }
    }
    *err = ORC_OK;
    return o;
}

int orc_set_phys(orc *o, const double *ph) {
    o->rho_l = ph[0]; o->rho_v = ph[1]; o->tau_l = ph[2]; o->tau_v = ph[3];
    o->sigma = ph[4]; o->xi = ph[5]; o->dt = ph[6];
    o->grav[0] = ph[7]; o->grav[1] = ph[8]; o->grav[2] = ph[9];
    double drho = o->rho_l - o->rho_v;
    if (!(drho > 0.0) || !(o->tau_l > 0.0) || !(o->tau_v > 0.0) || !(o->dt > 0.0) ||
        !(o->xi > 0.0) || o->sigma < 0.0)
        return ORC_EINVAL;
    /* beta and kappa from sigma and xi (Section 2.1) */
    o->beta = 12.0 * o->sigma / (o->xi * pow(drho, 4));
    o->kappa = 1.5 * o->xi * o->sigma / (drho * drho);
    o->have_phys = 1;
    return ORC_OK;
}

int orc_set_options(orc *o, int mass_mode, int lap_mode, double cg_tol, int cg_maxit) {
    if (mass_mode != 0 && mass_mode != 1) return ORC_EINVAL;
    if (lap_mode != 0 && lap_mode != 1) return ORC_EINVAL;
    o->mass_mode = mass_mode;
    o->lap_mode = lap_mode;
    if (cg_tol > 0) o->cg_tol = cg_tol;
    if (cg_maxit > 0) o->cg_maxit = cg_maxit;
    return ORC_OK;
}

/* ---- element-by-element operators -------------------------------------- */

/* y = M x with M = int N N^T */
int orc_apply_M(const orc *o, const double *x, double *y) {
    int nv = o->nv;
    memset(y, 0, (size_t)o->N * sizeof(double));
    for (int64_t e = 0; e < o->E; e++) {
        const int32_t *c = &o->conn[e * nv];
        double V = o->vol[e];
        for (int a = 0; a < nv; a++) {
            double s = 0.0;
            for (int b = 0; b < nv; b++)
                s += V * (a == b ? 2.0 : 1.0) / (nv * (nv + 1)) * x[c[b]];
            y[c[a]] += s;
        }
    }
    return ORC_OK;
}

/* y = (dt C_alpha + dt^2 D_alpha) x, the streaming operator of direction alpha:
 * C[a][b] = int N_a c_r d_r N_b = (V/(d+1)) c.grad N_b
 * D[a][b] = 1/2 int (c.grad N_a)(c.grad N_b) = V/2 (c.grad N_a)(c.grad N_b)   */
int orc_apply_A(const orc *o, int alpha, const double *x, double *y) {
    if (alpha < 0 || alpha >= o->L.Q) return ORC_EINVAL;
    int nv = o->nv, dim = o->dim;
    const double *c = o->L.e[alpha];
    double dt = o->dt;
    memset(y, 0, (size_t)o->N * sizeof(double));
    for (int64_t e = 0; e < o->E; e++) {
        const int32_t *cn = &o->conn[e * nv];
        const double *g = &o->grad[e * nv * dim];
        double V = o->vol[e];
        double cg[4];
        for (int a = 0; a < nv; a++) {
            cg[a] = 0.0;
            for (int r = 0; r < dim; r++) cg[a] += c[r] * g[a * dim + r];
        }
        for (int a = 0; a < nv; a++) {
            double s = 0.0;
            for (int b = 0; b < nv; b++) {
                double Cab = V / nv * cg[b];
                double Dab = 0.5 * V * cg[a] * cg[b];
                s += (dt * Cab + dt * dt * Dab) * x[cn[b]];
            }
            y[cn[a]] += s;
        }
    }
    return ORC_OK;
}

/* Volume-weighted nodal recovery of the element gradients (Section 2.3).
 * out is [N][dim]. */
int orc_recover_grad(const orc *o, const double *phi, double *out) {
    int nv = o->nv, dim = o->dim;
    double *den = (double *)xcalloc((size_t)o->N, sizeof(double));
    if (!den) return ORC_ENOMEM;
    memset(out, 0, (size_t)o->N * dim * sizeof(double));
    for (int64_t e = 0; e < o->E; e++) {
        const int32_t *cn = &o->conn[e * nv];
        const double *g = &o->grad[e * nv * dim];
        double gT[3] = {0, 0, 0};
        for (int b = 0; b < nv; b++)
            for (int r = 0; r < dim; r++) gT[r] += phi[cn[b]] * g[b * dim + r];
        for (int a = 0; a < nv; a++) {
            for (int r = 0; r < dim; r++) out[(int64_t)cn[a] * dim + r] += o->vol[e] * gT[r];
            den[cn[a]] += o->vol[e];
        }
    }
    for (int64_t k = 0; k < o->N; k++)
        for (int r = 0; r < dim; r++) out[k * dim + r] /= den[k];
    free(den);
    return ORC_OK;
}

int orc_lumped_mass(const orc *o, double *m) {
    memcpy(m, o->mlump, (size_t)o->N * sizeof(double));
    return ORC_OK;
}

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/* Solve M x = b by conjugate gradients preconditioned with diag(M), from
 * x = 0, until |r| <= tol |b| or the residual stops decreasing. */
int orc_solve_M(const orc *o, const double *b, double *x, int *iters, double *relres) {
    int64_t N = o->N;
    double *r = (double *)xcalloc((size_t)N, sizeof(double));
    double *z = (double *)xcalloc((size_t)N, sizeof(double));
    double *p = (double *)xcalloc((size_t)N, sizeof(double));
    double *q = (double *)xcalloc((size_t)N, sizeof(double));
    double *xbest = (double *)xcalloc((size_t)N, sizeof(double));
    if (!r || !z || !p || !q || !xbest) {
        free(r); free(z); free(p); free(q); free(xbest);
        return ORC_ENOMEM;
    }
    memset(x, 0, (size_t)N * sizeof(double));
    double bn = sqrt(dot(N, b, b));
    int it = 0, rc = ORC_OK;
    double rel = 0.0;
    if (bn > 0.0) {
        memcpy(r, b, (size_t)N * sizeof(double));
        for (int64_t i = 0; i < N; i++) z[i] = r[i] / o->mdiag[i];
        memcpy(p, z, (size_t)N * sizeof(double));
        double rz = dot(N, r, z);
        double best = 1.0;
        int since_best = 0;
        rel = 1.0;
        while (it < o->cg_maxit) {
            orc_apply_M(o, p, q);
            double alpha = rz / dot(N, p, q);
            for (int64_t i = 0; i < N; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            it++;
            rel = sqrt(dot(N, r, r)) / bn;
            if (rel < best) {
                best = rel;
                since_best = 0;
                memcpy(xbest, x, (size_t)N * sizeof(double));
            } else if (++since_best >= 8) {
                break;
            }
            if (rel <= o->cg_tol) break;
            for (int64_t i = 0; i < N; i++) z[i] = r[i] / o->mdiag[i];
            double rz_new = dot(N, r, z);
            double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < N; i++) p[i] = z[i] + beta * p[i];
        }
        memcpy(x, xbest, (size_t)N * sizeof(double));
        rel = best;
        if (rel > 1e-12) rc = ORC_ENOTCONV;
    }
    if (iters) *iters = it;
    if (relres) *relres = rel;
    free(r); free(z); free(p); free(q); free(xbest);
    return rc;
}

/* ---- local collision and forcing (Sections 2.1, 2.2) -------------------- */

typedef struct {
    double rho, u[3], p, tau;
    double gradrho[3], S[3], gradmu[3];
} nodefields_t;

/* Gamma_a(u) = f_eq / rho */
static double Gamma(const lattice_t *L, int a, const double u[3]) {
    double eu = 0.0, uu = 0.0;
    for (int r = 0; r < 3; r++) { eu += L->e[a][r] * u[r]; uu += u[r] * u[r]; }
    return L->w[a] * (1.0 + eu / CS2 + (eu * eu - CS2 * uu) / (2.0 * CS2 * CS2));
}

static double feq_a(const lattice_t *L, int a, double rho, const double u[3]) {
    return rho * Gamma(L, a, u);
}

static double geq_a(const lattice_t *L, int a, double rho, double p, const double u[3]) {
    const double zero[3] = {0, 0, 0};
    return L->w[a] * p / CS2 + rho * (Gamma(L, a, u) - Gamma(L, a, zero));
}

/* Per-direction terms at one node: equilibria, forcing F (order parameter),
 * G (pressure-momentum) and the exact-difference body force. */
static void node_terms(const orc *o, int a, const nodefields_t *nf, double *feq, double *geq,
                       double *F, double *G, double *Gb) {
    const lattice_t *L = &o->L;
    const double zero[3] = {0, 0, 0};
    double dt = o->dt;
    double Gu = Gamma(L, a, nf->u), G0 = Gamma(L, a, zero);
    double emu_f = 0.0, emu_g1 = 0.0, emu_S = 0.0;
    for (int r = 0; r < 3; r++) {
        double em = L->e[a][r] - nf->u[r];
        emu_f += em * (nf->gradrho[r] * CS2 - nf->rho * nf->gradmu[r]);
        emu_g1 += em * nf->gradrho[r];
        emu_S += em * nf->S[r];
    }
    *feq = feq_a(L, a, nf->rho, nf->u);
    *geq = geq_a(L, a, nf->rho, nf->p, nf->u);
    *F = 0.5 * dt * emu_f / CS2 * Gu;
    *G = 0.5 * dt * emu_g1 * (Gu - G0) + 0.5 * dt * emu_S / CS2 * Gu;
    double u2[3];
    for (int r = 0; r < 3; r++) u2[r] = nf->u[r] + o->grav[r] * dt;
    *Gb = 0.5 * (geq_a(L, a, nf->rho, nf->p, u2) - *geq);
}

/* Exposed for the moment pins: terms of every direction at one node. */
int orc_node_terms(const orc *o, const double *in, double *feq, double *geq, double *F, double *G,
                   double *Gb) {
    /* in = rho, u[3], p, gradrho[3], S[3], gradmu[3] */
    nodefields_t nf;
    nf.rho = in[0];
    for (int r = 0; r < 3; r++) {
        nf.u[r] = in[1 + r];
        nf.gradrho[r] = in[5 + r];
        nf.S[r] = in[8 + r];
        nf.gradmu[r] = in[11 + r];
    }
    nf.p = in[4];
    for (int a = 0; a < o->L.Q; a++) node_terms(o, a, &nf, &feq[a], &geq[a], &F[a], &G[a], &Gb[a]);
    return ORC_OK;
}

/* Weak-form Laplacian: lap = -m^-1 K phi with K = int grad N . grad N^T
 * (natural boundary), i.e. the Galerkin Laplacian with lumped mass. */
int orc_weak_laplacian(const orc *o, const double *phi, double *out) {
    int nv = o->nv, dim = o->dim;
    memset(out, 0, (size_t)o->N * sizeof(double));
    for (int64_t e = 0; e < o->E; e++) {
        const int32_t *cn = &o->conn[e * nv];
        const double *g = &o->grad[e * nv * dim];
        for (int a = 0; a < nv; a++) {
            double s = 0.0;
            for (int b = 0; b < nv; b++) {
                double gg = 0.0;
                for (int r = 0; r < dim; r++) gg += g[a * dim + r] * g[b * dim + r];
                s += o->vol[e] * gg * phi[cn[b]];
            }
            out[cn[a]] -= s;
        }
    }
    for (int64_t k = 0; k < o->N; k++) out[k] /= o->mlump[k];
    return ORC_OK;
}

static double mu_phi(const orc *o, double rho) {
    return 4.0 * o->beta * (rho - o->rho_v) * (rho - o->rho_l) * (rho - 0.5 * (o->rho_v + o->rho_l));
}

static double tau_of(const orc *o, double rho) {
    double C = (rho - o->rho_v) / (o->rho_l - o->rho_v);
    if (C < 0.0) C = 0.0;
    if (C > 1.0) C = 1.0;
    return 1.0 / (C / o->tau_l + (1.0 - C) / o->tau_v);
}

/* Derivatives of Section 2.3 for a nodal density field:
 * grad rho, Laplacian (recovered divergence of recovered gradient), stress
 * vector S_i = kappa [d_i(|grad rho|^2) - d_j(d_i rho d_j rho)], chemical
 * potential mu = mu_phi(rho) - kappa lap rho, and grad mu. */
static int derivatives(orc *o, const double *rho) {
    int64_t N = o->N;
    int dim = o->dim;
    double *comp = (double *)xcalloc((size_t)N, sizeof(double));
    double *gtmp = (double *)xcalloc((size_t)N * dim, sizeof(double));
    if (!comp || !gtmp) { free(comp); free(gtmp); return ORC_ENOMEM; }
    orc_recover_grad(o, rho, o->gradrho);
    if (o->lap_mode == 0) {
        memset(o->lap, 0, (size_t)N * sizeof(double));
        for (int r = 0; r < dim; r++) {
            for (int64_t k = 0; k < N; k++) comp[k] = o->gradrho[k * dim + r];
            orc_recover_grad(o, comp, gtmp);
            for (int64_t k = 0; k < N; k++) o->lap[k] += gtmp[k * dim + r];
        }
    } else {
        orc_weak_laplacian(o, rho, o->lap);
    }
    /* S_i = kappa [ d_i E - sum_j d_j T_ij ], E = |grad rho|^2, T_ij = d_i rho d_j rho */
    memset(o->S, 0, (size_t)N * dim * sizeof(double));
    for (int64_t k = 0; k < N; k++) {
        double E = 0.0;
        for (int r = 0; r < dim; r++) E += o->gradrho[k * dim + r] * o->gradrho[k * dim + r];
        comp[k] = E;
    }
    orc_recover_grad(o, comp, gtmp);
    for (int64_t k = 0; k < N * dim; k++) o->S[k] += o->kappa * gtmp[k];
    for (int i = 0; i < dim; i++)
        for (int j = 0; j < dim; j++) {
            for (int64_t k = 0; k < N; k++) comp[k] = o->gradrho[k * dim + i] * o->gradrho[k * dim + j];
            orc_recover_grad(o, comp, gtmp);
            for (int64_t k = 0; k < N; k++) o->S[k * dim + i] -= o->kappa * gtmp[k * dim + j];
        }
    for (int64_t k = 0; k < N; k++) o->mu[k] = mu_phi(o, rho[k]) - o->kappa * o->lap[k];
    orc_recover_grad(o, o->mu, o->gradmu);
    free(comp);
    free(gtmp);
    return ORC_OK;
}

static void load_nodefields(const orc *o, int64_t k, nodefields_t *nf) {
    int dim = o->dim;
    memset(nf, 0, sizeof(*nf));
    nf->rho = o->rho[k];
    nf->p = o->p[k];
    for (int r = 0; r < dim; r++) {
        nf->u[r] = o->u[k * dim + r];
        nf->gradrho[r] = o->gradrho[k * dim + r];
        nf->S[r] = o->S[k * dim + r];
        nf->gradmu[r] = o->gradmu[k * dim + r];
    }
    nf->tau = tau_of(o, nf->rho);
}

static int alloc_state(orc *o) {
    int64_t N = o->N;
    int Q = o->L.Q, dim = o->dim;
    if (o->psibar) return ORC_OK;
    o->psibar = (double *)xcalloc((size_t)2 * Q * N, sizeof(double));
    o->delta = (double *)xcalloc((size_t)2 * Q * N, sizeof(double));
    o->rho = (double *)xcalloc((size_t)N, sizeof(double));
    o->u = (double *)xcalloc((size_t)N * dim, sizeof(double));
    o->p = (double *)xcalloc((size_t)N, sizeof(double));
    o->gradrho = (double *)xcalloc((size_t)N * dim, sizeof(double));
    o->lap = (double *)xcalloc((size_t)N, sizeof(double));
    o->S = (double *)xcalloc((size_t)N * dim, sizeof(double));
    o->mu = (double *)xcalloc((size_t)N, sizeof(double));
    o->gradmu = (double *)xcalloc((size_t)N * dim, sizeof(double));
    if (!o->psibar || !o->delta || !o->rho || !o->u || !o->p || !o->gradrho || !o->lap || !o->S ||
        !o->mu || !o->gradmu)
        return ORC_ENOMEM;
    return ORC_OK;
}

/* Initial state: psi = psi_eq(rho, u, p); psibar = psi + forcing (the BGK
 * part of the pre-streaming collision vanishes at equilibrium). */
int orc_init(orc *o, const double *rho, const double *u, const double *p) {
    if (!o->have_phys) return ORC_ESTATE;
    int rc = alloc_state(o);
    if (rc) return rc;
    int64_t N = o->N;
    int Q = o->L.Q, dim = o->dim;
    memcpy(o->rho, rho, (size_t)N * sizeof(double));
    memcpy(o->u, u, (size_t)N * dim * sizeof(double));
    memcpy(o->p, p, (size_t)N * sizeof(double));
    rc = derivatives(o, o->rho);
    if (rc) return rc;
    for (int64_t k = 0; k < N; k++) {
        nodefields_t nf;
        load_nodefields(o, k, &nf);
        for (int a = 0; a < Q; a++) {
            double feq, geq, F, G, Gb;
            node_terms(o, a, &nf, &feq, &geq, &F, &G, &Gb);
            o->psibar[(int64_t)a * N + k] = feq + F;
            o->psibar[(int64_t)(Q + a) * N + k] = geq + G + Gb;
        }
    }
    memset(o->delta, 0, (size_t)2 * Q * N * sizeof(double));
    o->have_state = 1;
    return ORC_OK;
}

/* Streams one population: M Delta = -(dt C_a + dt^2 D_a) psibar,
 * psibar_s = psibar + Delta.  Touches only that population's slices, so
 * the populations of a step are independent of each other. */
static int stream_population(orc *o, int pop, int *iters, double *relres) {
    int64_t N = o->N;
    int a = pop % o->L.Q;
    double *x = &o->psibar[(int64_t)pop * N];
    double *d = &o->delta[(int64_t)pop * N];
    double *rhs = (double *)xcalloc((size_t)N, sizeof(double));
    if (!rhs) return ORC_ENOMEM;
    int rc = ORC_OK;
    *iters = 0;
    *relres = 0.0;
    orc_apply_A(o, a, x, rhs);
    for (int64_t k = 0; k < N; k++) rhs[k] = -rhs[k];
    if (o->mass_mode == 1) {
        for (int64_t k = 0; k < N; k++) d[k] = rhs[k] / o->mlump[k];
    } else {
        rc = orc_solve_M(o, rhs, d, iters, relres);
    }
    if (rc != ORC_ENOMEM)
        for (int64_t k = 0; k < N; k++) x[k] += d[k];
    free(rhs);
    return rc;
}

static int one_step(orc *o) {
    int64_t N = o->N;
    int Q = o->L.Q, dim = o->dim;
    const lattice_t *L = &o->L;
    int rc = ORC_OK;
    int maxit = 0;
    double worst = 0.0;

    /* Streaming of all 2Q populations.  Each population is streamed and
     * solved on its own (the same operations in the same order whatever the
     * thread count, so the result does not depend on it); with OpenMP the
     * populations are spread over threads. */
    int pop_rc[38], pop_it[38];
    double pop_rel[38];
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(o->threads > 0 ? o->threads : omp_get_max_threads())
#endif
    for (int pop = 0; pop < 2 * Q; pop++)
        pop_rc[pop] = stream_population(o, pop, &pop_it[pop], &pop_rel[pop]);
    for (int pop = 0; pop < 2 * Q; pop++) {
        if (pop_rc[pop] == ORC_ENOMEM) return ORC_ENOMEM;
        if (pop_rc[pop] == ORC_ENOTCONV) rc = ORC_ENOTCONV;
        if (pop_it[pop] > maxit) maxit = pop_it[pop];
        if (pop_rel[pop] > worst) worst = pop_rel[pop];
    }
    o->last_cg_iters = maxit;
    o->last_cg_relres = worst;

    /* Walls: populations entering the fluid take the value of their opposite */
    for (int64_t k = 0; k < N; k++) {
        if (!o->wall[k]) continue;
        for (int a = 0; a < Q; a++) {
            double cn = 0.0;
            for (int r = 0; r < dim; r++) cn += L->e[a][r] * o->wnormal[k * dim + r];
            if (cn > 1e-12) {
                int b = L->opp[a];
                o->psibar[(int64_t)a * N + k] = o->psibar[(int64_t)b * N + k];
                o->psibar[(int64_t)(Q + a) * N + k] = o->psibar[(int64_t)(Q + b) * N + k];
            }
        }
    }

    /* Density: zeroth moment of the streamed f */
    for (int64_t k = 0; k < N; k++) {
        double s = 0.0;
        for (int a = 0; a < Q; a++) s += o->psibar[(int64_t)a * N + k];
        o->rho[k] = s;
    }
    int drc = derivatives(o, o->rho);
    if (drc) return drc;

    /* Momentum and pressure from the streamed g with the dt/2 corrections */
    for (int64_t k = 0; k < N; k++) {
        double mom[3] = {0, 0, 0}, sg = 0.0;
        for (int a = 0; a < Q; a++) {
            double g = o->psibar[(int64_t)(Q + a) * N + k];
            sg += g;
            for (int r = 0; r < dim; r++) mom[r] += L->e[a][r] * g;
        }
        double rho = o->rho[k];
        double ugr = 0.0;
        for (int r = 0; r < dim; r++) {
            mom[r] += 0.5 * o->dt * o->S[k * dim + r] + 0.5 * o->dt * rho * o->grav[r];
            o->u[k * dim + r] = mom[r] / rho;
            ugr += o->u[k * dim + r] * o->gradrho[k * dim + r];
        }
        o->p[k] = CS2 * sg + 0.5 * o->dt * ugr * CS2;
    }

    /* Post-streaming collision, then pre-streaming collision of the next step */
    for (int64_t k = 0; k < N; k++) {
        nodefields_t nf;
        load_nodefields(o, k, &nf);
        double tau = nf.tau;
        for (int a = 0; a < Q; a++) {
            double feq, geq, F, G, Gb;
            node_terms(o, a, &nf, &feq, &geq, &F, &G, &Gb);
            double *fb = &o->psibar[(int64_t)a * N + k];
            double *gb = &o->psibar[(int64_t)(Q + a) * N + k];
            double f = *fb + 2.0 * tau / (2.0 * tau + 1.0) * (-(*fb - feq) / (2.0 * tau) + F);
            double g = *gb + 2.0 * tau / (2.0 * tau + 1.0) * (-(*gb - geq) / (2.0 * tau) + G + Gb);
            *fb = f - (f - feq) / (2.0 * tau) + F;
            *gb = g - (g - geq) / (2.0 * tau) + G + Gb;
        }
    }
    return rc;
}

int orc_step(orc *o, int n) {
    if (!o->have_state) return ORC_ESTATE;
    int rc = ORC_OK;
    for (int s = 0; s < n; s++) {
        int r = one_step(o);
        if (r == ORC_ENOMEM) return r;
        if (r != ORC_OK) rc = r;
    }
    return rc;
}

/* Fields of the last step (or of the initial state): rho, u [N][dim], p, C */
int orc_fields(const orc *o, double *rho, double *u, double *p, double *C) {
    if (!o->have_state) return ORC_ESTATE;
    int64_t N = o->N;
    if (rho) memcpy(rho, o->rho, (size_t)N * sizeof(double));
    if (u) memcpy(u, o->u, (size_t)N * o->dim * sizeof(double));
    if (p) memcpy(p, o->p, (size_t)N * sizeof(double));
    if (C)
        for (int64_t k = 0; k < N; k++) C[k] = (o->rho[k] - o->rho_v) / (o->rho_l - o->rho_v);
    return ORC_OK;
}

/* which: 0 grad rho [N][dim], 1 lap rho [N], 2 S [N][dim], 3 mu [N],
 *        4 grad mu [N][dim], 5 Delta [2Q][N] of the last streaming */
int orc_aux(const orc *o, int which, double *out) {
    if (!o->have_state) return ORC_ESTATE;
    int64_t N = o->N;
    int dim = o->dim, Q = o->L.Q;
    switch (which) {
    case 0: memcpy(out, o->gradrho, (size_t)N * dim * sizeof(double)); break;
    case 1: memcpy(out, o->lap, (size_t)N * sizeof(double)); break;
    case 2: memcpy(out, o->S, (size_t)N * dim * sizeof(double)); break;
    case 3: memcpy(out, o->mu, (size_t)N * sizeof(double)); break;
    case 4: memcpy(out, o->gradmu, (size_t)N * dim * sizeof(double)); break;
    case 5: memcpy(out, o->delta, (size_t)2 * Q * N * sizeof(double)); break;
    default: return ORC_EINVAL;
    }
    return ORC_OK;
}

int orc_last_cg(const orc *o, int *iters, double *relres) {
    *iters = o->last_cg_iters;
    *relres = o->last_cg_relres;
    return ORC_OK;
}

/* out = sum m rho, sum m C, sum m (1 - C), sum m sum_a e_a gbar_a (3 comps),
 * with m the lumped mass, rho = sum_a fbar_a of the current state. */
int orc_conserved(const orc *o, double *out) {
    if (!o->have_state) return ORC_ESTATE;
    int64_t N = o->N;
    int Q = o->L.Q, dim = o->dim;
    for (int i = 0; i < 6; i++) out[i] = 0.0;
    for (int64_t k = 0; k < N; k++) {
        double rho = 0.0, mom[3] = {0, 0, 0};
        for (int a = 0; a < Q; a++) {
            rho += o->psibar[(int64_t)a * N + k];
            for (int r = 0; r < dim; r++) mom[r] += o->L.e[a][r] * o->psibar[(int64_t)(Q + a) * N + k];
        }
        double C = (rho - o->rho_v) / (o->rho_l - o->rho_v);
        double m = o->mlump[k];
        out[0] += m * rho;
        out[1] += m * C;
        out[2] += m * (1.0 - C);
        for (int r = 0; r < dim; r++) out[3 + r] += m * mom[r];
    }
    return ORC_OK;
}

int orc_get_state(const orc *o, double *psibar) {
    if (!o->have_state) return ORC_ESTATE;
    memcpy(psibar, o->psibar, (size_t)2 * o->L.Q * o->N * sizeof(double));
    return ORC_OK;
}

int orc_set_state(orc *o, const double *psibar) {
    if (!o->have_phys) return ORC_ESTATE;
    int rc = alloc_state(o);
    if (rc) return rc;
    memcpy(o->psibar, psibar, (size_t)2 * o->L.Q * o->N * sizeof(double));
    o->have_state = 1;
    return ORC_OK;
}

/* Threads the streaming of a step's populations may use (0 = the OpenMP
 * default; 1 = serial).  Results do not depend on it. */
int orc_set_threads(orc *o, int n) {
    if (n < 0) return ORC_EINVAL;
    o->threads = n;
    return ORC_OK;
}

/* Threads the OpenMP runtime offers by default (1 without OpenMP). */
int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_beta_kappa(const orc *o, double *bk) {
    bk[0] = o->beta;
    bk[1] = o->kappa;
    return ORC_OK;
}
