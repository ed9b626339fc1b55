/*
 * Plain serial FP64 reference of the Thetis hot path -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the package smoke check and the benchmark's CPU
 * baseline may load this file's library.  It shares no code, header, table
 * or helper with the HIP library; the only thing both sides see is the LP
 * instance produced by the seeded generators.
 *
 * What it computes (Sridhar et al., "An Approximate, Efficient LP Solver for
 * LP Rounding"):
 *   - the standard-form LP of Section 3.1 with [0,u] bounds and one slack
 *     column per inequality row (Appendix C: covering rows get -1, packing
 *     rows +1), y = (x, s);
 *   - the penalty objective of equation (eq:QP) in Section 3.2,
 *       F(y) = c^T x - ubar^T (A y - b) + beta/2 ||A y - b||^2
 *              + rho/2 ||y - ybar||^2,          rho in {0, 1/beta};
 *   - the SCD iteration of Algorithm 1 (Section 3.3): per coordinate j,
 *       y_j <- clip(y_j - gamma * g_j / L, 0, u_j),
 *       g_j = c_j - A_j^T ubar + beta A_j^T (A y - b) + rho (y_j - ybar_j),
 *     with L = Lmax of (eq:Lmax) or the coordinate's own curvature;
 *   - the block variant with projection onto the k-simplex used for
 *     multiway cut (Appendix E);
 *   - the pre-rounding scalings of Lemma (infeasible:rounded:vc) and the
 *     covering (with q(P)) and packing lemmas of Appendix C, the threshold
 *     and randomized roundings of Section 2 and Appendix B (vertex cover,
 *     independent set, set cover, integer covering, weighted packing,
 *     multiway cut), the node-based roundings (argmax, sampling) of the
 *     MAP-inference LP of the experiments, and the feasibility check;
 *   - the multiplier step of the augmented-Lagrangian framework (Section
 *     3.2) with the LP's Lagrangian dual bound.
 *
 * Everything is FP64 with no fused multiply-add (built -ffp-contract=off),
 * plain loops in the order the algorithm states them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the
 * published round function: two 64x64->128 multiplies per round, the key
 * advanced by the Weyl constants between rounds. */
static const uint64_t PH_M0 = 0xD2E7470EE14C6C93ULL, PH_M1 = 0xCA5A826395121157ULL;
static const uint64_t PH_W0 = 0x9E3779B97F4A7C15ULL, PH_W1 = 0xBB67AE8584CAA73BULL;

void orc_philox(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PH_W0; k1 += PH_W1; }
        unsigned __int128 p0 = (unsigned __int128)PH_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PH_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0, n1 = lo1, n2 = hi0 ^ x3 ^ k1, n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* independent draw streams, fixed for both sides of the parity tests */
enum { ST_CLASS_ORDER = 1, ST_UNIFORM = 2, ST_PERM = 3, ST_ROUND = 4 };

static uint64_t ph_word(uint64_t seed, uint64_t stream, uint64_t c0, uint64_t c1, uint64_t c2) {
    uint64_t ctr[4] = {c0, c1, c2, 0}, key[2] = {seed, stream}, out[4];
    orc_philox(ctr, key, out);
    return out[0];
}
static double u53(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t m, n, N;                 /* N = n + m; column n+i is row i's slack */
    int64_t *row_ptr; int32_t *col_idx; double *val;   /* CSR of A (structural) */
    double *b, *c, *ub;              /* c, ub over N (slack cost 0, ub inf or 0) */
    int8_t *sense;
    /* CSC of [A | slacks] over all N columns */
    int64_t *cptr; int64_t *ridx; double *cval;
    /* simplex blocks */
    int64_t nblocks; int32_t k; int64_t *bfirst; int32_t *fixed; int64_t *col_block;
    /* update units: unit u is a free block (kind 1, id = block) or a single
       free column (kind 0, id = column) */
    int64_t nunits; int8_t *ukind; int64_t *uid; int32_t *ucolour; int32_t nclasses;
    /* pairwise factors of a MAP-inference LP: factor e joins blocks
       pw_ends[2e], pw_ends[2e+1]; its k*k columns start at pw_first[e],
       row-major in (label of the first block, label of the second) */
    int64_t npw; int64_t *pw_ends; int64_t *pw_first;
} orc_lp;

typedef struct {
    orc_lp *lp;
    double beta, gamma, rho; int step_rule, schedule; uint64_t seed;
    double *ybar, *ubar, *ctil;      /* ybar over N, ubar over m, ctil over N */
    double *y, *r;                   /* y over N, r = A y - b over m */
    double *L;                       /* curvature per unit */
    double Lmax;
    int64_t epoch;
    /* scratch */
    int64_t *order; double *g; double *v; double *w;
} orc_solver;

enum { STEP_PER_COORD = 0, STEP_GLOBAL_LMAX = 1 };
enum { SCHED_DET = 0, SCHED_PERM = 1, SCHED_UNIFORM = 2 };
enum { RULE_VC_THRESH = 1, RULE_MIS_THRESH = 2, RULE_MIS_RAND = 3, RULE_MC_CKR = 4,
       RULE_COVER_THRESH = 5, RULE_COVER_RAND = 6, RULE_PACK_RAND = 7,
       RULE_MAP_ARGMAX = 8, RULE_MAP_SAMPLE = 9 };

void orc_lp_free(orc_lp *p) {
    if (!p) return;
    free(p->row_ptr); free(p->col_idx); free(p->val); free(p->b); free(p->c); free(p->ub);
    free(p->sense); free(p->cptr); free(p->ridx); free(p->cval); free(p->bfirst);
    free(p->fixed); free(p->col_block); free(p->ukind); free(p->uid); free(p->ucolour);
    free(p->pw_ends); free(p->pw_first);
    free(p);
}

/* greedy colouring of the structural units in unit order; slack units form
 * one extra class.  Two units conflict when their columns share a row. */
static int build_units(orc_lp *p) {
    int64_t n = p->n, m = p->m;
    free(p->ukind); free(p->uid); free(p->ucolour);
    int64_t cap = n + m;
    p->ukind = (int8_t *)malloc(cap); p->uid = (int64_t *)malloc(cap * 8);
    p->ucolour = (int32_t *)malloc(cap * 4);
    int64_t *unit_of_col = (int64_t *)malloc((n > 0 ? n : 1) * 8);
    if (!p->ukind || !p->uid || !p->ucolour || !unit_of_col) { free(unit_of_col); return -1; }
    int64_t nu = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t bl = p->col_block[j];
        if (bl >= 0) {
            if (p->fixed[bl] >= 0) { unit_of_col[j] = -1; continue; }
            if (j == p->bfirst[bl]) { p->ukind[nu] = 1; p->uid[nu] = bl; ++nu; }
            unit_of_col[j] = nu - 1;
        } else {
            p->ukind[nu] = 0; p->uid[nu] = j; unit_of_col[j] = nu; ++nu;
        }
    }
    int64_t nstruct = nu;
    /* colouring: stamp[colour] = unit that last forbade it */
    int64_t maxc = 64;
    int64_t *stamp = (int64_t *)malloc(maxc * 8);
    for (int64_t q = 0; q < maxc; ++q) stamp[q] = -1;
    int32_t ncol = 0;
    for (int64_t t = 0; t < nstruct; ++t) {
        int64_t j0, j1;
        if (p->ukind[t] == 1) { j0 = p->bfirst[p->uid[t]]; j1 = j0 + p->k; }
        else { j0 = p->uid[t]; j1 = j0 + 1; }
        for (int64_t j = j0; j < j1; ++j)
            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) {
                int64_t i = p->ridx[e];
                for (int64_t q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
                    int64_t o = unit_of_col[p->col_idx[q]];
                    if (o >= 0 && o < t) stamp[p->ucolour[o]] = t;
                }
            }
        int32_t cc = 0;
        while (cc < maxc && stamp[cc] == t) ++cc;
        if (cc == maxc) {
            int64_t nm = maxc * 2;
            stamp = (int64_t *)realloc(stamp, nm * 8);
            for (int64_t q = maxc; q < nm; ++q) stamp[q] = -1;
            maxc = nm;
        }
        p->ucolour[t] = cc;
        if (cc + 1 > ncol) ncol = cc + 1;
    }
    free(stamp);
    int any_slack = 0;
    for (int64_t i = 0; i < m; ++i)
        if (p->sense[i] != 0) {
            p->ukind[nu] = 0; p->uid[nu] = n + i; p->ucolour[nu] = ncol; ++nu; any_slack = 1;
        }
    p->nunits = nu;
    p->nclasses = ncol + any_slack;
    free(unit_of_col);
    return 0;
}

orc_lp *orc_lp_create(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                      const double *val, const double *b, const double *c, const double *u,
                      const int8_t *sense) {
    if (m < 0 || n < 0) return NULL;
    orc_lp *p = (orc_lp *)calloc(1, sizeof(orc_lp));
    p->m = m; p->n = n; p->N = n + m;
    int64_t nnz = row_ptr[m];
    p->row_ptr = (int64_t *)malloc((m + 1) * 8);
    p->col_idx = (int32_t *)malloc((nnz > 0 ? nnz : 1) * 4);
    p->val = (double *)malloc((nnz > 0 ? nnz : 1) * 8);
    p->b = (double *)malloc((m > 0 ? m : 1) * 8);
    p->sense = (int8_t *)malloc(m > 0 ? m : 1);
    p->c = (double *)calloc(p->N > 0 ? p->N : 1, 8);
    p->ub = (double *)malloc((p->N > 0 ? p->N : 1) * 8);
    memcpy(p->row_ptr, row_ptr, (m + 1) * 8);
    for (int64_t i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) { orc_lp_free(p); return NULL; }
        p->b[i] = b[i];
        p->sense[i] = sense ? sense[i] : 0;
    }
    for (int64_t e = 0; e < nnz; ++e) {
        if (col_idx[e] < 0 || col_idx[e] >= n) { orc_lp_free(p); return NULL; }
        p->col_idx[e] = col_idx[e];
        p->val[e] = val ? val[e] : 1.0;
    }
    for (int64_t j = 0; j < n; ++j) { p->c[j] = c[j]; p->ub[j] = u ? u[j] : INFINITY; }
    for (int64_t i = 0; i < m; ++i) p->ub[n + i] = p->sense[i] != 0 ? INFINITY : 0.0;
    /* CSC of the augmented matrix: count, prefix, fill (rows ascending) */
    p->cptr = (int64_t *)calloc(p->N + 1, 8);
    for (int64_t e = 0; e < nnz; ++e) p->cptr[p->col_idx[e] + 1]++;
    for (int64_t i = 0; i < m; ++i) p->cptr[n + i + 1] = 1;
    for (int64_t j = 0; j < p->N; ++j) p->cptr[j + 1] += p->cptr[j];
    int64_t tot = p->cptr[p->N];
    p->ridx = (int64_t *)malloc((tot > 0 ? tot : 1) * 8);
    p->cval = (double *)malloc((tot > 0 ? tot : 1) * 8);
    int64_t *fill = (int64_t *)malloc((p->N > 0 ? p->N : 1) * 8);
    for (int64_t j = 0; j < p->N; ++j) fill[j] = p->cptr[j];
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t j = p->col_idx[e];
            p->ridx[fill[j]] = i; p->cval[fill[j]] = p->val[e]; fill[j]++;
        }
    for (int64_t i = 0; i < m; ++i) {
        /* covering (>=) rows: A x - s = b; packing (<=): A x + s = b */
        p->ridx[fill[n + i]] = i;
        p->cval[fill[n + i]] = p->sense[i] > 0 ? -1.0 : (p->sense[i] < 0 ? 1.0 : 0.0);
    }
    free(fill);
    p->col_block = (int64_t *)malloc((n > 0 ? n : 1) * 8);
    for (int64_t j = 0; j < n; ++j) p->col_block[j] = -1;
    p->fixed = (int32_t *)malloc(4); p->bfirst = (int64_t *)malloc(8);
    if (build_units(p) != 0) { orc_lp_free(p); return NULL; }
    return p;
}

int orc_lp_set_blocks(orc_lp *p, int64_t nblocks, int32_t k, const int64_t *first,
                      const int32_t *fixed_label) {
    if (k < 1 || k > 256) return -1;
    free(p->bfirst); free(p->fixed);
    p->nblocks = nblocks; p->k = k;
    p->bfirst = (int64_t *)malloc((nblocks > 0 ? nblocks : 1) * 8);
    p->fixed = (int32_t *)malloc((nblocks > 0 ? nblocks : 1) * 4);
    for (int64_t j = 0; j < p->n; ++j) p->col_block[j] = -1;
    for (int64_t t = 0; t < nblocks; ++t) {
        p->bfirst[t] = first[t];
        p->fixed[t] = fixed_label ? fixed_label[t] : -1;
        if (first[t] < 0 || first[t] + k > p->n) return -1;
        for (int32_t i = 0; i < k; ++i) {
            if (p->col_block[first[t] + i] != -1) return -1;
            p->col_block[first[t] + i] = t;
        }
    }
    /* a row may hold at most one column of each block, so the block of
       A^T A is diagonal (Appendix E takes the block minimiser of that form) */
    int64_t *last_row = (int64_t *)malloc((nblocks > 0 ? nblocks : 1) * 8);
    for (int64_t t = 0; t < nblocks; ++t) last_row[t] = -1;
    int shared = 0;
    for (int64_t i = 0; i < p->m && !shared; ++i)
        for (int64_t q = p->row_ptr[i]; q < p->row_ptr[i + 1]; ++q) {
            int64_t t = p->col_block[p->col_idx[q]];
            if (t < 0) continue;
            if (last_row[t] == i) { shared = 1; break; }
            last_row[t] = i;
        }
    free(last_row);
    if (shared) return -1;
    return build_units(p);
}

/* pairwise factors for the MAP roundings' energy; -1 on bad input */
int orc_lp_set_pairwise(orc_lp *p, int64_t nf, const int32_t *ends, const int64_t *first) {
    if (p->nblocks <= 0 || nf < 0) return -1;
    int64_t kk = (int64_t)p->k * p->k;
    free(p->pw_ends); free(p->pw_first);
    p->pw_ends = (int64_t *)malloc((2 * nf + 1) * 8);
    p->pw_first = (int64_t *)malloc((nf + 1) * 8);
    p->npw = -1;
    for (int64_t e = 0; e < nf; ++e) {
        for (int q = 0; q < 2; ++q) {
            if (ends[2 * e + q] < 0 || ends[2 * e + q] >= p->nblocks) return -1;
            p->pw_ends[2 * e + q] = ends[2 * e + q];
        }
        if (first[e] < 0 || first[e] + kk > p->n) return -1;
        for (int64_t j = first[e]; j < first[e] + kk; ++j) if (p->col_block[j] >= 0) return -1;
        p->pw_first[e] = first[e];
    }
    p->npw = nf;
    return 0;
}

/* energy of a labelling: node terms of every block, then the factor terms,
 * read off the objective */
static double map_energy(const orc_lp *p, const int32_t *lab) {
    double en = 0.0;
    for (int64_t t = 0; t < p->nblocks; ++t) en += p->c[p->bfirst[t] + lab[t]];
    for (int64_t e = 0; e < p->npw; ++e)
        en += p->c[p->pw_first[e] + (int64_t)lab[p->pw_ends[2 * e]] * p->k + lab[p->pw_ends[2 * e + 1]]];
    return en;
}

int64_t orc_num_units(const orc_lp *p) { return p->nunits; }
int32_t orc_num_classes(const orc_lp *p) { return p->nclasses; }
void orc_units(const orc_lp *p, int8_t *kind, int64_t *id, int32_t *colour) {
    for (int64_t t = 0; t < p->nunits; ++t) {
        kind[t] = p->ukind[t]; id[t] = p->uid[t]; colour[t] = p->ucolour[t];
    }
}

/* ------------------------------------------------------------------------ */
/* Euclidean projection onto {w >= 0, sum w = 1}: sort descending, find the
 * largest prefix whose shifted entries stay positive (Held, Wolfe & Crowder
 * 1974; Duchi et al. 2008). */
static int cmp_desc(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x < y) - (x > y);
}
void orc_simplex_project(const double *v, int32_t k, double *out) {
    double mu[256];
    for (int32_t i = 0; i < k; ++i) mu[i] = v[i];
    qsort(mu, k, sizeof(double), cmp_desc);
    double csum = 0.0, theta = 0.0;
    for (int32_t j = 0; j < k; ++j) {
        csum += mu[j];
        double t = (csum - 1.0) / (double)(j + 1);
        if (mu[j] - t > 0.0) theta = t;
    }
    for (int32_t i = 0; i < k; ++i) out[i] = v[i] - theta > 0.0 ? v[i] - theta : 0.0;
}

/* ------------------------------------------------------------------------ */
static double unit_curvature(const orc_solver *s, int64_t t) {
    const orc_lp *p = s->lp;
    if (p->ukind[t] == 0) {
        int64_t j = p->uid[t];
        double a2 = 0.0;
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) a2 += p->cval[e] * p->cval[e];
        return s->beta * a2 + s->rho;
    }
    /* block: its columns share no row, so the block of A^T A is
       diag(||A_i||^2); the largest entry bounds the block's curvature */
    int64_t j0 = p->bfirst[p->uid[t]];
    double best = 0.0;
    for (int32_t i = 0; i < p->k; ++i) {
        double a2 = 0.0;
        for (int64_t e = p->cptr[j0 + i]; e < p->cptr[j0 + i + 1]; ++e) a2 += p->cval[e] * p->cval[e];
        if (a2 > best) best = a2;
    }
    return s->beta * best + s->rho;
}

static void recompute_residual(orc_solver *s) {
    const orc_lp *p = s->lp;
    for (int64_t i = 0; i < p->m; ++i) {
        double acc = 0.0;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e)
            acc += p->val[e] * s->y[p->col_idx[e]];
        if (p->sense[i] > 0) acc -= s->y[p->n + i];
        else if (p->sense[i] < 0) acc += s->y[p->n + i];
        s->r[i] = acc - p->b[i];
    }
}

void orc_solver_free(orc_solver *s) {
    if (!s) return;
    free(s->ybar); free(s->ubar); free(s->ctil); free(s->y); free(s->r); free(s->L);
    free(s->order); free(s->g); free(s->v); free(s->w); free(s);
}

orc_solver *orc_solver_create(orc_lp *p, double beta, int32_t step_rule, double step_scale,
                              int32_t prox, const double *ybar, const double *ubar,
                              int32_t schedule, uint64_t seed) {
    if (!(beta > 0.0)) return NULL;
    orc_solver *s = (orc_solver *)calloc(1, sizeof(orc_solver));
    s->lp = p; s->beta = beta; s->gamma = step_scale; s->rho = prox ? 1.0 / beta : 0.0;
    s->step_rule = step_rule; s->schedule = schedule; s->seed = seed;
    int64_t N = p->N, m = p->m;
    s->ybar = (double *)calloc(N + 1, 8); s->ubar = (double *)calloc(m + 1, 8);
    s->ctil = (double *)calloc(N + 1, 8); s->y = (double *)calloc(N + 1, 8);
    s->r = (double *)calloc(m + 1, 8); s->L = (double *)calloc(p->nunits + 1, 8);
    s->order = (int64_t *)calloc(p->nunits + 1, 8);
    s->g = (double *)calloc(p->k + 1, 8); s->v = (double *)calloc(p->k + 1, 8);
    s->w = (double *)calloc(p->k + 1, 8);
    if (ybar) for (int64_t j = 0; j < N; ++j) s->ybar[j] = ybar[j];
    if (ubar) for (int64_t i = 0; i < m; ++i) s->ubar[i] = ubar[i];
    for (int64_t j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) acc += p->cval[e] * s->ubar[p->ridx[e]];
        s->ctil[j] = p->c[j] - acc;
    }
    /* starting point y = 0, fixed blocks at their unit vector (Section 3.3
       leaves x_0 free) */
    for (int64_t t = 0; t < p->nblocks; ++t)
        if (p->fixed[t] >= 0) s->y[p->bfirst[t] + p->fixed[t]] = 1.0;
    recompute_residual(s);
    s->Lmax = 0.0;
    for (int64_t t = 0; t < p->nunits; ++t) {
        s->L[t] = unit_curvature(s, t);
        if (s->L[t] > s->Lmax) s->Lmax = s->L[t];
    }
    return s;
}

/* one SCD step on unit t (the coordinate update of Algorithm 1; block form of Appendix E) */
static void update_unit(orc_solver *s, int64_t t) {
    const orc_lp *p = s->lp;
    double L = s->step_rule == STEP_GLOBAL_LMAX ? s->Lmax : s->L[t];
    if (p->ukind[t] == 0) {
        int64_t j = p->uid[t];
        double dot = 0.0;
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) dot += p->cval[e] * s->r[p->ridx[e]];
        double g = s->ctil[j] + s->beta * dot + s->rho * (s->y[j] - s->ybar[j]);
        double yn;
        if (L > 0.0) {
            yn = s->y[j] - s->gamma * g / L;
        } else {            /* empty column, no prox: move to the cheaper bound */
            yn = g > 0.0 ? 0.0 : (g < 0.0 ? p->ub[j] : s->y[j]);
        }
        if (yn < 0.0) yn = 0.0;
        if (yn > p->ub[j]) yn = p->ub[j];
        double d = yn - s->y[j];
        s->y[j] = yn;
        if (d != 0.0)
            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) s->r[p->ridx[e]] += d * p->cval[e];
        return;
    }
    int64_t j0 = p->bfirst[p->uid[t]];
    int32_t k = p->k;
    for (int32_t i = 0; i < k; ++i) {
        int64_t j = j0 + i;
        double dot = 0.0;
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) dot += p->cval[e] * s->r[p->ridx[e]];
        s->g[i] = s->ctil[j] + s->beta * dot + s->rho * (s->y[j] - s->ybar[j]);
    }
    for (int32_t i = 0; i < k; ++i) s->v[i] = s->y[j0 + i] - (L > 0.0 ? s->gamma * s->g[i] / L : 0.0);
    orc_simplex_project(s->v, k, s->w);
    for (int32_t i = 0; i < k; ++i) {
        int64_t j = j0 + i;
        double d = s->w[i] - s->y[j];
        s->y[j] = s->w[i];
        if (d != 0.0)
            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) s->r[p->ridx[e]] += d * p->cval[e];
    }
}

typedef struct { uint64_t key; int64_t idx; } keyed;
static int cmp_keyed(const void *a, const void *b) {
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* class order of epoch e: classes sorted by (Philox word, class id) */
void orc_class_order(const orc_lp *p, uint64_t seed, int64_t epoch, int32_t *order) {
    keyed *ks = (keyed *)malloc((p->nclasses + 1) * sizeof(keyed));
    for (int32_t c = 0; c < p->nclasses; ++c) {
        ks[c].key = ph_word(seed, ST_CLASS_ORDER, (uint64_t)epoch, (uint64_t)c, 0);
        ks[c].idx = c;
    }
    qsort(ks, p->nclasses, sizeof(keyed), cmp_keyed);
    for (int32_t c = 0; c < p->nclasses; ++c) order[c] = (int32_t)ks[c].idx;
    free(ks);
}

/* the unit sequence of one epoch under the solver's schedule */
static int64_t epoch_sequence(orc_solver *s, int32_t within_reverse) {
    const orc_lp *p = s->lp;
    int64_t U = p->nunits;
    if (s->schedule == SCHED_DET) {
        int32_t *ord = (int32_t *)malloc((p->nclasses + 1) * 4);
        orc_class_order(p, s->seed, s->epoch, ord);
        int64_t q = 0;
        for (int32_t ci = 0; ci < p->nclasses; ++ci) {
            if (!within_reverse) {
                for (int64_t t = 0; t < U; ++t) if (p->ucolour[t] == ord[ci]) s->order[q++] = t;
            } else {
                for (int64_t t = U - 1; t >= 0; --t) if (p->ucolour[t] == ord[ci]) s->order[q++] = t;
            }
        }
        free(ord);
        return q;
    }
    if (s->schedule == SCHED_PERM) {
        keyed *ks = (keyed *)malloc((U + 1) * sizeof(keyed));
        for (int64_t t = 0; t < U; ++t) {
            ks[t].key = ph_word(s->seed, ST_PERM, (uint64_t)s->epoch, (uint64_t)t, 0);
            ks[t].idx = t;
        }
        qsort(ks, U, sizeof(keyed), cmp_keyed);
        for (int64_t t = 0; t < U; ++t) s->order[t] = ks[t].idx;
        free(ks);
        return U;
    }
    /* uniform with replacement (the coordinate choice of Algorithm 1) */
    for (int64_t t = 0; t < U; ++t) {
        int64_t pick = (int64_t)(u53(ph_word(s->seed, ST_UNIFORM, (uint64_t)s->epoch, (uint64_t)t, 0)) * (double)U);
        if (pick >= U) pick = U - 1;
        s->order[t] = pick;
    }
    return U;
}

double orc_penalty(const orc_solver *s);

int32_t orc_run_epochs(orc_solver *s, int32_t nepochs, int32_t within_reverse, double *F_after) {
    for (int32_t e = 0; e < nepochs; ++e) {
        int64_t q = epoch_sequence(s, within_reverse);
        for (int64_t t = 0; t < q; ++t) update_unit(s, s->order[t]);
        s->epoch++;
        if (F_after) F_after[e] = orc_penalty(s);
    }
    return 0;
}

/* tiny instances: F after every single update of one epoch */
int64_t orc_trace_epoch(orc_solver *s, double *F_after_step, int64_t cap) {
    int64_t q = epoch_sequence(s, 0);
    int64_t w = 0;
    for (int64_t t = 0; t < q; ++t) {
        update_unit(s, s->order[t]);
        if (w < cap) F_after_step[w++] = orc_penalty(s);
    }
    s->epoch++;
    return w;
}

/* a single update of unit t, outside any schedule (used by the step pins) */
void orc_step_unit(orc_solver *s, int64_t t) { if (t >= 0 && t < s->lp->nunits) update_unit(s, t); }

void orc_get_y(const orc_solver *s, double *y) { memcpy(y, s->y, s->lp->N * 8); }
void orc_get_r(const orc_solver *s, double *r) { memcpy(r, s->r, s->lp->m * 8); }
void orc_set_y(orc_solver *s, const double *y) { memcpy(s->y, y, s->lp->N * 8); recompute_residual(s); }
int64_t orc_epoch(const orc_solver *s) { return s->epoch; }
double orc_lmax(const orc_solver *s) { return s->Lmax; }
void orc_set_epoch(orc_solver *s, int64_t e) { s->epoch = e; }

/* ------------------------------------------------------------------------ */
/* objective values, all recomputed from y in fixed order */

double orc_penalty(const orc_solver *s) {
    const orc_lp *p = s->lp;
    double f = 0.0;
    for (int64_t j = 0; j < p->n; ++j) f += p->c[j] * s->y[j];
    for (int64_t i = 0; i < p->m; ++i) {
        double acc = 0.0;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) acc += p->val[e] * s->y[p->col_idx[e]];
        if (p->sense[i] > 0) acc -= s->y[p->n + i];
        else if (p->sense[i] < 0) acc += s->y[p->n + i];
        double w = acc - p->b[i];
        f += -s->ubar[i] * w + 0.5 * s->beta * w * w;
    }
    if (s->rho > 0.0)
        for (int64_t j = 0; j < p->N; ++j) {
            if (j >= p->n && p->sense[j - p->n] == 0) continue;   /* not a variable */
            double d = s->y[j] - s->ybar[j];
            f += 0.5 * s->rho * d * d;
        }
    return f;
}

/* min over [0,U] of red*y + rho/2 (y - yb)^2 */
static double box_min(double red, double U, double rho, double yb) {
    if (rho > 0.0) {
        double y = yb - red / rho;
        if (y < 0.0) y = 0.0;
        if (y > U) y = U;
        return red * y + 0.5 * rho * (y - yb) * (y - yb);
    }
    if (red >= 0.0) return 0.0;
    return isinf(U) ? -INFINITY : red * U;
}

/* out: [0] F  [1] c^T x  [2] ||A y - b||_inf  [3] ||A y - b||_2
 *      [4] max original-row violation  [5] dual bound Phi  [6] relative gap */
void orc_metrics(const orc_solver *s, double *out) {
    const orc_lp *p = s->lp;
    int64_t m = p->m, n = p->n;
    double *u = (double *)malloc((m + 1) * 8);
    double linf = 0.0, l2 = 0.0, viol = 0.0, bu = 0.0, uu = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double ax = 0.0;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) ax += p->val[e] * s->y[p->col_idx[e]];
        double acc = ax;
        if (p->sense[i] > 0) acc -= s->y[n + i];
        else if (p->sense[i] < 0) acc += s->y[n + i];
        double w = acc - p->b[i];
        if (fabs(w) > linf) linf = fabs(w);
        l2 += w * w;
        double vi = p->sense[i] > 0 ? p->b[i] - ax : (p->sense[i] < 0 ? ax - p->b[i] : fabs(ax - p->b[i]));
        if (vi > viol) viol = vi;
        /* dual estimate u = ubar - beta w; without prox the unbounded slack
           columns need a non-negative reduced cost: covering u>=0, packing u<=0 */
        double ui = s->ubar[i] - s->beta * w;
        if (s->rho == 0.0) {
            if (p->sense[i] > 0 && ui < 0.0) ui = 0.0;
            if (p->sense[i] < 0 && ui > 0.0) ui = 0.0;
        }
        u[i] = ui;
        bu += p->b[i] * ui;
        uu += (ui - s->ubar[i]) * (ui - s->ubar[i]);
    }
    double phi = bu - uu / (2.0 * s->beta);
    /* sum over variables of min of the reduced-cost term over its feasible set */
    for (int64_t j = 0; j < p->N; ++j) {
        if (j < n && p->col_block[j] >= 0) continue;
        if (j >= n && p->sense[j - n] == 0) continue;
        double red = p->c[j];
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) red -= p->cval[e] * u[p->ridx[e]];
        phi += box_min(red, p->ub[j], s->rho, s->ybar[j]);
    }
    for (int64_t t = 0; t < p->nblocks; ++t) {
        int64_t j0 = p->bfirst[t];
        int32_t k = p->k;
        double red[256], yb[256], w[256];
        for (int32_t i = 0; i < k; ++i) {
            int64_t j = j0 + i;
            red[i] = p->c[j];
            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) red[i] -= p->cval[e] * u[p->ridx[e]];
            yb[i] = s->ybar[j];
        }
        if (p->fixed[t] >= 0) {
            /* fixed block contributes its value at the unit vector (plus the
               prox distance of that fixed point) */
            int32_t f = p->fixed[t];
            double v = red[f];
            if (s->rho > 0.0)
                for (int32_t i = 0; i < k; ++i) {
                    double d = (i == f ? 1.0 : 0.0) - yb[i];
                    v += 0.5 * s->rho * d * d;
                }
            phi += v;
            continue;
        }
        if (s->rho > 0.0) {
            double v[256];
            for (int32_t i = 0; i < k; ++i) v[i] = yb[i] - red[i] / s->rho;
            orc_simplex_project(v, k, w);
            double val = 0.0;
            for (int32_t i = 0; i < k; ++i) val += red[i] * w[i] + 0.5 * s->rho * (w[i] - yb[i]) * (w[i] - yb[i]);
            phi += val;
        } else {
            double mn = red[0];
            for (int32_t i = 1; i < k; ++i) if (red[i] < mn) mn = red[i];
            phi += mn;
        }
    }
    free(u);
    double F = orc_penalty(s);
    double cx = 0.0;
    for (int64_t j = 0; j < n; ++j) cx += p->c[j] * s->y[j];
    out[0] = F; out[1] = cx; out[2] = linf; out[3] = sqrt(l2); out[4] = viol; out[5] = phi;
    double den = fabs(F) > 1.0 ? fabs(F) : 1.0;
    out[6] = (F - phi) / den;
}

/* ------------------------------------------------------------------------ */
/* One multiplier update between two penalty solves: the augmented
 * Lagrangian framework of Section 3.2 (a proximal method of multipliers when
 * prox is on).  With w = A y - b recomputed from y:
 *     ubar <- ubar - beta w;   ybar <- y (move_centre, prox on only);
 *     beta <- new_beta when new_beta > 0 (rho = 1/beta follows with prox);
 *     ctil = c - A^T ubar and every unit's curvature recomputed.
 * The statistics describe the iterate y at which the step is taken:
 *   out[0] = c^T x, out[1] = ||w||_inf,
 *   out[2] = D(u), the Lagrangian dual function of the LP of Section 3.1,
 *            D(u) = b^T u + sum over variables of min over its feasible set
 *            (box, or simplex for a free block, the unit vector for a fixed
 *            block) of its reduced cost term, at u = the new ubar with each
 *            inequality row's entry clipped to the sign its slack allows
 *            (covering >= 0, packing <= 0), so that D(u) <= LP*,
 *   out[3] = (out[0] - out[2]) / max(1, |out[0]|). */
void orc_multiplier_step(orc_solver *s, int32_t move_centre, double new_beta, double *out) {
    const orc_lp *p = s->lp;
    int64_t m = p->m, n = p->n, N = p->N;
    recompute_residual(s);
    double *u = (double *)malloc((m + 1) * 8);
    double linf = 0.0, bu = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double w = s->r[i];
        if (fabs(w) > linf) linf = fabs(w);
        s->ubar[i] = s->ubar[i] - s->beta * w;
        double ui = s->ubar[i];
        if (p->sense[i] > 0 && ui < 0.0) ui = 0.0;
        if (p->sense[i] < 0 && ui > 0.0) ui = 0.0;
        u[i] = ui;
        bu += p->b[i] * ui;
    }
    double d = bu;
    for (int64_t j = 0; j < N; ++j) {
        if (j < n && p->col_block[j] >= 0) continue;
        if (j >= n && p->sense[j - n] == 0) continue;
        double red = p->c[j];
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) red -= p->cval[e] * u[p->ridx[e]];
        d += box_min(red, p->ub[j], 0.0, 0.0);
    }
    for (int64_t t = 0; t < p->nblocks; ++t) {
        double best = INFINITY;
        for (int32_t i = 0; i < p->k; ++i) {
            if (p->fixed[t] >= 0 && i != p->fixed[t]) continue;
            int64_t j = p->bfirst[t] + i;
            double red = p->c[j];
            for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) red -= p->cval[e] * u[p->ridx[e]];
            if (red < best) best = red;
        }
        d += best;
    }
    free(u);
    double cx = 0.0;
    for (int64_t j = 0; j < n; ++j) cx += p->c[j] * s->y[j];
    out[0] = cx; out[1] = linf; out[2] = d;
    out[3] = (cx - d) / (fabs(cx) > 1.0 ? fabs(cx) : 1.0);
    if (move_centre && s->rho > 0.0)
        for (int64_t j = 0; j < N; ++j) s->ybar[j] = s->y[j];
    if (new_beta > 0.0) {
        int prox = s->rho > 0.0;
        s->beta = new_beta;
        s->rho = prox ? 1.0 / new_beta : 0.0;
    }
    for (int64_t j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int64_t e = p->cptr[j]; e < p->cptr[j + 1]; ++e) acc += p->cval[e] * s->ubar[p->ridx[e]];
        s->ctil[j] = p->c[j] - acc;
    }
    s->Lmax = 0.0;
    for (int64_t t = 0; t < p->nunits; ++t) {
        s->L[t] = unit_curvature(s, t);
        if (s->L[t] > s->Lmax) s->Lmax = s->L[t];
    }
}

void orc_get_ubar(const orc_solver *s, double *ubar) { memcpy(ubar, s->ubar, s->lp->m * 8); }
void orc_get_ybar(const orc_solver *s, double *ybar) { memcpy(ybar, s->ybar, s->lp->N * 8); }
double orc_beta(const orc_solver *s) { return s->beta; }

/* ------------------------------------------------------------------------ */
/* rounding (Section 2; Appendix B; Appendix C scalings).  x is the
 * structural part of y; sol is 0/1 per column (VC, MIS) or a label per
 * block (MC).  Returns 0, or -1 when the instance does not have the shape
 * the rule needs. */

static int edge_rows_ok(const orc_lp *p, int want_sense) {
    for (int64_t i = 0; i < p->m; ++i) {
        if (p->row_ptr[i + 1] - p->row_ptr[i] != 2) return 0;
        if (p->sense[i] != want_sense || p->b[i] != 1.0) return 0;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) if (p->val[e] != 1.0) return 0;
    }
    return 1;
}

/* binary columns and rows of one sense with non-negative entries (and,
 * for covering, integer entries and right-hand sides) */
static int general_rows_ok(const orc_lp *p, int want_sense, int integral) {
    if (p->nblocks > 0) return 0;
    for (int64_t j = 0; j < p->n; ++j) if (p->ub[j] != 1.0) return 0;
    for (int64_t i = 0; i < p->m; ++i) {
        if (p->sense[i] != want_sense) return 0;
        if (integral && p->b[i] != floor(p->b[i])) return 0;
        if (!integral && !(p->b[i] > 0.0)) return 0;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
            if (p->val[e] < 0.0) return 0;
            if (integral && p->val[e] != floor(p->val[e])) return 0;
        }
    }
    return 1;
}

static int set_cover_rows_ok(const orc_lp *p) {
    if (!general_rows_ok(p, 1, 1)) return 0;
    for (int64_t i = 0; i < p->m; ++i) {
        if (p->b[i] != 1.0) return 0;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) if (p->val[e] != 1.0) return 0;
    }
    return 1;
}

/* q(P) of the covering lemma (Appendix C): over the rows, the smallest
 * b_j - A_j x among binary x with A_j x < b_j.  The sums A_j x reachable
 * below b_j come from the textbook subset-sum table over 0..b_j-1.  Rows
 * with b_j <= 0 have no such x.  Rows with b_j above 2^24 take the lower
 * bound 1 (valid for integer data).  Returns INFINITY without rows that
 * count, -1 when the instance is not an integer covering program. */
double orc_cover_q(const orc_lp *p) {
    if (!general_rows_ok(p, 1, 1)) return -1.0;
    double q = INFINITY;
    for (int64_t i = 0; i < p->m; ++i) {
        double bj = p->b[i];
        if (bj <= 0.0) continue;
        if (bj > 16777216.0) { if (1.0 < q) q = 1.0; continue; }
        int64_t B = (int64_t)bj;
        char *reach = (char *)calloc(B, 1);
        reach[0] = 1;
        for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
            int64_t a = (int64_t)p->val[e];
            if (a <= 0) continue;
            for (int64_t t = B - 1; t >= a; --t) if (reach[t - a]) reach[t] = 1;
        }
        int64_t top = B - 1;
        while (!reach[top]) --top;
        free(reach);
        if (bj - (double)top < q) q = bj - (double)top;
    }
    return q;
}

int32_t orc_round(const orc_lp *p, const double *x, int32_t rule, uint64_t seed, int32_t reps,
                  int32_t *sol, double *cost, double *aux) {
    int64_t n = p->n, m = p->m;
    if (rule == RULE_COVER_THRESH) {
        if (!set_cover_rows_ok(p)) return -1;
        /* Hochbaum's f-threshold (Appendix B, set cover) after the covering
           scaling with q = 1: keep s iff x_s/(1-eps) >= 1/f, i.e.
           x_s >= min(1, min_j S_j)/f with S_j the row sums, f the largest row
           length; each row's largest entry caps the threshold so that every
           row keeps a set in floating point as it does in exact arithmetic */
        int64_t f = 1;
        for (int64_t i = 0; i < m; ++i) if (p->row_ptr[i + 1] - p->row_ptr[i] > f) f = p->row_ptr[i + 1] - p->row_ptr[i];
        double T = 1.0 / (double)f;
        for (int64_t i = 0; i < m; ++i) {
            double sm = 0.0, mx = -INFINITY;
            for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
                double xv = x[p->col_idx[e]];
                sm += xv;
                if (xv > mx) mx = xv;
            }
            if (sm / (double)f < T) T = sm / (double)f;
            if (mx < T) T = mx;
        }
        double cst = 0.0;
        for (int64_t j = 0; j < n; ++j) { sol[j] = x[j] >= T ? 1 : 0; cst += sol[j] ? p->c[j] : 0.0; }
        *cost = cst;
        if (aux) { aux[0] = T; aux[1] = 0.0; }
        return 0;
    }
    if (rule == RULE_COVER_RAND) {
        double q = orc_cover_q(p);
        if (q < 0.0) return -1;
        /* covering lemma (Appendix C): eps = max_j (b_j - A_j x)_+,
           alpha = eps/q(P), xt = min(1, x/(1-alpha)) (all ones when alpha >= 1);
           randomized rounding (Appendix B, set cover): t = ceil(ln(2m))
           independent rounds each keep s with probability xt_s, their union
           is kept; a row still short is completed, from the union alone, by
           its unkept sets in decreasing xt (ties: entry order) */
        double eps = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double ax = 0.0;
            for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) ax += p->val[e] * x[p->col_idx[e]];
            if (p->b[i] - ax > eps) eps = p->b[i] - ax;
        }
        double alpha = isinf(q) ? 0.0 : eps / q;
        int32_t t = m > 0 ? (int32_t)ceil(log(2.0 * (double)m)) : 1;
        if (t < 1) t = 1;
        double *xt = (double *)malloc((n + 1) * 8);
        for (int64_t j = 0; j < n; ++j) {
            double v = alpha < 1.0 ? x[j] / (1.0 - alpha) : 1.0;
            xt[j] = v > 1.0 ? 1.0 : v;
        }
        int32_t *pick = (int32_t *)malloc((n + 1) * 4);
        int32_t *add = (int32_t *)malloc((n + 1) * 4);
        char *used = (char *)malloc(n + 1);
        double best = INFINITY;
        for (int32_t rep = 0; rep < (reps > 0 ? reps : 1); ++rep) {
            for (int64_t j = 0; j < n; ++j) {
                pick[j] = 0; add[j] = 0;
                for (int32_t r = 0; r < t; ++r)
                    if (u53(ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)j, 16 + (uint64_t)r)) < xt[j]) pick[j] = 1;
            }
            for (int64_t i = 0; i < m; ++i) {
                double cov = 0.0;
                for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) cov += p->val[e] * (double)pick[p->col_idx[e]];
                for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) used[p->col_idx[e]] = 0;
                while (cov < p->b[i]) {
                    int64_t pickc = -1; double bx = -1.0, ba = 0.0;
                    for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
                        int64_t j = p->col_idx[e];
                        if (pick[j] || used[j] || p->val[e] <= 0.0) continue;
                        if (xt[j] > bx) { bx = xt[j]; pickc = j; ba = p->val[e]; }
                    }
                    if (pickc < 0) break;
                    used[pickc] = 1;
                    add[pickc] = 1;
                    cov += ba;
                }
            }
            double cst = 0.0;
            for (int64_t j = 0; j < n; ++j) if (pick[j] || add[j]) cst += p->c[j];
            if (cst < best) {
                best = cst;
                for (int64_t j = 0; j < n; ++j) sol[j] = pick[j] || add[j];
                if (aux) aux[1] = rep;
            }
        }
        free(xt); free(pick); free(add); free(used);
        *cost = best;
        if (aux) aux[0] = alpha;
        return 0;
    }
    if (rule == RULE_PACK_RAND) {
        if (!general_rows_ok(p, -1, 0)) return -1;
        /* packing lemma (Appendix C): alpha = max_j ((A_j x - b_j)/b_j)_+,
           xt = x/(1+alpha); Bansal et al.'s alteration with theta = 1/k:
           choose s with probability xt_s; with weights w = A_js/b_j, drop a
           chosen s when, in some row where it has weight, the chosen sets of
           weight >= its own (itself included) weigh more than 1 */
        double alpha = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double ax = 0.0;
            for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) ax += p->val[e] * x[p->col_idx[e]];
            double v = (ax - p->b[i]) / p->b[i];
            if (v > alpha) alpha = v;
        }
        int32_t *pick = (int32_t *)malloc((n + 1) * 4);
        int32_t *drop = (int32_t *)malloc((n + 1) * 4);
        double best = INFINITY;
        for (int32_t rep = 0; rep < (reps > 0 ? reps : 1); ++rep) {
            for (int64_t j = 0; j < n; ++j) {
                double xt = x[j] / (1.0 + alpha);
                pick[j] = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)j, 0)) < xt ? 1 : 0;
                drop[j] = 0;
            }
            for (int64_t i = 0; i < m; ++i)
                for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
                    int64_t j = p->col_idx[e];
                    if (!pick[j] || p->val[e] <= 0.0) continue;
                    double w = p->val[e] / p->b[i], tot = 0.0;
                    for (int64_t e2 = p->row_ptr[i]; e2 < p->row_ptr[i + 1]; ++e2) {
                        if (!pick[p->col_idx[e2]]) continue;
                        double w2 = p->val[e2] / p->b[i];
                        if (w2 >= w) tot += w2;
                    }
                    if (tot > 1.0) drop[j] = 1;
                }
            double cst = 0.0;
            for (int64_t j = 0; j < n; ++j) if (pick[j] && !drop[j]) cst += p->c[j];
            if (cst < best) {
                best = cst;
                for (int64_t j = 0; j < n; ++j) sol[j] = pick[j] && !drop[j];
                if (aux) aux[1] = rep;
            }
        }
        free(pick); free(drop);
        *cost = best;
        if (aux) aux[0] = alpha;
        return 0;
    }
    if (rule == RULE_VC_THRESH) {
        if (!edge_rows_ok(p, 1)) return -1;
        /* Lemma (infeasible:rounded:vc): with eps = max_e (1 - x_u - x_v)_+,
           keeping x/(1-eps) >= 1/2 is keeping x_v >= T, T = min(1/2, min_e (x_u+x_v)/2) */
        double T = 0.5;
        for (int64_t i = 0; i < m; ++i) {
            double s2 = (x[p->col_idx[p->row_ptr[i]]] + x[p->col_idx[p->row_ptr[i] + 1]]) * 0.5;
            if (s2 < T) T = s2;
        }
        double cst = 0.0;
        for (int64_t j = 0; j < n; ++j) { sol[j] = x[j] >= T ? 1 : 0; cst += sol[j] ? p->c[j] : 0.0; }
        *cost = cst;
        if (aux) aux[0] = T;
        return 0;
    }
    if (rule == RULE_MIS_THRESH) {
        if (!edge_rows_ok(p, -1)) return -1;
        double T = 0.5;
        for (int64_t i = 0; i < m; ++i) {
            double s2 = (x[p->col_idx[p->row_ptr[i]]] + x[p->col_idx[p->row_ptr[i] + 1]]) * 0.5;
            if (s2 > T) T = s2;
        }
        double cst = 0.0;
        for (int64_t j = 0; j < n; ++j) { sol[j] = x[j] > T ? 1 : 0; cst += sol[j] ? p->c[j] : 0.0; }
        *cost = cst;
        if (aux) aux[0] = T;
        return 0;
    }
    if (rule == RULE_MIS_RAND) {
        if (!edge_rows_ok(p, -1)) return -1;
        /* packing lemma (Appendix C): alpha = max_e (x_u + x_v - 1)_+ ,
           xt = x/(1+alpha); keep v with probability xt_v (theta = 1/k); then
           drop every kept vertex that has a kept neighbour */
        double alpha = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            double sm = x[p->col_idx[p->row_ptr[i]]] + x[p->col_idx[p->row_ptr[i] + 1]];
            if (sm - 1.0 > alpha) alpha = sm - 1.0;
        }
        int32_t *pick = (int32_t *)malloc((n + 1) * 4);
        int32_t *drop = (int32_t *)malloc((n + 1) * 4);
        double best = INFINITY;
        for (int32_t rep = 0; rep < (reps > 0 ? reps : 1); ++rep) {
            for (int64_t j = 0; j < n; ++j) {
                double xt = x[j] / (1.0 + alpha);
                pick[j] = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)j, 0)) < xt ? 1 : 0;
                drop[j] = 0;
            }
            for (int64_t i = 0; i < m; ++i) {
                int32_t a = p->col_idx[p->row_ptr[i]], b = p->col_idx[p->row_ptr[i] + 1];
                if (pick[a] && pick[b]) { drop[a] = 1; drop[b] = 1; }
            }
            double cst = 0.0;
            for (int64_t j = 0; j < n; ++j) if (pick[j] && !drop[j]) cst += p->c[j];
            if (cst < best) {
                best = cst;
                for (int64_t j = 0; j < n; ++j) sol[j] = pick[j] && !drop[j];
                if (aux) aux[1] = rep;
            }
        }
        free(pick); free(drop);
        *cost = best;
        if (aux) aux[0] = alpha;
        return 0;
    }
    if (rule == RULE_MAP_ARGMAX || rule == RULE_MAP_SAMPLE) {
        if (p->nblocks <= 0 || p->npw < 0 || !p->pw_ends) return -1;
        /* node-based roundings of the local-polytope LP (Ravikumar et al.,
           cited for the MAP experiments): a fixed block keeps its label;
           otherwise the label of the largest marginal (ties: the lower
           label), or a label drawn from the marginal by inverse CDF in label
           order (u below the running sum; past the end, the last label with
           positive mass); best of reps by energy */
        int32_t k = p->k;
        int64_t nb = p->nblocks;
        int32_t *lab = (int32_t *)malloc((nb + 1) * 4);
        int32_t nrep = rule == RULE_MAP_ARGMAX ? 1 : (reps > 0 ? reps : 1);
        double best = INFINITY;
        for (int32_t rep = 0; rep < nrep; ++rep) {
            for (int64_t t = 0; t < nb; ++t) {
                const double *mu = x + p->bfirst[t];
                int32_t l = 0;
                if (p->fixed[t] >= 0) {
                    l = p->fixed[t];
                } else if (rule == RULE_MAP_ARGMAX) {
                    for (int32_t a = 1; a < k; ++a) if (mu[a] > mu[l]) l = a;
                } else {
                    double u = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)t, 3)), cum = 0.0;
                    l = -1;
                    int32_t lastpos = 0;
                    for (int32_t a = 0; a < k; ++a) {
                        if (mu[a] > 0.0) lastpos = a;
                        cum += mu[a];
                        if (l < 0 && u < cum) l = a;
                    }
                    if (l < 0) l = lastpos;
                }
                lab[t] = l;
            }
            double en = map_energy(p, lab);
            if (en < best) {
                best = en;
                for (int64_t t = 0; t < nb; ++t) sol[t] = lab[t];
                if (aux) aux[1] = rep;
            }
        }
        free(lab);
        *cost = best;
        if (aux) aux[0] = 0.0;
        return 0;
    }
    if (rule == RULE_MC_CKR) {
        if (p->nblocks <= 0) return -1;
        /* region growing: radius rho ~ U[0,1), terminal order sigma random;
           for i < k, every unassigned block with x^{sigma(i)} >= 1 - rho takes
           label sigma(i); the rest take sigma(k).  Cut cost = sum of c_e over
           edges whose endpoint labels differ, read off the objective of the z
           columns (each cut edge contributes 1/2 c_e for two labels). */
        int32_t k = p->k;
        int64_t nb = p->nblocks;
        int32_t *lab = (int32_t *)malloc((nb + 1) * 4);
        double best = INFINITY;
        for (int32_t rep = 0; rep < (reps > 0 ? reps : 1); ++rep) {
            double rad = u53(ph_word(seed, ST_ROUND, (uint64_t)rep, 0, 1));
            keyed ks[256];
            for (int32_t i = 0; i < k; ++i) {
                ks[i].key = ph_word(seed, ST_ROUND, (uint64_t)rep, (uint64_t)i, 2);
                ks[i].idx = i;
            }
            qsort(ks, k, sizeof(keyed), cmp_keyed);
            for (int64_t t = 0; t < nb; ++t) {
                lab[t] = (int32_t)ks[k - 1].idx;
                for (int32_t q = 0; q < k - 1; ++q) {
                    int32_t i = (int32_t)ks[q].idx;
                    if (x[p->bfirst[t] + i] >= 1.0 - rad) { lab[t] = i; break; }
                }
            }
            /* cost: for each row (z - x_u + x_v >= 0 style), the structural
               columns outside blocks are the edge variables; an edge is cut
               when the blocks in its rows carry different labels */
            double cst = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                int64_t zc = -1, b1 = -1, b2 = -1;
                for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
                    int64_t j = p->col_idx[e];
                    int64_t bl = p->col_block[j];
                    if (bl < 0) zc = j; else if (b1 < 0) b1 = bl; else b2 = bl;
                }
                if (zc < 0 || b1 < 0 || b2 < 0) continue;
                /* the z column of label i is charged when exactly one endpoint has label i */
                int64_t li = -1;
                for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) {
                    int64_t j = p->col_idx[e];
                    if (p->col_block[j] == b1) li = j - p->bfirst[b1];
                }
                if ((lab[b1] == li) != (lab[b2] == li)) cst += p->c[zc];
            }
            cst *= 0.5;     /* each (edge,label) pair owns two rows */
            if (cst < best) {
                best = cst;
                for (int64_t t = 0; t < nb; ++t) sol[t] = lab[t];
                if (aux) { aux[0] = rad; aux[1] = rep; }
            }
        }
        free(lab);
        *cost = best;
        return 0;
    }
    return -1;
}

/* feasibility of an integer solution for the original rows */
int32_t orc_check(const orc_lp *p, int32_t rule, const int32_t *sol, int32_t *feasible,
                  int64_t *nviol) {
    int64_t bad = 0;
    if (rule == RULE_MC_CKR || rule == RULE_MAP_ARGMAX || rule == RULE_MAP_SAMPLE) {
        for (int64_t t = 0; t < p->nblocks; ++t) {
            if (sol[t] < 0 || sol[t] >= p->k) { ++bad; continue; }
            if (p->fixed[t] >= 0 && sol[t] != p->fixed[t]) ++bad;
        }
    } else if ((rule >= RULE_VC_THRESH && rule <= RULE_MIS_RAND) ||
               (rule >= RULE_COVER_THRESH && rule <= RULE_PACK_RAND)) {
        for (int64_t j = 0; j < p->n; ++j) if (sol[j] != 0 && sol[j] != 1) ++bad;
        for (int64_t i = 0; i < p->m; ++i) {
            double ax = 0.0;
            for (int64_t e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) ax += p->val[e] * (double)sol[p->col_idx[e]];
            int ok = p->sense[i] > 0 ? ax >= p->b[i] : (p->sense[i] < 0 ? ax <= p->b[i] : ax == p->b[i]);
            if (!ok) ++bad;
        }
    } else {
        return -1;
    }
    *nviol = bad;
    *feasible = bad == 0;
    return 0;
}
