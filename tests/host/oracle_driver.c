/* Drives every entry point of the oracle on the given instance files, for
 * the address / undefined-behaviour sanitizer build of the oracle.  Test
 * infrastructure: compiled together with oracle/thetis_oracle.c. */
#include <string.h>

#include "read_inst.h"

typedef struct orc_lp orc_lp;
typedef struct orc_solver orc_solver;
orc_lp *orc_lp_create(int64_t, int64_t, const int64_t *, const int32_t *, const double *, const double *,
                      const double *, const double *, const int8_t *);
int orc_lp_set_blocks(orc_lp *, int64_t, int32_t, const int64_t *, const int32_t *);
int orc_lp_set_pairwise(orc_lp *, int64_t, const int32_t *, const int64_t *);
void orc_lp_free(orc_lp *);
int64_t orc_num_units(const orc_lp *);
int32_t orc_num_classes(const orc_lp *);
void orc_units(const orc_lp *, int8_t *, int64_t *, int32_t *);
void orc_class_order(const orc_lp *, uint64_t, int64_t, int32_t *);
double orc_cover_q(const orc_lp *);
orc_solver *orc_solver_create(orc_lp *, double, int32_t, double, int32_t, const double *, const double *,
                              int32_t, uint64_t);
void orc_solver_free(orc_solver *);
int32_t orc_run_epochs(orc_solver *, int32_t, int32_t, double *);
int64_t orc_trace_epoch(orc_solver *, double *, int64_t);
void orc_metrics(const orc_solver *, double *);
void orc_multiplier_step(orc_solver *, int32_t, double, double *);
void orc_get_y(const orc_solver *, double *);
void orc_set_y(orc_solver *, const double *);
int32_t orc_round(const orc_lp *, const double *, int32_t, uint64_t, int32_t, int32_t *, double *, double *);
int32_t orc_check(const orc_lp *, int32_t, const int32_t *, int32_t *, int64_t *);

int main(int argc, char **argv) {
    for (int a = 1; a < argc; ++a) {
        inst_file I = read_inst(argv[a]);
        orc_lp *p = orc_lp_create(I.m, I.n, I.row_ptr, I.col_idx, I.val, I.b, I.c, I.u, I.sense);
        if (!p) { fprintf(stderr, "%s: create failed\n", argv[a]); return 1; }
        if (I.nblocks && orc_lp_set_blocks(p, I.nblocks, (int32_t)I.k, I.bfirst, I.fixed) != 0) return 1;
        if (I.npw && orc_lp_set_pairwise(p, I.npw, I.pw_ends, I.pw_first) != 0) return 1;
        int64_t nu = orc_num_units(p);
        int32_t nc = orc_num_classes(p);
        int8_t *kind = (int8_t *)malloc(nu + 1);
        int64_t *uid = (int64_t *)malloc(8 * (nu + 1));
        int32_t *col = (int32_t *)malloc(4 * (nu + 1)), *ord = (int32_t *)malloc(4 * (nc + 1));
        orc_units(p, kind, uid, col);
        orc_class_order(p, 3, 5, ord);
        (void)orc_cover_q(p);
        double *zm = (double *)calloc(I.m + 1, 8), *zN = (double *)calloc(I.n + I.m + 1, 8);
        double *y = (double *)malloc(8 * (I.n + I.m + 1)), *tr = (double *)malloc(8 * (I.n + I.m + 2));
        double mt[8], st[4], Fs[4];
        for (int prox = 0; prox < 2; ++prox)
            for (int sched = 0; sched < 3; ++sched) {
                orc_solver *s = orc_solver_create(p, 10.0, sched == 2, 1.0, prox, prox ? zN : NULL, zm, sched, 7);
                orc_run_epochs(s, 3, sched == 0, Fs);
                (void)orc_trace_epoch(s, tr, I.n + I.m + 1);
                orc_metrics(s, mt);
                orc_multiplier_step(s, prox, 20.0, st);
                orc_run_epochs(s, 1, 0, NULL);
                orc_get_y(s, y);
                orc_set_y(s, y);
                orc_metrics(s, mt);
                orc_solver_free(s);
            }
        int64_t nsol = I.nblocks > I.n ? I.nblocks : I.n;
        int32_t *sol = (int32_t *)malloc(4 * (nsol + 1));
        for (int32_t rule = 1; rule <= 9; ++rule) {
            double cost, aux[4];
            if (orc_round(p, I.x, rule, 11, 3, sol, &cost, aux) == 0) {
                int32_t feas; int64_t nv;
                orc_check(p, rule, sol, &feas, &nv);
            }
        }
        free(sol); free(kind); free(uid); free(col); free(ord); free(zm); free(zN); free(y); free(tr);
        orc_lp_free(p);
        free_inst(&I);
    }
    printf("oracle driver ok\n");
    return 0;
}
