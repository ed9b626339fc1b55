/* Reads the instance files the sanitizer test writes (little-endian):
 * int64 m, n, nnz, nblocks, k, npw; int64 row_ptr[m+1]; int32 col_idx[nnz];
 * double val[nnz], b[m], c[n], u[n]; int8 sense[m]; int64 bfirst[nblocks];
 * int32 fixed[nblocks]; int32 pw_ends[2 npw]; int64 pw_first[npw];
 * double x[n] (a point to round).  Test infrastructure. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t m, n, nnz, nblocks, k, npw;
    int64_t *row_ptr; int32_t *col_idx; double *val, *b, *c, *u; int8_t *sense;
    int64_t *bfirst; int32_t *fixed; int32_t *pw_ends; int64_t *pw_first; double *x;
} inst_file;

static void *rd(FILE *f, size_t sz, int64_t cnt) {
    void *p = malloc(sz * (size_t)(cnt > 0 ? cnt : 1));
    if (cnt > 0 && fread(p, sz, (size_t)cnt, f) != (size_t)cnt) { fprintf(stderr, "short read\n"); exit(2); }
    return p;
}

static inst_file read_inst(const char *path) {
    inst_file I;
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    int64_t h[6];
    if (fread(h, 8, 6, f) != 6) { fprintf(stderr, "short header\n"); exit(2); }
    I.m = h[0]; I.n = h[1]; I.nnz = h[2]; I.nblocks = h[3]; I.k = h[4]; I.npw = h[5];
    I.row_ptr = (int64_t *)rd(f, 8, I.m + 1);
    I.col_idx = (int32_t *)rd(f, 4, I.nnz);
    I.val = (double *)rd(f, 8, I.nnz);
    I.b = (double *)rd(f, 8, I.m);
    I.c = (double *)rd(f, 8, I.n);
    I.u = (double *)rd(f, 8, I.n);
    I.sense = (int8_t *)rd(f, 1, I.m);
    I.bfirst = (int64_t *)rd(f, 8, I.nblocks);
    I.fixed = (int32_t *)rd(f, 4, I.nblocks);
    I.pw_ends = (int32_t *)rd(f, 4, 2 * I.npw);
    I.pw_first = (int64_t *)rd(f, 8, I.npw);
    I.x = (double *)rd(f, 8, I.n);
    fclose(f);
    return I;
}

static void free_inst(inst_file *I) {
    free(I->row_ptr); free(I->col_idx); free(I->val); free(I->b); free(I->c); free(I->u);
    free(I->sense); free(I->bfirst); free(I->fixed); free(I->pw_ends); free(I->pw_first); free(I->x);
}
