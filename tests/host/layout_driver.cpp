// Drives the host side of the library's C ABI (instance creation, blocks,
// pairwise factors, the layout with its colouring and plans, the rounding
// shapes, rejected inputs) on the given instance files, for the address /
// undefined-behaviour sanitizer build of layout.cpp.  Test infrastructure.
#include <cstdio>
#include <cstring>
#include <vector>

extern "C" {
#include "read_inst.h"
}
#include "../../include/thetis.h"

int main(int argc, char **argv) {
    for (int a = 1; a < argc; ++a) {
        inst_file I = read_inst(argv[a]);
        thetis_inst *h = nullptr;
        if (thetis_inst_create_csr(I.m, I.n, I.nnz, I.row_ptr, I.col_idx, I.val, I.b, I.c, I.u, I.sense, &h)) {
            fprintf(stderr, "%s: %s\n", argv[a], thetis_last_error());
            return 1;
        }
        if (I.nblocks && thetis_inst_set_simplex_blocks(h, I.nblocks, (int32_t)I.k, I.bfirst, I.fixed)) return 1;
        if (I.npw && thetis_inst_set_pairwise(h, I.npw, I.pw_ends, I.pw_first)) return 1;
        int32_t nc = 0;
        int64_t nu = 0;
        if (thetis_inst_classes(h, &nc, &nu, nullptr)) return 1;
        std::vector<int32_t> cls(nu + 1);
        if (thetis_inst_classes(h, &nc, &nu, cls.data())) return 1;
        int32_t flags = 0;
        double q = 0;
        if (thetis_inst_rounding_shape(h, &flags, &q)) return 1;
        thetis_inst_destroy(h);
        // rejected inputs leave nothing behind
        if (I.nnz > 0) {
            std::vector<int32_t> bad(I.col_idx, I.col_idx + I.nnz);
            bad[0] = (int32_t)I.n;
            if (thetis_inst_create_csr(I.m, I.n, I.nnz, I.row_ptr, bad.data(), I.val, I.b, I.c, I.u, I.sense, &h) ==
                THETIS_OK)
                return 1;
            std::vector<double> badc(I.c, I.c + I.n);
            badc[0] = 0.0 / 0.0;
            if (thetis_inst_create_csr(I.m, I.n, I.nnz, I.row_ptr, I.col_idx, I.val, I.b, badc.data(), I.u, I.sense,
                                       &h) == THETIS_OK)
                return 1;
        }
        free_inst(&I);
    }
    printf("layout driver ok\n");
    return 0;
}
