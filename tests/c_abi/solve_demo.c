/*
 * The solver driven through the C interface alone (include/saamg.h and the HIP runtime's C
 * API; no Python): build the 33^3 cylinder's domain, set up the hierarchy, solve A x = b,
 * refresh the hierarchy for a longer pipe on the same lattice and solve again.
 *
 *   solve_demo RHS OUT      RHS: nx*ny*nz fp64 box vector (x fastest), read;
 *                           OUT: the first solution, written in the same layout.
 * Prints one line per step; exits non-zero on any failure.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "saamg.h"

#define CHECK(call)                                                                  \
    do {                                                                             \
        int rc_ = (call);                                                            \
        if (rc_ != 0) {                                                              \
            fprintf(stderr, "%s failed: %d %s\n", #call, rc_, saamg_last_error());   \
            return 1;                                                                \
        }                                                                            \
    } while (0)
#define HCHECK(call)                                                                 \
    do {                                                                             \
        if ((call) != hipSuccess) {                                                  \
            fprintf(stderr, "%s failed\n", #call);                                   \
            return 1;                                                                \
        }                                                                            \
    } while (0)

/* Domain of a cylinder of radius 1 and length `len` on n^3 nodes; arrays malloc'ed. */
static int cylinder(int n, double len, saamg_domain* d, uint8_t** mask, int64_t** wn,
                    uint8_t** wd, double** ws) {
    const size_t nbox = (size_t)n * n * n;
    int64_t nw = 0;
    *mask = (uint8_t*)malloc(nbox);
    CHECK(saamg_domain_from_shape(SAAMG_SHAPE_CYLINDER, 1.0, 1.0, len, 0.0, 0.0, n, n, n, 0,
                                  *mask, 0, NULL, NULL, NULL, &nw));
    *wn = (int64_t*)malloc(8 * (nw + 1));
    *wd = (uint8_t*)malloc(nw + 1);
    *ws = (double*)malloc(8 * (nw + 1));
    CHECK(saamg_domain_from_shape(SAAMG_SHAPE_CYLINDER, 1.0, 1.0, len, 0.0, 0.0, n, n, n, 0,
                                  *mask, nw, *wn, *wd, *ws, &nw));
    d->nx = d->ny = d->nz = n;
    d->hx = d->hy = 2.0 / (n - 1);
    d->hz = len / (n - 1);
    d->mask = *mask;
    d->n_wall = nw;
    d->wall_node = *wn;
    d->wall_dir = *wd;
    d->wall_s = *ws;
    d->robin_d = 0.0;
    return 0;
}

int main(int argc, char** argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s RHS OUT\n", argv[0]);
        return 2;
    }
    const int n = 33;
    const size_t nbox = (size_t)n * n * n;
    double* hb = (double*)malloc(8 * nbox);
    FILE* f = fopen(argv[1], "rb");
    if (!f || fread(hb, 8, nbox, f) != nbox) {
        fprintf(stderr, "cannot read %s\n", argv[1]);
        return 1;
    }
    fclose(f);

    saamg_domain dom;
    uint8_t* mask;
    int64_t* wn;
    uint8_t* wd;
    double* ws;
    if (cylinder(n, 2.0, &dom, &mask, &wn, &wd, &ws)) return 1;
    saamg_hierarchy* H = NULL;
    CHECK(saamg_setup(&dom, SAAMG_VARIANT_LIN, NULL, NULL, &H));
    saamg_info info;
    CHECK(saamg_hierarchy_info(H, &info));
    printf("setup levels=%d unknowns=%lld\n", info.n_levels, (long long)info.n_unknowns[0]);

    double *db = NULL, *dx = NULL;
    HCHECK(hipMalloc((void**)&db, 8 * nbox));
    HCHECK(hipMalloc((void**)&dx, 8 * nbox));
    HCHECK(hipMemcpy(db, hb, 8 * nbox, hipMemcpyHostToDevice));
    saamg_result res;
    CHECK(saamg_solve(H, db, NULL, dx, 1e-10, 500, NULL, &res));
    printf("solve iterations=%d rel_res=%.3e\n", res.iterations, res.rel_res_true);
    if (res.status != 0 || !(res.rel_res_true <= 1e-10)) return 1;
    double* hx = (double*)malloc(8 * nbox);
    HCHECK(hipMemcpy(hx, dx, 8 * nbox, hipMemcpyDeviceToHost));
    f = fopen(argv[2], "wb");
    if (!f || fwrite(hx, 8, nbox, f) != nbox) {
        fprintf(stderr, "cannot write %s\n", argv[2]);
        return 1;
    }
    fclose(f);

    /* the same lattice for a pipe of length 2.5: only h_z changes */
    saamg_domain dom2;
    uint8_t* mask2;
    int64_t* wn2;
    uint8_t* wd2;
    double* ws2;
    if (cylinder(n, 2.5, &dom2, &mask2, &wn2, &wd2, &ws2)) return 1;
    CHECK(saamg_refresh(H, &dom2, NULL));
    CHECK(saamg_solve(H, db, dx, dx, 1e-10, 500, NULL, &res));
    printf("refresh+solve iterations=%d rel_res=%.3e\n", res.iterations, res.rel_res_true);
    if (res.status != 0 || !(res.rel_res_true <= 1e-10)) return 1;

    CHECK(saamg_destroy(H));
    HCHECK(hipFree(db));
    HCHECK(hipFree(dx));
    free(hb); free(hx); free(mask); free(wn); free(wd); free(ws);
    free(mask2); free(wn2); free(wd2); free(ws2);
    printf("ok\n");
    return 0;
}
