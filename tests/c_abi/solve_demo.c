/*
 * The solver driven through the C interface alone (include/saamg.h and the HIP runtime's C
 * API; no Python): build the 33^3 cylinder's domain, set up the hierarchy, solve A x = b,
 * refresh the hierarchy for a longer pipe on the same lattice and solve again; then set up
 * and solve once more with a caller-supplied allocator (saamg_options.alloc / free), and
 * check that a too-small allocator makes the setup fail cleanly.
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
    double h[4];
    *mask = (uint8_t*)malloc(nbox);
    CHECK(saamg_domain_from_shape(SAAMG_SHAPE_CYLINDER, 1.0, 1.0, len, 0.0, 0.0, n, n, n, 0,
                                  *mask, 0, NULL, NULL, NULL, &nw, NULL));
    *wn = (int64_t*)malloc(8 * (nw + 1));
    *wd = (uint8_t*)malloc(nw + 1);
    *ws = (double*)malloc(8 * (nw + 1));
    CHECK(saamg_domain_from_shape(SAAMG_SHAPE_CYLINDER, 1.0, 1.0, len, 0.0, 0.0, n, n, n, 0,
                                  *mask, nw, *wn, *wd, *ws, &nw, h));
    d->nx = d->ny = d->nz = n;
    d->hx = h[0];
    d->hy = h[1];
    d->hz = h[2];
    d->mask = *mask;
    d->n_wall = nw;
    d->wall_node = *wn;
    d->wall_dir = *wd;
    d->wall_s = *ws;
    d->robin_d = h[3];
    return 0;
}

/* A caller's allocator: bump allocation from one slab the caller owns, with counts. */
typedef struct {
    char* base;
    size_t cap, used;
    long n_alloc, n_free;
} slab_t;

static void* slab_alloc(void* ctx, size_t bytes, void* stream) {
    slab_t* sl = (slab_t*)ctx;
    (void)stream;
    size_t off = (sl->used + 255) & ~(size_t)255;
    if (off + bytes > sl->cap) return NULL;
    sl->used = off + bytes;
    sl->n_alloc++;
    return sl->base + off;
}

static void slab_free(void* ctx, void* ptr, void* stream) {
    slab_t* sl = (slab_t*)ctx;
    (void)stream;
    if ((char*)ptr >= sl->base && (char*)ptr < sl->base + sl->cap) sl->n_free++;
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

    /* the same setup and solve with every buffer from the caller's slab: the library
       keeps no device memory of its own (free device memory does not drop over the run;
       the runtime may hand back memory cached from the hipFree'd run above), returns every
       buffer, and the solution is bitwise the first one */
    slab_t sl = {NULL, (size_t)256 << 20, 0, 0, 0};
    HCHECK(hipMalloc((void**)&sl.base, sl.cap));
    HCHECK(hipDeviceSynchronize());
    size_t free0 = 0, free1 = 0, total = 0;
    HCHECK(hipMemGetInfo(&free0, &total));
    saamg_options opt;
    saamg_default_options(&opt);
    opt.alloc = slab_alloc;
    opt.free = slab_free;
    opt.alloc_ctx = &sl;
    CHECK(saamg_setup(&dom, SAAMG_VARIANT_LIN, &opt, NULL, &H));
    CHECK(saamg_solve(H, db, NULL, dx, 1e-10, 500, NULL, &res));
    CHECK(saamg_destroy(H));
    HCHECK(hipDeviceSynchronize());
    HCHECK(hipMemGetInfo(&free1, &total));
    double* hx2 = (double*)malloc(8 * nbox);
    HCHECK(hipMemcpy(hx2, dx, 8 * nbox, hipMemcpyDeviceToHost));
    int same = 1;
    for (size_t i = 0; i < nbox; ++i) same &= hx2[i] == hx[i];
    printf("caller allocator: allocs=%ld frees=%ld slab_bytes=%zu free_delta=%lld same=%d\n",
           sl.n_alloc, sl.n_free, sl.used, (long long)free0 - (long long)free1, same);
    if (sl.n_alloc == 0 || sl.n_free != sl.n_alloc || free1 < free0 || !same) return 1;

    /* a slab too small: setup fails with SAAMG_NOMEM and returns what it took */
    slab_t small = {sl.base, (size_t)64 << 10, 0, 0, 0};
    opt.alloc_ctx = &small;
    int rc = saamg_setup(&dom, SAAMG_VARIANT_LIN, &opt, NULL, &H);
    printf("small slab: rc=%d allocs=%ld frees=%ld (%s)\n", rc, small.n_alloc, small.n_free,
           saamg_last_error());
    if (rc != SAAMG_NOMEM || H != NULL || small.n_free != small.n_alloc) return 1;
    HCHECK(hipFree(sl.base));
    free(hx2);

    HCHECK(hipFree(db));
    HCHECK(hipFree(dx));
    free(hb); free(hx); free(mask); free(wn); free(wd); free(ws);
    free(mask2); free(wn2); free(wd2); free(ws2);
    printf("ok\n");
    return 0;
}
