/* Host-side checks of the C ABI for the sanitizer build (AddressSanitizer and
 * UndefinedBehaviorSanitizer on the library's host code, no GPU needed): every entry point
 * rejects invalid arguments before touching a device, context creation without a usable
 * device fails cleanly, and the status strings are defined.  Exit status 0 when every check
 * holds; each failed check is printed. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "genp.h"

static int failures = 0;

static void expect(int got, int want, const char* what) {
    if (got != want) {
        printf("FAIL %s: status %d, expected %d\n", what, got, want);
        ++failures;
    }
}

int main(void) {
    for (int code = -12; code <= 12; ++code) {
        const char* s = genp_strerror(code);
        if (!s || !s[0]) {
            printf("FAIL strerror(%d) empty\n", code);
            ++failures;
        }
    }
    genp_ctx* h = NULL;
    expect(genp_create(NULL, 16, GENP_F64, 64, NULL), GENP_EINVAL, "create(NULL handle)");
    expect(genp_create(&h, 0, GENP_F64, 256, NULL), GENP_EINVAL, "create(n = 0)");
    expect(genp_create(&h, 10, 7, 256, NULL), GENP_EINVAL, "create(bad precision)");
    expect(genp_create(&h, 10, GENP_F64, 96, NULL), GENP_EINVAL, "create(nb = 96)");
    if (h) {
        printf("FAIL create wrote a handle on error\n");
        ++failures;
    }
    int st = genp_create(&h, 16, GENP_F64, 64, NULL);
    if (st == GENP_OK) {
        /* a usable device: the remaining checks are for hosts without one */
        genp_destroy(h);
        printf("device present: checks without a device skipped\n");
    } else {
        expect(st, GENP_EDEVICE, "create without a device");
        if (h) {
            printf("FAIL create wrote a handle without a device\n");
            ++failures;
        }
    }
    expect(genp_destroy(NULL), GENP_OK, "destroy(NULL)");
    double x[4] = {0, 0, 0, 0};
    int64_t bk = 0;
    genp_info info;
    genp_refine_opts opts;
    memset(&opts, 0, sizeof opts);
    expect(genp_precondition(NULL, x, 1, GENP_G_DENSE, x, 1), GENP_EINVAL, "precondition(NULL)");
    expect(genp_precondition2(NULL, x, 1, GENP_G_NONE, NULL, 0, GENP_G_DENSE, x, 1), GENP_EINVAL,
           "precondition2(NULL)");
    expect(genp_factor(NULL, 0.0, &bk), GENP_EINVAL, "factor(NULL)");
    expect(genp_factor_block(NULL, 0.0, &bk), GENP_EINVAL, "factor_block(NULL)");
    expect(genp_block_pivots(NULL, x, 1), GENP_EINVAL, "block_pivots(NULL)");
    expect(genp_row_perm(NULL, NULL), GENP_EINVAL, "row_perm(NULL)");
    expect(genp_solve(NULL, x, 1, 1, x, 1), GENP_EINVAL, "solve(NULL)");
    expect(genp_refine(NULL, x, 1, 1, x, 1, 2, 0.0, GENP_SOLVER_LUIR, NULL), GENP_EINVAL, "refine(NULL)");
    expect(genp_refine_ex(NULL, x, 1, 1, x, 1, &opts, NULL), GENP_EINVAL, "refine_ex(NULL)");
    expect(genp_solve_backward(NULL, x, 1, x, 1, 1, x, 1, NULL, 0, 0), GENP_EINVAL, "solve_backward(NULL)");
    expect(genp_solve_backward_ex(NULL, x, 1, x, 1, 1, x, 1, NULL, 0, &opts, NULL), GENP_EINVAL,
           "solve_backward_ex(NULL)");
    expect(genp_condest(NULL, x, x + 1, x + 2), GENP_EINVAL, "condest(NULL)");
    expect(genp_get_info(NULL, &info), GENP_EINVAL, "get_info(NULL)");
    expect(genp_copy_work(NULL, x, 1), GENP_EINVAL, "copy_work(NULL)");
    genp_lr_info lri;
    genp_nrank_info nri;
    expect(genp_lowrank(NULL, 4, 4, 4, GENP_G_DENSE, x, 4, 2, 1e-8, 1e-8, x, 2, x, 2, NULL, 0, NULL, &lri, NULL),
           GENP_EINVAL, "lowrank(NULL A)");
    expect(genp_numerical_rank(NULL, 10, 10, 10, x, 4, 0, 4, 1e6, x, 4, &nri, NULL), GENP_EINVAL,
           "numerical_rank(NULL A)");
    expect(genp_numerical_rank_noalloc(NULL, 10, 10, 10, x, 4, 0, 4, 1e6, x, 4, &nri, NULL), GENP_EINVAL,
           "numerical_rank_noalloc(NULL A)");
    /* a problem larger than the fixed scratch array is refused before any device work */
    expect(genp_numerical_rank_noalloc(x, 200000, 200000, 200000, x, 64, 0, 64, 1e6, x, 64, &nri, NULL),
           GENP_ESCRATCH, "numerical_rank_noalloc(oversize)");
    if (failures) printf("%d check(s) failed\n", failures);
    else printf("all host checks passed\n");
    return failures ? 1 : 0;
}
