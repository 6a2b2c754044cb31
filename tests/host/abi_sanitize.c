/* Host-side checks of the C ABI, built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_host_sanitizers.py): parameter
 * validation, layout and workspace sizes over a randomized sweep of
 * parameters including extreme and invalid values, the size query of
 * lbm_create_static, argument checks that return before any device work,
 * and an empty batch's life cycle.  Nothing here touches a GPU. */
#include "lbmgrow.h"

#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

static uint64_t rs = 0x9E3779B97F4A7C15ull;
static uint64_t next(void)
{
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return rs;
}

static lbm_params base(void)
{
    lbm_params p;
    memset(&p, 0, sizeof p);
    p.abi_version = LBM_ABI_VERSION;
    p.struct_size = sizeof p;
    p.L = 256;
    p.H = 512;
    p.precision = LBM_FP32;
    p.growth = LBM_GROWTH_BULK;
    p.tau = 1.0;
    p.mu = 1e-3;
    p.rho_c = 0.5;
    p.rho_init = 1.0;
    p.init_amp = 1e-3;
    p.init_rows = 64;
    p.growth_rate = 1e-4;
    p.sigma = 1e-3;
    p.wall_min_gap = 50;
    p.wall_w_factor = 10.0;
    p.rho_ref = 1.0;
    p.rho_cell = 0.1;
    p.rho0 = 2.0;
    return p;
}

static const int32_t kInts[] = {0, 1, 2, 3, 4, 5, 7, 8, 9, 16, 63, 64, 65, 255, 256, 4096,
                                (1 << 24) - 1, 1 << 24, (1 << 24) + 1, INT_MAX, INT_MIN, -1, -2};
static const double kReals[] = {0.0, -0.0, 0.5, 0.5000001, 1.0, 2.0, 1e-300, 1e300, -1.0,
                                0.999999, 1e-3, 8.0, 64.0};

static int32_t any_int(void)
{
    if (next() & 1) return kInts[next() % (sizeof kInts / sizeof kInts[0])];
    return (int32_t)(next() % 20000) - 100;
}
static double any_real(void)
{
    const uint64_t k = next() % 16;
    if (k == 0) return NAN;
    if (k == 1) return INFINITY;
    if (k == 2) return -INFINITY;
    if (k < 8) return kReals[next() % (sizeof kReals / sizeof kReals[0])];
    return (double)(next() % 100000) / 1000.0 - 5.0;
}

static void mutate(lbm_params *p)
{
    const int n = 1 + (int)(next() % 4);
    for (int i = 0; i < n; ++i) {
        switch (next() % 24) {
        case 0: p->L = any_int(); break;
        case 1: p->H = any_int(); break;
        case 2: p->precision = any_int() % 6; break;
        case 3: p->growth = any_int() % 6; break;
        case 4: p->tau = any_real(); break;
        case 5: p->mu = any_real(); break;
        case 6: p->rho_c = any_real(); break;
        case 7: p->init_amp = any_real(); break;
        case 8: p->init_rows = any_int(); break;
        case 9: p->region = any_int() % 4; break;
        case 10: p->region_width = any_int(); break;
        case 11: p->ybc = any_int() % 4; break;
        case 12: p->sigma = any_real(); break;
        case 13: p->flags = (int32_t)(next() & 0x3F); break;
        case 14: p->kernel_vb = any_int() % 20; break;
        case 15: p->kernel_ty = any_int() % 80; break;
        case 16: p->lattice = any_int() % 3; break;
        case 17: p->kernel_order = any_int() % 6; break;
        case 18: p->rho_cell = any_real(); break;
        case 19: p->rho0 = any_real(); break;
        case 20: p->growth_rate = any_real(); break;
        case 21: p->wall_min_gap = any_int(); break;
        case 22: p->struct_size = (uint32_t)(next() % 512); break;
        default: p->abi_version = (uint32_t)(next() % 8); break;
        }
    }
}

int main(void)
{
    const char *v = lbm_version();
    CHECK(v != NULL && strncmp(v, "lbmgrow", 7) == 0);
    CHECK(strcmp(lbm_last_error(NULL), "") != 0);

    /* a valid configuration and the calls that reject bad arguments before
       any device work */
    lbm_params p = base();
    const size_t ws = lbm_workspace_bytes(&p);
    CHECK(ws > (size_t)2 * 9 * 256 * 512 * 4);
    CHECK(lbm_tiles(&p) > 0);
    CHECK(lbm_workspace_bytes(NULL) == 0 && lbm_tiles(NULL) == 0);
    lbm_handle *h = (lbm_handle *)&p;   /* must be overwritten */
    CHECK(lbm_create(NULL, (void *)(uintptr_t)4096, ws, NULL, &h) == LBM_E_INVALID && h == NULL);
    CHECK(lbm_create(&p, NULL, ws, NULL, &h) == LBM_E_INVALID);
    CHECK(lbm_create(&p, (void *)(uintptr_t)4100, ws, NULL, &h) == LBM_E_INVALID);   /* unaligned */
    CHECK(lbm_create(&p, (void *)(uintptr_t)4096, ws - 1, NULL, &h) == LBM_E_NOMEM);
    CHECK(lbm_create(&p, (void *)(uintptr_t)4096, ws, NULL, NULL) == LBM_E_INVALID);
    size_t pops = 0;
    CHECK(lbm_create_static(&p, NULL, &pops, NULL, NULL) == LBM_OK && pops > 0 && pops < ws);
    CHECK(lbm_create_static(&p, NULL, NULL, NULL, NULL) == LBM_E_INVALID);
    CHECK(lbm_step(NULL, 1) < 0 && lbm_destroy(NULL) < 0);
    CHECK(lbm_stream_copy(NULL, NULL, 16, NULL) == LBM_E_INVALID);
    CHECK(lbm_stream_copy((void *)(uintptr_t)4096, (void *)(uintptr_t)4104, 16, NULL) == LBM_E_INVALID);

    /* randomized sweep: the size queries agree on validity and never
       overflow */
    int valid = 0;
    for (int it = 0; it < 200000; ++it) {
        lbm_params q = base();
        mutate(&q);
        const size_t b = lbm_workspace_bytes(&q);
        const int64_t t = lbm_tiles(&q);
        CHECK((b == 0) == (t == 0));
        size_t sp = 0;
        const int rc = lbm_create_static(&q, NULL, &sp, NULL, NULL);
        CHECK(b != 0 || rc == LBM_E_INVALID);
        if (b != 0) {
            ++valid;
            const int nq = q.lattice == LBM_LATTICE_D2Q7 ? 7 : 9;
            const size_t es = q.precision == LBM_FP64 ? 8 : q.precision == LBM_FP32 ? 4 : 2;
            CHECK(b >= (size_t)2 * nq * (size_t)q.L * (size_t)q.H * es);
            CHECK(rc == LBM_E_NOMEM || (rc == LBM_OK && sp < b));
        }
        lbm_handle *hh = NULL;
        if (b == 0) CHECK(lbm_create(&q, (void *)(uintptr_t)4096, (size_t)1 << 40, NULL, &hh) == LBM_E_INVALID);
    }
    CHECK(valid > 1000);

    /* batch sizes and an empty batch's life cycle (host only) */
    CHECK(lbm_batch_workspace_bytes(0, 1) == 0 && lbm_batch_workspace_bytes(1, 0) == 0);
    CHECK(lbm_batch_workspace_bytes(INT_MAX, INT64_MAX / 1024) > 0 ||
          lbm_batch_workspace_bytes(INT_MAX, INT64_MAX / 1024) == 0);
    const size_t bw = lbm_batch_workspace_bytes(8, 4096);
    CHECK(bw > 0);
    lbm_batch *bt = NULL;
    CHECK(lbm_batch_create((void *)(uintptr_t)4096, bw - 1, 8, 4096, NULL, &bt) == LBM_E_NOMEM);
    CHECK(lbm_batch_create((void *)(uintptr_t)4097, bw, 8, 4096, NULL, &bt) == LBM_E_INVALID);
    CHECK(lbm_batch_create((void *)(uintptr_t)4096, bw, 8, 4096, NULL, &bt) == LBM_OK && bt);
    CHECK(lbm_batch_add(bt, NULL) == LBM_E_INVALID);
    CHECK(lbm_batch_step(bt, -1) == LBM_E_INVALID);
    CHECK(lbm_batch_step(bt, 10) == LBM_OK);   /* no members: nothing to do */
    CHECK(lbm_batch_destroy(bt) == LBM_OK);
    CHECK(lbm_batch_destroy(NULL) == LBM_E_INVALID);

    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("abi_sanitize ok: %d valid configurations\n", valid);
    return 0;
}
