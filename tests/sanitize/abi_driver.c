/* Drives the host side of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
 * without a GPU: parameter validation, the back-off, context creation with an allocator that
 * fails, NULL handles, the scratch check of the solve that allocates nothing, server and batch
 * argument checks, and the thread-local error message.  Exit status 0 when every call behaves
 * as documented. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "bssmppi.h"

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("failed: %s (line %d): %s\n", #c, __LINE__, bss_last_error()); ++fails; } } while (0)

static void* no_alloc(size_t n, void* user) { (void)n; (void)user; return NULL; }
static void no_release(void* p, void* user) { (void)p; (void)user; }

int main(void)
{
    bss_params p;
    bss_params_default(&p);
    CHECK(bss_validate(&p) == BSS_OK);
    double nu = 0.0;
    CHECK(bss_backoff(&p, &nu) == BSS_OK && fabs(nu - 1.6448536269514722) < 1e-12);
    /* each invalid field is rejected */
    bss_params q = p; q.K = 0; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.M = 513; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.T = 100000; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.delta = 0.7; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.gamma = NAN; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.lambda = -1; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.belief = 2; q.M = 7; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.n_obs = 9; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.n_con = 1; q.con_a[0] = INFINITY; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.lanes = 24; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.ell_a = 3; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.vehicle = 1; q.shield_iters = 2; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.vehicle = 1; q.track_len = 5; CHECK(bss_validate(&q) == BSS_E_INVAL);
    q = p; q.vehicle = 1; CHECK(bss_validate(&q) == BSS_OK);
    CHECK(bss_validate(NULL) == BSS_E_INVAL);
    /* a failing allocator: BSS_E_NOMEM, no context, nothing leaked (LeakSanitizer) */
    bss_allocator a = {no_alloc, no_release, NULL};
    bss_ctx* c = (bss_ctx*)1;
    for (int i = 0; i < 100; ++i) {
        CHECK(bss_create(&p, &a, NULL, &c) == BSS_E_NOMEM);
        CHECK(c == NULL);
    }
    CHECK(strstr(bss_last_error(), "allocator returned NULL") != NULL);
    bss_allocator half = {no_alloc, NULL, NULL};
    CHECK(bss_create(&p, &half, NULL, &c) == BSS_E_INVAL);
    /* NULL handles */
    double u0[2];
    double x0[6] = {30, 0, 1.57, 5, 0, 0};
    CHECK(bss_solve(NULL, x0, NULL, u0, NULL) == BSS_E_INVAL);
    CHECK(bss_step_shift(NULL) == BSS_E_INVAL);
    CHECK(bss_get_controls(NULL, u0) == BSS_E_INVAL);
    bss_destroy(NULL);
    /* the solve that allocates nothing checks its scratch before any device call */
    q = p; q.K = 8192; q.M = 128; q.T = 200;
    CHECK(bss_noalloc_scratch_bytes(&q) > BSS_NOALLOC_SCRATCH_BYTES);
    double dummy[16];
    CHECK(bss_solve_noalloc(&q, 0, dummy, NULL, dummy, dummy + 8, dummy, NULL) == BSS_E_INVAL);
    CHECK(strstr(bss_last_error(), "scratch") != NULL);
    CHECK(bss_solve_noalloc(&p, 0, dummy, NULL, dummy, dummy, dummy, NULL) == BSS_E_INVAL);
    CHECK(bss_noalloc_scratch_bytes(NULL) == 0);
    /* server configuration checks */
    bss_server_config cfg;
    bss_server_config_default(&cfg);
    cfg.n_vehicles = 0;
    bss_server* srv = NULL;
    CHECK(bss_server_create(&cfg, &p, &srv) == BSS_E_INVAL && srv == NULL);
    /* batches need contexts */
    bss_batch* b = NULL;
    CHECK(bss_batch_create(NULL, 1, 0, 0, &b) == BSS_E_INVAL);
    if (fails) return 1;
    puts("abi driver: ok");
    return 0;
}
