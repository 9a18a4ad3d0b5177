/*
 * abi_sanitize.c -- driver for the host side of the C ABI under
 * AddressSanitizer and UndefinedBehaviorSanitizer: every entry point's
 * validation runs on valid and invalid sizes, null pointers, bad options and
 * short workspaces, none of which reaches the GPU.  Linked against a
 * host-only build of the library (the device code is not compiled); built
 * and run by tests/test_oracle_sanitize.py.  Exit status 0 when every
 * validation answered as documented in include/gspca*.h.
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "gspca.h"
#include "gspca_block.h"
#include "gspca_ws.h"

static int failures = 0;
#define CHECK(c)                                                                           \
    do {                                                                                   \
        if (!(c)) {                                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);                \
            ++failures;                                                                    \
        }                                                                                  \
    } while (0)

#define FAKE(x) ((void *)(uintptr_t)(x))

static gspca_problem prob(int32_t dtype, int64_t M, int64_t N, int64_t K)
{
    gspca_problem p;
    memset(&p, 0, sizeof p);
    p.dtype = dtype;
    p.X = FAKE(0x10000);
    p.ldx = M;
    p.M = M;
    p.N = N;
    p.K = K;
    p.col_scale = (const float *)FAKE(0x20000);
    return p;
}

static void fit_validation(void)
{
    gspca_options op;
    gspca_default_options(&op);
    CHECK(op.algo == GSPCA_GS && op.max_iter == 10000);
    gspca_default_options(NULL);
    const int64_t shapes[][3] = {{1, 1, 1}, {100, 20, 4}, {3000, 700, 8}, {513, 4097, 3},
                                 {70000, 8192, 32}, {40, 9000, 2}, {5, 3, 3}};
    for (int dt = 0; dt < 4; ++dt)
        for (size_t i = 0; i < sizeof shapes / sizeof shapes[0]; ++i) {
            gspca_problem p = prob(dt, shapes[i][0], shapes[i][1], shapes[i][2]);
            for (int impl = 0; impl < 2; ++impl)
                for (int algo = 0; algo < 2; ++algo)
                    for (int reorth = 0; reorth < 3; ++reorth) {
                        op.implicit_deflation = impl;
                        op.algo = algo;
                        op.reorth = reorth;
                        const size_t w = gspca_workspace_bytes(&p, &op);
                        if (dt >= 2 && (!impl || algo != 0))
                            CHECK(w == 0); /* codes need implicit GS-PCA */
                        gspca_result r = {FAKE(0x1000), FAKE(0x2000), (double *)FAKE(0x3000),
                                          NULL, NULL, NULL};
                        if (w > 0)
                            CHECK(gspca_fit_ex(&p, &op, &r, FAKE(0x4000), w - 1, NULL) ==
                                  GSPCA_EWORKSPACE);
                        else
                            CHECK(gspca_fit_ex(&p, &op, &r, FAKE(0x4000), 1u << 30, NULL) < 0);
                    }
        }
    gspca_default_options(&op);
    gspca_problem p = prob(1, 100, 20, 4);
    gspca_result r = {FAKE(0x1000), FAKE(0x2000), (double *)FAKE(0x3000), NULL, NULL, NULL};
    gspca_result empty;
    memset(&empty, 0, sizeof empty);
    CHECK(gspca_fit_ex(NULL, &op, &r, FAKE(0x4000), 1u << 30, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_ex(&p, NULL, &r, FAKE(0x4000), 1u << 30, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_ex(&p, &op, NULL, FAKE(0x4000), 1u << 30, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_ex(&p, &op, &empty, FAKE(0x4000), 1u << 30, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_ex(&p, &op, &r, NULL, 1u << 30, NULL) == GSPCA_EWORKSPACE);
    CHECK(gspca_fit_ex(&p, &op, &r, FAKE(0x4001), 1u << 30, NULL) == GSPCA_EINVAL);
    gspca_options bad = op;
    bad.tol = -1.0;
    CHECK(gspca_workspace_bytes(&p, &bad) == 0);
    bad = op;
    bad.max_iter = 0;
    CHECK(gspca_workspace_bytes(&p, &bad) == 0);
    bad = op;
    bad.init = GSPCA_INIT_GIVEN;
    CHECK(gspca_workspace_bytes(&p, &bad) == 0);
    bad = op;
    bad.stop = 5;
    CHECK(gspca_workspace_bytes(&p, &bad) == 0);
    bad = op;
    bad.algo = 9;
    CHECK(gspca_workspace_bytes(&p, &bad) == 0);
    bad = op;
    bad.reorth = 7;
    CHECK(gspca_workspace_bytes(&p, &bad) == 0);
    gspca_problem q = p;
    q.ldx = 50;
    CHECK(gspca_workspace_bytes(&q, &op) == 0);
    q = p;
    q.K = 21;
    CHECK(gspca_workspace_bytes(&q, &op) == 0);
    q = p;
    q.X = NULL;
    CHECK(gspca_workspace_bytes(&q, &op) == 0);
    CHECK(gspca_fit(NULL, 10, 5, 2, 1e-7, 100, NULL, NULL, NULL, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_f32((const float *)FAKE(0x1000), 10, 5, 6, 1e-7, 100, (float *)FAKE(1),
                        (float *)FAKE(1), (double *)FAKE(1), NULL) == GSPCA_EINVAL);
}

static void quantize_validation(void)
{
    CHECK(gspca_quantized_bytes(100, 20, GSPCA_F32) == 0);
    CHECK(gspca_quantized_bytes(100, 9000, GSPCA_BF16) == 0);
    CHECK(gspca_quantized_bytes(0, 20, GSPCA_BF16) == 0);
    CHECK(gspca_quantized_bytes(100, 20, GSPCA_BF16) > 0);
    CHECK(gspca_quantized_bytes(100, 8192, GSPCA_FP8_E4M3) > 0);
    CHECK(gspca_quantize(NULL, 10, 5, 10, GSPCA_BF16, FAKE(1), (float *)FAKE(1), FAKE(256), 256,
                         NULL) == GSPCA_EINVAL);
    CHECK(gspca_quantize((const float *)FAKE(1), 10, 5, 9, GSPCA_BF16, FAKE(1), (float *)FAKE(1),
                         FAKE(256), 256, NULL) == GSPCA_EINVAL);
    CHECK(gspca_quantize((const float *)FAKE(1), 10, 5, 10, GSPCA_BF16, FAKE(1),
                         (float *)FAKE(1), FAKE(256), 8, NULL) == GSPCA_EWORKSPACE);
}

static void batched_validation(void)
{
    gspca_batch_problem b[3];
    memset(b, 0, sizeof b);
    for (int i = 0; i < 3; ++i) {
        b[i].X = (const float *)FAKE(0x1000);
        b[i].ldx = 64 + i;
        b[i].M = 64 + i;
        b[i].N = 16 + i;
        b[i].K = 4;
        b[i].T = (float *)FAKE(0x2000);
        b[i].P = (float *)FAKE(0x3000);
        b[i].lambda = (double *)FAKE(0x4000);
    }
    CHECK(gspca_batched_workspace_bytes(b, 3) > 0);
    CHECK(gspca_batched_workspace_bytes(NULL, 3) == 0);
    CHECK(gspca_batched_workspace_bytes(b, 0) == 0);
    gspca_batch_problem bad = b[1];
    bad.M = 5000;
    CHECK(gspca_batched_workspace_bytes(&bad, 1) == 0);
    bad = b[1];
    bad.K = 65;
    CHECK(gspca_batched_workspace_bytes(&bad, 1) == 0);
    gspca_options op;
    gspca_default_options(&op);
    gspca_batch_plan plan;
    op.algo = GSPCA_NIPALS;
    CHECK(gspca_batched_prepare(b, 3, &op, FAKE(0x10000), 1u << 20, &plan, NULL) == GSPCA_EINVAL);
    gspca_default_options(&op);
    op.reorth = GSPCA_REORTH_MGS;
    CHECK(gspca_batched_prepare(b, 3, &op, FAKE(0x10000), 1u << 20, &plan, NULL) == GSPCA_EINVAL);
    gspca_default_options(&op);
    CHECK(gspca_batched_prepare(b, 3, &op, FAKE(0x10000), 8, &plan, NULL) == GSPCA_EWORKSPACE);
    op.init = GSPCA_INIT_GIVEN; /* no T0 given */
    CHECK(gspca_batched_prepare(b, 3, &op, FAKE(0x10000), 1u << 20, &plan, NULL) == GSPCA_EINVAL);
    memset(&plan, 0, sizeof plan);
    CHECK(gspca_batched_launch(&plan, NULL) == GSPCA_EINVAL);
    CHECK(gspca_batched_launch(NULL, NULL) == GSPCA_EINVAL);
    CHECK(gspca_batched_tune(&plan, NULL) == GSPCA_EINVAL);
}

static void block_and_ws_validation(void)
{
    CHECK(gspca_block_workspace_bytes(100, 50, 32) > 0);
    CHECK(gspca_block_workspace_bytes(100, 50, 48) == 0);
    CHECK(gspca_block_workspace_bytes(20, 50, 32) == 0);
    gspca_block_options bo;
    memset(&bo, 0, sizeof bo);
    bo.r = 32;
    bo.max_iter = 5;
    bo.tol = 1e-6;
    bo.Omega = (const float *)FAKE(0x1000);
    float *T = (float *)FAKE(0x2000), *P = (float *)FAKE(0x3000);
    double *lam = (double *)FAKE(0x4000);
    CHECK(gspca_fit_block(NULL, 100, 100, 50, 4, &bo, T, P, lam, NULL, NULL, FAKE(0x5000),
                          1u << 30, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_block((const float *)FAKE(0x10000), 100, 100, 50, 40, &bo, T, P, lam, NULL,
                          NULL, FAKE(0x5000), 1u << 30, NULL) == GSPCA_EINVAL);
    CHECK(gspca_fit_block((const float *)FAKE(0x10000), 100, 100, 50, 4, &bo, T, P, lam, NULL,
                          NULL, FAKE(0x5000), 16, NULL) == GSPCA_EWORKSPACE);
    CHECK(gspca_mlp_param_count(32, 256, 256, 16) == 32 * 256 + 256 + 256 * 256 + 256 + 256 * 16 + 16);
    CHECK(gspca_sketch_workspace_bytes(2048, 256, 32) > 0);
    CHECK(gspca_sketch_workspace_bytes(2048, 256, 40) == 0);
    CHECK(gspca_sketch(NULL, 10, 10, 10, NULL, 32, NULL, NULL) == GSPCA_EINVAL);
    CHECK(gspca_whiten_sketch(NULL, 100, 32, NULL, NULL, NULL, NULL, 0, NULL) < 0);
    gspca_mlp net;
    memset(&net, 0, sizeof net);
    net.d0 = 32;
    net.d1 = 8; /* below the allowed range */
    net.d2 = 256;
    net.d3 = 16;
    CHECK(gspca_mlp_workspace_bytes(&net, 2048, 4, 32) == 0);
    CHECK(gspca_mlp_sync(&net, NULL) == GSPCA_EINVAL);
    CHECK(gspca_mlp_forward(&net, NULL, 10, NULL, NULL, 0, NULL) == GSPCA_EINVAL);
    CHECK(gspca_mlp_adam(NULL, 1e-3f, 0.9f, 0.999f, 1e-8f, NULL) == GSPCA_EINVAL);
}

int main(void)
{
    for (int s = -6; s <= 2; ++s)
        CHECK(gspca_status_string(s) != NULL);
    CHECK(strcmp(gspca_status_string(12345), "unknown status") == 0);
    CHECK(gspca_version() >= 100);
    fit_validation();
    quantize_validation();
    batched_validation();
    block_and_ws_validation();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host validation under sanitizers: ok\n");
    return 0;
}
