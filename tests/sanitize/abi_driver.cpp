// Host-side driver for the sanitizer build of the C-ABI layer: it calls
// every argument-validation and workspace-sizing path of include/tc.h that
// returns before any device work (so it runs without a GPU) and checks the
// status codes.  Built with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host code of tc_api.cpp by tests/test_host_sanitizers.py.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "tc.h"

static int failures = 0;
#define EXPECT(cond)                                                            \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "FAILED line %d: %s\n", __LINE__, #cond);      \
            ++failures;                                                         \
        }                                                                       \
    } while (0)

static tc_instance inst(int n, int R_f, int R_N)
{
    tc_instance I;
    std::memset(&I, 0, sizeof I);
    static double dummy[1];
    for (int l = 0; l < 3; ++l) {
        I.n[l] = n;
        I.p[l] = dummy;
        I.U[l] = dummy;
    }
    I.R_f = R_f;
    I.R_N = R_N;
    I.c = dummy;
    I.J = dummy;
    return I;
}

int main()
{
    const tc_precision precs[] = {TC_FP64, TC_FP32, TC_BF16X3, TC_BF16X6, TC_OZAKI_I8};
    // workspace sizes over many shapes, ops and precisions (host arithmetic only)
    const int ns[] = {1, 2, 5, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257, 1000, 4096, 4097,
                      8191, 65536};
    const int rfs[] = {1, 7, 64, 65, 255, 256, 257, 330, 1024};
    for (int n : ns)
        for (int R_f : rfs)
            for (tc_precision p : precs) {
                tc_instance I[3] = {inst(n, R_f, 5), inst(n, R_f, 5), inst(n / 2 + 1, R_f, 3)};
                I[1].G_saved = I[0].J;
                for (int op = 0; op < 4; ++op)
                    for (int count = 1; count <= 3; ++count) {
                        const size_t w = tc_workspace_bytes(op, I, count, p);
                        EXPECT(w != (size_t)-1);
                    }
            }
    tc_instance I = inst(64, 8, 4);
    EXPECT(tc_workspace_bytes(7, &I, 1, TC_FP64) == (size_t)-1);
    EXPECT(tc_workspace_bytes(TC_OP_TEI_GRAM, &I, 1, (tc_precision)42) == (size_t)-1);
    EXPECT(tc_workspace_bytes(TC_OP_TEI_GRAM, nullptr, 1, TC_FP64) == (size_t)-1);
    tc_instance bad = inst(0, 8, 4);
    EXPECT(tc_workspace_bytes(TC_OP_TEI_GRAM, &bad, 1, TC_FP64) == (size_t)-1);
    bad = inst(70000, 8, 4);
    EXPECT(tc_tei_gram(&bad, 1, TC_FP64, nullptr, 0, nullptr) == TC_ERR_INVALID_ARG);
    bad = inst(64, 8, 1000);
    EXPECT(tc_tei_gram(&bad, 1, TC_FP64, nullptr, 0, nullptr) == TC_ERR_INVALID_ARG);
    bad = inst(64, 8, 4);
    bad.U[1] = nullptr;
    EXPECT(tc_tei_gram(&bad, 1, TC_FP64, nullptr, 0, nullptr) == TC_ERR_INVALID_ARG);
    EXPECT(tc_tei_gram(&I, 0, TC_FP64, nullptr, 0, nullptr) == TC_ERR_INVALID_ARG);
    EXPECT(tc_tei_gram(&I, 1, TC_FP64, nullptr, 0, nullptr) == TC_ERR_WORKSPACE);
    EXPECT(tc_tei_gram_noalloc(&bad, 1, TC_FP64, nullptr) == TC_ERR_INVALID_ARG);
    tc_instance big = inst(4096, 1024, 32);
    EXPECT(tc_tei_gram_noalloc(&big, 1, TC_FP64, nullptr) == TC_ERR_WORKSPACE);
    const double *jb[1] = {nullptr};
    double *du[3] = {nullptr, nullptr, nullptr};
    EXPECT(tc_tei_gram_backward(&I, 1, jb, du, TC_FP64, nullptr, 0, nullptr) ==
           TC_ERR_INVALID_ARG);
    EXPECT(tc_autotune(&I, 1, TC_FP64, nullptr, 0, nullptr, nullptr) == TC_ERR_WORKSPACE);
    EXPECT(tc_convolve(0, 1, 1, nullptr, nullptr, nullptr, TC_FP64, nullptr, 0, nullptr) ==
           TC_ERR_INVALID_ARG);
    double t[4], c[4];
    EXPECT(tc_newton_kernel(0, 1.0, 4, -1.0, 0.5, t, c, nullptr, nullptr) == TC_ERR_INVALID_ARG);
    // tuning table round trip
    EXPECT(tc_tune_set(1024, 8, 20, TC_FP64, TC_ALGO_DIRECT) == TC_OK);
    EXPECT(tc_tune_get(1024, 8, 20, TC_FP64) == TC_ALGO_DIRECT);
    EXPECT(tc_tune_set(1024, 8, 20, TC_FP64, TC_ALGO_AUTO) == TC_OK);
    EXPECT(tc_tune_set(0, 8, 20, TC_FP64, TC_ALGO_FFT) == TC_ERR_INVALID_ARG);
    // status strings for every code and an unknown one
    for (int s = -1; s < 8; ++s)
        EXPECT(tc_status_string((tc_status)s) != nullptr);
    // other sizing calls
    int n3[3] = {64, 64, 64}, r3[3] = {8, 8, 8};
    EXPECT(tc_canonical_to_tucker_workspace_bytes(n3, 16, r3) > 0);
    EXPECT(tc_density_fit_workspace_bytes(64, 10, 8) > 0);
    EXPECT(tc_tei_cholesky_workspace_bytes(10, 8, 4, 8) > 0);
    if (failures) {
        std::fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    std::printf("abi driver: all checks passed\n");
    return 0;
}
