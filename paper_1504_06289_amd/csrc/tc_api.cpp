// C-ABI layer (include/tc.h): argument validation, workspace layout and
// kernel dispatch.  Nothing here allocates, frees or synchronises; every
// launch goes to the caller's stream, so a call can be captured in a HIP
// graph.
#include "tc.h"

#include <cmath>
#include <cstdint>
#include <vector>

#include "tc_internal.h"

namespace {

using tc::launch_adjoint_d;
using tc::launch_adjoint_gemm_f64;
using tc::launch_gram_f64;
using tc::launch_hadamard_sum;
using tc::launch_newton_kernel;
using tc::launch_toeplitz_f64;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool size_ok(int n, int R_f, int R_N)
{
    return n >= 1 && n <= TC_MAX_N && R_f >= 1 && R_f <= TC_MAX_RF && R_N >= 1 &&
           R_N <= TC_MAX_RN;
}

bool prec_ok(tc_precision prec) { return prec == TC_FP64; }

bool prec_known(tc_precision prec)
{
    return prec == TC_FP64 || prec == TC_FP32 || prec == TC_SPLIT3;
}

bool instance_ok(const tc_instance &I)
{
    if (!I.c || !I.J)
        return false;
    for (int l = 0; l < 3; ++l) {
        if (!size_ok(I.n[l], I.R_f, I.R_N) || !I.p[l] || !I.U[l])
            return false;
    }
    return true;
}

int max_n(const tc_instance &I)
{
    int m = I.n[0];
    if (I.n[1] > m)
        m = I.n[1];
    if (I.n[2] > m)
        m = I.n[2];
    return m;
}

// Workspace of one instance (bytes), forward.
size_t gram_ws(const tc_instance &I)
{
    const size_t F2 = (size_t)I.R_f * I.R_f;
    size_t w = align_up(sizeof(double) * (size_t)I.R_N * I.R_f * max_n(I));
    if (!I.G_saved)
        w += align_up(sizeof(double) * 3 * (size_t)I.R_N * F2);
    return w;
}

// Workspace of one instance (bytes), backward.
size_t gram_bwd_ws(const tc_instance &I)
{
    const size_t F2 = (size_t)I.R_f * I.R_f;
    size_t w = align_up(sizeof(double) * (size_t)I.R_N * I.R_f * max_n(I));  // W of one mode
    w += align_up(sizeof(double) * (size_t)I.R_N * F2);                      // D of one mode
    if (!I.G_saved)
        w += align_up(sizeof(double) * 3 * (size_t)I.R_N * F2);  // recomputed Grams
    return w;
}

tc_status hip_status(hipError_t e) { return e == hipSuccess ? TC_OK : TC_ERR_HIP; }

// Forward of one instance: Grams of every mode into G (3 x R_N x R_f^2),
// then the Hadamard/sum-over-k contraction into J.
tc_status run_forward(const tc_instance &I, char *ws, hipStream_t st)
{
    const size_t F2 = (size_t)I.R_f * I.R_f;
    double *W = reinterpret_cast<double *>(ws);
    double *G = I.G_saved;
    if (!G)
        G = reinterpret_cast<double *>(ws + align_up(sizeof(double) * (size_t)I.R_N * I.R_f *
                                                     max_n(I)));
    for (int l = 0; l < 3; ++l) {
        double *Gl = G + (size_t)l * I.R_N * F2;
        hipError_t e = launch_toeplitz_f64(I.p[l], I.U[l], W, I.n[l], I.R_f, I.R_N, st);
        if (e != hipSuccess)
            return TC_ERR_HIP;
        e = launch_gram_f64(I.U[l], W, Gl, I.n[l], I.R_f, I.R_N, st);
        if (e != hipSuccess)
            return TC_ERR_HIP;
    }
    return hip_status(launch_hadamard_sum(I.c, G, G + (size_t)I.R_N * F2,
                                          G + 2 * (size_t)I.R_N * F2, I.J, I.R_f, I.R_N, st));
}

}  // namespace

extern "C" {

const char *tc_status_string(tc_status s)
{
    switch (s) {
    case TC_OK:
        return "TC_OK";
    case TC_ERR_INVALID_ARG:
        return "TC_ERR_INVALID_ARG: invalid argument";
    case TC_ERR_WORKSPACE:
        return "TC_ERR_WORKSPACE: workspace missing or too small";
    case TC_ERR_UNSUPPORTED:
        return "TC_ERR_UNSUPPORTED: precision or size not supported";
    case TC_ERR_HIP:
        return "TC_ERR_HIP: HIP launch or runtime error";
    }
    return "unknown tc_status";
}

int tc_version(void) { return 100; }

size_t tc_workspace_bytes(int op, const tc_instance *inst, int count, tc_precision prec)
{
    if (!inst || count < 1 || !prec_known(prec))
        return (size_t)-1;
    if (op == TC_OP_CONVOLVE) {
        if (!size_ok(inst[0].n[0], inst[0].R_f, inst[0].R_N))
            return (size_t)-1;
        return 0;
    }
    size_t w = 0;
    for (int i = 0; i < count; ++i) {
        const tc_instance &I = inst[i];
        for (int l = 0; l < 3; ++l)
            if (!size_ok(I.n[l], I.R_f, I.R_N))
                return (size_t)-1;
        size_t wi;
        if (op == TC_OP_TEI_GRAM)
            wi = gram_ws(I);
        else if (op == TC_OP_TEI_GRAM_BACKWARD)
            wi = gram_bwd_ws(I);
        else
            return (size_t)-1;
        if (wi > w)
            w = wi;
    }
    return w;
}

tc_status tc_newton_kernel(int n, double h, int R_N, double u0, double hu, double *t_host,
                           double *c_host, double *p_dev, void *stream)
{
    if (n < 1 || n > TC_MAX_N || R_N < 1 || R_N > TC_MAX_RN || !p_dev)
        return TC_ERR_INVALID_ARG;
    if (!(std::isfinite(h) && h > 0.0 && std::isfinite(u0) && std::isfinite(hu) && hu > 0.0))
        return TC_ERR_INVALID_ARG;
    // nodes t_k = exp(u0 + k hu) (sinc rule in u = log t); weights a_k = (2/sqrt(pi)) hu t_k
    std::vector<double> t(R_N);
    for (int k = 0; k < R_N; ++k) {
        t[k] = std::exp(u0 + (double)k * hu);
        if (!std::isfinite(t[k]) || t[k] <= 0.0)
            return TC_ERR_INVALID_ARG;
    }
    const double two_over_sqrtpi = 1.1283791670955125739;
    hipError_t e = launch_newton_kernel(t.data(), R_N, n, h, p_dev, (hipStream_t)stream);
    if (e != hipSuccess)
        return TC_ERR_HIP;
    for (int k = 0; k < R_N; ++k) {
        if (t_host)
            t_host[k] = t[k];
        if (c_host)
            c_host[k] = two_over_sqrtpi * hu * t[k] * (h * h * h);
    }
    return TC_OK;
}

tc_status tc_convolve(int n, int R_f, int R_N, const double *p_dev, const double *U_dev,
                      double *W_dev, tc_precision prec, void *ws, size_t ws_bytes,
                      void *stream)
{
    (void)ws;
    (void)ws_bytes;
    if (!size_ok(n, R_f, R_N) || !p_dev || !U_dev || !W_dev)
        return TC_ERR_INVALID_ARG;
    if (!prec_known(prec))
        return TC_ERR_INVALID_ARG;
    if (!prec_ok(prec))
        return TC_ERR_UNSUPPORTED;
    return hip_status(launch_toeplitz_f64(p_dev, U_dev, W_dev, n, R_f, R_N, (hipStream_t)stream));
}

tc_status tc_tei_gram(const tc_instance *inst, int count, tc_precision prec, void *ws,
                      size_t ws_bytes, void *stream)
{
    if (!inst || count < 1 || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!instance_ok(inst[i]))
            return TC_ERR_INVALID_ARG;
    if (!prec_ok(prec))
        return TC_ERR_UNSUPPORTED;
    const size_t need = tc_workspace_bytes(TC_OP_TEI_GRAM, inst, count, prec);
    if (need > 0 && (!ws || ws_bytes < need))
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
        tc_status s = run_forward(inst[i], (char *)ws, st);
        if (s != TC_OK)
            return s;
    }
    return TC_OK;
}

tc_status tc_tei_gram_backward(const tc_instance *inst, int count, const double *const *Jbar,
                               double *const *dU, tc_precision prec, void *ws, size_t ws_bytes,
                               void *stream)
{
    if (!inst || count < 1 || !Jbar || !dU || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        const tc_instance &I = inst[i];
        if (!I.c || !Jbar[i])
            return TC_ERR_INVALID_ARG;
        for (int l = 0; l < 3; ++l)
            if (!size_ok(I.n[l], I.R_f, I.R_N) || !I.p[l] || !I.U[l] || !dU[3 * i + l])
                return TC_ERR_INVALID_ARG;
    }
    if (!prec_ok(prec))
        return TC_ERR_UNSUPPORTED;
    const size_t need = tc_workspace_bytes(TC_OP_TEI_GRAM_BACKWARD, inst, count, prec);
    if (!ws || ws_bytes < need)
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
        const tc_instance &I = inst[i];
        const size_t F2 = (size_t)I.R_f * I.R_f;
        char *base = (char *)ws;
        double *W = reinterpret_cast<double *>(base);
        base += align_up(sizeof(double) * (size_t)I.R_N * I.R_f * max_n(I));
        double *D = reinterpret_cast<double *>(base);
        base += align_up(sizeof(double) * (size_t)I.R_N * F2);
        double *G = I.G_saved;
        if (!G) {
            G = reinterpret_cast<double *>(base);
            for (int l = 0; l < 3; ++l) {
                if (launch_toeplitz_f64(I.p[l], I.U[l], W, I.n[l], I.R_f, I.R_N, st) !=
                    hipSuccess)
                    return TC_ERR_HIP;
                if (launch_gram_f64(I.U[l], W, G + (size_t)l * I.R_N * F2, I.n[l], I.R_f,
                                    I.R_N, st) != hipSuccess)
                    return TC_ERR_HIP;
            }
        }
        for (int l = 0; l < 3; ++l) {
            const double *Ga = G + (size_t)((l + 1) % 3) * I.R_N * F2;
            const double *Gb = G + (size_t)((l + 2) % 3) * I.R_N * F2;
            if (launch_adjoint_d(I.c, Jbar[i], Ga, Gb, D, I.R_f, I.R_N, st) != hipSuccess)
                return TC_ERR_HIP;
            if (launch_toeplitz_f64(I.p[l], I.U[l], W, I.n[l], I.R_f, I.R_N, st) != hipSuccess)
                return TC_ERR_HIP;
            if (launch_adjoint_gemm_f64(D, W, dU[3 * i + l], I.n[l], I.R_f, I.R_N, 2.0, st) !=
                hipSuccess)
                return TC_ERR_HIP;
        }
    }
    return TC_OK;
}

}  // extern "C"
