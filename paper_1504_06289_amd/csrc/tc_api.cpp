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

using namespace tc;

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool size_ok(int n, int R_f, int R_N)
{
    return n >= 1 && n <= TC_MAX_N && R_f >= 1 && R_f <= TC_MAX_RF && R_N >= 1 &&
           R_N <= TC_MAX_RN;
}

bool prec_known(tc_precision prec)
{
    return prec == TC_FP64 || prec == TC_FP32 || prec == TC_OZAKI_I8;
}

bool prec_supported(tc_precision prec) { return prec == TC_FP64 || prec == TC_OZAKI_I8; }

bool instance_ok(const tc_instance &I)
{
    if (!I.c || !I.J)
        return false;
    for (int l = 0; l < 3; ++l)
        if (!size_ok(I.n[l], I.R_f, I.R_N) || !I.p[l] || !I.U[l])
            return false;
    return true;
}

// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures, so the same code computes tc_workspace_bytes and the layout.
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T> T *take(size_t count)
    {
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += align_up(sizeof(T) * count);
        return p;
    }
};

// Scratch of one mode's Toeplitz product (slices of U and of the kernel).
struct ToeplitzScratch {
    int8_t *US = nullptr;
    int *EU = nullptr;
    int8_t *PS = nullptr;
    int *EP = nullptr;
};

ToeplitzScratch carve_toeplitz(Carver &c, tc_precision prec, int n, int R_f, int R_N)
{
    ToeplitzScratch s;
    if (prec == TC_OZAKI_I8) {
        const OzakiLayout L = ozaki_layout(n, R_f, R_N);
        s.US = c.take<int8_t>(4 * (size_t)L.uplane);
        s.EU = c.take<int>(L.R_f_pad);
        s.PS = c.take<int8_t>(4 * (size_t)L.pplane);
        s.EP = c.take<int>(R_N);
    }
    return s;
}

// Scratch of one mode's Gram on top of the Toeplitz scratch (slices of W).
struct GramScratch {
    int8_t *WS = nullptr;
    int *EW = nullptr;
};

GramScratch carve_gram(Carver &c, tc_precision prec, int n, int R_f, int R_N)
{
    GramScratch s;
    if (prec == TC_OZAKI_I8) {
        const OzakiLayout L = ozaki_layout(n, R_f, R_N);
        s.WS = c.take<int8_t>(4 * (size_t)L.wplane);
        s.EW = c.take<int>((size_t)R_N * L.R_f_pad);
    }
    return s;
}

// W = T_k U for all k of one mode.  For the int8 path the slices of U are
// left in `ts` for a following Gram.
hipError_t mode_toeplitz(tc_precision prec, int n, int R_f, int R_N, const double *p,
                         const double *U, double *W, const ToeplitzScratch &ts, hipStream_t st)
{
    if (prec == TC_FP64)
        return launch_toeplitz_f64(p, U, W, n, R_f, R_N, st);
    const OzakiLayout L = ozaki_layout(n, R_f, R_N);
    hipError_t e =
        launch_split_rows(U, 1, R_f, n, L.R_f_pad, L.n_pad, L.uplane, ts.US, ts.EU, st);
    if (e != hipSuccess)
        return e;
    e = launch_split_kernel_vectors(p, n, R_N, L, ts.PS, ts.EP, st);
    if (e != hipSuccess)
        return e;
    return launch_toeplitz_i8(ts.US, ts.EU, ts.PS, ts.EP, L, W, n, R_f, R_N, st);
}

// G_k = U^T W_k for all k of one mode (W from mode_toeplitz with the same ts).
hipError_t mode_gram(tc_precision prec, int n, int R_f, int R_N, const double *U,
                     const double *W, double *G, const ToeplitzScratch &ts,
                     const GramScratch &gs, hipStream_t st)
{
    if (prec == TC_FP64)
        return launch_gram_f64(U, W, G, n, R_f, R_N, st);
    const OzakiLayout L = ozaki_layout(n, R_f, R_N);
    hipError_t e =
        launch_split_rows(W, R_N, R_f, n, L.R_f_pad, L.n_pad, L.wplane, gs.WS, gs.EW, st);
    if (e != hipSuccess)
        return e;
    return launch_gram_i8(ts.US, ts.EU, gs.WS, gs.EW, L, G, R_f, R_N, st);
}

int max_n(const tc_instance &I)
{
    int m = I.n[0];
    for (int l = 1; l < 3; ++l)
        if (I.n[l] > m)
            m = I.n[l];
    return m;
}

// Workspace plan of one instance.  Layout: [W][G?][D?][per-mode scratch];
// the per-mode scratch is sized for the largest mode and reused.
struct InstancePlan {
    double *W, *G, *D;
    ToeplitzScratch ts[3];
    GramScratch gs[3];
    size_t bytes;
};

InstancePlan plan_instance(void *ws, const tc_instance &I, tc_precision prec, bool backward)
{
    InstancePlan P{};
    Carver c(ws);
    const size_t F2 = (size_t)I.R_f * I.R_f;
    P.W = c.take<double>((size_t)I.R_N * I.R_f * max_n(I));
    P.G = I.G_saved ? I.G_saved : c.take<double>(3 * (size_t)I.R_N * F2);
    P.D = backward ? c.take<double>((size_t)I.R_N * F2) : nullptr;
    const size_t scratch0 = c.used;
    size_t scratch_max = 0;
    for (int l = 0; l < 3; ++l) {
        c.used = scratch0;
        P.ts[l] = carve_toeplitz(c, prec, I.n[l], I.R_f, I.R_N);
        P.gs[l] = carve_gram(c, prec, I.n[l], I.R_f, I.R_N);
        if (c.used - scratch0 > scratch_max)
            scratch_max = c.used - scratch0;
    }
    P.bytes = scratch0 + scratch_max;
    return P;
}

size_t convolve_ws(int n, int R_f, int R_N, tc_precision prec)
{
    Carver c(nullptr);
    carve_toeplitz(c, prec, n, R_f, R_N);
    return c.used;
}

tc_status forward_instance(const tc_instance &I, tc_precision prec, void *ws, hipStream_t st)
{
    const InstancePlan P = plan_instance(ws, I, prec, false);
    const size_t F2 = (size_t)I.R_f * I.R_f;
    for (int l = 0; l < 3; ++l) {
        double *Gl = P.G + (size_t)l * I.R_N * F2;
        if (mode_toeplitz(prec, I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], P.W, P.ts[l], st) !=
            hipSuccess)
            return TC_ERR_HIP;
        if (mode_gram(prec, I.n[l], I.R_f, I.R_N, I.U[l], P.W, Gl, P.ts[l], P.gs[l], st) !=
            hipSuccess)
            return TC_ERR_HIP;
    }
    if (launch_hadamard_sum(I.c, P.G, P.G + (size_t)I.R_N * F2, P.G + 2 * (size_t)I.R_N * F2,
                            I.J, I.R_f, I.R_N, st) != hipSuccess)
        return TC_ERR_HIP;
    return TC_OK;
}

tc_status backward_instance(const tc_instance &I, const double *Jbar, double *const *dU,
                            tc_precision prec, void *ws, hipStream_t st)
{
    const InstancePlan P = plan_instance(ws, I, prec, true);
    const size_t F2 = (size_t)I.R_f * I.R_f;
    if (!I.G_saved) {
        for (int l = 0; l < 3; ++l) {
            if (mode_toeplitz(prec, I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], P.W, P.ts[l], st) !=
                hipSuccess)
                return TC_ERR_HIP;
            if (mode_gram(prec, I.n[l], I.R_f, I.R_N, I.U[l], P.W, P.G + (size_t)l * I.R_N * F2,
                          P.ts[l], P.gs[l], st) != hipSuccess)
                return TC_ERR_HIP;
        }
    }
    for (int l = 0; l < 3; ++l) {
        const double *Ga = P.G + (size_t)((l + 1) % 3) * I.R_N * F2;
        const double *Gb = P.G + (size_t)((l + 2) % 3) * I.R_N * F2;
        if (launch_adjoint_d(I.c, Jbar, Ga, Gb, P.D, I.R_f, I.R_N, st) != hipSuccess)
            return TC_ERR_HIP;
        if (mode_toeplitz(prec, I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], P.W, P.ts[l], st) !=
            hipSuccess)
            return TC_ERR_HIP;
        if (launch_adjoint_gemm_f64(P.D, P.W, dU[l], I.n[l], I.R_f, I.R_N, 2.0, st) !=
            hipSuccess)
            return TC_ERR_HIP;
    }
    return TC_OK;
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

int tc_version(void) { return 200; }

size_t tc_workspace_bytes(int op, const tc_instance *inst, int count, tc_precision prec)
{
    if (!inst || count < 1 || !prec_known(prec))
        return (size_t)-1;
    if (op == TC_OP_CONVOLVE) {
        if (!size_ok(inst[0].n[0], inst[0].R_f, inst[0].R_N))
            return (size_t)-1;
        return convolve_ws(inst[0].n[0], inst[0].R_f, inst[0].R_N, prec);
    }
    if (op != TC_OP_TEI_GRAM && op != TC_OP_TEI_GRAM_BACKWARD)
        return (size_t)-1;
    size_t w = 0;
    for (int i = 0; i < count; ++i) {
        for (int l = 0; l < 3; ++l)
            if (!size_ok(inst[i].n[l], inst[i].R_f, inst[i].R_N))
                return (size_t)-1;
        const size_t wi =
            plan_instance(nullptr, inst[i], prec, op == TC_OP_TEI_GRAM_BACKWARD).bytes;
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
    if (launch_newton_kernel(t.data(), R_N, n, h, p_dev, (hipStream_t)stream) != hipSuccess)
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
                      double *W_dev, tc_precision prec, void *ws, size_t ws_bytes, void *stream)
{
    if (!size_ok(n, R_f, R_N) || !p_dev || !U_dev || !W_dev || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    if (!prec_supported(prec))
        return TC_ERR_UNSUPPORTED;
    const size_t need = convolve_ws(n, R_f, R_N, prec);
    if (need > 0 && (!ws || ws_bytes < need))
        return TC_ERR_WORKSPACE;
    Carver c(ws);
    const ToeplitzScratch ts = carve_toeplitz(c, prec, n, R_f, R_N);
    if (mode_toeplitz(prec, n, R_f, R_N, p_dev, U_dev, W_dev, ts, (hipStream_t)stream) !=
        hipSuccess)
        return TC_ERR_HIP;
    return TC_OK;
}

tc_status tc_tei_gram(const tc_instance *inst, int count, tc_precision prec, void *ws,
                      size_t ws_bytes, void *stream)
{
    if (!inst || count < 1 || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!instance_ok(inst[i]))
            return TC_ERR_INVALID_ARG;
    if (!prec_supported(prec))
        return TC_ERR_UNSUPPORTED;
    const size_t need = tc_workspace_bytes(TC_OP_TEI_GRAM, inst, count, prec);
    if (need > 0 && (!ws || ws_bytes < need))
        return TC_ERR_WORKSPACE;
    for (int i = 0; i < count; ++i) {
        const tc_status s = forward_instance(inst[i], prec, ws, (hipStream_t)stream);
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
    if (!prec_supported(prec))
        return TC_ERR_UNSUPPORTED;
    const size_t need = tc_workspace_bytes(TC_OP_TEI_GRAM_BACKWARD, inst, count, prec);
    if (!ws || ws_bytes < need)
        return TC_ERR_WORKSPACE;
    for (int i = 0; i < count; ++i) {
        const tc_status s =
            backward_instance(inst[i], Jbar[i], dU + 3 * i, prec, ws, (hipStream_t)stream);
        if (s != TC_OK)
            return s;
    }
    return TC_OK;
}

}  // extern "C"
