// C-ABI layer (include/tc.h): argument validation, workspace layout,
// algorithm choice (tuning table) and kernel dispatch.  Nothing here
// allocates or frees device memory.  Only the calls whose comment in tc.h
// says so synchronise (autotuning, the pivoted Cholesky drivers, the lattice
// energy, the epsilon-truncated canonical-to-Tucker transform and the kernel
// timing read-out); every other call only enqueues work on the caller's
// stream, so it can be captured in a HIP graph.
#include "tc.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <algorithm>
#include <initializer_list>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
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
    return prec == TC_FP64 || prec == TC_FP32 || prec == TC_OZAKI_I8 || prec == TC_BF16X3 ||
           prec == TC_BF16X6;
}

// Precisions whose contractions read binary64 operands scaled per row by 2^-e.
bool row_scaled(tc_precision prec)
{
    return prec == TC_FP32 || prec == TC_BF16X3 || prec == TC_BF16X6;
}

int bf16_pieces(tc_precision prec) { return prec == TC_BF16X6 ? 3 : 2; }

bool prec_supported(tc_precision prec) { return prec_known(prec); }

bool instance_ok(const tc_instance &I)
{
    if (!I.c || !I.J)
        return false;
    for (int l = 0; l < 3; ++l)
        if (!size_ok(I.n[l], I.R_f, I.R_N) || !I.p[l] || !I.U[l])
            return false;
    return true;
}

// ---------------------------------------------------------------------------
// tuning table
// ---------------------------------------------------------------------------
using TuneKey = std::tuple<int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

// Built-in rule: the FFT route once the grid is long enough for the n^2
// Toeplitz product to dominate (measured crossover on MI355X, refined by
// tc_autotune), the direct matrix-core product otherwise.
constexpr int kFftMinN = 256;

// an FFT route exists for n cells (LDS-resident or four-step)
bool fft_any(int n) { return fft_supported(n) || fft_large_supported(n); }

tc_algorithm resolve(int n, int R_f, int R_N, tc_precision prec)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(TuneKey(n, R_f, R_N, (int)prec));
        if (it != g_tune.end()) {
            const tc_algorithm a = (tc_algorithm)it->second;
            if (a != TC_ALGO_FFT || fft_any(n))
                return a;
        }
    }
    return (fft_supported(n) && n >= kFftMinN) || fft_large_supported(n) ? TC_ALGO_FFT
                                                                          : TC_ALGO_DIRECT;
}

// the int8 route whose convolution writes W's int8 slices directly (and
// treats narrow and smooth kernel terms apart): the LDS-resident FFT lengths
bool i8_fused_fft(tc_precision prec, tc_algorithm algo, int n)
{
    return prec == TC_OZAKI_I8 && algo == TC_ALGO_FFT && fft_supported(n);
}

// Batch routes: one entry per batch signature (precision, count and every
// instance's sizes), set by tc_batch_tune_set or tc_autotune.
std::map<uint64_t, int> g_batch_tune;

uint64_t batch_signature(const tc_instance *inst, int count, tc_precision prec)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    auto mix = [&](long v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (uint64_t)((v >> (8 * b)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    mix((long)prec);
    mix(count);
    for (int i = 0; i < count; ++i) {
        for (int l = 0; l < 3; ++l)
            mix(inst[i].n[l]);
        mix(inst[i].R_f);
        mix(inst[i].R_N);
        mix(inst[i].G_saved != nullptr);
    }
    return h;
}

// Built-in: fork-join.  On the 64-instance workload (int8) it measured
// 31.7 ms against 33.3 ms for the work queue: the queue's Grams start only
// once every instance has its slices, so they no longer overlap the other
// instances' convolutions; tc_autotune measures both per batch.
constexpr int kBatchDefaultI8 = TC_BATCH_FORK_JOIN;

int batch_route(const tc_instance *inst, int count, tc_precision prec)
{
    if (prec != TC_OZAKI_I8 || count < 2)
        return TC_BATCH_FORK_JOIN;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_batch_tune.find(batch_signature(inst, count, prec));
    return it != g_batch_tune.end() ? it->second : kBatchDefaultI8;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
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

// Scratch of one mode (every buffer any algorithm/precision may need).
struct ModeScratch {
    int8_t *US = nullptr;  // int8 slices of U
    int *EU = nullptr;
    int8_t *PS = nullptr;  // int8 slices of the kernel vectors (direct route)
    int *EP = nullptr;
    int8_t *WS = nullptr;  // int8 slices of W
    int *EW = nullptr;
    double2 *twN = nullptr;    // FFT twiddles
    double2 *Uspec = nullptr;  // half spectra of U rows
    double2 *Cspec = nullptr;  // half spectra of the kernel embeddings
    // int8 FFT route: term classes and the low-rank Grams of smooth terms
    int *cls = nullptr;        // class of each kernel term (launch_term_class)
    double *Q = nullptr;       // [kPolyRank][n] orthonormal polynomials
    double *X = nullptr;       // [R_f][kPolyRank] projections of U's rows
    double *Xp = nullptr;      // partial sums of X over cell ranges
    double2 *Qspec = nullptr;  // half spectra of Q's rows
    double *Sp = nullptr;      // partial sums of S over frequency ranges
    double *S = nullptr;       // [R_N][kPolyRank][kPolyRank] = Q T_k Q^T
    // FFT route beyond 4096 cells (four-step transforms)
    double2 *Zl = nullptr;     // spectra of the pairs of U rows
    double2 *Cl = nullptr;     // spectra of the kernel embeddings
    double2 *Tl = nullptr;     // inverse scratch
    int *El = nullptr;         // row exponents of U (the pairs' scales)
    double *tail = nullptr;    // later K parts of the int8 Gram's split tail items
};

// large_fft: reserve the scratch of the four-step FFT route (n > 4096)
ModeScratch carve_mode(Carver &c, tc_precision prec, int n, int R_f, int R_N, bool gram,
                       bool large_fft = true)
{
    ModeScratch s;
    if (prec == TC_OZAKI_I8) {
        const OzakiLayout L = ozaki_layout(n, R_f, R_N);
        s.US = c.take<int8_t>(4 * (size_t)L.uplane);
        s.EU = c.take<int>(L.R_f_pad);
        s.PS = c.take<int8_t>(4 * (size_t)L.pplane);
        s.EP = c.take<int>(R_N);
        if (gram) {
            s.WS = c.take<int8_t>(4 * (size_t)L.wplane);
            s.EW = c.take<int>((size_t)R_N * L.R_f_pad);
            if (gram_i8_wide(R_f, L.R_f_pad))
                s.tail = c.take<double>(kOzakiTailBytes / sizeof(double));
        }
    }
    if (row_scaled(prec)) {
        s.EU = c.take<int>(R_f);
        s.EP = c.take<int>(R_N);
        if (gram)
            s.EW = c.take<int>((size_t)R_N * R_f);
    }
    if (fft_large_supported(n) && large_fft) {
        const LargeFftLayout L = fft_large_layout(n, R_f, R_N);
        s.twN = c.take<double2>(L.N);
        s.Zl = c.take<double2>(L.z_entries);
        s.Cl = c.take<double2>(L.c_entries);
        s.Tl = c.take<double2>(L.t_entries);
        s.El = c.take<int>(R_f);
    }
    if (fft_supported(n)) {
        const int N = fft_length(n);
        s.twN = c.take<double2>(N);
        s.Uspec = c.take<double2>((size_t)R_f * (N / 2 + 1));
        s.Cspec = c.take<double2>((size_t)R_N * (N / 2 + 1));
        if (prec == TC_OZAKI_I8 && gram) {
            s.cls = c.take<int>(R_N);
            if (smooth_terms_supported(n)) {
                s.Q = c.take<double>((size_t)kPolyRank * n);
                s.X = c.take<double>((size_t)R_f * kPolyRank);
                s.Xp = c.take<double>((size_t)kProjectSplit * R_f * kPolyRank);
                s.Qspec = c.take<double2>((size_t)kPolyRank * (N / 2 + 1));
                s.Sp = c.take<double>((size_t)R_N * kSpectralSplit * kPolyRank * kPolyRank);
                s.S = c.take<double>((size_t)R_N * kPolyRank * kPolyRank);
            }
        }
    }
    return s;
}

// ---------------------------------------------------------------------------
// kernel timing (tc_profile_*): when enabled, every launch is bracketed by a
// pair of HIP events recorded on the launch stream; tc_profile_read
// synchronises the recorded events and returns per-kernel totals.
// ---------------------------------------------------------------------------
struct ProfRecord {
    const char *name;
    hipEvent_t e0, e1;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event()
{
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess)
        return nullptr;
    return e;
}

struct ProfScope {
    const char *name;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    ProfScope(const char *n, hipStream_t s) : name(n), st(s)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on)
            return;
        e0 = prof_event();
        if (e0 && hipEventRecord(e0, st) != hipSuccess) {
            g_prof_pool.push_back(e0);
            e0 = nullptr;
        }
    }
    void end()
    {
        if (!e0)
            return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        hipEvent_t e1 = prof_event();
        if (e1 && hipEventRecord(e1, st) == hipSuccess) {
            g_prof_pending.push_back({name, e0, e1});
        } else {
            g_prof_pool.push_back(e0);
            if (e1)
                g_prof_pool.push_back(e1);
        }
        e0 = nullptr;
    }
};

// launch `expr` (returns hipError_t) under the kernel name `name` on stream st;
// with TC_DEBUG_SYNC set, synchronise st after it and report a failure
#define TRYK(name, expr)                                                                       \
    do {                                                                                       \
        ProfScope ps_(name, st);                                                               \
        if ((expr) != hipSuccess)                                                              \
            return TC_ERR_HIP;                                                                 \
        ps_.end();                                                                             \
        if (debug_sync_on() && !debug_sync_check(name, st))                                    \
            return TC_ERR_HIP;                                                                 \
    } while (0)

// With TC_CHECK_FINITE set: TC_ERR_INVALID_ARG when any of the arrays holds a
// NaN or Inf (checked on the device before any other work; synchronises st).
tc_status finite_inputs(std::initializer_list<FiniteSpan> spans, hipStream_t st)
{
    if (!check_finite_on())
        return TC_OK;
    const std::vector<FiniteSpan> v(spans);
    const int r = scan_nonfinite(v.data(), (int)v.size(), st);
    return r < 0 ? TC_ERR_HIP : r > 0 ? TC_ERR_INVALID_ARG : TC_OK;
}

tc_status finite_instance(const tc_instance &I, hipStream_t st)
{
    tc_status s = finite_inputs({{I.c, I.R_N}}, st);
    for (int l = 0; l < 3 && s == TC_OK; ++l)
        s = finite_inputs({{I.p[l], (long)I.R_N * (2L * I.n[l] - 1)},
                           {I.U[l], (long)I.R_f * I.n[l]}}, st);
    return s;
}

// spectra of U's rows and of the kernel embeddings (FFT route)
tc_status fft_spectra(int n, int R_f, int R_N, const double *p, const double *U,
                      const ModeScratch &s, hipStream_t st)
{
    const int N = fft_length(n);
    TRYK("fft_twiddles", launch_fft_twiddles(s.twN, N, st));
    TRYK("rfft_rows", launch_rfft_rows(U, R_f, n, N, s.twN, s.Uspec, st));
    TRYK("rfft_kernel_embed", launch_rfft_kernel_embed(p, n, R_N, N, s.twN, s.Cspec, st));
    return TC_OK;
}

// W = T_k U (binary64 output) for all k of one mode.
tc_status mode_W(tc_precision prec, tc_algorithm algo, int n, int R_f, int R_N, const double *p,
                 const double *U, double *W, const ModeScratch &s, hipStream_t st)
{
    if (algo == TC_ALGO_FFT && fft_large_supported(n)) {
        if (!s.Zl)
            return TC_ERR_WORKSPACE;
        TRYK("fft_twiddles", launch_fft_twiddles(s.twN, fft_length(n), st));
        TRYK("row_exponents", launch_row_exponents(U, R_f, n, s.El, st));
        TRYK("fft_large",
             launch_fft_large_W(p, U, s.El, n, R_f, R_N, s.twN, s.Zl, s.Cl, s.Tl, W, st));
        return TC_OK;
    }
    if (algo == TC_ALGO_FFT) {
        const tc_status r = fft_spectra(n, R_f, R_N, p, U, s, st);
        if (r != TC_OK)
            return r;
        TRYK("fft_conv", launch_fft_conv(s.Uspec, s.Cspec, n, fft_length(n), R_f, R_N, s.twN, W,
                                         nullptr, nullptr, 0, 0, 0, nullptr, nullptr, nullptr,
                                         st));
        return TC_OK;
    }
    if (prec == TC_FP64) {
        TRYK("toeplitz_f64", launch_toeplitz_f64(p, U, W, n, R_f, R_N, st));
        return TC_OK;
    }
    if (row_scaled(prec)) {
        TRYK("row_exponents", launch_row_exponents(U, R_f, n, s.EU, st));
        TRYK("row_exponents", launch_row_exponents(p, R_N, 2 * n - 1, s.EP, st));
        if (prec == TC_FP32)
            TRYK("toeplitz_f32", launch_toeplitz_f32(p, s.EP, U, s.EU, W, n, R_f, R_N, st));
        else
            TRYK("toeplitz_bf16", launch_toeplitz_bf16(p, s.EP, U, s.EU, W, n, R_f, R_N,
                                                       bf16_pieces(prec), st));
        return TC_OK;
    }
    const OzakiLayout L = ozaki_layout(n, R_f, R_N);
    TRYK("split_rows", launch_split_rows(U, 1, R_f, n, L.R_f_pad, L.n_pad, L.uplane, s.US, s.EU, st));
    TRYK("split_kernel_vectors", launch_split_kernel_vectors(p, n, R_N, L, s.PS, s.EP, st));
    TRYK("toeplitz_i8", launch_toeplitz_i8(s.US, s.EU, s.PS, s.EP, L, W, n, R_f, R_N, st));
    return TC_OK;
}

// int8 FFT route, the part of a mode that depends only on the kernel vectors
// (and n): twiddles, kernel spectra, term classes and, for smooth terms, the
// polynomial basis Q, its spectra and S_k = Q T_k Q^T.
tc_status int8fft_kernel_part(int n, int R_N, const double *p, const ModeScratch &s,
                              hipStream_t st)
{
    const int N = fft_length(n);
    TRYK("fft_twiddles", launch_fft_twiddles(s.twN, N, st));
    TRYK("rfft_kernel_embed", launch_rfft_kernel_embed(p, n, R_N, N, s.twN, s.Cspec, st));
    TRYK("term_class", launch_term_class(p, n, R_N, s.cls, st));
    if (smooth_terms_supported(n)) {
        TRYK("poly_rows", launch_poly_rows(n, s.Q, st));
        TRYK("rfft_rows", launch_rfft_rows(s.Q, kPolyRank, n, N, s.twN, s.Qspec, st));
        TRYK("spectral_gram",
             launch_spectral_gram(s.Qspec, s.Cspec, N, R_N, s.cls, s.Sp, s.S, st));
    }
    return TC_OK;
}

// The part that depends on U, in the mode's scratch s, reading the kernel
// part's results from kp: s itself, or the scratch of an earlier mode with the
// same kernel vectors and n whose kernel part ran earlier on the same stream.
// (Running the small smooth-term kernels before the convolution instead of
// after the int8 Gram measured 0.1 ms slower per step with concurrent modes.)
// The part of a mode that does not need the kernel part: twiddles (when
// borrowing), the spectra of U and its int8 slices.
tc_status int8fft_u_prep(int n, int R_f, int R_N, const double *U, const ModeScratch &s,
                         bool borrowing, hipStream_t st)
{
    const int N = fft_length(n);
    const OzakiLayout L = ozaki_layout(n, R_f, R_N);
    if (borrowing)
        TRYK("fft_twiddles", launch_fft_twiddles(s.twN, N, st));
    TRYK("rfft_rows", launch_rfft_rows(U, R_f, n, N, s.twN, s.Uspec, st));
    TRYK("split_rows", launch_split_rows(U, 1, R_f, n, L.R_f_pad, L.n_pad, L.uplane, s.US, s.EU, st));
    return TC_OK;
}

// with_gram == false leaves the int8 Gram of the listed terms to the caller
// (the work queue of a batch); the smooth terms' Grams are still formed here
tc_status int8fft_u_main(int n, int R_f, int R_N, const double *p, const double *U, double *G,
                         const ModeScratch &s, const ModeScratch &kp, bool mirror,
                         hipStream_t st, bool with_gram = true)
{
    const int N = fft_length(n);
    const OzakiLayout L = ozaki_layout(n, R_f, R_N);
    TRYK("fft_conv_split", launch_fft_conv(s.Uspec, kp.Cspec, n, N, R_f, R_N, s.twN, nullptr,
                                           s.WS, s.EW, L.R_f_pad, L.n_pad, L.wplane, U, p,
                                           kp.cls, st));
    if (with_gram)
        TRYK("gram_i8",
             launch_gram_i8(s.US, s.EU, s.WS, s.EW, L, G, R_f, R_N, kp.cls, mirror, s.tail, st));
    if (smooth_terms_supported(n)) {
        // smooth terms: G_k = X S_k X^T with X = U Q^T
        TRYK("poly_project", launch_poly_project(U, n, R_f, kp.Q, s.Xp, s.X, st));
        TRYK("lowrank_gram",
             launch_lowrank_gram(s.X, kp.S, kp.cls, G, R_f, R_N, mirror, st));
    }
    return TC_OK;
}

tc_status int8fft_u_part(int n, int R_f, int R_N, const double *p, const double *U, double *G,
                         const ModeScratch &s, const ModeScratch &kp, bool mirror,
                         hipStream_t st)
{
    const tc_status r = int8fft_u_prep(n, R_f, R_N, U, s, &kp != &s, st);
    if (r != TC_OK)
        return r;
    return int8fft_u_main(n, R_f, R_N, p, U, G, s, kp, mirror, st);
}

// G_k = U^T T_k U for all k of one mode (W is scratch).
tc_status mode_grams(tc_precision prec, tc_algorithm algo, int n, int R_f, int R_N,
                     const double *p, const double *U, double *W, double *G,
                     const ModeScratch &s, hipStream_t st, bool mirror = true,
                     bool with_gram = true)
{
    if (prec == TC_FP64) {
        const tc_status r = mode_W(prec, algo, n, R_f, R_N, p, U, W, s, st);
        if (r != TC_OK)
            return r;
        TRYK("gram_f64", launch_gram_f64(U, W, G, n, R_f, R_N, mirror, st));
        return TC_OK;
    }
    if (row_scaled(prec)) {
        const tc_status r = mode_W(prec, algo, n, R_f, R_N, p, U, W, s, st);
        if (r != TC_OK)
            return r;
        TRYK("row_exponents", launch_row_exponents(U, R_f, n, s.EU, st));
        TRYK("row_exponents", launch_row_exponents(W, (long)R_N * R_f, n, s.EW, st));
        if (prec == TC_FP32)
            TRYK("gram_f32", launch_gram_f32(U, s.EU, W, s.EW, G, n, R_f, R_N, mirror, st));
        else
            TRYK("gram_bf16", launch_gram_bf16(U, s.EU, W, s.EW, G, n, R_f, R_N,
                                               bf16_pieces(prec), mirror, st));
        return TC_OK;
    }
    if (i8_fused_fft(prec, algo, n)) {
        const tc_status r = int8fft_kernel_part(n, R_N, p, s, st);
        if (r != TC_OK)
            return r;
        return int8fft_u_part(n, R_f, R_N, p, U, G, s, s, mirror, st);
    }
    const OzakiLayout L = ozaki_layout(n, R_f, R_N);
    const tc_status r = mode_W(prec, algo, n, R_f, R_N, p, U, W, s, st);
    if (r != TC_OK)
        return r;
    // the direct route split U's rows for its own product; the four-step FFT
    // route (n > 4096) did not
    if (algo == TC_ALGO_FFT)
        TRYK("split_rows", launch_split_rows(U, 1, R_f, n, L.R_f_pad, L.n_pad, L.uplane, s.US, s.EU, st));
    TRYK("split_rows_W", launch_split_rows(W, R_N, R_f, n, L.R_f_pad, L.n_pad, L.wplane, s.WS, s.EW, st));
    if (with_gram)
        TRYK("gram_i8",
             launch_gram_i8(s.US, s.EU, s.WS, s.EW, L, G, R_f, R_N, nullptr, mirror, s.tail, st));
    return TC_OK;
}

// Workspace plan of one instance.  Layout: [G?][D?] and then either one
// [W][per-mode scratch] region sized for the largest mode and reused by the
// three modes in turn, or (split) one such region per mode, so that the modes
// can run concurrently.
struct InstancePlan {
    double *G, *D;
    double *part;  // adjoint: partial sums of the split contraction (or null)
    double *W[3];
    ModeScratch ms[3];
    size_t bytes;
};

InstancePlan plan_instance(void *ws, const tc_instance &I, tc_precision prec, bool backward,
                           bool split = false, bool by_route = false)
{
    InstancePlan P{};
    Carver c(ws);
    const size_t F2 = (size_t)I.R_f * I.R_f;
    P.G = I.G_saved ? I.G_saved : c.take<double>(3 * (size_t)I.R_N * F2);
    P.D = backward ? c.take<double>((size_t)I.R_N * F2) : nullptr;
    P.part = nullptr;
    if (backward) {
        size_t np = 0;
        for (int l = 0; l < 3; ++l) {
            const size_t nl = (size_t)(adjoint_splits(I.n[l], I.R_f, I.R_N) - 1) * I.R_f * I.n[l];
            if (nl > np)
                np = nl;
        }
        if (np > 0)
            P.part = c.take<double>(np);
    }
    // binary64 W: every route but the forward int8 FFT route, which writes
    // the int8 slices of W straight from the convolution; by_route == false
    // keeps it for every mode (any route may run: the autotuner)
    // The four-step FFT scratch (n > 4096) likewise only where that route runs.
    bool needW[3], largeF[3];
    for (int l = 0; l < 3; ++l) {
        const tc_algorithm a = resolve(I.n[l], I.R_f, I.R_N, prec);
        needW[l] = backward || !by_route || !i8_fused_fft(prec, a, I.n[l]);
        largeF[l] = !by_route || a == TC_ALGO_FFT;
    }
    if (split) {
        for (int l = 0; l < 3; ++l) {
            P.W[l] = needW[l] ? c.take<double>((size_t)I.R_N * I.R_f * I.n[l]) : nullptr;
            P.ms[l] = carve_mode(c, prec, I.n[l], I.R_f, I.R_N, true, largeF[l]);
        }
        P.bytes = c.used;
        return P;
    }
    size_t wn = 0;
    for (int l = 0; l < 3; ++l)
        if (needW[l] && (size_t)I.n[l] > wn)
            wn = I.n[l];
    P.W[0] = P.W[1] = P.W[2] = wn ? c.take<double>((size_t)I.R_N * I.R_f * wn) : nullptr;
    const size_t scratch0 = c.used;
    size_t scratch_max = 0;
    for (int l = 0; l < 3; ++l) {
        c.used = scratch0;
        P.ms[l] = carve_mode(c, prec, I.n[l], I.R_f, I.R_N, true, largeF[l]);
        if (c.used - scratch0 > scratch_max)
            scratch_max = c.used - scratch0;
    }
    P.bytes = scratch0 + scratch_max;
    return P;
}

size_t convolve_ws(int n, int R_f, int R_N, tc_precision prec)
{
    Carver c(nullptr);
    carve_mode(c, prec, n, R_f, R_N, false, resolve(n, R_f, R_N, prec) == TC_ALGO_FFT);
    return c.used;
}

// Coulomb entries against a density: every size and pointer present
bool density_ok(const tc_density &D)
{
    if (!D.c || !D.d || !D.Jd)
        return false;
    for (int l = 0; l < 3; ++l)
        if (!size_ok(D.n[l], D.R_f, D.R_N) || !size_ok(D.n[l], D.R_rho, D.R_N) || !D.p[l] ||
            !D.U[l] || !D.V[l])
            return false;
    return true;
}

// Workspace: [H: 3 x R_N x R_f x R_rho][W: R_N x R_rho x max n][one mode's
// convolution scratch, sized for the largest mode and reused]
struct DensityPlan {
    double *H, *W;
    ModeScratch ms[3];
    size_t bytes;
};

DensityPlan plan_density(void *ws, const tc_density &D)
{
    DensityPlan P{};
    Carver c(ws);
    P.H = c.take<double>(3 * (size_t)D.R_N * D.R_f * D.R_rho);
    int nmax = D.n[0];
    for (int l = 1; l < 3; ++l)
        nmax = D.n[l] > nmax ? D.n[l] : nmax;
    P.W = c.take<double>((size_t)D.R_N * D.R_rho * nmax);
    const size_t scratch0 = c.used;
    size_t scratch_max = 0;
    for (int l = 0; l < 3; ++l) {
        c.used = scratch0;
        P.ms[l] = carve_mode(c, TC_FP64, D.n[l], D.R_rho, D.R_N, false,
                             resolve(D.n[l], D.R_rho, D.R_N, TC_FP64) == TC_ALGO_FFT);
        if (c.used - scratch0 > scratch_max)
            scratch_max = c.used - scratch0;
    }
    P.bytes = scratch0 + scratch_max;
    return P;
}

// ---------------------------------------------------------------------------
// batches: independent instances run on a fixed pool of internal streams
// (created once, default priority), forked from and joined back into the
// caller's stream with events, so a captured batch is one graph with
// parallel branches.  Instances are assigned greedily (largest first) to the
// least-loaded branch; each branch owns one workspace region sized for its
// largest instance.
// ---------------------------------------------------------------------------
constexpr int kBranches = 4;

double instance_cost(const tc_instance &I)
{
    double c = 0.0;
    for (int l = 0; l < 3; ++l) {
        const double n = I.n[l], f = I.R_f;
        c += I.R_N * (n * std::log2(n + 1.0) * f + n * f * f);
    }
    return c;
}

struct BatchPlan {
    std::vector<int> branch;       // branch of each instance
    size_t offset[kBranches] = {};  // workspace region of each branch
    size_t bytes = 0;
};

// by_route == false sizes the regions for any route of every mode (the
// autotuner changes the routes while it runs)
BatchPlan plan_batch(const tc_instance *inst, int count, tc_precision prec, bool by_route = true)
{
    BatchPlan B;
    B.branch.assign(count, 0);
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return instance_cost(inst[a]) > instance_cost(inst[b]);
    });
    double load[kBranches] = {};
    size_t need[kBranches] = {};
    for (int i : order) {
        int best = 0;
        for (int b = 1; b < kBranches; ++b)
            if (load[b] < load[best])
                best = b;
        B.branch[i] = best;
        load[best] += instance_cost(inst[i]);
        const size_t wi = plan_instance(nullptr, inst[i], prec, false, false, by_route).bytes;
        if (wi > need[best])
            need[best] = wi;
    }
    for (int b = 0; b < kBranches; ++b) {
        B.offset[b] = B.bytes;
        B.bytes += align_up(need[b]);
    }
    return B;
}

struct BranchPool {
    bool ok = false;
    hipStream_t st[kBranches] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBranches] = {};
    hipEvent_t kpart[3] = {};  // a mode's kernel part done (borrowed by later modes)
};
std::mutex g_pool_mu;
BranchPool g_pool;

bool pool_init()
{
    if (g_pool.ok)
        return true;
    for (int b = 0; b < kBranches; ++b)
        if (hipStreamCreateWithFlags(&g_pool.st[b], hipStreamNonBlocking) != hipSuccess)
            return false;
    if (hipEventCreateWithFlags(&g_pool.fork, hipEventDisableTiming) != hipSuccess)
        return false;
    for (int b = 0; b < kBranches; ++b)
        if (hipEventCreateWithFlags(&g_pool.join[b], hipEventDisableTiming) != hipSuccess)
            return false;
    for (int l = 0; l < 3; ++l)
        if (hipEventCreateWithFlags(&g_pool.kpart[l], hipEventDisableTiming) != hipSuccess)
            return false;
    g_pool.ok = true;
    return true;
}

bool profiling()
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return g_prof_on;
}

// One instance: the Grams of the three modes, then the Hadamard sum.  With
// `split` the workspace plan has one region per mode and the modes run
// concurrently: the first on st, the other two on pool branches forked from
// and joined back into st (the caller holds g_pool_mu and the pool is
// initialised), except while kernel timing is on, when they run in turn on st.
//
// On the int8 FFT route a mode whose kernel vectors and n equal those of an
// earlier mode (the same pointer: the common case of one grid spacing in all
// three directions) reuses that mode's kernel part (spectra, term classes,
// S_k) instead of recomputing it.  With concurrent modes the owner computes
// it first on its stream and records an event; a borrowing branch prepares
// its own U (spectra, int8 slices) meanwhile and waits for the event only
// before its convolution (2.59 -> 2.55 ms per step against computing the
// shared part before the fork, which in turn beat three copies).  The
// smooth-term Grams stay after the int8 Gram of their mode: moving them first
// measured 2.5% slower.
tc_status forward_instance(const tc_instance &I, tc_precision prec, void *ws, size_t ws_bytes,
                           hipStream_t st, bool split_plan = false)
{
    const InstancePlan P = plan_instance(ws, I, prec, false, split_plan, true);
    // the plan follows the tuning table: a table changed since the caller
    // sized the workspace may need more
    if (P.bytes > ws_bytes)
        return TC_ERR_WORKSPACE;
    const size_t F2 = (size_t)I.R_f * I.R_f;
    const bool split = split_plan && !profiling();
    // the Hadamard sum reads only the upper triangles: the lower ones are
    // written only into a caller's G_saved
    const bool mirror = I.G_saved != nullptr;
    tc_algorithm algo[3];
    int owner[3];
    for (int l = 0; l < 3; ++l) {
        algo[l] = resolve(I.n[l], I.R_f, I.R_N, prec);
        owner[l] = l;
    }
    for (int l = 0; l < 3; ++l) {
        if (!i8_fused_fft(prec, algo[l], I.n[l]))
            continue;
        auto same_part = [&](int m) {
            return owner[m] == m && algo[m] == algo[l] && I.p[m] == I.p[l] && I.n[m] == I.n[l];
        };
        if (split_plan) {
            // one scratch region per mode: any earlier owner's part stays intact
            for (int m = 0; m < l; ++m)
                if (same_part(m)) {
                    owner[l] = m;
                    break;
                }
        } else if (l > 0 && i8_fused_fft(prec, algo[l - 1], I.n[l - 1]) &&
                   same_part(owner[l - 1])) {
            // one region shared by the modes in turn: only the part the
            // previous mode left there (its own or the one it borrowed) is
            // still intact; a mode in between with another part overwrites it
            owner[l] = owner[l - 1];
        }
    }
    // The owner of a borrowed kernel part computes it on its own stream and
    // records kpart[owner]; a borrowing branch waits for that event before its
    // convolution.
    if (split && hipEventRecord(g_pool.fork, st) != hipSuccess)
        return TC_ERR_HIP;
    tc_status status = TC_OK;
    for (int l = 0; l < 3 && status == TC_OK; ++l) {
        // the first mode stays on the caller's stream (no cross-queue wait
        // before it starts); the other two fork onto branches
        hipStream_t sl = (split && l > 0) ? g_pool.st[l] : st;
        if (split && l > 0 && hipStreamWaitEvent(sl, g_pool.fork, 0) != hipSuccess) {
            status = TC_ERR_HIP;
            break;
        }
        double *Gl = P.G + (size_t)l * I.R_N * F2;
        const bool i8fft = i8_fused_fft(prec, algo[l], I.n[l]);
        if (!i8fft) {
            status = mode_grams(prec, algo[l], I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], P.W[l], Gl,
                                P.ms[l], sl, mirror);
            continue;
        }
        const int o = owner[l];
        if (o == l) {
            status = int8fft_kernel_part(I.n[l], I.R_N, I.p[l], P.ms[l], sl);
            if (status == TC_OK && split && hipEventRecord(g_pool.kpart[l], sl) != hipSuccess)
                status = TC_ERR_HIP;
        }
        if (status == TC_OK)
            status = int8fft_u_prep(I.n[l], I.R_f, I.R_N, I.U[l], P.ms[l], o != l, sl);
        // a borrowing branch waits for the owner's kernel part only now
        if (status == TC_OK && split && o != l &&
            hipStreamWaitEvent(sl, g_pool.kpart[o], 0) != hipSuccess)
            status = TC_ERR_HIP;
        if (status == TC_OK)
            status = int8fft_u_main(I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], Gl, P.ms[l], P.ms[o],
                                    mirror, sl);
    }
    if (split) {
        // join both branches, also after a failed launch
        for (int l = 1; l < 3; ++l)
            if (hipEventRecord(g_pool.join[l], g_pool.st[l]) != hipSuccess ||
                hipStreamWaitEvent(st, g_pool.join[l], 0) != hipSuccess)
                status = TC_ERR_HIP;
    }
    if (status != TC_OK)
        return status;
    TRYK("hadamard_sum", launch_hadamard_sum(I.c, P.G, P.G + (size_t)I.R_N * F2,
                                             P.G + 2 * (size_t)I.R_N * F2, I.J, I.R_f, I.R_N, st));
    return TC_OK;
}

// ---------------------------------------------------------------------------
// int8 batches through the work queue: every mode of every instance prepares
// its int8 slices (and its smooth-term Grams) on the branch of its instance,
// then one persistent launch forms all the int8 Grams, then the Hadamard sums.
// ---------------------------------------------------------------------------
// Batch routes (tc_batch_route): fork-join, or the queue with 128-tiles or
// with 64-tiles below R_f = 256, each with one or two K parts.
struct QueueShape {
    bool small_tiles;  // 64-tiles for R_f < 256
    int kparts;
};
QueueShape queue_shape(int route)
{
    return {route == TC_BATCH_QUEUE_T64 || route == TC_BATCH_QUEUE_T64_K2,
            route == TC_BATCH_QUEUE_K2 || route == TC_BATCH_QUEUE_T64_K2 ? 2 : 1};
}

bool queue_route(int route) { return route >= TC_BATCH_QUEUE && route <= TC_BATCH_QUEUE_T64_K2; }

// Layout of the queue plan: per instance one split-plan region (its Grams and
// one scratch region per mode), then the job table, the counter and, for two
// K parts, one slab of Grams per job.
struct QueuePlan {
    std::vector<size_t> offset;  // of each instance's region
    size_t jobs = 0, counter = 0, slabs = 0, bytes = 0;
};

QueuePlan plan_queue(const tc_instance *inst, int count, tc_precision prec, bool by_route = true)
{
    QueuePlan Q;
    Q.offset.resize(count);
    size_t used = 0;
    for (int i = 0; i < count; ++i) {
        Q.offset[i] = used;
        used += align_up(plan_instance(nullptr, inst[i], prec, false, true, by_route).bytes);
    }
    Q.jobs = used;
    used += align_up(sizeof(GramJob) * 3 * (size_t)count);
    Q.counter = used;
    used += align_up(sizeof(int));
    Q.slabs = used;
    for (int i = 0; i < count; ++i)
        used += 3 * align_up(sizeof(double) * (size_t)inst[i].R_N * inst[i].R_f * inst[i].R_f);
    Q.bytes = used;
    return Q;
}

tc_status forward_batch_queue(const tc_instance *inst, int count, tc_precision prec, int route,
                              void *ws, size_t ws_bytes, hipStream_t st)
{
    const QueuePlan Q = plan_queue(inst, count, prec);
    if (Q.bytes > ws_bytes)
        return TC_ERR_WORKSPACE;
    const QueueShape shape = queue_shape(route);
    char *base = (char *)ws;
    const BatchPlan B = plan_batch(inst, count, prec);  // branch of each instance
    if (hipEventRecord(g_pool.fork, st) != hipSuccess)
        return TC_ERR_HIP;
    for (int b = 0; b < kBranches; ++b)
        if (hipStreamWaitEvent(g_pool.st[b], g_pool.fork, 0) != hipSuccess)
            return TC_ERR_HIP;
    std::vector<GramJob> jobs;
    jobs.reserve(3 * (size_t)count);
    double *slab = (double *)(base + Q.slabs);
    tc_status status = TC_OK;
    for (int i = 0; i < count && status == TC_OK; ++i) {
        const tc_instance &I = inst[i];
        hipStream_t sb = g_pool.st[B.branch[i]];
        const InstancePlan P = plan_instance(base + Q.offset[i], I, prec, false, true, true);
        const size_t F2 = (size_t)I.R_f * I.R_f;
        const bool mirror = I.G_saved != nullptr;
        tc_algorithm algo[3];
        int owner[3];
        for (int l = 0; l < 3; ++l) {
            algo[l] = resolve(I.n[l], I.R_f, I.R_N, prec);
            owner[l] = l;
            if (i8_fused_fft(prec, algo[l], I.n[l]))
                for (int m = 0; m < l; ++m)
                    if (owner[m] == m && i8_fused_fft(prec, algo[m], I.n[m]) &&
                        I.p[m] == I.p[l] && I.n[m] == I.n[l]) {
                        owner[l] = m;
                        break;
                    }
        }
        for (int l = 0; l < 3 && status == TC_OK; ++l) {
            double *Gl = P.G + (size_t)l * I.R_N * F2;
            const bool fused = i8_fused_fft(prec, algo[l], I.n[l]);
            // the modes of an instance run in turn on its branch, so a
            // borrowed kernel part is complete before it is read
            if (!fused) {
                status = mode_grams(prec, algo[l], I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], P.W[l],
                                    Gl, P.ms[l], sb, mirror, false);
            } else {
                if (owner[l] == l)
                    status = int8fft_kernel_part(I.n[l], I.R_N, I.p[l], P.ms[l], sb);
                if (status == TC_OK)
                    status = int8fft_u_prep(I.n[l], I.R_f, I.R_N, I.U[l], P.ms[l],
                                            owner[l] != l, sb);
                if (status == TC_OK)
                    status = int8fft_u_main(I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], Gl, P.ms[l],
                                            P.ms[owner[l]], mirror, sb, false);
            }
            const OzakiLayout L = ozaki_layout(I.n[l], I.R_f, I.R_N);
            GramJob J{};
            J.US = P.ms[l].US;
            J.EU = P.ms[l].EU;
            J.WS = P.ms[l].WS;
            J.EW = P.ms[l].EW;
            J.cls = fused ? P.ms[owner[l]].cls : nullptr;
            J.G = Gl;
            J.uplane = L.uplane;
            J.wplane = L.wplane;
            J.n_pad = L.n_pad;
            J.R_f_pad = L.R_f_pad;
            J.R_f = I.R_f;
            J.R_N = I.R_N;
            J.tile = shape.small_tiles && I.R_f < 256 ? 64 : 128;
            const int nt = (L.R_f_pad + J.tile - 1) / J.tile;
            J.ntri = nt * (nt + 1) / 2;
            J.kparts = shape.kparts;
            J.slab = J.kparts > 1 ? slab : nullptr;
            J.mirror = mirror ? 1 : 0;
            jobs.push_back(J);
            slab += align_up(sizeof(double) * (size_t)I.R_N * F2) / sizeof(double);
        }
    }
    for (int b = 0; b < kBranches; ++b)
        if (hipEventRecord(g_pool.join[b], g_pool.st[b]) != hipSuccess ||
            hipStreamWaitEvent(st, g_pool.join[b], 0) != hipSuccess)
            status = TC_ERR_HIP;
    if (status != TC_OK)
        return status;
    // the queue: costliest jobs first (contraction length, then tile rows)
    std::stable_sort(jobs.begin(), jobs.end(), [](const GramJob &a, const GramJob &b) {
        if (a.n_pad != b.n_pad)
            return a.n_pad > b.n_pad;
        return a.R_f_pad > b.R_f_pad;
    });
    long total = 0;
    for (GramJob &J : jobs) {
        J.item_begin = (int)total;
        total += (long)J.R_N * J.ntri * J.kparts;
    }
    if (total > 0x7fffffff)
        return TC_ERR_UNSUPPORTED;
    TRYK("gram_queue", launch_gram_queue(jobs.data(), (int)jobs.size(), (int)total,
                                         (GramJob *)(base + Q.jobs), (int *)(base + Q.counter),
                                         st));
    // the Hadamard sums, spread over the branches again
    if (hipEventRecord(g_pool.fork, st) != hipSuccess)
        return TC_ERR_HIP;
    for (int b = 0; b < kBranches; ++b)
        if (hipStreamWaitEvent(g_pool.st[b], g_pool.fork, 0) != hipSuccess)
            return TC_ERR_HIP;
    for (int i = 0; i < count && status == TC_OK; ++i) {
        const tc_instance &I = inst[i];
        hipStream_t sb = g_pool.st[B.branch[i]];
        const InstancePlan P = plan_instance(base + Q.offset[i], I, prec, false, true, true);
        const size_t F2 = (size_t)I.R_f * I.R_f;
        ProfScope ps_("hadamard_sum", sb);
        if (launch_hadamard_sum(I.c, P.G, P.G + (size_t)I.R_N * F2, P.G + 2 * (size_t)I.R_N * F2,
                                I.J, I.R_f, I.R_N, sb) != hipSuccess)
            status = TC_ERR_HIP;
        ps_.end();
        if (status == TC_OK && debug_sync_on() && !debug_sync_check("hadamard_sum", sb))
            status = TC_ERR_HIP;
    }
    for (int b = 0; b < kBranches; ++b)
        if (hipEventRecord(g_pool.join[b], g_pool.st[b]) != hipSuccess ||
            hipStreamWaitEvent(st, g_pool.join[b], 0) != hipSuccess)
            status = TC_ERR_HIP;
    return status;
}

// Workspace of tc_autotune's batch timing: copies of the instances with J in
// the workspace and no G_saved, run through every batch route.
size_t autotune_batch_bytes(const tc_instance *inst, int count, tc_precision prec)
{
    std::vector<tc_instance> cp(inst, inst + count);
    size_t js = 0;
    for (tc_instance &I : cp) {
        I.G_saved = nullptr;
        js += align_up(sizeof(double) * (size_t)I.R_f * I.R_f);
    }
    return js + std::max(plan_batch(cp.data(), count, prec, false).bytes,
                         plan_queue(cp.data(), count, prec, false).bytes);
}

// A batch through the fork-join route: every instance on a branch, its
// modes in turn, its own per-mode launches.
tc_status forward_batch_fork_join(const tc_instance *inst, int count, tc_precision prec, void *ws,
                                  size_t ws_bytes, hipStream_t st)
{
    const BatchPlan B = plan_batch(inst, count, prec);
    if (B.bytes > ws_bytes)
        return TC_ERR_WORKSPACE;
    // fork: every branch waits for the work already queued on the caller's stream
    if (hipEventRecord(g_pool.fork, st) != hipSuccess)
        return TC_ERR_HIP;
    for (int b = 0; b < kBranches; ++b)
        if (hipStreamWaitEvent(g_pool.st[b], g_pool.fork, 0) != hipSuccess)
            return TC_ERR_HIP;
    tc_status status = TC_OK;
    for (int i = 0; i < count && status == TC_OK; ++i) {
        const int b = B.branch[i];
        const size_t end = b + 1 < kBranches ? B.offset[b + 1] : B.bytes;
        status = forward_instance(inst[i], prec, (char *)ws + B.offset[b], end - B.offset[b],
                                  g_pool.st[b]);
    }
    // join (also after a failed launch, so no branch is left forked)
    for (int b = 0; b < kBranches; ++b) {
        if (hipEventRecord(g_pool.join[b], g_pool.st[b]) != hipSuccess ||
            hipStreamWaitEvent(st, g_pool.join[b], 0) != hipSuccess)
            status = TC_ERR_HIP;
    }
    return status;
}

tc_status backward_instance(const tc_instance &I, const double *Jbar, double *const *dU,
                            tc_precision prec, void *ws, hipStream_t st)
{
    const InstancePlan P = plan_instance(ws, I, prec, true);
    const size_t F2 = (size_t)I.R_f * I.R_f;
    if (!I.G_saved) {
        for (int l = 0; l < 3; ++l) {
            const tc_algorithm algo = resolve(I.n[l], I.R_f, I.R_N, prec);
            const tc_status r = mode_grams(prec, algo, I.n[l], I.R_f, I.R_N, I.p[l], I.U[l],
                                           P.W[l], P.G + (size_t)l * I.R_N * F2, P.ms[l], st);
            if (r != TC_OK)
                return r;
        }
    }
    for (int l = 0; l < 3; ++l) {
        const double *Ga = P.G + (size_t)((l + 1) % 3) * I.R_N * F2;
        const double *Gb = P.G + (size_t)((l + 2) % 3) * I.R_N * F2;
        TRYK("adjoint_d", launch_adjoint_d(I.c, Jbar, Ga, Gb, P.D, I.R_f, I.R_N, st));
        const tc_algorithm algo = resolve(I.n[l], I.R_f, I.R_N, prec);
        const tc_status r =
            mode_W(prec, algo, I.n[l], I.R_f, I.R_N, I.p[l], I.U[l], P.W[l], P.ms[l], st);
        if (r != TC_OK)
            return r;
        TRYK("adjoint_gemm_f64",
             launch_adjoint_gemm_f64(P.D, P.W[l], dU[l], I.n[l], I.R_f, I.R_N, 2.0, P.part, st));
    }
    return TC_OK;
}

// ---- pivoted Cholesky drivers --------------------------------------------

// Scratch of one pivoted Cholesky: residual diagonal, pivot column, device
// pivots, pivot state and statistics, and (fit only) the factor L.
struct CholScratch {
    double *d, *d2, *col, *L, *y, *Yd, *stats;
    int *piv, *state, *ispiv;
};

CholScratch carve_chol(Carver &c, int N, int R_max, bool own_L, size_t y_len,
                       size_t Yd_len = 0)
{
    CholScratch s{};
    s.d = c.take<double>(N);
    s.d2 = c.take<double>(N);  // the other residual diagonal of the formed-matrix steps
    s.col = c.take<double>(N);
    s.L = own_L ? c.take<double>((size_t)R_max * N) : nullptr;
    s.y = y_len ? c.take<double>(y_len) : nullptr;
    s.Yd = Yd_len ? c.take<double>(Yd_len) : nullptr;
    s.stats = c.take<double>(2);
    s.piv = c.take<int>(R_max);
    s.state = c.take<int>(3);
    s.ispiv = c.take<int>(N);
    return s;
}

// Runs the loop: `column` enqueues the column of A at the pivot into s.col.
// thr_rel: the steps run while the residual trace exceeds thr_rel * trace(A).
// After one synchronisation for trace(A), the steps are enqueued in groups of
// 16, 32, then 64 steps; the device stops itself (done flag: the rest of a
// group are no-ops) and the host checks the flag once per group.  Each check
// leaves the device idle for a round trip to the host, and the growing groups
// take fewer of them on long factorisations at the cost of at most 63 no-op
// steps after the last.
constexpr int kCholGroup = 16;
constexpr int kCholGroupMax = 64;

template <class Column>
// A: the formed matrix [N][N] (its pivot rows are the columns), or null and
// `column` computes each pivot's column into s.col.
tc_status pivoted_cholesky(int N, int R_max, double thr_rel, const CholScratch &s, double *L,
                           Column column, const double *A, int *pivots_host, int *R_out,
                           double *residual_out, hipStream_t st)
{
    double stats[2];
    int state[3];
    auto fetch = [&]() {
        return hipMemcpyAsync(stats, s.stats, sizeof stats, hipMemcpyDeviceToHost, st) ==
                       hipSuccess &&
               hipMemcpyAsync(state, s.state, sizeof state, hipMemcpyDeviceToHost, st) ==
                       hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    TRYK("chol_init", launch_fill_int(s.state, 3, 0, st));
    TRYK("chol_init", launch_fill_int(s.ispiv, N, 0, st));
    TRYK("chol_select",
         launch_chol_select(s.d, N, 0, 0, -1.0, R_max, s.state, s.stats, s.piv, s.ispiv, st));
    if (!fetch())
        return TC_ERR_HIP;
    const double thr = thr_rel * stats[1];
    if (!state[1] && !(stats[1] > thr)) {  // nothing to do: zero steps
        state[1] = 1;
        state[2] = 0;
    }
    int r = 0;
    int group = kCholGroup;
    while (!state[1]) {
        for (int g = 0; g < group && r < R_max; ++g, ++r) {
            if (A) {
                // formed matrix: the selection of step r's pivot and the step
                // in one launch (the diagonal alternates between d and d2;
                // step r reads the one step r - 1 wrote)
                double *din = (r & 1) ? s.d2 : s.d, *dout = (r & 1) ? s.d : s.d2;
                TRYK("chol_step", launch_chol_select_step(A, L, N, r, s.ispiv, s.state, din,
                                                          dout, thr, R_max, s.stats, s.piv, st));
                continue;
            }
            const tc_status cs = column(st);
            if (cs != TC_OK)
                return cs;
            TRYK("chol_step", launch_chol_step(s.col, A, L, N, r, s.ispiv, s.state, s.d, st));
            TRYK("chol_select", launch_chol_select(s.d, N, 1, r + 1, thr, R_max, s.state,
                                                   s.stats, s.piv, s.ispiv, st));
        }
        if (A && r >= R_max && !state[1]) {
            // every step enqueued: one more selection records the end (r = R_max)
            double *din = (r & 1) ? s.d2 : s.d, *dout = (r & 1) ? s.d : s.d2;
            TRYK("chol_step", launch_chol_select_step(A, L, N, r, s.ispiv, s.state, din, dout,
                                                      thr, R_max, s.stats, s.piv, st));
        }
        if (!fetch())
            return TC_ERR_HIP;
        group = std::min(2 * group, kCholGroupMax);
    }
    const int R = state[2];
    *R_out = R;
    if (residual_out)
        *residual_out = stats[1];
    if (pivots_host && R > 0 &&
        (hipMemcpyAsync(pivots_host, s.piv, sizeof(int) * R, hipMemcpyDeviceToHost, st) !=
             hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
        return TC_ERR_HIP;
    return TC_OK;
}

// The fit forms A = F^T F (n x n) when it is at most 512 MiB (n <= 8192):
// each step then reads the pivot's row instead of a pass over F.
constexpr int kFitFormedMaxN = 8192;

size_t fit_ws(int n, int N_pair, int R_max)
{
    Carver c(nullptr);
    carve_chol(c, n, R_max, true, (size_t)fit_column_parts() * n, (size_t)R_max * R_max);
    if (n <= kFitFormedMaxN) {
        c.take<double>((size_t)n * N_pair);
        c.take<double>((size_t)n * n);
    }
    return c.used;
}

// B is formed (each step then reads the pivot's row) when it is at most
// 128 MiB (N_pair <= 4096); its terms go through Z in chunks of about 256 MiB
constexpr int kTeiFormedMaxN = 4096;
int tei_form_chunk(int N_pair, int R_N)
{
    const size_t per = (size_t)3 * N_pair * N_pair * sizeof(double);
    size_t kc = ((size_t)256 << 20) / per;
    kc = kc < 1 ? 1 : kc;
    return (int)(kc < (size_t)R_N ? kc : (size_t)R_N);
}

size_t tei_chol_ws(int N_pair, int R, int R_N, int R_max)
{
    Carver c(nullptr);
    carve_chol(c, N_pair, R_max, false, 0, (size_t)3 * R_N * N_pair * R);
    if (N_pair <= kTeiFormedMaxN) {
        c.take<double>((size_t)N_pair * N_pair);
        c.take<double>((size_t)3 * tei_form_chunk(N_pair, R_N) * N_pair * N_pair);
    }
    return c.used;
}

}  // namespace

namespace tc {
// tc_tei_gram on a given workspace
tc_status tei_gram_check(const tc_instance *inst, int count, tc_precision prec)
{
    if (!inst || count < 1 || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!instance_ok(inst[i]))
            return TC_ERR_INVALID_ARG;
    if (!prec_supported(prec))
        return TC_ERR_UNSUPPORTED;
    return TC_OK;
}

tc_status tei_gram_call(const tc_instance *inst, int count, tc_precision prec, void *ws,
                        size_t ws_bytes, void *stream)
{
    const tc_status chk = tei_gram_check(inst, count, prec);
    if (chk != TC_OK)
        return chk;
    const size_t need = tc_workspace_bytes(TC_OP_TEI_GRAM, inst, count, prec);
    if (need > 0 && (!ws || ws_bytes < need))
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
        const tc_status f = finite_instance(inst[i], st);
        if (f != TC_OK)
            return f;
    }
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!pool_init())
        return TC_ERR_HIP;
    if (count == 1)  // one instance: its three modes on three branches
        return forward_instance(inst[0], prec, ws, ws_bytes, st, true);

    const int route = batch_route(inst, count, prec);
    if (queue_route(route))
        return forward_batch_queue(inst, count, prec, route, ws, ws_bytes, st);
    return forward_batch_fork_join(inst, count, prec, ws, ws_bytes, st);
}
}  // namespace tc

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
    default:
        break;
    }
    return "unknown tc_status";
}

int tc_version(void) { return 300; }

size_t tc_workspace_bytes(int op, const tc_instance *inst, int count, tc_precision prec)
{
    if (!inst || count < 1 || !prec_known(prec))
        return (size_t)-1;
    if (op == TC_OP_CONVOLVE) {
        if (!size_ok(inst[0].n[0], inst[0].R_f, inst[0].R_N))
            return (size_t)-1;
        return convolve_ws(inst[0].n[0], inst[0].R_f, inst[0].R_N, prec);
    }
    if (op != TC_OP_TEI_GRAM && op != TC_OP_TEI_GRAM_BACKWARD && op != TC_OP_AUTOTUNE)
        return (size_t)-1;
    for (int i = 0; i < count; ++i)
        for (int l = 0; l < 3; ++l)
            if (!size_ok(inst[i].n[l], inst[i].R_f, inst[i].R_N))
                return (size_t)-1;
    if (op == TC_OP_TEI_GRAM) {
        if (count == 1)
            return plan_instance(nullptr, inst[0], prec, false, true, true).bytes;
        // every batch route the tuning table may select
        const size_t fj = plan_batch(inst, count, prec).bytes;
        if (prec != TC_OZAKI_I8)
            return fj;
        return std::max(fj, plan_queue(inst, count, prec).bytes);
    }
    size_t w = 0;
    for (int i = 0; i < count; ++i) {
        // the autotuner's Grams go to the workspace, never to G_saved
        tc_instance Ii = inst[i];
        if (op == TC_OP_AUTOTUNE)
            Ii.G_saved = nullptr;
        const size_t wi = plan_instance(nullptr, Ii, prec, op == TC_OP_TEI_GRAM_BACKWARD).bytes;
        if (wi > w)
            w = wi;
    }
    if (op == TC_OP_AUTOTUNE && count > 1 && prec == TC_OZAKI_I8)
        w = std::max(w, autotune_batch_bytes(inst, count, prec));
    return w;
}

tc_status tc_tune_set(int n, int R_f, int R_N, tc_precision prec, tc_algorithm algo)
{
    if (!size_ok(n, R_f, R_N) || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    if (algo != TC_ALGO_AUTO && algo != TC_ALGO_DIRECT && algo != TC_ALGO_FFT)
        return TC_ERR_INVALID_ARG;
    if (algo == TC_ALGO_FFT && !fft_any(n))
        return TC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneKey key(n, R_f, R_N, (int)prec);
    if (algo == TC_ALGO_AUTO)
        g_tune.erase(key);
    else
        g_tune[key] = (int)algo;
    return TC_OK;
}

tc_status tc_batch_tune_set(const tc_instance *inst, int count, tc_precision prec,
                            tc_batch_route route)
{
    if (!inst || count < 1 || !prec_known(prec) || route < TC_BATCH_AUTO ||
        route > TC_BATCH_QUEUE_T64_K2)
        return TC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        for (int l = 0; l < 3; ++l)
            if (!size_ok(inst[i].n[l], inst[i].R_f, inst[i].R_N))
                return TC_ERR_INVALID_ARG;
    if (queue_route(route) && prec != TC_OZAKI_I8)
        return TC_ERR_UNSUPPORTED;
    const uint64_t key = batch_signature(inst, count, prec);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (route == TC_BATCH_AUTO)
        g_batch_tune.erase(key);
    else
        g_batch_tune[key] = (int)route;
    return TC_OK;
}

tc_batch_route tc_batch_tune_get(const tc_instance *inst, int count, tc_precision prec)
{
    if (!inst || count < 1 || !prec_known(prec))
        return TC_BATCH_AUTO;
    return (tc_batch_route)batch_route(inst, count, prec);
}

tc_algorithm tc_tune_get(int n, int R_f, int R_N, tc_precision prec)
{
    if (!size_ok(n, R_f, R_N) || !prec_known(prec))
        return TC_ALGO_AUTO;
    return resolve(n, R_f, R_N, prec);
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
    hipStream_t st = (hipStream_t)stream;
    TRYK("newton_kernel", launch_newton_kernel(t.data(), R_N, n, h, p_dev, st));
    for (int k = 0; k < R_N; ++k) {
        if (t_host)
            t_host[k] = t[k];
        if (c_host)
            c_host[k] = two_over_sqrtpi * hu * t[k] * (h * h * h);
    }
    return TC_OK;
}

tc_status tc_term_classes(int n, int R_N, const double *p_dev, int *cls_dev, void *stream)
{
    if (!size_ok(n, 1, R_N) || !p_dev || !cls_dev)
        return TC_ERR_INVALID_ARG;
    if (launch_term_class(p_dev, n, R_N, cls_dev, (hipStream_t)stream) != hipSuccess)
        return TC_ERR_HIP;
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
    const tc_status f = finite_inputs({{p_dev, (long)R_N * (2L * n - 1)}, {U_dev, (long)R_f * n}},
                                      (hipStream_t)stream);
    if (f != TC_OK)
        return f;
    Carver c(ws);
    const tc_algorithm algo = resolve(n, R_f, R_N, prec);
    const ModeScratch s = carve_mode(c, prec, n, R_f, R_N, false, algo == TC_ALGO_FFT);
    if (c.used > ws_bytes && c.used > 0)
        return TC_ERR_WORKSPACE;
    return mode_W(prec, algo, n, R_f, R_N, p_dev, U_dev, W_dev, s, (hipStream_t)stream);
}


size_t tc_density_fit_workspace_bytes(int n, int N_pair, int R_max)
{
    if (n < 1 || n > TC_MAX_N || N_pair < 1 || N_pair > TC_MAX_RF || R_max < 1 || R_max > n)
        return (size_t)-1;
    return fit_ws(n, N_pair, R_max);
}

tc_status tc_density_fit(int n, int N_pair, const double *F_dev, double tol, int R_max,
                         double *U_dev, double *V_dev, int *pivots_host, int *R_out,
                         double *residual_out, void *ws, size_t ws_bytes, void *stream)
{
    if (n < 1 || n > TC_MAX_N || N_pair < 1 || N_pair > TC_MAX_RF || R_max < 1 || R_max > n ||
        !F_dev || !U_dev || !V_dev || !R_out || !(tol >= 0.0) || !std::isfinite(tol))
        return TC_ERR_INVALID_ARG;
    if (!ws || ws_bytes < fit_ws(n, N_pair, R_max))
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carver c(ws);
    const CholScratch s =
        carve_chol(c, n, R_max, true, (size_t)fit_column_parts() * n, (size_t)R_max * R_max);
    double *A = nullptr;
    if (n <= kFitFormedMaxN && !chol_columns_on()) {
        double *Ft = c.take<double>((size_t)n * N_pair);
        A = c.take<double>((size_t)n * n);
        TRYK("fit_gram", launch_fit_gram(F_dev, n, N_pair, Ft, A, st));
        // the formed matrix's diagonal, so that the steps and the pivot
        // choices read one matrix
        TRYK("fit_diag", launch_diag_copy(A, n, s.d, st));
    } else {
        TRYK("fit_diag", launch_fit_diag(F_dev, n, N_pair, s.d, st));
    }
    auto column = [&](hipStream_t st) -> tc_status {
        TRYK("fit_column", launch_fit_column(F_dev, n, N_pair, s.state, s.y, s.col, st));
        return TC_OK;
    };
    const tc_status r = pivoted_cholesky(n, R_max, tol * tol, s, s.L, column, A, pivots_host,
                                         R_out, residual_out, st);
    if (r != TC_OK)
        return r;
    TRYK("fit_finish", launch_fit_finish(F_dev, s.L, n, N_pair, *R_out, R_max, s.piv, s.Yd,
                                         U_dev, V_dev, st));
    return hipStreamSynchronize(st) == hipSuccess ? TC_OK : TC_ERR_HIP;
}

size_t tc_tei_cholesky_workspace_bytes(int N_pair, int R, int R_N, int R_max)
{
    if (N_pair < 1 || N_pair > TC_MAX_RF || R < 1 || R > TC_MAX_RF || R_N < 1 ||
        R_N > TC_MAX_RN || R_max < 1 || R_max > N_pair)
        return (size_t)-1;
    return tei_chol_ws(N_pair, R, R_N, R_max);
}

tc_status tc_tei_cholesky(int N_pair, int R, int R_N, const double *c_dev,
                          const double *const *V_dev, const double *const *M_dev, double tol,
                          int R_max, double *L_dev, int *pivots_host, int *R_out,
                          double *residual_out, void *ws, size_t ws_bytes, void *stream)
{
    if (N_pair < 1 || N_pair > TC_MAX_RF || R < 1 || R > TC_MAX_RF || R_N < 1 ||
        R_N > TC_MAX_RN || R_max < 1 || R_max > N_pair || !c_dev || !V_dev || !M_dev ||
        !L_dev || !R_out || !(tol >= 0.0) || !std::isfinite(tol))
        return TC_ERR_INVALID_ARG;
    for (int l = 0; l < 3; ++l)
        if (!V_dev[l] || !M_dev[l])
            return TC_ERR_INVALID_ARG;
    if (!ws || ws_bytes < tei_chol_ws(N_pair, R, R_N, R_max))
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    Carver c(ws);
    // s.Yd: Y = V M
    const CholScratch s = carve_chol(c, N_pair, R_max, false, 0, (size_t)3 * R_N * N_pair * R);
    TRYK("tei_diag", launch_tei_diag(c_dev, V_dev, M_dev, R, R_N, N_pair, s.Yd, s.d, st));
    double *B = nullptr;
    if (N_pair <= kTeiFormedMaxN && !chol_columns_on()) {
        // B formed once (GEMMs of V with Y on matrix cores); its diagonal
        // replaces d, so that the steps and the pivot choices read one matrix
        B = c.take<double>((size_t)N_pair * N_pair);
        const int kc = tei_form_chunk(N_pair, R_N);
        double *Z = c.take<double>((size_t)3 * kc * N_pair * N_pair);
        TRYK("tei_form_b",
             launch_tei_form_b(c_dev, V_dev, s.Yd, R, R_N, N_pair, kc, Z, B, s.d, st));
    }
    // the pivot's column from V and the rows of Y = V M at the pivot (one
    // launch; M symmetric, so M v_p is row p of Y)
    auto column = [&](hipStream_t st) -> tc_status {
        TRYK("tei_column", launch_tei_entries(c_dev, V_dev, s.Yd, R, R_N, N_pair, s.state, s.col, st));
        return TC_OK;
    };
    return pivoted_cholesky(N_pair, R_max, tol, s, L_dev, column, B, pivots_host, R_out,
                            residual_out, st);
}

// ---- canonical-to-Tucker transform ------------------------------------------
static bool tucker_sizes_ok(const int *n, int R, const int *r)
{
    if (!n || !r || R < 1 || R > (1 << 24))
        return false;
    for (int l = 0; l < 3; ++l)
        if (n[l] < 1 || n[l] > TC_MAX_N || r[l] < 1 || r[l] > kTuckerMaxRank || r[l] > n[l] ||
            r[l] > R)
            return false;
    return true;
}

static int tucker_sub(int n, int r)
{
    return std::min(std::min(n, kTuckerMaxSub), std::max(2 * r, r + 8));
}

// Workspace: [X: 64 x nmax][P: 64 x mmax][part: slices x 64 x max(nmax, mmax)]
// [H: 64 x 64][lam: 64][Vt: 64 x 64][Ut: 3 x 48 x R][K: 48^2 x R][Mt: 48^2 x nmax]
struct TuckerPlan {
    double *X, *P, *P2, *Gm, *part, *H, *lam, *Vt, *Ut[3], *K, *Mt, *D, *nrm, *Linv, *lamA;
    int *flag;
    size_t bytes;
};

// Orthogonal iteration in the space of B's rows (Y <- orth(Y B B^T), k x m)
// instead of on X (k x n) when forming B B^T once costs less than the
// products it saves: 2 m^2 n flops in one square product against
// 2 its k m n in skinny ones, which run at about half the rate
// (m^2 <= 2 its k n).  The workspace holds B B^T for m up to 4096 where that
// holds at the default of 20 steps; a call checks its own step count too.
constexpr int kTuckerGramIts = 20;
constexpr int kTuckerGramMaxM = 4096;
static bool tucker_gram_pays(long m, long n, long k, long its)
{
    return m >= k && m * m <= 2 * its * k * n;
}
static bool tucker_gram_form(int m, int n, int k)
{
    return m <= kTuckerGramMaxM && tucker_gram_pays(m, n, k, kTuckerGramIts);
}

static TuckerPlan plan_tucker(void *ws, const int *n, int R, const int *r)
{
    TuckerPlan T{};
    Carver c(ws);
    int nmax = std::max(n[0], std::max(n[1], n[2]));
    long rr = 0;
    for (int l = 0; l < 3; ++l)
        for (int m = l + 1; m < 3; ++m)
            rr = std::max(rr, (long)r[l] * r[m]);
    const long mmax = std::max((long)R, rr);
    // the Gram form's B B^T: the largest m that takes it
    long gmax = 0;
    for (int l = 0; l < 3; ++l) {
        const int k = tucker_sub(n[l], r[l]);
        const int m1 = l == 0 ? 1 : 0, m2 = l == 2 ? 1 : 2;
        for (long m : {(long)R, (long)r[m1] * r[m2]})
            if (tucker_gram_form((int)m, n[l], k))
                gmax = std::max(gmax, m);
    }
    T.X = c.take<double>((size_t)kTuckerMaxSub * nmax);
    T.P = c.take<double>((size_t)kTuckerMaxSub * mmax);
    T.P2 = c.take<double>((size_t)kTuckerMaxSub * mmax);
    T.Gm = c.take<double>((size_t)gmax * gmax);
    // split-slice scratch: the largest of the products the transform forms
    size_t part = 0;
    auto need = [&](long I, long N, long K) {
        part = std::max(part, (size_t)gemm_splits((int)I, (int)N, (int)K) * I * N);
    };
    for (int l = 0; l < 3; ++l) {
        const int k = tucker_sub(n[l], r[l]);
        const int m1 = l == 0 ? 1 : 0, m2 = l == 2 ? 1 : 2;
        const long q = (long)r[m1] * r[m2];
        for (long m : {(long)R, q}) {
            need(k, m, n[l]);
            need(k, n[l], m);
            need(k, k, m);
        }
        need(r[l], n[l], k);
        need(r[l], R, n[l]);
        need(q, n[l], R);
        need(k, k, n[l]);
        for (long m : {(long)R, q})
            if (tucker_gram_form((int)m, n[l], k)) {
                need(m, m, n[l]);  // B B^T
                need(k, m, m);     // Y (B B^T)
            }
    }
    need(r[0], (long)r[1] * r[2], R);
    T.part = c.take<double>(part);
    T.H = c.take<double>((size_t)kTuckerMaxSub * kTuckerMaxSub);
    T.lam = c.take<double>(kTuckerMaxSub);
    T.Vt = c.take<double>((size_t)kTuckerMaxSub * kTuckerMaxSub);
    for (int l = 0; l < 3; ++l)
        T.Ut[l] = c.take<double>((size_t)r[l] * R);
    T.K = c.take<double>((size_t)rr * R);
    T.Mt = c.take<double>((size_t)rr * nmax);
    T.D = c.take<double>((size_t)kOrthRows * kOrthRows);
    T.nrm = c.take<double>(kOrthRows);
    T.Linv = c.take<double>((size_t)kOrthRows * kOrthRows);
    T.flag = c.take<int>(1);
    T.lamA = c.take<double>(3 * (size_t)kTuckerMaxSub);
    T.bytes = c.used;
    return T;
}

// The r dominant left singular vectors of B^T (B [m][n] rows) as the rows of
// Z [r][n]: orthogonal iteration, then Rayleigh-Ritz.  warm: the first r rows
// of the start are Z itself.  Only the last step's rows enter the
// Rayleigh-Ritz step, so the steps before it take one Cholesky-QR pass (rows
// orthonormal to about (condition number)^2 u, enough to keep the next
// product well conditioned) and the last takes two.  The first step, where
// the start (random rows, or a basis of another matrix) is furthest from the
// dominant subspace, orthonormalises between X B^T and its product with B:
// each half then raises the condition number of the rows once, not twice (the
// same subspace in exact arithmetic).  That needs m >= k; with fewer rows in
// B the product has rank below k anyway and the fallback refills it.
static tc_status dominant_rows(const TuckerPlan &T, const double *B, int m, int n, int r,
                               int its, bool warm, double *Z, double *sv,
                               unsigned long long salt, hipStream_t st)
{
    const int k = tucker_sub(n, r);
    if (warm && hipMemcpyAsync(T.X, Z, sizeof(double) * (size_t)r * n, hipMemcpyDeviceToDevice,
                               st) != hipSuccess)
        return TC_ERR_HIP;
    auto orth = [&](double *X, int len, int passes, unsigned long long s) {
        return launch_orth_rows(X, k, len, passes, T.D, T.nrm, T.Linv, T.flag, T.part, s, st);
    };
    TRYK("random_rows", launch_random_rows(T.X, warm ? r : 0, k, n, salt, st));
    TRYK("orth_rows", orth(T.X, n, 1, salt + 1));
    if (tucker_gram_form(m, n, k) && tucker_gram_pays(m, n, k, its)) {
        // Y_0 = orth(X B^T), Y_t = orth(Y_{t-1} B B^T), X = orth2(Y_{its-1} B): the
        // subspaces of the loop below (its applications of B^T B) with one
        // product of k x m by m x m per step
        TRYK("gemm_f64", launch_gemm_f64(false, B, B, T.Gm, m, m, n, T.part, st));  // B B^T
        TRYK("gemm_f64", launch_gemm_f64(false, T.X, B, T.P, k, m, n, T.part, st));  // X B^T
        TRYK("orth_rows", orth(T.P, m, 1, salt + 1 + its + 1));
        double *Y = T.P, *Yn = T.P2;
        for (int it = 1; it < its; ++it) {
            TRYK("gemm_f64", launch_gemm_f64(false, Y, T.Gm, Yn, k, m, m, T.part, st));
            std::swap(Y, Yn);
            TRYK("orth_rows", orth(Y, m, 1, salt + 2 + it));
        }
        TRYK("gemm_f64", launch_gemm_f64(true, Y, B, T.X, k, n, m, T.part, st));  // Y B
        TRYK("orth_rows", orth(T.X, n, 2, salt + 2));
        its = 0;  // the steps are done
    }
    for (int it = 0; it < its; ++it) {
        TRYK("gemm_f64", launch_gemm_f64(false, T.X, B, T.P, k, m, n, T.part, st));  // X B^T
        if (it == 0 && m >= k)
            TRYK("orth_rows", orth(T.P, m, 1, salt + 1 + its + 1));
        TRYK("gemm_f64", launch_gemm_f64(true, T.P, B, T.X, k, n, m, T.part, st));   // (X B^T) B
        TRYK("orth_rows", orth(T.X, n, it == its - 1 ? 2 : 1, salt + 2 + it));
    }
    TRYK("gemm_f64", launch_gemm_f64(false, T.X, B, T.P, k, m, n, T.part, st));
    TRYK("gemm_f64", launch_gemm_f64(false, T.P, T.P, T.H, k, k, m, T.part, st));
    TRYK("jacobi_eig", launch_jacobi_eig(T.H, k, T.lam, T.Vt, st));
    TRYK("gemm_f64", launch_gemm_f64(true, T.Vt, T.X, Z, r, n, k, T.part, st));
    TRYK("sign_rows", launch_sign_rows(Z, r, n, T.lam, sv, st));
    return TC_OK;
}

size_t tc_canonical_to_tucker_workspace_bytes(const int *n, int R, const int *r)
{
    if (!tucker_sizes_ok(n, R, r))
        return (size_t)-1;
    return plan_tucker(nullptr, n, R, r).bytes;
}

tc_status tc_canonical_to_tucker(const int *n, int R, const double *c_dev,
                                 const double *const *A_dev, const int *r, int m_max, int its,
                                 double eps, double *const *Z_dev, double *beta_dev,
                                 double *sv_dev, int *r_out, void *ws, size_t ws_bytes,
                                 void *stream)
{
    if (!tucker_sizes_ok(n, R, r) || !c_dev || !A_dev || !Z_dev || !beta_dev || m_max < 0 ||
        m_max > 100 || its < 1 || its > 1000 || !std::isfinite(eps) || eps >= 1.0)
        return TC_ERR_INVALID_ARG;
    for (int l = 0; l < 3; ++l) {
        if (!A_dev[l] || !Z_dev[l])
            return TC_ERR_INVALID_ARG;
        const int m1 = l == 0 ? 1 : 0, m2 = l == 2 ? 1 : 2;
        if (m_max > 0 && (long)r[l] > (long)r[m1] * r[m2])
            return TC_ERR_INVALID_ARG;
    }
    const TuckerPlan T = plan_tucker(ws, n, R, r);
    if (!ws || ws_bytes < T.bytes)
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double *sv3[3] = {sv_dev, sv_dev ? sv_dev + r[0] : nullptr,
                      sv_dev ? sv_dev + r[0] + r[1] : nullptr};
    // (A) dominant subspaces of the side matrices
    int rk[3] = {r[0], r[1], r[2]};
    for (int l = 0; l < 3; ++l) {
        const tc_status s = dominant_rows(T, A_dev[l], R, n[l], r[l], its, false, Z_dev[l],
                                          sv3[l], 1000ull * (l + 1), st);
        if (s != TC_OK)
            return s;
        if (eps > 0.0 && hipMemcpyAsync(T.lamA + l * kTuckerMaxSub, T.lam, sizeof(double) * r[l],
                                        hipMemcpyDeviceToDevice, st) != hipSuccess)
            return TC_ERR_HIP;
    }
    if (eps > 0.0) {
        // epsilon truncation: singular values sqrt(lam) against eps times the largest
        double lam[3 * kTuckerMaxSub];
        if (hipMemcpyAsync(lam, T.lamA, sizeof lam, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return TC_ERR_HIP;
        for (int l = 0; l < 3; ++l) {
            const double *ll = lam + l * kTuckerMaxSub;
            const double s0 = std::sqrt(std::max(ll[0], 0.0));
            int cnt = 0;
            for (int i = 0; i < r[l]; ++i)
                cnt += std::sqrt(std::max(ll[i], 0.0)) >= eps * s0;
            rk[l] = std::max(1, std::min(r[l], cnt));
        }
        for (int l = 0; l < 3; ++l) {
            const int m1 = l == 0 ? 1 : 0, m2 = l == 2 ? 1 : 2;
            rk[l] = std::min(rk[l], rk[m1] * rk[m2]);
        }
    }
    if (r_out)
        for (int l = 0; l < 3; ++l)
            r_out[l] = rk[l];
    // (B) projections (basis rows beyond the chosen ranks zero)
    for (int l = 0; l < 3; ++l) {
        TRYK("zero_rows", launch_zero_rows(Z_dev[l], rk[l], r[l], n[l], st));
        TRYK("gemm_f64", launch_gemm_f64(false, Z_dev[l], A_dev[l], T.Ut[l], r[l], R, n[l],
                                         T.part, st));
    }
    // (C, D) sweeps: mode l from the image projected on the other two modes
    for (int sweep = 0; sweep < m_max; ++sweep)
        for (int l = 0; l < 3; ++l) {
            const int m1 = l == 0 ? 1 : 0, m2 = l == 2 ? 1 : 2;
            const int rr = r[m1] * r[m2];
            TRYK("khatri_rao",
                 launch_khatri_rao(c_dev, T.Ut[m1], T.Ut[m2], r[m1], r[m2], R, T.K, st));
            TRYK("gemm_f64", launch_gemm_f64(true, T.K, A_dev[l], T.Mt, rr, n[l], R, T.part, st));
            const tc_status s =
                dominant_rows(T, T.Mt, rr, n[l], r[l], its, true, Z_dev[l], sv3[l],
                              1000000ull + 1000ull * (3 * sweep + l), st);
            if (s != TC_OK)
                return s;
            TRYK("zero_rows", launch_zero_rows(Z_dev[l], rk[l], r[l], n[l], st));
            TRYK("gemm_f64", launch_gemm_f64(false, Z_dev[l], A_dev[l], T.Ut[l], r[l], R, n[l],
                                             T.part, st));
        }
    // (E) core: beta[i][(j m)] = sum_t Ut1[i][t] (c_t Ut2[j][t] Ut3[m][t])
    TRYK("khatri_rao", launch_khatri_rao(c_dev, T.Ut[1], T.Ut[2], r[1], r[2], R, T.K, st));
    TRYK("gemm_f64", launch_gemm_f64(false, T.Ut[0], T.K, beta_dev, r[0], r[1] * r[2], R,
                                     T.part, st));
    return TC_OK;
}

// ---- nuclear potential matrix ----------------------------------------------
static bool nuclear_ok(const tc_nuclear_problem &P)
{
    if (!P.c || !P.V || !P.Z || !P.pos || P.M < 1 || (long)P.M * P.R_N > 65535)
        return false;
    for (int l = 0; l < 3; ++l) {
        if (!size_ok(P.n[l], P.R_f, P.R_N) || !P.p[l] || !P.U[l] || !(P.h[l] > 0.0) ||
            !std::isfinite(P.h[l]))
            return false;
    }
    for (int a = 0; a < P.M; ++a) {
        if (!std::isfinite(P.Z[a]))
            return false;
        for (int l = 0; l < 3; ++l)
            if (P.pos[3 * a + l] < 0 || P.pos[3 * a + l] >= P.n[l])
                return false;
    }
    return true;
}

// Workspace: [shift: 3 x M ints][cls: 3 x R_N ints][cw: M R_N][G: 3 x M R_N x R_f x R_f]
struct NuclearPlan {
    int *shift, *cls;
    double *cw, *G;
    size_t bytes;
};

static NuclearPlan plan_nuclear(void *ws, const tc_nuclear_problem &P)
{
    NuclearPlan N{};
    Carver c(ws);
    const size_t T = (size_t)P.M * P.R_N;
    N.shift = c.take<int>(3 * (size_t)P.M);
    N.cls = c.take<int>(3 * (size_t)P.R_N);  // term classes of each mode's kernel vectors
    N.cw = c.take<double>(T);
    N.G = c.take<double>(3 * T * P.R_f * P.R_f);
    N.bytes = c.used;
    return N;
}

size_t tc_nuclear_workspace_bytes(const tc_nuclear_problem *prob)
{
    if (!prob || !nuclear_ok(*prob))
        return (size_t)-1;
    return plan_nuclear(nullptr, *prob).bytes;
}

tc_status tc_nuclear(const tc_nuclear_problem *prob, void *ws, size_t ws_bytes, void *stream)
{
    if (!prob || !nuclear_ok(*prob))
        return TC_ERR_INVALID_ARG;
    const tc_nuclear_problem &P = *prob;
    const NuclearPlan N = plan_nuclear(ws, P);
    if (!ws || ws_bytes < N.bytes)
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    tc_status f = finite_inputs({{P.c, P.R_N}}, st);
    for (int l = 0; l < 3 && f == TC_OK; ++l)
        f = finite_inputs({{P.p[l], (long)P.R_N * (2L * P.n[l] - 1)},
                           {P.U[l], (long)P.R_f * P.n[l]}}, st);
    if (f != TC_OK)
        return f;
    const double inv_vol = 1.0 / (P.h[0] * P.h[1] * P.h[2]);
    for (int base = 0; base < P.M; base += kNuclearChunk) {
        NuclearChunk ch{};
        ch.base = base;
        ch.count = std::min(kNuclearChunk, P.M - base);
        for (int a = 0; a < ch.count; ++a) {
            ch.Z[a] = P.Z[base + a];
            for (int l = 0; l < 3; ++l)
                ch.pos[l][a] = P.pos[3 * (base + a) + l];
        }
        TRYK("nuclear_table",
             launch_nuclear_table(ch, P.c, P.R_N, P.M, inv_vol, N.shift, N.cw, st));
    }
    const size_t plane = (size_t)P.M * P.R_N * P.R_f * P.R_f;
    for (int l = 0; l < 3; ++l) {
        // narrow terms' Grams sum only over the cells near their nuclei
        TRYK("term_class", launch_term_class(P.p[l], P.n[l], P.R_N, N.cls + l * P.R_N, st));
        TRYK("diag_gram_f64", launch_diag_gram_f64(P.U[l], P.p[l], N.shift + l * P.M,
                                                   N.cls + l * P.R_N, N.G + l * plane, P.n[l],
                                                   P.R_f, P.R_N, P.M, false, st));
    }
    TRYK("hadamard_sum", launch_hadamard_sum(N.cw, N.G, N.G + plane, N.G + 2 * plane, P.V, P.R_f,
                                             P.M * P.R_N, st));
    return TC_OK;
}

static bool lattice_ok(int n0, const int *L, int R_N, const double *const *p)
{
    if (n0 < 1 || !L || !p || R_N < 1 || R_N > TC_MAX_RN)
        return false;
    for (int l = 0; l < 3; ++l)
        if (L[l] < 1 || (long)n0 * L[l] > TC_MAX_N || !p[l])
            return false;
    return true;
}

tc_status tc_lattice_sum(int n0, const int *L, int R_N, const double *const *p_dev,
                         double *const *A_dev, void *stream)
{
    if (!lattice_ok(n0, L, R_N, p_dev) || !A_dev || !A_dev[0] || !A_dev[1] || !A_dev[2])
        return TC_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    TRYK("lattice_sum", launch_lattice_sum(n0, L, R_N, p_dev, A_dev, st));
    return TC_OK;
}

tc_status tc_lattice_energy(int n0, const int *L, int R_N, const double *c_dev, const double *h,
                            const double *const *p_dev, double Z, double *E_host, void *ws,
                            size_t ws_bytes, void *stream)
{
    if (!lattice_ok(n0, L, R_N, p_dev) || !c_dev || !h || !E_host || !std::isfinite(Z))
        return TC_ERR_INVALID_ARG;
    for (int l = 0; l < 3; ++l)
        if (!(h[l] > 0.0) || !std::isfinite(h[l]))
            return TC_ERR_INVALID_ARG;
    if (!ws || ws_bytes < sizeof(double) * ((size_t)R_N + 1))
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    double *term = (double *)ws;
    double *E = term + R_N;
    TRYK("lattice_energy", launch_lattice_energy(n0, L, R_N, c_dev, h, p_dev, Z, term, E, st));
    if (hipMemcpyAsync(E_host, E, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return TC_ERR_HIP;
    return TC_OK;
}

size_t tc_coulomb_workspace_bytes(const tc_density *prob, tc_precision prec)
{
    if (!prob || !prec_known(prec))
        return (size_t)-1;
    for (int l = 0; l < 3; ++l)
        if (!size_ok(prob->n[l], prob->R_f, prob->R_N) ||
            !size_ok(prob->n[l], prob->R_rho, prob->R_N))
            return (size_t)-1;
    return plan_density(nullptr, *prob).bytes;
}

tc_status tc_coulomb(const tc_density *prob, tc_precision prec, void *ws, size_t ws_bytes,
                     void *stream)
{
    if (!prob || !prec_known(prec) || !density_ok(*prob))
        return TC_ERR_INVALID_ARG;
    if (prec != TC_FP64)
        return TC_ERR_UNSUPPORTED;
    const tc_density &D = *prob;
    const DensityPlan P = plan_density(ws, D);
    if (!ws || ws_bytes < P.bytes)
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    tc_status f = finite_inputs({{D.c, D.R_N}, {D.d, D.R_rho}}, st);
    for (int l = 0; l < 3 && f == TC_OK; ++l)
        f = finite_inputs({{D.p[l], (long)D.R_N * (2L * D.n[l] - 1)},
                           {D.U[l], (long)D.R_f * D.n[l]},
                           {D.V[l], (long)D.R_rho * D.n[l]}}, st);
    if (f != TC_OK)
        return f;
    const size_t plane = (size_t)D.R_N * D.R_f * D.R_rho;
    for (int l = 0; l < 3; ++l) {
        // the factors T_q V of the Hartree potential, then their scalar
        // products with the product functions
        const tc_status r = mode_W(TC_FP64, resolve(D.n[l], D.R_rho, D.R_N, TC_FP64), D.n[l],
                                   D.R_rho, D.R_N, D.p[l], D.V[l], P.W, P.ms[l], st);
        if (r != TC_OK)
            return r;
        TRYK("cross_gram_f64", launch_cross_gram_f64(D.U[l], P.W, P.H + l * plane, D.n[l],
                                                     D.R_f, D.R_rho, D.R_N, st));
    }
    TRYK("coulomb_reduce",
         launch_coulomb_reduce(D.c, D.d, P.H, D.R_f, D.R_rho, D.R_N, D.Jd, st));
    return TC_OK;
}

tc_status tc_tei_gram(const tc_instance *inst, int count, tc_precision prec, void *ws,
                      size_t ws_bytes, void *stream)
{
    return tc::tei_gram_call(inst, count, prec, ws, ws_bytes, stream);
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
        const tc_instance &I = inst[i];
        const long F2 = (long)I.R_f * I.R_f;
        tc_status f = finite_instance(I, (hipStream_t)stream);
        if (f == TC_OK)
            f = finite_inputs({{Jbar[i], F2}, {I.G_saved, I.G_saved ? 3L * I.R_N * F2 : 0}},
                              (hipStream_t)stream);
        if (f != TC_OK)
            return f;
    }
    for (int i = 0; i < count; ++i) {
        const tc_status s =
            backward_instance(inst[i], Jbar[i], dU + 3 * i, prec, ws, (hipStream_t)stream);
        if (s != TC_OK)
            return s;
    }
    return TC_OK;
}

tc_status tc_autotune(const tc_instance *inst, int count, tc_precision prec, void *ws,
                      size_t ws_bytes, void *stream, double *ms_out)
{
    if (!inst || count < 1 || !prec_known(prec))
        return TC_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i)
        if (!instance_ok(inst[i]))
            return TC_ERR_INVALID_ARG;
    if (!prec_supported(prec))
        return TC_ERR_UNSUPPORTED;
    // the Grams of the measurement runs go to the workspace, never to G_saved
    const size_t need = tc_workspace_bytes(TC_OP_AUTOTUNE, inst, count, prec);
    if (!ws || ws_bytes < need)
        return TC_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return TC_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return TC_ERR_HIP;
    }
    tc_status status = TC_OK;
    std::map<TuneKey, std::pair<double, double>> measured;
    for (int i = 0; i < count && status == TC_OK; ++i) {
        const tc_instance &I = inst[i];
        // scratch Grams: never the caller's G_saved
        tc_instance scratchI = I;
        scratchI.G_saved = nullptr;
        const InstancePlan P = plan_instance(ws, scratchI, prec, false);
        for (int l = 0; l < 3 && status == TC_OK; ++l) {
            const TuneKey key(I.n[l], I.R_f, I.R_N, (int)prec);
            auto it = measured.find(key);
            if (it == measured.end()) {
                double ms[2] = {-1.0, -1.0};
                const tc_algorithm cand[2] = {TC_ALGO_DIRECT, TC_ALGO_FFT};
                for (int a = 0; a < 2 && status == TC_OK; ++a) {
                    if (cand[a] == TC_ALGO_FFT && !fft_any(I.n[l]))
                        continue;
                    for (int rep = 0; rep < 4 && status == TC_OK; ++rep) {
                        if (rep == 1 && hipEventRecord(e0, st) != hipSuccess)
                            status = TC_ERR_HIP;
                        if (status == TC_OK)
                            status = mode_grams(prec, cand[a], I.n[l], I.R_f, I.R_N, I.p[l],
                                                I.U[l], P.W[l], P.G, P.ms[l], st);
                    }
                    float t = 0.0f;
                    if (status == TC_OK &&
                        (hipEventRecord(e1, st) != hipSuccess ||
                         hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                        status = TC_ERR_HIP;
                    ms[a] = t / 3.0;
                }
                it = measured.emplace(key, std::make_pair(ms[0], ms[1])).first;
                if (status == TC_OK) {
                    const bool fft_wins = ms[1] >= 0.0 && ms[1] < ms[0];
                    std::lock_guard<std::mutex> lk(g_tune_mu);
                    g_tune[key] = fft_wins ? (int)TC_ALGO_FFT : (int)TC_ALGO_DIRECT;
                }
            }
            if (ms_out) {
                ms_out[(i * 3 + l) * 2 + 0] = it->second.first;
                ms_out[(i * 3 + l) * 2 + 1] = it->second.second;
            }
        }
    }
    if (status == TC_OK && count > 1 && prec == TC_OZAKI_I8) {
        // the whole batch on every route: copies of the instances with J in
        // the workspace (the callers' J stay untouched) and no saved Grams
        std::vector<tc_instance> cp(inst, inst + count);
        size_t off = 0;
        for (tc_instance &I : cp) {
            I.G_saved = nullptr;
            I.J = (double *)((char *)ws + off);
            off += align_up(sizeof(double) * (size_t)I.R_f * I.R_f);
        }
        void *bws = (char *)ws + off;
        const size_t bbytes = ws_bytes - off;
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (!pool_init())
            status = TC_ERR_HIP;
        float best = -1.0f;
        int best_route = TC_BATCH_FORK_JOIN;
        for (int route = TC_BATCH_FORK_JOIN; route <= TC_BATCH_QUEUE_T64_K2 && status == TC_OK;
             ++route) {
            for (int rep = 0; rep < 3 && status == TC_OK; ++rep) {
                if (rep == 1 && hipEventRecord(e0, st) != hipSuccess)
                    status = TC_ERR_HIP;
                if (status == TC_OK)
                    status = queue_route(route)
                                 ? forward_batch_queue(cp.data(), count, prec, route, bws, bbytes,
                                                       st)
                                 : forward_batch_fork_join(cp.data(), count, prec, bws, bbytes, st);
            }
            float t = 0.0f;
            if (status == TC_OK &&
                (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                 hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                status = TC_ERR_HIP;
            if (status == TC_OK && (best < 0.0f || t < best)) {
                best = t;
                best_route = route;
            }
        }
        if (status == TC_OK) {
            std::lock_guard<std::mutex> lt(g_tune_mu);
            g_batch_tune[batch_signature(inst, count, prec)] = best_route;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}


tc_status tc_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return TC_OK;
}

int tc_profile_read(int max_kernels, char (*names)[64], double *total_ms, long *calls)
{
    std::vector<ProfRecord> recs;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        recs.swap(g_prof_pending);
    }
    std::map<std::string, std::pair<double, long>> tot;
    int status = 0;
    for (const ProfRecord &r : recs) {
        float ms = 0.0f;
        if (hipEventSynchronize(r.e1) != hipSuccess ||
            hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess)
            status = -1;
        auto &e = tot[r.name];
        e.first += ms;
        e.second += 1;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        for (const ProfRecord &r : recs) {
            g_prof_pool.push_back(r.e0);
            g_prof_pool.push_back(r.e1);
        }
    }
    if (status != 0)
        return -1;
    int i = 0;
    for (const auto &kv : tot) {
        if (i >= max_kernels)
            break;
        if (names) {
            std::snprintf(names[i], 64, "%s", kv.first.c_str());
        }
        if (total_ms)
            total_ms[i] = kv.second.first;
        if (calls)
            calls[i] = kv.second.second;
        ++i;
    }
    return (int)tot.size();
}

}  // extern "C"
