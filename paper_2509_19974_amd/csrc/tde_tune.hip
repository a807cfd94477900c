// Engine and tile selection for TDE_PATH_AUTO: a tuning table measured on the
// device (tde_tune), saved and loaded as text, with a cost model and a tile
// rule as the default.
//
// Buckets: m = round(log2(max(nu, nv))) clamped to [10, 23]; lag class by the
// fraction of the full linear range requested (narrow <= 1/16, part <= 1/2,
// full above); code class by Ku Kv (ternary = 1, small <= 49, large). Each
// bucket holds the engine that ran fastest on codes of that class, and for
// the matrix-core engine its tile width (4 or 8 accumulator blocks: 4096 or
// 8192 lags per tile); the engine is only taken where it applies to the
// request, and the tile width applies to any matrix-core correlation of the
// bucket (also one forced by the caller's path).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "tde_internal.h"

namespace tde {

namespace {

constexpr int kMinLog = 10, kMaxLog = 23;
constexpr int kNB = kMaxLog - kMinLog + 1;

struct Table {
    bool valid = false;
    int eng[3][3][kNB] = {};   // [code class][lag class][size bucket], 0 = unset
    int tb[3][3][kNB] = {};    // matrix-core tile blocks (4 or 8), 0 = the rule
};

std::mutex g_mu;
Table g_tab;
// while tde_tune measures a tile width (its own thread only)
thread_local int t_force_tb = 0;

int size_bucket(int64_t nu, int64_t nv) {
    const double m = std::log2((double)std::max(nu, nv));
    return std::clamp((int)std::lround(m), kMinLog, kMaxLog) - kMinLog;
}

int lag_class(int64_t nu, int64_t nv, int64_t lag_lo, int64_t lag_hi) {
    const double f = (double)(lag_hi - lag_lo + 1) / (double)(nu + nv - 1);
    return f <= 1.0 / 16 ? 0 : (f <= 0.5 ? 1 : 2);
}

int code_class(int kuv) { return kuv == 1 ? 0 : (kuv <= 49 ? 1 : 2); }

// Approximate sum over tau in [lo, hi] of the overlap (the multiply-adds of
// a direct engine): the overlap is piecewise linear, integrated per piece.
double overlap_sum(int64_t nu, int64_t nv, int64_t lo, int64_t hi) {
    lo = std::max<int64_t>(lo, -(nu - 1));
    hi = std::min<int64_t>(hi, nv - 1);
    if (lo > hi) return 0.0;
    auto ov = [&](int64_t t) {
        return (double)(std::min(nu, nv - t) - std::max<int64_t>(0, -t));
    };
    int64_t br[4] = {lo, std::clamp<int64_t>(0, lo, hi), std::clamp<int64_t>(nv - nu, lo, hi), hi};
    std::sort(br, br + 4);
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const int64_t a = br[k], b = br[k + 1];
        if (b > a) s += 0.5 * (ov(a) + ov(b)) * (double)(b - a);   // linear on [a, b]
    }
    return s + 0.5 * (ov(br[0]) + ov(br[3]));
}

// Default when no table is installed: seconds from rates measured on MI355X
// (matrix-core engine ~1.17e15 MAC/s with int8 operands and ~1.9e15 with
// FP4/FP6 operands on 64 x 65536 batches; bit-plane engine ~1.5e14 MAC/s;
// transform engine ~4e-11 s per residue and prime of the transform length).
int model_choice(int64_t nu, int64_t nv, int kuv, int kmax, int64_t lo, int64_t hi) {
    const double macs = overlap_sum(nu, nv, lo, hi);
    const double rate = mfma_choose_fmt(kmax, true) == kFmtI8 ? 1.17e15 : 1.9e15;
    double best = macs / rate + 4e-6;
    int eng = TDE_PATH_MFMA;
    NttPlan P;
    if (ntt_plan(nu, nv, kuv, lo, hi, P)) {
        const double t = 4e-11 * (double)P.nprimes * (double)((int64_t)1 << P.log_n) + 12e-6;
        if (t < best) {
            best = t;
            eng = TDE_PATH_NTT;
        }
    }
    return eng;
}

bool applicable(int eng, int64_t nu, int64_t nv, int kuv, int64_t lo, int64_t hi) {
    if (eng == TDE_PATH_MFMA) return true;
    if (eng == TDE_PATH_POPC) return kuv == 1;
    if (eng == TDE_PATH_NTT) {
        NttPlan P;
        return ntt_plan(nu, nv, kuv, lo, hi, P);
    }
    return false;
}

uint32_t lcg(uint64_t& s) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(s >> 33);
}

}  // namespace

int tuned_tile_blocks(int64_t nu, int64_t nv, int kuv, int64_t lag_lo, int64_t lag_hi) {
    if (t_force_tb) return t_force_tb;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_tab.valid) return 0;
    return g_tab.tb[code_class(kuv)][lag_class(nu, nv, lag_lo, lag_hi)][size_bucket(nu, nv)];
}

int auto_engine(int64_t nu, int64_t nv, int kuv, int kmax, int64_t lag_lo, int64_t lag_hi) {
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (g_tab.valid) {
            const int e = g_tab.eng[code_class(kuv)][lag_class(nu, nv, lag_lo, lag_hi)][size_bucket(nu, nv)];
            if (e && applicable(e, nu, nv, kuv, lag_lo, lag_hi)) return e;
        }
    }
    return model_choice(nu, nv, kuv, kmax, lag_lo, lag_hi);
}

}  // namespace tde

using namespace tde;

extern "C" {

int tde_tune_query(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi) {
    if (nu < 1 || nv < 1 || lag_lo > lag_hi || kmax_u < 1 || kmax_u > 127 || kmax_v < 1 || kmax_v > 127)
        return set_error(TDE_ERR_ARG, "tde_tune_query: invalid request");
    return auto_engine(nu, nv, kmax_u * kmax_v, kmax_u > kmax_v ? kmax_u : kmax_v, lag_lo, lag_hi);
}

int tde_tune_reset(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    g_tab = Table{};
    return TDE_OK;
}

int tde_tune_save(const char* path) {
    if (!path) return set_error(TDE_ERR_ARG, "tde_tune_save: null path");
    Table t;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        t = g_tab;
    }
    if (!t.valid) return set_error(TDE_ERR_ARG, "tde_tune_save: no tuning table installed");
    FILE* f = fopen(path, "w");
    if (!f) return set_error(TDE_ERR_IO, "tde_tune_save: cannot open %s", path);
    fprintf(f, "tde-tune 2\n");
    for (int c = 0; c < 3; ++c)
        for (int l = 0; l < 3; ++l)
            for (int b = 0; b < kNB; ++b)
                if (t.eng[c][l][b])
                    fprintf(f, "%d %d %d %d %d\n", c, l, b + kMinLog, t.eng[c][l][b], t.tb[c][l][b]);
    const bool ok = fclose(f) == 0;
    return ok ? TDE_OK : set_error(TDE_ERR_IO, "tde_tune_save: write to %s failed", path);
}

int tde_tune_load(const char* path) {
    if (!path) return set_error(TDE_ERR_ARG, "tde_tune_load: null path");
    FILE* f = fopen(path, "r");
    if (!f) return set_error(TDE_ERR_IO, "tde_tune_load: cannot open %s", path);
    Table t;
    char head[32] = {0};
    int ver = 0;
    if (fscanf(f, "%31s %d", head, &ver) != 2 || strcmp(head, "tde-tune") != 0 || (ver != 1 && ver != 2)) {
        fclose(f);
        return set_error(TDE_ERR_IO, "tde_tune_load: %s is not a tuning file", path);
    }
    // version 1 lines: code lag log2n engine; version 2 adds the tile blocks
    const int fields = ver == 1 ? 4 : 5;
    int c, l, m, e, tb = 0, n = 0;
    int got;
    while ((got = ver == 1 ? fscanf(f, "%d %d %d %d", &c, &l, &m, &e)
                           : fscanf(f, "%d %d %d %d %d", &c, &l, &m, &e, &tb)) == fields) {
        if (c < 0 || c > 2 || l < 0 || l > 2 || m < kMinLog || m > kMaxLog || e < TDE_PATH_MFMA ||
            e > TDE_PATH_NTT || (tb != 0 && tb != 4 && tb != 8)) {
            fclose(f);
            return set_error(TDE_ERR_IO, "tde_tune_load: bad entry %d %d %d %d %d in %s", c, l, m, e, tb, path);
        }
        t.eng[c][l][m - kMinLog] = e;
        t.tb[c][l][m - kMinLog] = tb;
        ++n;
    }
    const bool clean_end = got == EOF;
    fclose(f);
    if (!clean_end) return set_error(TDE_ERR_IO, "tde_tune_load: trailing garbage in %s", path);
    t.valid = n > 0;
    std::lock_guard<std::mutex> lock(g_mu);
    g_tab = t;
    return TDE_OK;
}

}  // extern "C"

namespace {

struct TuneBufs {
    float* x = nullptr;
    float* y = nullptr;
    tde_peak* out = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneBufs() {
        if (x) (void)hipFree(x);
        if (y) (void)hipFree(y);
        if (out) (void)hipFree(out);
        if (ws) (void)hipFree(ws);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

constexpr int kTunePairs = 512;     // most pairs of one bucket's batch

// Seconds per pair of engine e on a batch of P identical pairs (the way the
// batch call runs it: one persistent launch over all their tiles), the mean
// of two calls after one warm-up call.
int time_engine(tde_ctx* ctx, TuneBufs& B, int64_t N, int bits, int64_t half, int P, int e, hipStream_t s,
                double* out_s) {
    std::vector<tde_pair> pairs(P);
    for (auto& q : pairs) {
        q = tde_pair{};
        q.x = B.x;
        q.y = B.y;
        q.nx = N;
        q.ny = N;
        q.lag_lo = -half;
        q.lag_hi = half;
        q.bits = bits;
    }
    tde_opts o{TDE_MODE_FULL, e, 0, 0, nullptr, 0.f, TDE_QUANT_UNIFORM};
    const size_t need = tde_estimate_workspace_size(pairs.data(), P, &o);
    if (need == 0) return set_error(TDE_ERR_ARG, "tde_tune: cannot plan bucket");
    if (need > B.ws_bytes) {
        if (B.ws) (void)hipFree(B.ws);
        B.ws = nullptr;
        B.ws_bytes = 0;
        if (hipMalloc(&B.ws, need) != hipSuccess) return set_error(TDE_ERR_HIP, "tde_tune: workspace allocation");
        B.ws_bytes = need;
    }
    float tot = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
        float ms = 0.f;
        TDE_HIP_CHECK(hipEventRecord(B.e0, s));
        const int st = tde_estimate_batch(ctx, pairs.data(), P, &o, B.out, B.ws, B.ws_bytes, s);
        if (st != TDE_OK) return st;
        TDE_HIP_CHECK(hipEventRecord(B.e1, s));
        TDE_HIP_CHECK(hipEventSynchronize(B.e1));
        TDE_HIP_CHECK(hipEventElapsedTime(&ms, B.e0, B.e1));
        if (rep > 0) tot += ms;
    }
    *out_s = tot / 2 * 1e-3 / P;
    return TDE_OK;
}

}  // namespace

extern "C" {

int tde_tune(tde_ctx* ctx, int max_log_n, void* stream) {
    if (max_log_n < kMinLog || max_log_n > 22) return set_error(TDE_ERR_ARG, "tde_tune: max_log_n in [10, 22]");
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_tune: null context");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nmax = (int64_t)1 << max_log_n;
    int prev = -1;
    TDE_HIP_CHECK(hipGetDevice(&prev));
    TDE_HIP_CHECK(hipSetDevice(ctx_device(ctx)));
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev};
    TuneBufs B;
    TDE_HIP_CHECK(hipMalloc(&B.x, nmax * sizeof(float)));
    TDE_HIP_CHECK(hipMalloc(&B.y, nmax * sizeof(float)));
    TDE_HIP_CHECK(hipMalloc(&B.out, kTunePairs * sizeof(tde_peak)));
    TDE_HIP_CHECK(hipEventCreate(&B.e0));
    TDE_HIP_CHECK(hipEventCreate(&B.e1));
    {
        // two independent noise signals (sums of uniforms from a host LCG)
        std::vector<float> hx(nmax), hy(nmax);
        uint64_t seed = 0x2509199740ull;
        for (int64_t k = 0; k < nmax; ++k) {
            hx[k] = (float)(lcg(seed) % 2001u) + (float)(lcg(seed) % 2001u) - 2000.f;
            hy[k] = (float)(lcg(seed) % 2001u) + (float)(lcg(seed) % 2001u) - 2000.f;
        }
        TDE_HIP_CHECK(hipMemcpy(B.x, hx.data(), nmax * sizeof(float), hipMemcpyHostToDevice));
        TDE_HIP_CHECK(hipMemcpy(B.y, hy.data(), nmax * sizeof(float), hipMemcpyHostToDevice));
    }
    Table t;
    const int cls_bits[3] = {1, 4, 8};          // one quantizer per code class
    for (int c = 0; c < 3; ++c) {
        const int bits = cls_bits[c];
        const int K = kmax_of_bits(bits);
        for (int m = kMinLog; m <= max_log_n; ++m) {
            const int64_t N = (int64_t)1 << m;
            for (int l = 0; l < 3; ++l) {
                const int64_t half = l == 0 ? std::max<int64_t>(16, N / 64) : (l == 1 ? N / 4 : N - 1);
                // enough pairs for about 2^38 multiply-adds (0.1 - 0.3 ms of
                // the matrix cores) and at least 2048 matrix-core work items
                // (8 per CU), so that the timing reflects a full device
                // rather than a few long items; at most kTunePairs
                const double macs = overlap_sum(N, N, -half, half);
                XItem probe{};
                probe.p.nu = N;
                probe.p.nv = N;
                probe.p.lag_lo = -half;
                probe.p.lag_hi = half;
                probe.p.kuv = K * K;
                probe.p.kmax = K;
                t_force_tb = 4;
                mfma_plan_pair(probe, true);
                t_force_tb = 0;
                const double items = (double)std::max<int64_t>(1, mfma_count_items(probe));
                const double want = std::max(274877906944.0 / std::max(macs, 1.0), 2048.0 / items);
                const int P = (int)std::clamp(std::ceil(want), 1.0, (double)kTunePairs);
                double best = 1e30, best_mfma = 1e30;
                int best_e = 0, best_tb = 0;
                // the matrix-core engine at both tile widths (int8 codes at 8
                // blocks take a launch of their own, one wave per SIMD), then
                // the other engines
                const int trials[4][2] = {{TDE_PATH_MFMA, 4}, {TDE_PATH_MFMA, 8}, {TDE_PATH_POPC, 0},
                                          {TDE_PATH_NTT, 0}};
                for (const auto& tr : trials) {
                    const int e = tr[0];
                    if (!applicable(e, N, N, K * K, -half, half)) continue;
                    double sec = 0.0;
                    t_force_tb = tr[1];
                    const int st = time_engine(ctx, B, N, bits, half, P, e, s, &sec);
                    t_force_tb = 0;
                    if (st != TDE_OK) return st;
                    if (e == TDE_PATH_MFMA && sec < best_mfma) {
                        best_mfma = sec;
                        best_tb = tr[1];
                    }
                    if (sec < best) {
                        best = sec;
                        best_e = e;
                    }
                }
                t.eng[c][l][m - kMinLog] = best_e;
                t.tb[c][l][m - kMinLog] = best_tb;
            }
        }
    }
    // sizes beyond the measured range take the largest measured bucket
    for (int c = 0; c < 3; ++c)
        for (int l = 0; l < 3; ++l)
            for (int m = max_log_n + 1; m <= kMaxLog; ++m) {
                t.eng[c][l][m - kMinLog] = t.eng[c][l][max_log_n - kMinLog];
                t.tb[c][l][m - kMinLog] = t.tb[c][l][max_log_n - kMinLog];
            }
    t.valid = true;
    std::lock_guard<std::mutex> lock(g_mu);
    g_tab = t;
    return TDE_OK;
}

}  // extern "C"
