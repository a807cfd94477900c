// C ABI of libtde.so (include/tde.h): argument validation, workspace layout,
// engine selection and launch sequencing. Every step of the estimator runs
// in the HIP kernels of this library; this file only plans and queues them.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "tde_internal.h"

struct tde_ctx {
    int device;
    int num_cu;
    // pinned staging for batch descriptors (host -> workspace copies)
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    std::mutex mu;
    // stage timing (measurement only)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Mark {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
};

namespace tde {

static thread_local char g_err[512] = "";

int set_error(int status, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return status;
}

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int64_t overlap(int64_t nu, int64_t nv, int64_t tau) {
    int64_t hi = std::min(nu, nv - tau), lo = std::max<int64_t>(0, -tau);
    return hi > lo ? hi - lo : 0;
}

// Largest overlap over [lo, hi]; overlap(tau) is concave, so its maximum over
// an interval is at an end or at a clamped corner of its plateau [0, nv-nu].
int64_t max_overlap(int64_t nu, int64_t nv, int64_t lo, int64_t hi) {
    int64_t c[4] = {lo, hi, std::clamp<int64_t>(0, lo, hi), std::clamp<int64_t>(nv - nu, lo, hi)};
    int64_t m = 0;
    for (int64_t t : c) m = std::max(m, overlap(nu, nv, t));
    return m;
}

bool valid_bits(int b) { return b == 1 || b == 2 || b == 4 || b == 8; }

// Bump allocator over the caller's workspace.
struct Carve {
    uint8_t* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<uint8_t*>(b)) {}
    void* take(size_t bytes) {
        void* p = base ? base + off : nullptr;
        off += align_bytes(bytes);
        return p;
    }
};

int upload(tde_ctx* ctx, void* dst_dev, const void* src_host, size_t bytes, hipStream_t s) {
    if (bytes == 0) return TDE_OK;
    if (ctx->upload_pending) {
        TDE_HIP_CHECK(hipEventSynchronize(ctx->upload_done));
        ctx->upload_pending = false;
    }
    if (bytes > ctx->pinned_bytes) {
        if (ctx->pinned) TDE_HIP_CHECK(hipHostFree(ctx->pinned));
        ctx->pinned = nullptr;
        size_t nb = std::max<size_t>(bytes, 1 << 20);
        TDE_HIP_CHECK(hipHostMalloc(&ctx->pinned, nb, hipHostMallocDefault));
        ctx->pinned_bytes = nb;
    }
    memcpy(ctx->pinned, src_host, bytes);
    TDE_HIP_CHECK(hipMemcpyAsync(dst_dev, ctx->pinned, bytes, hipMemcpyHostToDevice, s));
    TDE_HIP_CHECK(hipEventRecord(ctx->upload_done, s));
    ctx->upload_pending = true;
    return TDE_OK;
}

hipEvent_t timing_event(tde_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// Records an event on s when timing is on; returns it (or null).
hipEvent_t mark(tde_ctx* c, hipStream_t s) {
    if (!c->timing) return nullptr;
    hipEvent_t e = timing_event(c);
    if (e) (void)hipEventRecord(e, s);
    return e;
}

void mark_stage(tde_ctx* c, int stage, hipEvent_t a, hipEvent_t b) {
    if (c->timing && a && b) c->marks.push_back({stage, a, b});
}

// Engine choice for one correlation. The direct engines are exact for every
// size; the bit-plane engine only takes ternary codes.
int choose_path(int path, int kuv) {
    if (path != TDE_PATH_AUTO) return path;
    (void)kuv;
    return TDE_PATH_MFMA;
}

}  // namespace
}  // namespace tde

using namespace tde;

extern "C" {

const char* tde_status_string(int status) {
    switch (status) {
        case TDE_OK: return "ok";
        case TDE_ERR_ARG: return "invalid argument";
        case TDE_ERR_RANGE: return "int32 result cannot hold the exact correlation";
        case TDE_ERR_WS: return "workspace missing or too small";
        case TDE_ERR_HIP: return "HIP runtime error";
        case TDE_ERR_UNSUPPORTED: return "unsupported request";
        case TDE_ERR_IO: return "file I/O error";
        default: return "unknown status";
    }
}

const char* tde_last_error(void) { return g_err; }

int tde_create(tde_ctx** out, int device) {
    if (!out) return set_error(TDE_ERR_ARG, "tde_create: null output pointer");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0)
        return set_error(TDE_ERR_HIP, "tde_create: no HIP device");
    if (device < 0 || device >= n) return set_error(TDE_ERR_ARG, "tde_create: device %d of %d", device, n);
    hipDeviceProp_t prop;
    TDE_HIP_CHECK(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(TDE_ERR_UNSUPPORTED, "tde_create: device %d is %s, this library is built for gfx950",
                         device, prop.gcnArchName);
    tde_ctx* c = new tde_ctx();
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    {
        DeviceGuard g(device);
        if (hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess) {
            delete c;
            return set_error(TDE_ERR_HIP, "tde_create: event creation failed");
        }
    }
    *out = c;
    return TDE_OK;
}

int tde_timing_enable(tde_ctx* c, int on) {
    if (!c) return set_error(TDE_ERR_ARG, "tde_timing_enable: null context");
    std::lock_guard<std::mutex> lock(c->mu);
    c->timing = on != 0;
    return TDE_OK;
}

int tde_timing_read(tde_ctx* c, double* ms, int64_t* count) {
    if (!c || !ms || !count) return set_error(TDE_ERR_ARG, "tde_timing_read: null pointer");
    std::lock_guard<std::mutex> lock(c->mu);
    DeviceGuard g(c->device);
    for (int k = 0; k < 4; ++k) {
        ms[k] = 0.0;
        count[k] = 0;
    }
    for (auto& m : c->marks) {
        TDE_HIP_CHECK(hipEventSynchronize(m.b));
        float t = 0.f;
        TDE_HIP_CHECK(hipEventElapsedTime(&t, m.a, m.b));
        ms[m.stage] += t;
        count[m.stage] += 1;
    }
    c->marks.clear();
    c->ev_used = 0;
    return TDE_OK;
}

void tde_destroy(tde_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->upload_pending) (void)hipEventSynchronize(c->upload_done);
    if (c->upload_done) (void)hipEventDestroy(c->upload_done);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
}

// ------------------------------------------------------------ quantize --

size_t tde_quantize_workspace_size(int64_t n) {
    if (n < 1) return 0;
    return align_bytes((size_t)quantize_gsum_doubles(n) * 8) + align_bytes(4);
}

int tde_quantize(tde_ctx* ctx, const float* x, int64_t n, int bits, float inv_step, int8_t* q,
                 tde_qstat* stat, void* ws, size_t ws_bytes, void* stream) {
    if (!x || !q) return set_error(TDE_ERR_ARG, "tde_quantize: null x or q");
    if (n < 1) return set_error(TDE_ERR_ARG, "tde_quantize: n = %lld < 1", (long long)n);
    if (!valid_bits(bits)) return set_error(TDE_ERR_ARG, "tde_quantize: bits = %d not in {1,2,4,8}", bits);
    if (!std::isfinite(inv_step)) return set_error(TDE_ERR_ARG, "tde_quantize: inv_step is not finite");
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_quantize: null context");
    const bool need_scale = bits != 1 && !(inv_step > 0.f);
    QSig one{};
    one.x = x;
    one.n = n;
    one.q = q;
    one.stat = stat;
    one.bits = bits;
    one.inv_fixed = (bits != 1 && inv_step > 0.f) ? inv_step : 0.f;
    if (need_scale) {
        size_t need = tde_quantize_workspace_size(n);
        if (!ws || ws_bytes < need)
            return set_error(TDE_ERR_WS, "tde_quantize: workspace %zu < %zu bytes", ws_bytes, need);
        Carve cv(ws);
        one.gsum = static_cast<double*>(cv.take((size_t)quantize_gsum_doubles(n) * 8));
        one.inv_out = static_cast<float*>(cv.take(4));
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_quantize: hipSetDevice failed");
    return launch_quantize(nullptr, one, 1, ceil_div(n, 256), ceil_div(n, kQuantBlock), need_scale,
                           static_cast<hipStream_t>(stream));
}

// --------------------------------------------------------- correlation --

static int check_xcorr(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int kmax_u, int kmax_v,
                       int64_t lag_lo, int64_t lag_hi, const void* r, int r_dtype, int path, const char* who) {
    if (!u || !v || !r) return set_error(TDE_ERR_ARG, "%s: null pointer", who);
    if (nu < 1 || nv < 1) return set_error(TDE_ERR_ARG, "%s: empty signal", who);
    if (lag_lo > lag_hi) return set_error(TDE_ERR_ARG, "%s: lag_lo > lag_hi", who);
    if (lag_hi - lag_lo + 1 > ((int64_t)1 << 40)) return set_error(TDE_ERR_ARG, "%s: lag range too large", who);
    if (kmax_u < 1 || kmax_u > 127 || kmax_v < 1 || kmax_v > 127)
        return set_error(TDE_ERR_ARG, "%s: kmax must be in [1, 127]", who);
    if (r_dtype != TDE_I32 && r_dtype != TDE_I64) return set_error(TDE_ERR_ARG, "%s: bad r_dtype", who);
    if (((uintptr_t)r) & (r_dtype == TDE_I32 ? 3 : 7))
        return set_error(TDE_ERR_ARG, "%s: r is not aligned to its element size", who);
    if (path < TDE_PATH_AUTO || path > TDE_PATH_NTT) return set_error(TDE_ERR_ARG, "%s: bad path", who);
    if (path == TDE_PATH_POPC && (kmax_u != 1 || kmax_v != 1))
        return set_error(TDE_ERR_ARG, "%s: the bit-plane engine needs ternary codes (kmax 1)", who);
    if (path == TDE_PATH_NTT) return set_error(TDE_ERR_UNSUPPORTED, "%s: NTT engine not available", who);
    if (r_dtype == TDE_I32) {
        const int64_t ov = max_overlap(nu, nv, lag_lo, lag_hi);
        if ((__int128)ov * kmax_u * kmax_v >= ((__int128)1 << 31))
            return set_error(TDE_ERR_RANGE, "%s: overlap %lld x %d x %d does not fit int32", who, (long long)ov,
                             kmax_u, kmax_v);
    }
    return TDE_OK;
}

size_t tde_xcorr_workspace_size(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi,
                                int path) {
    if (nu < 1 || nv < 1 || lag_lo > lag_hi || kmax_u < 1 || kmax_v < 1) return 0;
    XItem it{};
    it.p.nu = nu;
    it.p.nv = nv;
    it.p.lag_lo = lag_lo;
    it.p.lag_hi = lag_hi;
    it.p.kuv = kmax_u * kmax_v;
    int eng = choose_path(path, it.p.kuv);
    if (eng == TDE_PATH_POPC) return popc_ws_bytes(it.p);
    mfma_plan_pair(it);
    return align_bytes((size_t)mfma_count_items(it) * sizeof(MWork)) + align_bytes(2 * sizeof(int));
}

int tde_xcorr_int(tde_ctx* ctx, const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int kmax_u, int kmax_v,
                  int64_t lag_lo, int64_t lag_hi, void* r, int r_dtype, int path, void* ws, size_t ws_bytes,
                  void* stream) {
    int rc = check_xcorr(u, nu, v, nv, kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path, "tde_xcorr_int");
    if (rc) return rc;
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_xcorr_int: null context");
    XItem it{};
    it.engine = choose_path(path, kmax_u * kmax_v);
    it.p.u = u;
    it.p.v = v;
    it.p.nu = nu;
    it.p.nv = nv;
    it.p.lag_lo = lag_lo;
    it.p.lag_hi = lag_hi;
    it.p.r = r;
    it.p.r_dtype = r_dtype;
    it.p.kuv = kmax_u * kmax_v;
    const int eng = choose_path(path, it.p.kuv);
    size_t need = tde_xcorr_workspace_size(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, eng);
    if (need && (!ws || ws_bytes < need))
        return set_error(TDE_ERR_WS, "tde_xcorr_int: workspace %zu < %zu bytes", ws_bytes, need);
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_xcorr_int: hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t rbytes = (lag_hi - lag_lo + 1) * (r_dtype == TDE_I32 ? 4 : 8);
    rc = launch_zero_r(nullptr, it, 1, rbytes, s);
    if (rc) return rc;
    if (eng == TDE_PATH_POPC) {
        popc_plan(it, ws);
        rc = launch_zero(ws, need, s);
        if (rc) return rc;
        rc = launch_popc_pack(nullptr, it, 1, std::max(it.nuw, it.nvw), s);
        if (rc) return rc;
        return launch_xcorr_popc(nullptr, it, 1, it.nsplit, it.ntiles, s);
    }
    mfma_plan_pair(it);
    std::vector<MWork> work;
    mfma_items(it, 0, work);
    mfma_sort_items(work);
    MWork* work_dev = static_cast<MWork*>(ws);
    int* counters = reinterpret_cast<int*>(static_cast<uint8_t*>(ws) +
                                           align_bytes((size_t)mfma_count_items(it) * sizeof(MWork)));
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        rc = upload(ctx, work_dev, work.data(), work.size() * sizeof(MWork), s);
    }
    if (rc) return rc;
    return launch_xcorr_mfma(nullptr, it, work_dev, (int)work.size(), counters, nullptr, ctx->num_cu, s);
}

// -------------------------------------------------------------- argmax --

size_t tde_argmax_workspace_size(int64_t nlags) {
    if (nlags < 1) return 0;
    return align_bytes((size_t)ceil_div(nlags, kArgChunk) * sizeof(ArgPart));
}

int tde_argmax_lag(tde_ctx* ctx, const void* r, int r_dtype, int64_t lag_lo, int64_t lag_hi, tde_peak* out,
                   void* ws, size_t ws_bytes, void* stream) {
    if (!r || !out) return set_error(TDE_ERR_ARG, "tde_argmax_lag: null pointer");
    if (lag_lo > lag_hi) return set_error(TDE_ERR_ARG, "tde_argmax_lag: lag_lo > lag_hi");
    if (r_dtype != TDE_I32 && r_dtype != TDE_I64) return set_error(TDE_ERR_ARG, "tde_argmax_lag: bad r_dtype");
    const int64_t L = lag_hi - lag_lo + 1;
    size_t need = tde_argmax_workspace_size(L);
    if (!ws || ws_bytes < need) return set_error(TDE_ERR_WS, "tde_argmax_lag: workspace %zu < %zu", ws_bytes, need);
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_argmax_lag: null context");
    ArgSeg one{};
    one.r = r;
    one.L = L;
    one.lag_lo = lag_lo;
    one.part_base = 0;
    one.nparts = (int32_t)ceil_div(L, kArgChunk);
    one.dtype = r_dtype;
    one.out = out;
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_argmax_lag: hipSetDevice failed");
    return launch_argmax(nullptr, one, 1, one.nparts, static_cast<ArgPart*>(ws), static_cast<hipStream_t>(stream));
}

// --------------------------------------------------------------- batch --

}  // extern "C"

namespace {

int validate_pairs(const tde_pair* pairs, int64_t np, const tde_opts* opts) {
    if (!pairs || np < 1) return set_error(TDE_ERR_ARG, "tde_estimate_batch: no pairs");
    if (np > 65535) return set_error(TDE_ERR_ARG, "tde_estimate_batch: at most 65535 pairs per call");
    int path = opts ? opts->path : TDE_PATH_AUTO;
    if (opts && opts->mode != TDE_MODE_FULL)
        return set_error(TDE_ERR_UNSUPPORTED, "tde_estimate_batch: only TDE_MODE_FULL is available");
    for (int64_t i = 0; i < np; ++i) {
        const tde_pair& q = pairs[i];
        if (!q.x || !q.y) return set_error(TDE_ERR_ARG, "pair %lld: null signal", (long long)i);
        if (q.nx < 1 || q.ny < 1) return set_error(TDE_ERR_ARG, "pair %lld: empty signal", (long long)i);
        if (q.lag_lo > q.lag_hi) return set_error(TDE_ERR_ARG, "pair %lld: lag_lo > lag_hi", (long long)i);
        if (q.lag_hi - q.lag_lo + 1 > ((int64_t)1 << 31))
            return set_error(TDE_ERR_ARG, "pair %lld: lag range too large", (long long)i);
        if (!valid_bits(q.bits)) return set_error(TDE_ERR_ARG, "pair %lld: bits %d", (long long)i, q.bits);
        if (!std::isfinite(q.inv_step_x) || !std::isfinite(q.inv_step_y))
            return set_error(TDE_ERR_ARG, "pair %lld: non-finite inv_step", (long long)i);
        if (q.r_out) {
            if (q.r_dtype != TDE_I32 && q.r_dtype != TDE_I64)
                return set_error(TDE_ERR_ARG, "pair %lld: bad r_dtype", (long long)i);
            if (((uintptr_t)q.r_out) & (q.r_dtype == TDE_I32 ? 3 : 7))
                return set_error(TDE_ERR_ARG, "pair %lld: r_out misaligned", (long long)i);
            const int K = kmax_of_bits(q.bits);
            if (q.r_dtype == TDE_I32 &&
                (__int128)max_overlap(q.nx, q.ny, q.lag_lo, q.lag_hi) * K * K >= ((__int128)1 << 31))
                return set_error(TDE_ERR_RANGE, "pair %lld: int32 r cannot hold the exact values", (long long)i);
        }
        if (path == TDE_PATH_POPC && q.bits > 2)
            return set_error(TDE_ERR_ARG, "pair %lld: the bit-plane engine needs ternary codes", (long long)i);
        if (path == TDE_PATH_NTT)
            return set_error(TDE_ERR_UNSUPPORTED, "tde_estimate_batch: NTT engine not available");
    }
    return TDE_OK;
}

// Per-pair decisions shared by the workspace size and the launch.
struct PairPlan {
    int eng;            // engine
    int rdt;            // r dtype
    bool fused;         // argmax from tile triples, no r array
    bool need_r;        // r materialized (requested or needed by the argmax kernel)
    XItem probe;        // MFMA plan of the pair (sizes only)
};

PairPlan plan_pair(const tde_pair& q, int path) {
    PairPlan pp{};
    const int K = kmax_of_bits(q.bits);
    pp.eng = choose_path(path, K * K);
    pp.rdt = q.r_out ? q.r_dtype
                     : ((__int128)max_overlap(q.nx, q.ny, q.lag_lo, q.lag_hi) * K * K < ((__int128)1 << 31) ? TDE_I32
                                                                                                          : TDE_I64);
    pp.probe.p.nu = q.nx;
    pp.probe.p.nv = q.ny;
    pp.probe.p.lag_lo = q.lag_lo;
    pp.probe.p.lag_hi = q.lag_hi;
    pp.probe.p.kuv = K * K;
    if (pp.eng == TDE_PATH_MFMA) {
        mfma_plan_pair(pp.probe);
        pp.fused = !pp.probe.segmented;
    } else {
        pp.fused = false;
    }
    pp.need_r = q.r_out != nullptr || !pp.fused;
    return pp;
}

struct BatchPlan {
    size_t total = 0;
    // offsets inside the workspace; [0, off_stats) is uploaded from the host
    size_t off_qsig, off_items, off_segs, off_work, off_counters, off_tparts, off_stats, off_inv, off_parts;
    int64_t nwork = 0, ntparts = 0, nsegs = 0, total_parts = 0;
    std::vector<PairPlan> pp;
    std::vector<size_t> off_q;      // per signal (2 per pair)
    std::vector<size_t> off_gsum;   // per signal
    std::vector<size_t> off_r;      // per pair (r materialized in the workspace)
    std::vector<size_t> off_planes; // per pair (bit-plane engine)
};

BatchPlan plan_batch(const tde_pair* pairs, int64_t np, const tde_opts* opts) {
    BatchPlan B;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_bytes(bytes);
        return o;
    };
    const int path = opts ? opts->path : TDE_PATH_AUTO;
    B.pp.resize(np);
    for (int64_t i = 0; i < np; ++i) {
        B.pp[i] = plan_pair(pairs[i], path);
        const PairPlan& pp = B.pp[i];
        if (pp.eng == TDE_PATH_MFMA) {
            B.nwork += mfma_count_items(pp.probe);
            if (pp.fused) B.ntparts += pp.probe.ntiles;
        }
        if (!pp.fused) {
            B.nsegs += 1;
            B.total_parts += ceil_div(pairs[i].lag_hi - pairs[i].lag_lo + 1, kArgChunk);
        }
    }
    B.off_qsig = take(sizeof(QSig) * 2 * np);
    B.off_items = take(sizeof(XItem) * np);
    B.off_segs = take(sizeof(ArgSeg) * (B.nsegs ? B.nsegs : 1));
    B.off_work = take(sizeof(MWork) * (B.nwork ? B.nwork : 1));
    B.off_counters = take(2 * sizeof(int));
    B.off_tparts = take(sizeof(ArgPart) * (B.ntparts ? B.ntparts : 1));
    B.off_stats = take(sizeof(tde_qstat) * 2 * np);
    B.off_inv = take(sizeof(float) * 2 * np);
    B.off_parts = take(sizeof(ArgPart) * (B.total_parts ? B.total_parts : 1));
    B.off_q.resize(2 * np);
    B.off_gsum.resize(2 * np);
    B.off_r.assign(np, 0);
    B.off_planes.assign(np, 0);
    for (int64_t i = 0; i < np; ++i) {
        const tde_pair& q = pairs[i];
        const PairPlan& pp = B.pp[i];
        B.off_q[2 * i] = take(q.nx);
        B.off_q[2 * i + 1] = take(q.ny);
        B.off_gsum[2 * i] = take((size_t)quantize_gsum_doubles(q.nx) * 8);
        B.off_gsum[2 * i + 1] = take((size_t)quantize_gsum_doubles(q.ny) * 8);
        const int64_t L = q.lag_hi - q.lag_lo + 1;
        if (pp.need_r && !q.r_out) B.off_r[i] = take((size_t)L * (pp.rdt == TDE_I32 ? 4 : 8));
        if (pp.eng == TDE_PATH_POPC) B.off_planes[i] = take(popc_ws_bytes(pp.probe.p));
    }
    B.total = off;
    return B;
}

}  // namespace

extern "C" {

size_t tde_estimate_workspace_size(const tde_pair* pairs, int64_t np, const tde_opts* opts) {
    if (validate_pairs(pairs, np, opts) != TDE_OK) return 0;
    return plan_batch(pairs, np, opts).total;
}

int tde_estimate_batch(tde_ctx* ctx, const tde_pair* pairs, int64_t np, const tde_opts* opts, tde_peak* out,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!out) return set_error(TDE_ERR_ARG, "tde_estimate_batch: null out");
    int rc = validate_pairs(pairs, np, opts);
    if (rc) return rc;
    BatchPlan B = plan_batch(pairs, np, opts);
    if (!ws || ws_bytes < B.total)
        return set_error(TDE_ERR_WS, "tde_estimate_batch: workspace %zu < %zu bytes", ws_bytes, B.total);
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_estimate_batch: null context");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_estimate_batch: hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t* W = static_cast<uint8_t*>(ws);
    hipEvent_t t_begin = mark(ctx, s);

    // ---- descriptors (host side)
    std::vector<QSig> sigs(2 * np);
    std::vector<XItem> items(np);
    std::vector<ArgSeg> segs;
    std::vector<MWork> work;
    int64_t gbase = 0, bbase = 0, pbase = 0, tbase = 0;
    tde_qstat* stats = reinterpret_cast<tde_qstat*>(W + B.off_stats);
    float* invs = reinterpret_cast<float*>(W + B.off_inv);
    ArgPart* tparts = reinterpret_cast<ArgPart*>(W + B.off_tparts);
    bool need_scale = false, any_popc = false, any_mfma = false, any_fused = false, any_r = false;
    int64_t max_rbytes = 0, p_split = 0, p_tiles = 0, p_words = 0;
    for (int64_t i = 0; i < np; ++i) {
        const tde_pair& q = pairs[i];
        const PairPlan& pp = B.pp[i];
        for (int side = 0; side < 2; ++side) {
            QSig& S = sigs[2 * i + side];
            S.x = side ? q.y : q.x;
            S.n = side ? q.ny : q.nx;
            S.q = reinterpret_cast<int8_t*>(W + B.off_q[2 * i + side]);
            S.stat = stats + 2 * i + side;
            S.gsum = reinterpret_cast<double*>(W + B.off_gsum[2 * i + side]);
            S.inv_out = invs + 2 * i + side;
            S.grp_base = gbase;
            S.blk_base = bbase;
            const float fixed = side ? q.inv_step_y : q.inv_step_x;
            S.inv_fixed = (q.bits != 1 && fixed > 0.f) ? fixed : 0.f;
            S.bits = q.bits;
            if (q.bits != 1 && !(fixed > 0.f)) need_scale = true;
            gbase += ceil_div(S.n, 256);
            bbase += ceil_div(S.n, kQuantBlock);
        }
        XItem& it = items[i];
        it = pp.probe;                     // plan (tiles, flags, outside triple)
        it.engine = pp.eng;
        it.p.u = sigs[2 * i].q;
        it.p.v = sigs[2 * i + 1].q;
        it.p.r = pp.need_r ? (q.r_out ? q.r_out : (void*)(W + B.off_r[i])) : nullptr;
        it.p.r_dtype = pp.rdt;
        it.stat_x = stats + 2 * i;
        it.stat_y = stats + 2 * i + 1;
        it.peak = out + i;
        it.fused = pp.fused ? 1 : 0;
        if (it.p.r) {
            any_r = true;
            max_rbytes = std::max<int64_t>(max_rbytes, (q.lag_hi - q.lag_lo + 1) * (pp.rdt == TDE_I32 ? 4 : 8));
        }
        if (pp.eng == TDE_PATH_MFMA) {
            any_mfma = true;
            if (pp.fused) {
                it.part_base = tbase;
                tbase += it.ntiles;
                any_fused = true;
            }
            mfma_items(it, (int)i, work);
        } else {
            popc_plan(it, W + B.off_planes[i]);
            p_split = std::max(p_split, it.nsplit);
            p_tiles = std::max(p_tiles, it.ntiles);
            p_words = std::max(p_words, std::max(it.nuw, it.nvw));
            any_popc = true;
        }
        if (!pp.fused) {
            ArgSeg sg{};
            sg.r = it.p.r;
            sg.L = q.lag_hi - q.lag_lo + 1;
            sg.lag_lo = q.lag_lo;
            sg.part_base = pbase;
            sg.nparts = (int32_t)ceil_div(sg.L, kArgChunk);
            sg.dtype = pp.rdt;
            sg.out = out + i;
            sg.stat_x = it.stat_x;
            sg.stat_y = it.stat_y;
            pbase += sg.nparts;
            segs.push_back(sg);
        }
    }
    mfma_sort_items(work);

    // ---- upload descriptors (one copy) and queue the kernels
    std::vector<uint8_t> blob(B.off_work + work.size() * sizeof(MWork));
    memcpy(blob.data() + B.off_qsig, sigs.data(), sizeof(QSig) * 2 * np);
    memcpy(blob.data() + B.off_items, items.data(), sizeof(XItem) * np);
    if (!segs.empty()) memcpy(blob.data() + B.off_segs, segs.data(), sizeof(ArgSeg) * segs.size());
    if (!work.empty()) memcpy(blob.data() + B.off_work, work.data(), work.size() * sizeof(MWork));
    rc = upload(ctx, W, blob.data(), blob.size(), s);
    if (rc) return rc;
    const QSig* sigs_dev = reinterpret_cast<const QSig*>(W + B.off_qsig);
    const XItem* items_dev = reinterpret_cast<const XItem*>(W + B.off_items);
    const ArgSeg* segs_dev = reinterpret_cast<const ArgSeg*>(W + B.off_segs);
    XItem none{};
    ArgSeg noseg{};
    QSig nosig{};

    hipEvent_t t_q0 = mark(ctx, s);
    rc = launch_quantize(sigs_dev, nosig, (int)(2 * np), gbase, bbase, need_scale, s);
    if (rc) return rc;
    hipEvent_t t_q1 = mark(ctx, s);
    mark_stage(ctx, 0, t_q0, t_q1);
    if (any_r) {
        rc = launch_zero_r(items_dev, none, (int)np, max_rbytes, s);
        if (rc) return rc;
    }
    hipEvent_t t_e0 = mark(ctx, s);
    if (any_popc) {
        // zero the plane buffers (padding must read as 0), then pack
        for (int64_t i = 0; i < np; ++i)
            if (B.pp[i].eng == TDE_PATH_POPC) {
                rc = launch_zero(W + B.off_planes[i], popc_ws_bytes(items[i].p), s);
                if (rc) return rc;
            }
        rc = launch_popc_pack(items_dev, none, (int)np, p_words, s);
        if (rc) return rc;
        rc = launch_xcorr_popc(items_dev, none, (int)np, p_split, p_tiles, s);
        if (rc) return rc;
    }
    if (any_mfma) {
        rc = launch_xcorr_mfma(items_dev, none, reinterpret_cast<const MWork*>(W + B.off_work), (int)work.size(),
                               reinterpret_cast<int*>(W + B.off_counters), tparts, ctx->num_cu, s);
        if (rc) return rc;
    }
    hipEvent_t t_e1 = mark(ctx, s);
    mark_stage(ctx, 1, t_e0, t_e1);
    if (any_fused) {
        rc = launch_tiles_final(items_dev, none, (int)np, tparts, s);
        if (rc) return rc;
    }
    if (!segs.empty()) {
        rc = launch_argmax(segs_dev, noseg, (int)segs.size(), pbase, reinterpret_cast<ArgPart*>(W + B.off_parts), s);
        if (rc) return rc;
    }
    hipEvent_t t_end = mark(ctx, s);
    mark_stage(ctx, 2, t_e1, t_end);
    mark_stage(ctx, 3, t_begin, t_end);
    return TDE_OK;
}

}  // extern "C"
