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

// pinned staging of a context, made once at tde_create (descriptor uploads
// larger than this go through it in chunks)
constexpr size_t kStagingBytes = (size_t)4 << 20;

// Static device scratch of tde_xcorr_int_noalloc: one copy per device, held
// from the library's load until the process ends. In host code `scratch` is
// only a handle: its device address (one per device) comes from
// hipGetSymbolAddress at tde_create and is kept in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

struct tde_ctx {
    int device;
    int num_cu;
    // pinned staging for batch descriptors (host -> workspace copies)
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    std::mutex mu;
    // captured batch graphs, keyed by the exact call signature
    struct Graph {
        std::vector<uint8_t> sig;
        uintptr_t ws_lo, ws_hi;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    hipStream_t cap_stream = nullptr;
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

int ctx_device(const tde_ctx* ctx) { return ctx->device; }
int ctx_num_cu(const tde_ctx* ctx) { return ctx->num_cu; }

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

// Host -> device copy through the context's pinned staging buffer (made at
// tde_create, never reallocated): chunks of at most its size, each staged
// only after the previous copy out of it has finished, so nothing here
// allocates.
int upload(tde_ctx* ctx, void* dst_dev, const void* src_host, size_t bytes, hipStream_t s) {
    size_t done = 0;
    while (done < bytes) {
        if (ctx->upload_pending) {
            TDE_HIP_CHECK(hipEventSynchronize(ctx->upload_done));
            ctx->upload_pending = false;
        }
        const size_t nb = std::min(bytes - done, ctx->pinned_bytes);
        memcpy(ctx->pinned, static_cast<const uint8_t*>(src_host) + done, nb);
        TDE_HIP_CHECK(hipMemcpyAsync(static_cast<uint8_t*>(dst_dev) + done, ctx->pinned, nb, hipMemcpyHostToDevice, s));
        TDE_HIP_CHECK(hipEventRecord(ctx->upload_done, s));
        ctx->upload_pending = true;
        done += nb;
    }
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

// A call that writes [ws, ws + bytes) clobbers the descriptors a cached graph
// keeps there: drop such graphs.
void drop_graphs_on(tde_ctx* c, const void* ws, size_t bytes) {
    if (!ws || c->graphs.empty()) return;
    const uintptr_t lo = (uintptr_t)ws, hi = lo + bytes;
    for (size_t k = 0; k < c->graphs.size();) {
        auto& gr = c->graphs[k];
        if (gr.ws_lo < hi && lo < gr.ws_hi) {
            (void)hipGraphExecDestroy(gr.exec);
            (void)hipGraphDestroy(gr.graph);
            c->graphs.erase(c->graphs.begin() + k);
        } else {
            ++k;
        }
    }
}

// Engine choice for one correlation: the caller's, or the tuning table's
// (every engine is exact; they differ in speed).
int choose_path(int path, int64_t nu, int64_t nv, int kuv, int kmax, int64_t lo, int64_t hi) {
    if (path == TDE_PATH_MFMA_I8) return TDE_PATH_MFMA;
    if (path != TDE_PATH_AUTO) return path;
    return auto_engine(nu, nv, kuv, kmax, lo, hi);
}

}  // namespace

// Scratch of tde_refine_ties, carved in this order; with ws = nullptr only
// the size is computed.
RefineWs refine_ws_carve(void* ws, int max_ties, size_t* bytes) {
    Carve cv(ws);
    RefineWs w;
    w.lags = static_cast<int64_t*>(cv.take((size_t)max_ties * 8));
    w.vals = static_cast<double*>(cv.take((size_t)max_ties * 8));
    w.errs = static_cast<double*>(cv.take((size_t)max_ties * 8));
    w.cand = static_cast<int*>(cv.take((size_t)max_ties * 4));
    w.ncand = static_cast<int*>(cv.take(sizeof(int)));
    w.count = static_cast<int*>(cv.take(sizeof(int)));
    w.hits = static_cast<int*>(cv.take((size_t)kRefineMaxChunks * sizeof(int)));
    w.limbs = static_cast<int64_t*>(cv.take((size_t)max_ties * kExactLimbs * 8));
    if (bytes) *bytes = cv.off;
    return w;
}
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
        if (hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming) != hipSuccess ||
            hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc(&c->pinned, kStagingBytes, hipHostMallocDefault) != hipSuccess) {
            tde_destroy(c);
            return set_error(TDE_ERR_HIP, "tde_create: event, stream or pinned staging creation failed");
        }
        c->pinned_bytes = kStagingBytes;
        if (device < kMaxDevices) {
            std::lock_guard<std::mutex> lock(g_scratch_mu);
            if (!g_scratch_ptr[device]) {
                void* p = nullptr;
                const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
                if (e != hipSuccess || !p) {
                    tde_destroy(c);
                    return set_error(TDE_ERR_HIP, "tde_create: address of the static scratch on device %d: %s",
                                     device, hipGetErrorString(e));
                }
                g_scratch_ptr[device] = p;
            }
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
    for (int k = 0; k < TDE_STAGES; ++k) {
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
    for (auto& gr : c->graphs) {
        (void)hipGraphExecDestroy(gr.exec);
        (void)hipGraphDestroy(gr.graph);
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
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
    return tde_quantize_ex(ctx, x, n, bits, TDE_QUANT_UNIFORM, inv_step, q, stat, ws, ws_bytes, stream);
}

int tde_quantizer_thresholds(int quantizer, int bits, float* out) {
    if (!out) return set_error(TDE_ERR_ARG, "tde_quantizer_thresholds: null out");
    if (quantizer != TDE_QUANT_MULAW && quantizer != TDE_QUANT_GAUSS)
        return set_error(TDE_ERR_ARG, "tde_quantizer_thresholds: not a non-uniform quantizer");
    const int K = quant_table(quantizer, bits, out);
    if (K == 0) return set_error(TDE_ERR_UNSUPPORTED, "tde_quantizer_thresholds: bits %d (2 or 4 only)", bits);
    return K;
}

int tde_quantize_ex(tde_ctx* ctx, const float* x, int64_t n, int bits, int quantizer, float inv_step, int8_t* q,
                    tde_qstat* stat, void* ws, size_t ws_bytes, void* stream) {
    if (!x || !q) return set_error(TDE_ERR_ARG, "tde_quantize: null x or q");
    if (n < 1) return set_error(TDE_ERR_ARG, "tde_quantize: n = %lld < 1", (long long)n);
    if (!valid_bits(bits)) return set_error(TDE_ERR_ARG, "tde_quantize: bits = %d not in {1,2,4,8}", bits);
    if (!std::isfinite(inv_step)) return set_error(TDE_ERR_ARG, "tde_quantize: inv_step is not finite");
    if (quantizer < TDE_QUANT_UNIFORM || quantizer > TDE_QUANT_GAUSS)
        return set_error(TDE_ERR_ARG, "tde_quantize: quantizer %d", quantizer);
    if (quantizer != TDE_QUANT_UNIFORM && bits == 8)
        return set_error(TDE_ERR_UNSUPPORTED, "tde_quantize: non-uniform quantizers take bits 1, 2 or 4");
    const bool need_scale = bits != 1 && !(inv_step > 0.f);
    // the exact sum of squares behind an undecided automatic scale counts
    // at most 2^32 - 1 digits per limb
    if (need_scale && n >= ((int64_t)1 << 32))
        return set_error(TDE_ERR_UNSUPPORTED, "tde_quantize: automatic scale of 2^32 or more samples");
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_quantize: null context");
    QSig one{};
    one.x = x;
    one.n = n;
    one.q = q;
    one.stat = stat;
    one.bits = bits;
    one.inv_fixed = (bits != 1 && inv_step > 0.f) ? inv_step : 0.f;
    if (quantizer != TDE_QUANT_UNIFORM && bits != 1) one.nthr = quant_table(quantizer, bits, one.thr);
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
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        drop_graphs_on(ctx, ws, ws_bytes);
    }
    return launch_quantize(nullptr, one, 1, ceil_div(n, kQuantBlock), need_scale, stat != nullptr, nullptr, 0,
                           static_cast<hipStream_t>(stream), n, n);
}

// --------------------------------------------------------- correlation --

// The request itself (sizes, code ranges, lag range, engine), without its
// buffers: what tde_xcorr_int and the workspace query both refuse.
static int check_xcorr_request(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi,
                               int path, const char* who) {
    if (nu < 1 || nv < 1) return set_error(TDE_ERR_ARG, "%s: empty signal", who);
    if (lag_lo > lag_hi) return set_error(TDE_ERR_ARG, "%s: lag_lo > lag_hi", who);
    if (lag_hi - lag_lo + 1 > ((int64_t)1 << 40)) return set_error(TDE_ERR_ARG, "%s: lag range too large", who);
    if (kmax_u < 1 || kmax_u > 127 || kmax_v < 1 || kmax_v > 127)
        return set_error(TDE_ERR_ARG, "%s: kmax must be in [1, 127]", who);
    if (path < TDE_PATH_AUTO || path > TDE_PATH_MFMA_I8) return set_error(TDE_ERR_ARG, "%s: bad path", who);
    if (path == TDE_PATH_POPC && (kmax_u != 1 || kmax_v != 1))
        return set_error(TDE_ERR_ARG, "%s: the bit-plane engine needs ternary codes (kmax 1)", who);
    if (path == TDE_PATH_NTT) {
        NttPlan P;
        if (!ntt_plan(nu, nv, kmax_u * kmax_v, lag_lo, lag_hi, P))
            return set_error(TDE_ERR_UNSUPPORTED, "%s: transform longer than 2^%d", who, kNttMaxLog);
    }
    return TDE_OK;
}

static int check_xcorr(const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int kmax_u, int kmax_v,
                       int64_t lag_lo, int64_t lag_hi, const void* r, int r_dtype, int path, const char* who) {
    if (!u || !v || !r) return set_error(TDE_ERR_ARG, "%s: null pointer", who);
    const int rc = check_xcorr_request(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path, who);
    if (rc) return rc;
    if (r_dtype != TDE_I32 && r_dtype != TDE_I64) return set_error(TDE_ERR_ARG, "%s: bad r_dtype", who);
    if (((uintptr_t)r) & (r_dtype == TDE_I32 ? 3 : 7))
        return set_error(TDE_ERR_ARG, "%s: r is not aligned to its element size", who);
    if (r_dtype == TDE_I32) {
        const int64_t ov = max_overlap(nu, nv, lag_lo, lag_hi);
        if ((__int128)ov * kmax_u * kmax_v >= ((__int128)1 << 31))
            return set_error(TDE_ERR_RANGE, "%s: overlap %lld x %d x %d does not fit int32", who, (long long)ov,
                             kmax_u, kmax_v);
    }
    return TDE_OK;
}

int tde_mfma_operand_bits(int kmax_u, int kmax_v, int path) {
    if (kmax_u < 1 || kmax_u > 127 || kmax_v < 1 || kmax_v > 127)
        return set_error(TDE_ERR_ARG, "tde_mfma_operand_bits: kmax must be in [1, 127]");
    if (path != TDE_PATH_AUTO && path != TDE_PATH_MFMA && path != TDE_PATH_MFMA_I8)
        return set_error(TDE_ERR_ARG, "tde_mfma_operand_bits: not a matrix-core path");
    const int f = mfma_choose_fmt(kmax_u > kmax_v ? kmax_u : kmax_v, path != TDE_PATH_MFMA_I8);
    return f == kFmtF4 ? 4 : (f == kFmtF6 ? 6 : 8);
}

size_t tde_xcorr_workspace_size(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi,
                                int path) {
    if (check_xcorr_request(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path, "tde_xcorr_workspace_size")) return 0;
    XItem it{};
    it.p.nu = nu;
    it.p.nv = nv;
    it.p.lag_lo = lag_lo;
    it.p.lag_hi = lag_hi;
    it.p.kuv = kmax_u * kmax_v;
    it.p.kmax = kmax_u > kmax_v ? kmax_u : kmax_v;
    int eng = choose_path(path, nu, nv, it.p.kuv, it.p.kmax, lag_lo, lag_hi);
    if (eng == TDE_PATH_POPC) return popc_ws_bytes(it.p);
    if (eng == TDE_PATH_NTT) {
        NttPlan P;
        if (!ntt_plan(nu, nv, it.p.kuv, lag_lo, lag_hi, P)) return 0;
        return align_bytes(sizeof(NttJob)) + align_bytes(ntt_tab_words(P) * 4) + align_bytes(ntt_res_bytes(P));
    }
    mfma_plan_pair(it, path != TDE_PATH_MFMA_I8);
    size_t pk = 0;
    if (it.fmt != kFmtI8) {
        const int wb = it.fmt == kFmtF6 ? 6 : 4;
        pk = align_bytes(packed_bytes(nu, wb)) + align_bytes(packed_bytes(nv, wb));
    }
    return align_bytes(sizeof(XItem)) + align_bytes((size_t)mfma_count_items(it) * sizeof(MWork)) +
           align_bytes(2 * sizeof(int)) + pk;
}

}  // extern "C"

namespace {

// Body of tde_xcorr_int, on the scratch ws (the caller's workspace, or the
// device's static scratch for tde_xcorr_int_noalloc).
int xcorr_run(tde_ctx* ctx, const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int kmax_u, int kmax_v,
              int64_t lag_lo, int64_t lag_hi, void* r, int r_dtype, int path, void* ws, size_t ws_bytes,
              void* stream) {
    int rc;
    XItem it{};
    it.p.u = u;
    it.p.v = v;
    it.p.nu = nu;
    it.p.nv = nv;
    it.p.lag_lo = lag_lo;
    it.p.lag_hi = lag_hi;
    it.p.r = r;
    it.p.r_dtype = r_dtype;
    it.p.kuv = kmax_u * kmax_v;
    it.p.kmax = kmax_u > kmax_v ? kmax_u : kmax_v;
    const int eng = choose_path(path, nu, nv, it.p.kuv, it.p.kmax, lag_lo, lag_hi);
    it.engine = eng;
    const int wpath = path == TDE_PATH_MFMA_I8 ? path : eng;
    size_t need = tde_xcorr_workspace_size(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, wpath);
    if (need && (!ws || ws_bytes < need))
        return set_error(TDE_ERR_WS, "tde_xcorr_int: workspace %zu < %zu bytes", ws_bytes, need);
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_xcorr_int: hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t rbytes = (lag_hi - lag_lo + 1) * (r_dtype == TDE_I32 ? 4 : 8);
    rc = launch_zero_r(nullptr, it, 1, rbytes, s);
    if (rc) return rc;
    if (eng == TDE_PATH_POPC) {
        {
            std::lock_guard<std::mutex> lock(ctx->mu);
            drop_graphs_on(ctx, ws, ws_bytes);
        }
        popc_plan(it, ws);
        rc = launch_zero(ws, need, s);
        if (rc) return rc;
        rc = launch_popc_pack(nullptr, it, 1, std::max(it.nuw, it.nvw), s);
        if (rc) return rc;
        return launch_xcorr_popc(nullptr, it, 1, it.nsplit, it.ntiles, s);
    }
    if (eng == TDE_PATH_NTT) {
        NttPlan P;
        ntt_plan(nu, nv, it.p.kuv, lag_lo, lag_hi, P);
        Carve cv(ws);
        NttJob* job_dev = static_cast<NttJob*>(cv.take(sizeof(NttJob)));
        uint32_t* tab = static_cast<uint32_t*>(cv.take(ntt_tab_words(P) * 4));
        NttJob job{};
        job.u = u;
        job.v = v;
        job.nu = nu;
        job.nv = nv;
        job.lag_lo = lag_lo;
        job.jlo = P.jlo;
        job.jhi = P.jhi;
        job.r = r;
        job.r_dtype = r_dtype;
        job.res = static_cast<uint32_t*>(cv.take(ntt_res_bytes(P)));
        job.parts = nullptr;
        {
            std::lock_guard<std::mutex> lock(ctx->mu);
            drop_graphs_on(ctx, ws, ws_bytes);
            rc = upload(ctx, job_dev, &job, sizeof(job), s);
        }
        if (rc) return rc;
        if (P.jlo > P.jhi) return TDE_OK;          // every requested lag is outside the support
        return launch_ntt(ntt_group(P, tab), job_dev, 1, s);
    }
    mfma_plan_pair(it, path != TDE_PATH_MFMA_I8);
    std::vector<MWork> work;
    mfma_items(it, 0, work);
    mfma_sort_items(work);
    // workspace: the item, the work list, two counters (one upload), then
    // the packed codes of FP operands
    const size_t off_w = align_bytes(sizeof(XItem));
    uint8_t* W = static_cast<uint8_t*>(ws);
    const size_t off_c = off_w + align_bytes(work.size() * sizeof(MWork));
    int* counters = reinterpret_cast<int*>(W + off_c);
    if (it.fmt != kFmtI8) {
        const int wb = it.fmt == kFmtF6 ? 6 : 4;
        uint32_t* upk = reinterpret_cast<uint32_t*>(W + off_c + align_bytes(2 * sizeof(int)));
        uint32_t* vpk = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(upk) + align_bytes(packed_bytes(nu, wb)));
        rc = launch_pack_fp(u, nu, upk, wb, s);
        if (!rc) rc = launch_pack_fp(v, nv, vpk, wb, s);
        if (rc) return rc;
        it.p.upk = upk;
        it.p.vpk = vpk;
    }
    std::vector<uint8_t> blob(off_w + work.size() * sizeof(MWork));
    memcpy(blob.data(), &it, sizeof(XItem));
    memcpy(blob.data() + off_w, work.data(), work.size() * sizeof(MWork));
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        drop_graphs_on(ctx, ws, ws_bytes);
        rc = upload(ctx, W, blob.data(), blob.size(), s);
    }
    if (rc) return rc;
    return launch_xcorr_mfma(reinterpret_cast<const XItem*>(W), reinterpret_cast<const MWork*>(W + off_w),
                             (int)work.size(), counters, false, nullptr, ctx->num_cu, s,
                             mfma_launch_of(it.fmt, it.mb) == 4 ? (int)work.size() : 0);
}

}  // namespace

extern "C" {

int tde_mfma_tile_lags(int64_t nu, int64_t nv, int kmax_u, int kmax_v, int64_t lag_lo, int64_t lag_hi, int path) {
    if (path != TDE_PATH_AUTO && path != TDE_PATH_MFMA && path != TDE_PATH_MFMA_I8)
        return set_error(TDE_ERR_ARG, "tde_mfma_tile_lags: path %d is not a matrix-core path", path);
    const int rc = check_xcorr_request(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path, "tde_mfma_tile_lags");
    if (rc) return rc;
    XItem it{};
    it.p.nu = nu;
    it.p.nv = nv;
    it.p.lag_lo = lag_lo;
    it.p.lag_hi = lag_hi;
    it.p.kuv = kmax_u * kmax_v;
    it.p.kmax = kmax_u > kmax_v ? kmax_u : kmax_v;
    mfma_plan_pair(it, path != TDE_PATH_MFMA_I8);
    return 1024 * it.mb;
}

int tde_xcorr_int(tde_ctx* ctx, const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int kmax_u, int kmax_v,
                  int64_t lag_lo, int64_t lag_hi, void* r, int r_dtype, int path, void* ws, size_t ws_bytes,
                  void* stream) {
    int rc = check_xcorr(u, nu, v, nv, kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path, "tde_xcorr_int");
    if (rc) return rc;
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_xcorr_int: null context");
    return xcorr_run(ctx, u, nu, v, nv, kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path, ws, ws_bytes, stream);
}

// tde_xcorr_int with the device's static scratch as its workspace.
int tde_xcorr_int_noalloc(tde_ctx* ctx, const int8_t* u, int64_t nu, const int8_t* v, int64_t nv, int kmax_u,
                          int kmax_v, int64_t lag_lo, int64_t lag_hi, void* r, int r_dtype, int path, void* stream) {
    int rc = check_xcorr(u, nu, v, nv, kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path, "tde_xcorr_int_noalloc");
    if (rc) return rc;
    const int wpath = path == TDE_PATH_MFMA_I8 ? path
                      : choose_path(path, nu, nv, kmax_u * kmax_v, kmax_u > kmax_v ? kmax_u : kmax_v, lag_lo, lag_hi);
    const size_t need = tde_xcorr_workspace_size(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, wpath);
    if (need > kNoAllocScratchBytes)
        return set_error(TDE_ERR_UNSUPPORTED,
                         "tde_xcorr_int_noalloc: this correlation needs %zu bytes of scratch; the static scratch "
                         "holds %zu", need, kNoAllocScratchBytes);
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_xcorr_int_noalloc: null context");
    void* ws = g_scratch_ptr[ctx->device];
    if (!ws) return set_error(TDE_ERR_HIP, "tde_xcorr_int_noalloc: no scratch address for device %d", ctx->device);
    return xcorr_run(ctx, u, nu, v, nv, kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path, ws, kNoAllocScratchBytes,
                     stream);
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
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        drop_graphs_on(ctx, ws, ws_bytes);
    }
    return launch_argmax(nullptr, one, 1, one.nparts, static_cast<ArgPart*>(ws), static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------ tie refinement --

size_t tde_refine_workspace_size(int max_ties) {
    if (max_ties < 2 || max_ties > 65536) return 0;
    size_t bytes = 0;
    refine_ws_carve(nullptr, max_ties, &bytes);
    return bytes;
}

int tde_refine_ties(tde_ctx* ctx, const float* x, int64_t nx, const float* y, int64_t ny, const void* r,
                    int r_dtype, int64_t lag_lo, int64_t lag_hi, tde_peak* peak, int max_ties, void* ws,
                    size_t ws_bytes, void* stream) {
    if (!x || !y || !r || !peak) return set_error(TDE_ERR_ARG, "tde_refine_ties: null pointer");
    if (nx < 1 || ny < 1) return set_error(TDE_ERR_ARG, "tde_refine_ties: empty signal");
    if (lag_lo > lag_hi) return set_error(TDE_ERR_ARG, "tde_refine_ties: lag_lo > lag_hi");
    // tie counts and chunk offsets are int
    if (lag_hi - lag_lo >= ((int64_t)1 << 31) - 1)
        return set_error(TDE_ERR_ARG, "tde_refine_ties: more than 2^31 - 1 lags");
    if (r_dtype != TDE_I32 && r_dtype != TDE_I64) return set_error(TDE_ERR_ARG, "tde_refine_ties: bad r_dtype");
    if (max_ties < 2 || max_ties > 65536) return set_error(TDE_ERR_ARG, "tde_refine_ties: max_ties in [2, 65536]");
    if (std::min(nx, ny) > ((int64_t)1 << 22))
        return set_error(TDE_ERR_UNSUPPORTED, "tde_refine_ties: overlaps longer than 2^22 samples");
    const size_t need = tde_refine_workspace_size(max_ties);
    if (!ws || ws_bytes < need) return set_error(TDE_ERR_WS, "tde_refine_ties: workspace %zu < %zu", ws_bytes, need);
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_refine_ties: null context");
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_refine_ties: hipSetDevice failed");
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        drop_graphs_on(ctx, ws, ws_bytes);
    }
    return launch_refine(x, nx, y, ny, r, r_dtype, lag_lo, lag_hi - lag_lo + 1, peak, max_ties,
                         refine_ws_carve(ws, max_ties, nullptr), static_cast<hipStream_t>(stream));
}

// --------------------------------------------------------------- batch --

}  // extern "C"

namespace {

int validate_pairs(const tde_pair* pairs, int64_t np, const tde_opts* opts) {
    if (!pairs || np < 1) return set_error(TDE_ERR_ARG, "tde_estimate_batch: no pairs");
    if (np > 65535) return set_error(TDE_ERR_ARG, "tde_estimate_batch: at most 65535 pairs per call");
    int path = opts ? opts->path : TDE_PATH_AUTO;
    const bool learned = opts && opts->mode == TDE_MODE_LEARNED;
    if (opts && opts->mode != TDE_MODE_FULL && !learned)
        return set_error(TDE_ERR_ARG, "tde_estimate_batch: unknown mode %d", opts->mode);
    if (path < TDE_PATH_AUTO || path > TDE_PATH_MFMA_I8)
        return set_error(TDE_ERR_ARG, "tde_estimate_batch: bad path %d", path);
    const int quantizer = opts ? opts->quantizer : TDE_QUANT_UNIFORM;
    if (quantizer < TDE_QUANT_UNIFORM || quantizer > TDE_QUANT_GAUSS)
        return set_error(TDE_ERR_ARG, "tde_estimate_batch: quantizer %d", quantizer);
    if (learned) {
        if (!opts->model) return set_error(TDE_ERR_ARG, "tde_estimate_batch: learned mode needs a model");
        if (opts->topk < 1 || opts->topk > kCnnMaxTop || opts->topk >= model_net(opts->model).nb)
            return set_error(TDE_ERR_ARG, "tde_estimate_batch: topk must be in [1, %d]", kCnnMaxTop);
        if (std::isnan(opts->margin)) return set_error(TDE_ERR_ARG, "tde_estimate_batch: NaN margin");
        if (path != TDE_PATH_AUTO && path != TDE_PATH_MFMA && path != TDE_PATH_MFMA_I8)
            return set_error(TDE_ERR_ARG, "tde_estimate_batch: learned mode falls back on TDE_PATH_MFMA");
        const CnnNet& net = model_net(opts->model);
        const int64_t n = 16 * (int64_t)net.ld, half = (int64_t)(net.nb / 2) * 256;
        for (int64_t i = 0; i < np; ++i) {
            const tde_pair& q = pairs[i];
            if (q.nx != n || q.ny != n || q.lag_lo != -half || q.lag_hi != half - 1 || q.r_out ||
                (q.bits != 2 && q.bits != 4 && q.bits != 8))
                return set_error(TDE_ERR_ARG,
                                 "pair %lld: learned mode needs nx = ny = %lld, lags [%lld, %lld], bits 2/4/8, no r_out",
                                 (long long)i, (long long)n, (long long)-half, (long long)(half - 1));
            // each window wave sums a quarter of the m range (plus the
            // tile's reach and whole groups of 4 steps) in int32
            const int K = kmax_of_bits(q.bits);
            if ((__int128)(n / 4 + 512) * K * K >= ((__int128)1 << 31))
                return set_error(TDE_ERR_UNSUPPORTED, "pair %lld: signals too long for int32 window sums", (long long)i);
        }
    }
    for (int64_t i = 0; i < np; ++i) {
        const tde_pair& q = pairs[i];
        if (!q.x || !q.y) return set_error(TDE_ERR_ARG, "pair %lld: null signal", (long long)i);
        if (q.nx < 1 || q.ny < 1) return set_error(TDE_ERR_ARG, "pair %lld: empty signal", (long long)i);
        if (q.lag_lo > q.lag_hi) return set_error(TDE_ERR_ARG, "pair %lld: lag_lo > lag_hi", (long long)i);
        if (q.lag_hi - q.lag_lo + 1 > ((int64_t)1 << 31))
            return set_error(TDE_ERR_ARG, "pair %lld: lag range too large", (long long)i);
        if (!valid_bits(q.bits)) return set_error(TDE_ERR_ARG, "pair %lld: bits %d", (long long)i, q.bits);
        if (quantizer != TDE_QUANT_UNIFORM && q.bits == 8)
            return set_error(TDE_ERR_UNSUPPORTED, "pair %lld: non-uniform quantizers take bits 1, 2 or 4",
                             (long long)i);
        if (!std::isfinite(q.inv_step_x) || !std::isfinite(q.inv_step_y))
            return set_error(TDE_ERR_ARG, "pair %lld: non-finite inv_step", (long long)i);
        if (q.bits != 1 && ((!(q.inv_step_x > 0.f) && q.nx >= ((int64_t)1 << 32)) ||
                            (!(q.inv_step_y > 0.f) && q.ny >= ((int64_t)1 << 32))))
            return set_error(TDE_ERR_UNSUPPORTED, "pair %lld: automatic scale of 2^32 or more samples",
                             (long long)i);
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
        if (path == TDE_PATH_NTT) {
            const int K = kmax_of_bits(q.bits);
            NttPlan P;
            if (!ntt_plan(q.nx, q.ny, K * K, q.lag_lo, q.lag_hi, P))
                return set_error(TDE_ERR_UNSUPPORTED, "pair %lld: transform longer than 2^%d", (long long)i,
                                 kNttMaxLog);
        }
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
    NttPlan ntt;        // NTT plan (engine NTT)
};

// Triple (value 0) of the lags of [lo, hi] outside the covered run [c_lo, c_hi].
void outside_triple(int64_t lo, int64_t hi, int64_t c_lo, int64_t c_hi, XItem& it) {
    const int64_t L = hi - lo + 1;
    c_lo = std::max(c_lo, lo);
    c_hi = std::min(c_hi, hi);
    const int64_t covered = c_hi >= c_lo ? c_hi - c_lo + 1 : 0;
    it.out_c = L - covered;
    if (it.out_c == 0) {
        it.out_v = INT64_MIN;
        it.out_i = INT64_MAX;
    } else {
        it.out_v = 0;
        it.out_i = (covered == 0 || c_lo > lo) ? 0 : (c_hi + 1 - lo);
    }
}

PairPlan plan_pair(const tde_pair& q, int path, bool learned) {
    PairPlan pp{};
    const int K = kmax_of_bits(q.bits);
    pp.eng = learned ? TDE_PATH_MFMA : choose_path(path, q.nx, q.ny, K * K, K, q.lag_lo, q.lag_hi);
    pp.rdt = q.r_out ? q.r_dtype
                     : ((__int128)max_overlap(q.nx, q.ny, q.lag_lo, q.lag_hi) * K * K < ((__int128)1 << 31) ? TDE_I32
                                                                                                          : TDE_I64);
    pp.probe.p.nu = q.nx;
    pp.probe.p.nv = q.ny;
    pp.probe.p.lag_lo = q.lag_lo;
    pp.probe.p.lag_hi = q.lag_hi;
    pp.probe.p.kuv = K * K;
    pp.probe.p.kmax = K;
    if (pp.eng == TDE_PATH_MFMA) {
        mfma_plan_pair(pp.probe, path != TDE_PATH_MFMA_I8);
        pp.fused = !pp.probe.segmented;
    } else if (pp.eng == TDE_PATH_NTT) {
        ntt_plan(q.nx, q.ny, K * K, q.lag_lo, q.lag_hi, pp.ntt);
        pp.fused = true;
        pp.probe.ntiles = pp.ntt.jlo <= pp.ntt.jhi ? pp.ntt.ntiles : 0;
        outside_triple(q.lag_lo, q.lag_hi, pp.ntt.jlo - (q.nx - 1), pp.ntt.jhi - (q.nx - 1), pp.probe);
    } else {
        pp.fused = false;
    }
    pp.need_r = q.r_out != nullptr || !pp.fused;
    return pp;
}

struct BatchPlan {
    size_t total = 0;
    // offsets inside the workspace; [0, off_stats) is uploaded from the host
    size_t off_qsig, off_items, off_segs, off_jobs, off_work, off_counters, off_tparts, off_stats, off_inv,
        off_parts;
    int64_t nwork = 0, ntparts = 0, nsegs = 0, total_parts = 0, njobs = 0;
    // NTT launch groups: pairs with the same transform length and prime count
    struct NGroup {
        int log_n, nprimes;
        std::vector<int64_t> pairs;
        size_t off_tab;
    };
    std::vector<NGroup> ngroups;
    std::vector<size_t> off_res;    // per pair (NTT residues)
    int quantizer = TDE_QUANT_UNIFORM;
    // learned mode
    bool learned = false;
    const tde_model* model = nullptr;
    int topk = 0;
    float theta = 0.f;
    size_t off_cnn = 0, off_top = 0, off_margin = 0, off_wparts = 0;
    std::vector<PairPlan> pp;
    std::vector<size_t> off_q;      // per signal (2 per pair)
    std::vector<size_t> off_gsum;   // per signal
    std::vector<size_t> off_r;      // per pair (r materialized in the workspace)
    std::vector<size_t> off_planes; // per pair (bit-plane engine)
    std::vector<size_t> off_pk;     // per signal: packed FP4/FP6 codes (0: none)
    // learned mode: the fallback's work list planned on the device (every pair
    // on 4-block matrix-core items with tile triples, no caller r)
    bool fb_dyn = false;
    int64_t fb_cap = 0, fb_slot_bytes = 0;
    size_t off_fbctl = 0, off_fbslots = 0, off_dwork = 0, off_rpool = 0, off_fbparts = 0;
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
    B.quantizer = opts ? opts->quantizer : TDE_QUANT_UNIFORM;
    B.learned = opts && opts->mode == TDE_MODE_LEARNED;
    B.pp.resize(np);
    for (int64_t i = 0; i < np; ++i) {
        B.pp[i] = plan_pair(pairs[i], path, B.learned);
        const PairPlan& pp = B.pp[i];
        if (pp.eng == TDE_PATH_MFMA) {
            B.nwork += mfma_count_items(pp.probe);
            if (pp.fused) B.ntparts += pp.probe.ntiles;
        }
        if (pp.eng == TDE_PATH_NTT && pp.probe.ntiles > 0) {
            B.ntparts += pp.probe.ntiles;
            B.njobs += 1;
            auto g = std::find_if(B.ngroups.begin(), B.ngroups.end(), [&](const BatchPlan::NGroup& x) {
                return x.log_n == pp.ntt.log_n && x.nprimes == pp.ntt.nprimes;
            });
            if (g == B.ngroups.end()) {
                B.ngroups.push_back({pp.ntt.log_n, pp.ntt.nprimes, {}, 0});
                g = B.ngroups.end() - 1;
            }
            g->pairs.push_back(i);
        }
        if (!pp.fused) {
            B.nsegs += 1;
            B.total_parts += ceil_div(pairs[i].lag_hi - pairs[i].lag_lo + 1, kArgChunk);
        }
    }
    B.off_qsig = take(sizeof(QSig) * 2 * np);
    B.off_items = take(sizeof(XItem) * np);
    B.off_segs = take(sizeof(ArgSeg) * (B.nsegs ? B.nsegs : 1));
    B.off_jobs = take(sizeof(NttJob) * (B.njobs ? B.njobs : 1));
    B.off_work = take(sizeof(MWork) * (B.nwork ? B.nwork : 1));
    B.off_counters = take(2 * sizeof(int));
    B.off_tparts = take(sizeof(ArgPart) * (B.ntparts ? B.ntparts : 1));
    B.off_stats = take(sizeof(tde_qstat) * 2 * np);
    B.off_inv = take(sizeof(float) * 2 * np);
    B.off_parts = take(sizeof(ArgPart) * (B.total_parts ? B.total_parts : 1));
    if (B.learned) {
        B.model = opts->model;
        B.topk = opts->topk;
        B.theta = opts->margin;
        B.off_cnn = take(cnn_infer_bytes(model_net(B.model), (int)np));
        B.off_top = take(sizeof(int32_t) * np * B.topk);
        B.off_margin = take(sizeof(float) * np);
        B.off_wparts = take(sizeof(ArgPart) * np * B.topk);
        bool dyn = true;
        int64_t max_items = 0, slot = 0;
        for (int64_t i = 0; i < np; ++i) {
            const PairPlan& pp = B.pp[i];
            if (pp.eng != TDE_PATH_MFMA || !pp.fused || pairs[i].r_out ||
                mfma_launch_of(pp.probe.fmt, pp.probe.mb) != 4) {
                dyn = false;
                break;
            }
            max_items = std::max<int64_t>(max_items, mfma_count_items(pp.probe));
            slot = std::max<int64_t>(slot, (pairs[i].lag_hi - pairs[i].lag_lo + 1) * (pp.rdt == TDE_I32 ? 4 : 8));
        }
        if (dyn && np > 0) {
            B.fb_dyn = true;
            B.fb_cap = std::max<int64_t>(B.nwork, (int64_t)kFbSlots * max_items * kFbMaxSplit);
            B.fb_slot_bytes = (int64_t)align_bytes((size_t)slot);
            B.off_fbctl = take(4 * sizeof(int));
            B.off_fbslots = take(kFbSlots * sizeof(int));
            B.off_dwork = take(sizeof(MWork) * B.fb_cap);
            B.off_rpool = take((size_t)(kFbSlots * B.fb_slot_bytes));
            B.off_fbparts = take(sizeof(ArgPart) * kFbSlots * 64);
        }
    }
    B.off_q.resize(2 * np);
    B.off_gsum.resize(2 * np);
    B.off_r.assign(np, 0);
    B.off_planes.assign(np, 0);
    B.off_res.assign(np, 0);
    B.off_pk.assign(2 * np, 0);
    for (auto& g : B.ngroups) {
        NttPlan P{};
        P.log_n = g.log_n;
        P.nprimes = g.nprimes;
        g.off_tab = take(ntt_tab_words(P) * 4);
    }
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
        if (pp.eng == TDE_PATH_MFMA && pp.probe.fmt != kFmtI8) {
            const int wb = pp.probe.fmt == kFmtF6 ? 6 : 4;
            B.off_pk[2 * i] = take(packed_bytes(q.nx, wb));
            B.off_pk[2 * i + 1] = take(packed_bytes(q.ny, wb));
        }
        if (pp.eng == TDE_PATH_NTT && pp.probe.ntiles > 0) B.off_res[i] = take(ntt_res_bytes(pp.ntt));
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

}  // extern "C"

namespace {

// Everything a batch call queues, prepared on the host.
struct BatchLaunch {
    std::vector<uint8_t> blob;       // descriptors for [0, blob.size()) of the workspace
    int64_t np = 0, bbase = 0, pbase = 0;
    int64_t min_n = INT64_MAX, max_n = 0;   // signal lengths
    bool need_scale = false, any_popc = false, any_mfma = false, any_fused = false, any_r = false;
    int64_t max_rbytes = 0, p_split = 0, p_tiles = 0, p_words = 0;
    int nwork = 0, nsegs = 0, n4 = 0;
    int win_formats = 0;                                  // learned mode: window kernels to launch
    std::vector<std::pair<NttGroup, int64_t>> ngroups;   // (group, first job index)
    std::vector<int> ngroup_jobs;
    int64_t p_zero_words = 0;                             // largest bit-plane region (words)
};

// Learned mode: the operand width (4 or 6) of the pair's FP window kernel, or
// 0 for the int8 one. The FP kernel takes codes up to 7 (the pair's
// matrix-core format is FP4/FP6), at most 8 windows in its one tile, and
// signals short enough that a wave's fp32 partial (a quarter of the m range
// in whole chunks, plus the tile's reach) stays below 2^24.
int win_fp_width(const tde_pair& q, const PairPlan& pp, const BatchPlan& B) {
    if (!B.learned || B.topk > 8 || pp.probe.fmt == kFmtI8) return 0;
    const int64_t K = kmax_of_bits(q.bits);
    // a wave's m range: a quarter of the steps, rounded up to whole 16-step chunks
    if ((std::max(q.nx, q.ny) / 4 + 2048) * K * K >= ((int64_t)1 << 24)) return 0;
    return pp.probe.fmt == kFmtF6 ? 6 : 4;
}

void batch_prepare(tde_ctx* ctx, const tde_pair* pairs, int64_t np, tde_peak* out, uint8_t* W, const BatchPlan& B,
                   BatchLaunch& L) {
    (void)ctx;
    std::vector<QSig> sigs(2 * np);
    std::vector<XItem> items(np);
    std::vector<ArgSeg> segs;
    std::vector<MWork> work;
    int64_t bbase = 0, pbase = 0, tbase = 0;
    tde_qstat* stats = reinterpret_cast<tde_qstat*>(W + B.off_stats);
    float* invs = reinterpret_cast<float*>(W + B.off_inv);
    L.np = np;
    for (int64_t i = 0; i < np; ++i) {
        const tde_pair& q = pairs[i];
        const PairPlan& pp = B.pp[i];
        for (int side = 0; side < 2; ++side) {
            QSig& S = sigs[2 * i + side];
            S.x = side ? q.y : q.x;
            S.n = side ? q.ny : q.nx;
            S.q = reinterpret_cast<int8_t*>(W + B.off_q[2 * i + side]);
            S.stat = stats + 2 * i + side;
            S.stat_lite = 1;
            S.gsum = reinterpret_cast<double*>(W + B.off_gsum[2 * i + side]);
            S.inv_out = invs + 2 * i + side;
            S.blk_base = bbase;
            const float fixed = side ? q.inv_step_y : q.inv_step_x;
            S.inv_fixed = (q.bits != 1 && fixed > 0.f) ? fixed : 0.f;
            S.bits = q.bits;
            if (B.quantizer != TDE_QUANT_UNIFORM && q.bits != 1) S.nthr = quant_table(B.quantizer, q.bits, S.thr);
            if (B.off_pk[2 * i + side]) {
                S.pk = reinterpret_cast<uint32_t*>(W + B.off_pk[2 * i + side]);
                S.pk_bits = pp.probe.fmt == kFmtF6 ? 6 : 4;
                // the FP engine reads only the packed codes; so does the
                // learned path's FP window kernel (the int8 one reads int8 codes)
                S.skip_q = B.learned && win_fp_width(q, pp, B) == 0 ? 0 : 1;
            }
            if (B.learned) {
                // decimated CNN input, written by the quantize kernel
                S.dec = reinterpret_cast<uint16_t*>(W + B.off_cnn) + (2 * i + side) * (int64_t)model_net(B.model).ld;
                S.dec_mul = 6.f / (float)(2 * kmax_of_bits(q.bits) + 1);
            }
            if (q.bits != 1 && !(fixed > 0.f)) L.need_scale = true;
            L.min_n = S.n < L.min_n ? S.n : L.min_n;
            L.max_n = S.n > L.max_n ? S.n : L.max_n;
            bbase += ceil_div(S.n, kQuantBlock);
        }
        XItem& it = items[i];
        it = pp.probe;                     // plan (tiles, flags, outside triple)
        it.engine = pp.eng;
        it.p.u = sigs[2 * i].q;
        it.p.v = sigs[2 * i + 1].q;
        it.p.upk = sigs[2 * i].pk;
        it.p.vpk = sigs[2 * i + 1].pk;
        it.p.r = pp.need_r ? (q.r_out ? q.r_out : (void*)(W + B.off_r[i])) : nullptr;
        it.p.r_dtype = pp.rdt;
        it.stat_x = stats + 2 * i;
        it.stat_y = stats + 2 * i + 1;
        it.peak = out + i;
        it.fused = pp.fused ? 1 : 0;
        if (B.learned) {
            it.margin = reinterpret_cast<const float*>(W + B.off_margin) + i;
            it.theta = B.theta;
            it.nwin = B.topk;
            it.win_parts = reinterpret_cast<const ArgPart*>(W + B.off_wparts) + i * B.topk;
            it.win_w = win_fp_width(q, pp, B);
            L.win_formats |= it.win_w == 6 ? 2 : it.win_w == 4 ? 4 : 1;
        }
        if (it.p.r) {
            L.any_r = true;
            L.max_rbytes = std::max<int64_t>(L.max_rbytes, (q.lag_hi - q.lag_lo + 1) * (pp.rdt == TDE_I32 ? 4 : 8));
        }
        if (pp.eng == TDE_PATH_MFMA) {
            L.any_mfma = true;
            if (pp.fused) {
                it.part_base = tbase;
                tbase += it.ntiles;
                L.any_fused = true;
            }
            it.work_first = (int32_t)work.size();
            mfma_items(it, (int)i, work);
            it.work_count = (int32_t)(work.size() - it.work_first);
        } else if (pp.eng == TDE_PATH_NTT) {
            it.part_base = tbase;
            tbase += it.ntiles;
            L.any_fused = true;
        } else {
            popc_plan(it, W + B.off_planes[i]);
            L.p_split = std::max(L.p_split, it.nsplit);
            L.p_tiles = std::max(L.p_tiles, it.ntiles);
            L.p_words = std::max(L.p_words, std::max(it.nuw, it.nvw));
            L.any_popc = true;
            L.p_zero_words = std::max(L.p_zero_words, it.plane_words);
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
            sg.nx = q.nx;
            sg.ny = q.ny;
            pbase += sg.nparts;
            segs.push_back(sg);
        }
    }
    // NTT jobs, grouped by transform length and prime count
    std::vector<NttJob> jobs;
    for (const auto& g : B.ngroups) {
        NttPlan P{};
        P.log_n = g.log_n;
        P.nprimes = g.nprimes;
        P.wc3 = B.pp[g.pairs[0]].ntt.wc3;
        L.ngroups.push_back({ntt_group(P, reinterpret_cast<uint32_t*>(W + g.off_tab)), (int64_t)jobs.size()});
        L.ngroup_jobs.push_back((int)g.pairs.size());
        for (int64_t i : g.pairs) {
            const tde_pair& q = pairs[i];
            const PairPlan& pp = B.pp[i];
            const XItem& it = items[i];
            NttJob J{};
            J.u = it.p.u;
            J.v = it.p.v;
            J.nu = q.nx;
            J.nv = q.ny;
            J.lag_lo = q.lag_lo;
            J.jlo = pp.ntt.jlo;
            J.jhi = pp.ntt.jhi;
            J.r = it.p.r;
            J.r_dtype = it.p.r_dtype;
            J.res = reinterpret_cast<uint32_t*>(W + B.off_res[i]);
            J.parts = reinterpret_cast<ArgPart*>(W + B.off_tparts) + it.part_base;
            jobs.push_back(J);
        }
    }
    // longest first; a list the device plans from keeps pair order (each
    // pair's items at work_first .. work_first + work_count - 1)
    if (!B.fb_dyn) mfma_sort_items(work);
    L.bbase = bbase;
    L.pbase = pbase;
    L.nwork = (int)work.size();
    L.n4 = 0;
    for (const MWork& w : work) L.n4 += mfma_launch_of(w.fmt, w.mb) == 4 ? 1 : 0;
    L.nsegs = (int)segs.size();
    L.blob.assign(B.off_work + work.size() * sizeof(MWork), 0);
    memcpy(L.blob.data() + B.off_qsig, sigs.data(), sizeof(QSig) * 2 * np);
    memcpy(L.blob.data() + B.off_items, items.data(), sizeof(XItem) * np);
    if (!segs.empty()) memcpy(L.blob.data() + B.off_segs, segs.data(), sizeof(ArgSeg) * segs.size());
    if (!work.empty()) memcpy(L.blob.data() + B.off_work, work.data(), work.size() * sizeof(MWork));
    if (!jobs.empty()) memcpy(L.blob.data() + B.off_jobs, jobs.data(), jobs.size() * sizeof(NttJob));
}

// Queues the kernels of a prepared batch on s (the descriptors are already in
// the workspace). No memset or copy nodes: safe to capture in a graph.
int batch_enqueue(tde_ctx* ctx, uint8_t* W, const BatchPlan& B, const BatchLaunch& L, hipStream_t s, bool timed) {
    const QSig* sigs_dev = reinterpret_cast<const QSig*>(W + B.off_qsig);
    const XItem* items_dev = reinterpret_cast<const XItem*>(W + B.off_items);
    const ArgSeg* segs_dev = reinterpret_cast<const ArgSeg*>(W + B.off_segs);
    ArgPart* tparts = reinterpret_cast<ArgPart*>(W + B.off_tparts);
    XItem none{};
    ArgSeg noseg{};
    QSig nosig{};
    auto mk = [&](void) { return timed ? mark(ctx, s) : nullptr; };
    hipEvent_t t_q0 = mk();
    int rc = launch_quantize(sigs_dev, nosig, (int)(2 * L.np), L.bbase, L.need_scale, false,
                             L.any_mfma ? reinterpret_cast<int*>(W + B.off_counters) : nullptr, 2, s, L.min_n, L.max_n);
    if (rc) return rc;
    hipEvent_t t_q1 = mk();
    if (timed) mark_stage(ctx, 0, t_q0, t_q1);
    if (L.any_r) {
        rc = launch_zero_r(items_dev, none, (int)L.np, L.max_rbytes, s);
        if (rc) return rc;
    }
    hipEvent_t t_e0 = mk();
    if (B.learned) {
        // proposer: decimate + encoder + head + top-k, then the windows
        int32_t* top = reinterpret_cast<int32_t*>(W + B.off_top);
        float* margin = reinterpret_cast<float*>(W + B.off_margin);
        hipEvent_t t_p0 = mk();
        rc = cnn_infer(B.model, reinterpret_cast<const uint16_t*>(W + B.off_cnn), (int)L.np, W + B.off_cnn, B.topk,
                       top, margin, nullptr, s, nullptr);
        if (rc) return rc;
        hipEvent_t t_p1 = mk();
        if (timed) mark_stage(ctx, 4, t_p0, t_p1);
        rc = launch_xcorr_win(items_dev, (int)L.np, top, margin, B.theta, B.topk, model_net(B.model).nb,
                              reinterpret_cast<ArgPart*>(W + B.off_wparts), s, L.win_formats);
        if (rc) return rc;
        hipEvent_t t_w1 = mk();
        if (timed) mark_stage(ctx, 5, t_p1, t_w1);
    }
    if (L.any_popc) {
        // zero the plane buffers (padding must read as 0), then pack
        rc = launch_popc_zero(items_dev, none, (int)L.np, L.p_zero_words, s);
        if (rc) return rc;
        rc = launch_popc_pack(items_dev, none, (int)L.np, L.p_words, s);
        if (rc) return rc;
        rc = launch_xcorr_popc(items_dev, none, (int)L.np, L.p_split, L.p_tiles, s);
        if (rc) return rc;
    }
    for (size_t k = 0; k < L.ngroups.size(); ++k) {
        rc = launch_ntt(L.ngroups[k].first, reinterpret_cast<const NttJob*>(W + B.off_jobs) + L.ngroups[k].second,
                        L.ngroup_jobs[k], s);
        if (rc) return rc;
    }
    int* fb_ctl = reinterpret_cast<int*>(W + B.off_fbctl);
    int* fb_slots = reinterpret_cast<int*>(W + B.off_fbslots);
    if (L.any_mfma) {
        hipEvent_t t_m0 = mk();
        if (B.fb_dyn) {
            // the fallback pairs' items, cut so that they fill the device
            // (about two items per resident workgroup of the engine)
            MWork* dwork = reinterpret_cast<MWork*>(W + B.off_dwork);
            rc = launch_fb_plan(items_dev, (int)L.np, reinterpret_cast<const MWork*>(W + B.off_work), dwork, fb_ctl,
                                fb_slots, 4 * ctx->num_cu, s);
            if (rc) return rc;
            rc = launch_fb_zero(items_dev, fb_ctl, fb_slots, W + B.off_rpool, B.fb_slot_bytes, s);
            if (rc) return rc;
            rc = launch_xcorr_mfma(items_dev, dwork, (int)B.fb_cap, reinterpret_cast<int*>(W + B.off_counters), true,
                                   tparts, ctx->num_cu, s, (int)B.fb_cap, fb_ctl + 1, W + B.off_rpool, B.fb_slot_bytes);
        } else {
            rc = launch_xcorr_mfma(items_dev, reinterpret_cast<const MWork*>(W + B.off_work), L.nwork,
                                   reinterpret_cast<int*>(W + B.off_counters), true, tparts, ctx->num_cu, s, L.n4);
        }
        if (rc) return rc;
        hipEvent_t t_m1 = mk();
        if (timed) mark_stage(ctx, 6, t_m0, t_m1);
    }
    hipEvent_t t_e1 = mk();
    if (timed) mark_stage(ctx, 1, t_e0, t_e1);
    if (L.any_fused) {
        rc = launch_tiles_final(items_dev, none, (int)L.np, tparts, s);
        if (rc) return rc;
    }
    if (B.fb_dyn && L.any_mfma) {
        rc = launch_fb_argmax(items_dev, fb_ctl, fb_slots, W + B.off_rpool, B.fb_slot_bytes,
                              reinterpret_cast<ArgPart*>(W + B.off_fbparts), s);
        if (rc) return rc;
    }
    if (L.nsegs) {
        rc = launch_argmax(segs_dev, noseg, L.nsegs, L.pbase, reinterpret_cast<ArgPart*>(W + B.off_parts), s);
        if (rc) return rc;
    }
    hipEvent_t t_end = mk();
    if (timed) mark_stage(ctx, 2, t_e1, t_end);
    return TDE_OK;
}

std::vector<uint8_t> batch_signature(const tde_pair* pairs, int64_t np, const tde_opts* opts, const void* ws,
                                     size_t ws_bytes, const tde_peak* out) {
    std::vector<uint8_t> sig(sizeof(tde_pair) * np + sizeof(tde_opts) + 3 * sizeof(uint64_t));
    uint8_t* d = sig.data();
    memcpy(d, pairs, sizeof(tde_pair) * np);
    d += sizeof(tde_pair) * np;
    memcpy(d, opts, sizeof(tde_opts));
    d += sizeof(tde_opts);
    uint64_t extra[3] = {(uint64_t)(uintptr_t)ws, (uint64_t)ws_bytes, (uint64_t)(uintptr_t)out};
    memcpy(d, extra, sizeof(extra));
    return sig;
}

}  // namespace

extern "C" {

int tde_estimate_batch(tde_ctx* ctx, const tde_pair* pairs, int64_t np, const tde_opts* opts, tde_peak* out,
                       void* ws, size_t ws_bytes, void* stream) {
    if (!out) return set_error(TDE_ERR_ARG, "tde_estimate_batch: null out");
    int rc = validate_pairs(pairs, np, opts);
    if (rc) return rc;
    const bool use_graph = opts && opts->use_graph;
    if (!ctx) {
        BatchPlan B = plan_batch(pairs, np, opts);
        if (!ws || ws_bytes < B.total)
            return set_error(TDE_ERR_WS, "tde_estimate_batch: workspace %zu < %zu bytes", ws_bytes, B.total);
        return set_error(TDE_ERR_ARG, "tde_estimate_batch: null context");
    }
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_estimate_batch: hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uint8_t> sig;
    if (use_graph) {
        sig = batch_signature(pairs, np, opts, ws, ws_bytes, out);
        for (auto& gr : ctx->graphs)
            if (gr.sig == sig) {
                TDE_HIP_CHECK(hipGraphLaunch(gr.exec, s));
                return TDE_OK;
            }
    }
    BatchPlan B = plan_batch(pairs, np, opts);
    if (!ws || ws_bytes < B.total)
        return set_error(TDE_ERR_WS, "tde_estimate_batch: workspace %zu < %zu bytes", ws_bytes, B.total);
    uint8_t* W = static_cast<uint8_t*>(ws);
    BatchLaunch L;
    batch_prepare(ctx, pairs, np, out, W, B, L);
    drop_graphs_on(ctx, ws, B.total);
    if (!use_graph) {
        hipEvent_t t_begin = mark(ctx, s);
        rc = upload(ctx, W, L.blob.data(), L.blob.size(), s);
        if (rc) return rc;
        rc = batch_enqueue(ctx, W, B, L, s, true);
        if (rc) return rc;
        hipEvent_t t_end = mark(ctx, s);
        mark_stage(ctx, 3, t_begin, t_end);
        return TDE_OK;
    }
    // graph: descriptors go in once, synchronously, then the kernels are
    // captured on the context's stream and replayed on the caller's.
    TDE_HIP_CHECK(hipStreamSynchronize(s));
    TDE_HIP_CHECK(hipMemcpy(W, L.blob.data(), L.blob.size(), hipMemcpyHostToDevice));
    TDE_HIP_CHECK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = batch_enqueue(ctx, W, B, L, ctx->cap_stream, false);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) return set_error(TDE_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ec != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return set_error(TDE_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(ec));
    }
    if (ctx->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(ctx->graphs.front().exec);
        (void)hipGraphDestroy(ctx->graphs.front().graph);
        ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({std::move(sig), (uintptr_t)ws, (uintptr_t)ws + B.total, graph, exec});
    TDE_HIP_CHECK(hipGraphLaunch(exec, s));
    return TDE_OK;
}

}  // extern "C"

// ------------------------------------------------------- model inputs --

namespace {

int check_model_pairs(const tde_model* M, const tde_pair* pairs, int64_t np, const char* who) {
    if (!pairs || np < 1 || np > 65535) return set_error(TDE_ERR_ARG, "%s: 1..65535 pairs", who);
    const int64_t n = M ? 16 * (int64_t)model_net(M).ld : -1;
    for (int64_t i = 0; i < np; ++i) {
        const tde_pair& q = pairs[i];
        if (!q.x || !q.y) return set_error(TDE_ERR_ARG, "%s: pair %lld: null signal", who, (long long)i);
        if (q.bits != 2 && q.bits != 4 && q.bits != 8)
            return set_error(TDE_ERR_ARG, "%s: pair %lld: bits must be 2, 4 or 8", who, (long long)i);
        if (M && (q.nx != n || q.ny != n))
            return set_error(TDE_ERR_ARG, "%s: pair %lld: signals must have 16 ld = %lld samples", who, (long long)i,
                             (long long)n);
        if (q.nx < 1 || q.ny < 1 || (q.nx % 16) || (q.ny % 16))
            return set_error(TDE_ERR_ARG, "%s: pair %lld: lengths must be multiples of 16", who, (long long)i);
        if (!std::isfinite(q.inv_step_x) || !std::isfinite(q.inv_step_y))
            return set_error(TDE_ERR_ARG, "%s: pair %lld: non-finite inv_step", who, (long long)i);
    }
    return TDE_OK;
}

struct PrepPlan {
    size_t off_qsig, off_csig, off_stats, off_inv, total;
    std::vector<size_t> off_q, off_gsum;
};

PrepPlan plan_prepare(const tde_pair* pairs, int64_t np) {
    PrepPlan P;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off += align_bytes(b);
        return o;
    };
    P.off_qsig = take(sizeof(QSig) * 2 * np);
    P.off_csig = take(sizeof(CnnSig) * 2 * np);
    P.off_stats = take(sizeof(tde_qstat) * 2 * np);
    P.off_inv = take(sizeof(float) * 2 * np);
    P.off_q.resize(2 * np);
    P.off_gsum.resize(2 * np);
    for (int64_t i = 0; i < 2 * np; ++i) {
        const int64_t n = (i & 1) ? pairs[i / 2].ny : pairs[i / 2].nx;
        P.off_q[i] = take(n);
        P.off_gsum[i] = take((size_t)quantize_gsum_doubles(n) * 8);
    }
    P.total = off;
    return P;
}

// Quantizer scales of every signal (and its codes, in the workspace) and the
// descriptors of their decimation; shared by tde_model_prepare and the
// learned batch mode. Returns the number of quantize blocks.
int64_t fill_prepare(const tde_pair* pairs, int64_t np, uint8_t* W, const PrepPlan& P, std::vector<uint8_t>& blob,
                     bool& need_scale) {
    blob.assign(P.off_stats, 0);
    QSig* sigs = reinterpret_cast<QSig*>(blob.data() + P.off_qsig);
    CnnSig* cs = reinterpret_cast<CnnSig*>(blob.data() + P.off_csig);
    tde_qstat* stats = reinterpret_cast<tde_qstat*>(W + P.off_stats);
    float* invs = reinterpret_cast<float*>(W + P.off_inv);
    int64_t bbase = 0;
    need_scale = false;
    for (int64_t i = 0; i < 2 * np; ++i) {
        const tde_pair& q = pairs[i / 2];
        const int side = (int)(i & 1);
        QSig S{};
        S.x = side ? q.y : q.x;
        S.n = side ? q.ny : q.nx;
        S.q = reinterpret_cast<int8_t*>(W + P.off_q[i]);
        S.stat = stats + i;
        S.gsum = reinterpret_cast<double*>(W + P.off_gsum[i]);
        S.inv_out = invs + i;
        S.blk_base = bbase;
        const float fixed = side ? q.inv_step_y : q.inv_step_x;
        S.inv_fixed = fixed > 0.f ? fixed : 0.f;
        S.bits = q.bits;
        if (!(fixed > 0.f)) need_scale = true;
        bbase += ceil_div(S.n, kQuantBlock);
        sigs[i] = S;
        cs[i] = CnnSig{S.x, S.inv_out, 6.f / (float)(2 * kmax_of_bits(q.bits) + 1)};
    }
    return bbase;
}

}  // namespace

extern "C" {

size_t tde_model_prepare_workspace_size(const tde_pair* pairs, int64_t np) {
    if (check_model_pairs(nullptr, pairs, np, "tde_model_prepare_workspace_size") != TDE_OK) return 0;
    return plan_prepare(pairs, np).total;
}

int tde_model_prepare(tde_ctx* ctx, const tde_model* M, const tde_pair* pairs, int64_t np, uint16_t* xdec, void* ws,
                      size_t ws_bytes, void* stream) {
    if (!M || !xdec) return set_error(TDE_ERR_ARG, "tde_model_prepare: null model or output");
    int rc = check_model_pairs(M, pairs, np, "tde_model_prepare");
    if (rc) return rc;
    PrepPlan P = plan_prepare(pairs, np);
    if (!ws || ws_bytes < P.total)
        return set_error(TDE_ERR_WS, "tde_model_prepare: workspace %zu < %zu bytes", ws_bytes, P.total);
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_model_prepare: null context");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return set_error(TDE_ERR_HIP, "tde_model_prepare: hipSetDevice failed");
    hipStream_t s = static_cast<hipStream_t>(stream);
    uint8_t* W = static_cast<uint8_t*>(ws);
    std::vector<uint8_t> blob;
    bool need_scale = false;
    const int64_t nblk = fill_prepare(pairs, np, W, P, blob, need_scale);
    drop_graphs_on(ctx, ws, P.total);
    rc = upload(ctx, W, blob.data(), blob.size(), s);
    if (rc) return rc;
    QSig none{};
    rc = launch_quantize(reinterpret_cast<const QSig*>(W + P.off_qsig), none, (int)(2 * np), nblk, need_scale, false,
                         nullptr, 0, s);
    if (rc) return rc;
    return launch_cnn_decimate(reinterpret_cast<const CnnSig*>(W + P.off_csig), (int)(2 * np), model_net(M).ld, xdec,
                               s);
}

}  // extern "C"
