// Correlation of a stream against a template, block by block (overlap-save):
// the extension to long and streaming signals that Section 5 names as future
// work, assembled from the steps of Algorithm 1 from quantization to argmax.
//
// The stream's codes live in two alternating buffers laid out as
//     [ last nx - 1 codes of the stream | the call's n new codes ]
// (zeros before the stream's start, and after its end for the finishing
// call). Buffer position p holds stream sample p - (nx - 1) + T for T samples
// before the call, so the correlation of the template with the buffer at
// buffer lags 0 .. n - 1 is r at stream lags T - nx + 1 .. T - nx + n
// (Eq. (1)), each with the template's whole overlap inside the buffer. The
// engines of tde_xcorr_int compute it exactly; tde_argmax_lag takes the
// call's peak, and k_peak_merge folds it into the running peak (later calls
// hold larger lags, so an equal maximum only adds to the count).
//
// Steady state: when the matrix-core engine takes calls of max_block samples
// without cutting tiles into segments, the stream plans that call once per
// buffer (item descriptors, sorted work list, packed template codes) and a
// push that asks for no r only launches kernels: quantize, pack the buffer's
// codes (FP4/FP6 operands), the engine with its fused per-tile argmax,
// the per-pair peak, the merge and the history copy; no host planning, no
// upload, no wait on the device.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tde_internal.h"

using namespace tde;

struct tde_stream {
    tde_ctx* ctx = nullptr;
    int device = 0;
    int64_t nx = 0;
    int bits = 0, kmax = 0, path = 0;
    float inv_y = 0.f;
    int64_t max_block = 0, cap = 0;   // cap: largest call (max(max_block, nx - 1))
    int8_t* u = nullptr;              // template codes
    int8_t* buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t* r = nullptr;             // r of a call when the caller passes none (int64)
    uint8_t* ws = nullptr;            // engine workspace, then argmax workspace
    size_t ws_x = 0, ws_a = 0;
    tde_peak* blk = nullptr;          // peak of the last call
    tde_peak* run = nullptr;          // running peak
    int64_t pos = 0;
    bool finished = false;
    // cached plan of a max_block call (matrix-core engine, no segments)
    bool fast = false;
    int fmt = 0;
    uint8_t* fdev = nullptr;          // [2 items][work list][2 counters][tile triples]
    XItem* fitems = nullptr;
    MWork* fwork = nullptr;
    int nwork = 0, n4 = 0;
    int* fcount = nullptr;
    ArgPart* ftparts = nullptr;
    uint32_t* upk = nullptr;          // packed template codes
    uint32_t* vpk[2] = {nullptr, nullptr};
};

namespace {

struct Dev {
    int prev = -1;
    explicit Dev(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~Dev() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// blk's lag is shifted by lag_add (buffer to stream lags; 0 when it already
// holds stream lags)
__global__ void k_peak_merge(tde_peak* blk, tde_peak* run, int first, tde_peak* blk_out, tde_peak* run_out,
                             int64_t lag_add) {
    if (threadIdx.x != 0) return;
    tde_peak b = *blk;
    b.lag += lag_add;
    b.flags = 0;
    *blk = b;
    tde_peak r = *run;
    if (first || b.rmax > r.rmax) {
        r = b;
    } else if (b.rmax == r.rmax) {
        r.n_ties += b.n_ties;
    }
    *run = r;
    if (blk_out) *blk_out = b;
    if (run_out) *run_out = r;
}

__global__ void k_peak_copy(const tde_peak* run, tde_peak* out) {
    if (threadIdx.x == 0) *out = *run;
}

bool stream_path_ok(int path, int bits) {
    if (path == TDE_PATH_POPC) return bits == 1;
    return path == TDE_PATH_AUTO || path == TDE_PATH_MFMA || path == TDE_PATH_MFMA_I8 || path == TDE_PATH_NTT;
}

// One call over n buffer lags: the codes are in buf[cur][nx - 1, nx - 1 + n).
int stream_step(tde_stream* st, int64_t n, void* r_out, int r_dtype, tde_peak* block_peak, tde_peak* running_peak,
                hipStream_t s) {
    const int64_t nx = st->nx;
    int8_t* b = st->buf[st->cur];
    void* r = r_out ? r_out : (void*)st->r;
    const int rdt = r_out ? r_dtype : TDE_I64;
    const size_t need = tde_xcorr_workspace_size(nx, nx - 1 + n, st->kmax, st->kmax, 0, n - 1, st->path);
    if (need > st->ws_x) return set_error(TDE_ERR_WS, "tde_stream: engine workspace %zu < %zu", st->ws_x, need);
    int rc = tde_xcorr_int(st->ctx, st->u, nx, b, nx - 1 + n, st->kmax, st->kmax, 0, n - 1, r, rdt, st->path,
                           st->ws, st->ws_x, s);
    if (rc) return rc;
    const int64_t lo = st->pos - nx + 1;
    rc = tde_argmax_lag(st->ctx, r, rdt, lo, lo + n - 1, st->blk, st->ws + st->ws_x, st->ws_a, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_peak_merge, dim3(1), dim3(64), 0, s, st->blk, st->run, st->pos == 0 ? 1 : 0, block_peak,
                       running_peak, (int64_t)0);
    TDE_HIP_CHECK(hipGetLastError());
    // the last nx - 1 codes become the next call's history
    const int nxt = 1 - st->cur;
    rc = launch_copy_bytes(st->buf[nxt], b + n, (size_t)(nx - 1), s);
    if (rc) return rc;
    st->cur = nxt;
    return TDE_OK;
}

// A max_block call on the cached plan (no r): the codes are in buf[cur].
int stream_step_fast(tde_stream* st, tde_peak* block_peak, tde_peak* running_peak, hipStream_t s) {
    const int64_t nx = st->nx, n = st->max_block;
    int8_t* b = st->buf[st->cur];
    int rc = TDE_OK;
    if (st->fmt != kFmtI8) rc = launch_pack_fp(b, nx - 1 + n, st->vpk[st->cur], st->fmt == kFmtF6 ? 6 : 4, s);
    if (rc) return rc;
    const XItem* it = st->fitems + st->cur;
    rc = launch_xcorr_mfma(it, st->fwork, st->nwork, st->fcount, false, st->ftparts, ctx_num_cu(st->ctx), s, st->n4);
    if (rc) return rc;
    XItem none{};
    rc = launch_tiles_final(it, none, 1, st->ftparts, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_peak_merge, dim3(1), dim3(64), 0, s, st->blk, st->run, st->pos == 0 ? 1 : 0, block_peak,
                       running_peak, st->pos - nx + 1);
    TDE_HIP_CHECK(hipGetLastError());
    const int nxt = 1 - st->cur;
    rc = launch_copy_bytes(st->buf[nxt], b + n, (size_t)(nx - 1), s);
    if (rc) return rc;
    st->cur = nxt;
    return TDE_OK;
}

// Plans a max_block call once per buffer when the matrix-core engine takes it
// whole (no segments); otherwise calls take the general path.
int stream_plan_fast(tde_stream* st, hipStream_t s) {
    const int64_t nx = st->nx, n = st->max_block;
    const int K = st->kmax;
    int eng = st->path;
    if (eng == TDE_PATH_AUTO) eng = tde_tune_query(nx, nx - 1 + n, K, K, 0, n - 1);
    if (eng != TDE_PATH_MFMA && eng != TDE_PATH_MFMA_I8) return TDE_OK;
    XItem it{};
    it.p.u = st->u;
    it.p.nu = nx;
    it.p.nv = nx - 1 + n;
    it.p.lag_lo = 0;
    it.p.lag_hi = n - 1;
    it.p.r = nullptr;
    it.p.r_dtype = TDE_I64;
    it.p.kuv = K * K;
    it.p.kmax = K;
    mfma_plan_pair(it, st->path != TDE_PATH_MFMA_I8);
    if (it.segmented) return TDE_OK;
    it.engine = TDE_PATH_MFMA;
    it.fused = 1;
    it.part_base = 0;
    it.peak = st->blk;
    std::vector<MWork> work;
    mfma_items(it, 0, work);
    mfma_sort_items(work);
    const int wb = it.fmt == kFmtF6 ? 6 : 4;
    const size_t o_items = 0, o_work = align_bytes(2 * sizeof(XItem));
    const size_t o_cnt = o_work + align_bytes(work.size() * sizeof(MWork));
    const size_t o_tp = o_cnt + align_bytes(2 * sizeof(int));
    size_t o_pk = o_tp + align_bytes((size_t)(it.ntiles > 0 ? it.ntiles : 1) * sizeof(ArgPart));
    size_t total = o_pk;
    size_t o_upk = 0, o_vpk0 = 0, o_vpk1 = 0;
    if (it.fmt != kFmtI8) {
        o_upk = total;
        total += align_bytes(packed_bytes(nx, wb));
        o_vpk0 = total;
        total += align_bytes(packed_bytes(nx - 1 + n, wb));
        o_vpk1 = total;
        total += align_bytes(packed_bytes(nx - 1 + n, wb));
    }
    if (hipMalloc(&st->fdev, total) != hipSuccess) return set_error(TDE_ERR_HIP, "tde_stream_create: allocation failed");
    uint8_t* D = st->fdev;
    if (it.fmt != kFmtI8) {
        st->upk = reinterpret_cast<uint32_t*>(D + o_upk);
        st->vpk[0] = reinterpret_cast<uint32_t*>(D + o_vpk0);
        st->vpk[1] = reinterpret_cast<uint32_t*>(D + o_vpk1);
        int rc = launch_pack_fp(st->u, nx, st->upk, wb, s);
        if (rc) return rc;
        it.p.upk = st->upk;
    }
    XItem two[2] = {it, it};
    for (int p = 0; p < 2; ++p) {
        two[p].p.v = st->buf[p];
        two[p].p.vpk = st->vpk[p];
    }
    std::vector<uint8_t> blob(o_cnt, 0);
    memcpy(blob.data() + o_items, two, sizeof(two));
    if (!work.empty()) memcpy(blob.data() + o_work, work.data(), work.size() * sizeof(MWork));
    TDE_HIP_CHECK(hipStreamSynchronize(s));
    TDE_HIP_CHECK(hipMemcpy(D, blob.data(), blob.size(), hipMemcpyHostToDevice));
    st->fitems = reinterpret_cast<XItem*>(D + o_items);
    st->fwork = reinterpret_cast<MWork*>(D + o_work);
    st->nwork = (int)work.size();
    st->n4 = mfma_launch_of(it.fmt, it.mb) == 4 ? (int)work.size() : 0;
    st->fcount = reinterpret_cast<int*>(D + o_cnt);
    st->ftparts = reinterpret_cast<ArgPart*>(D + o_tp);
    st->fmt = it.fmt;
    st->fast = true;
    return TDE_OK;
}

}  // namespace

extern "C" {

int tde_stream_create(tde_ctx* ctx, const float* x, int64_t nx, int bits, float inv_step_x, float inv_step_y,
                      int64_t max_block, int path, tde_stream** out, void* stream) {
    if (!out) return set_error(TDE_ERR_ARG, "tde_stream_create: null output");
    *out = nullptr;
    if (!x) return set_error(TDE_ERR_ARG, "tde_stream_create: null template");
    if (nx < 1) return set_error(TDE_ERR_ARG, "tde_stream_create: nx < 1");
    if (bits != 1 && bits != 2 && bits != 4 && bits != 8)
        return set_error(TDE_ERR_ARG, "tde_stream_create: bits = %d not in {1,2,4,8}", bits);
    if (!std::isfinite(inv_step_x) || inv_step_x < 0.f || !std::isfinite(inv_step_y) || inv_step_y < 0.f)
        return set_error(TDE_ERR_ARG, "tde_stream_create: scales must be finite and >= 0");
    if (bits != 1 && !(inv_step_y > 0.f))
        return set_error(TDE_ERR_ARG, "tde_stream_create: the stream needs a fixed scale inv_step_y > 0");
    if (max_block < 1) return set_error(TDE_ERR_ARG, "tde_stream_create: max_block < 1");
    if (!stream_path_ok(path, bits)) return set_error(TDE_ERR_ARG, "tde_stream_create: path %d", path);
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_stream_create: null context");
    const int K = kmax_of_bits(bits);
    const int64_t cap = max_block > nx - 1 ? max_block : nx - 1;
    // The largest call must be plannable (the NTT has a largest transform).
    // Each engine's workspace grows with the call's length, so sizing for the
    // largest call covers every call; under AUTO a call may take any engine
    // that fits, so the workspace covers all of them.
    size_t ws_x = tde_xcorr_workspace_size(nx, nx - 1 + cap, K, K, 0, cap - 1, path);
    if (ws_x == 0) return set_error(TDE_ERR_UNSUPPORTED, "tde_stream_create: no engine plan for %lld-sample calls",
                                    (long long)cap);
    if (path == TDE_PATH_AUTO)
        for (int e : {TDE_PATH_MFMA, TDE_PATH_POPC, TDE_PATH_NTT}) {
            if (e == TDE_PATH_POPC && bits != 1) continue;
            const size_t w = tde_xcorr_workspace_size(nx, nx - 1 + cap, K, K, 0, cap - 1, e);
            if (w > ws_x) ws_x = w;
        }
    tde_stream* st = new tde_stream();
    st->ctx = ctx;
    st->device = ctx_device(ctx);
    st->nx = nx;
    st->bits = bits;
    st->kmax = K;
    st->path = path;
    st->inv_y = inv_step_y;
    st->max_block = max_block;
    st->cap = cap;
    st->ws_x = align_bytes(ws_x);
    st->ws_a = align_bytes(tde_argmax_workspace_size(cap));
    Dev dv(st->device);
    const size_t qws = tde_quantize_workspace_size(nx);
    void* qtmp = nullptr;
    if (hipMalloc(&st->u, (size_t)nx) != hipSuccess || hipMalloc(&st->buf[0], (size_t)(nx - 1 + cap)) != hipSuccess ||
        hipMalloc(&st->buf[1], (size_t)(nx - 1 + cap)) != hipSuccess ||
        hipMalloc(&st->r, (size_t)cap * 8) != hipSuccess || hipMalloc(&st->ws, st->ws_x + st->ws_a) != hipSuccess ||
        hipMalloc(&st->blk, 2 * sizeof(tde_peak)) != hipSuccess || hipMalloc(&qtmp, qws) != hipSuccess) {
        if (qtmp) (void)hipFree(qtmp);
        tde_stream_destroy(st);
        return set_error(TDE_ERR_HIP, "tde_stream_create: allocation failed");
    }
    st->run = st->blk + 1;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = tde_quantize(ctx, x, nx, bits, inv_step_x, st->u, nullptr, qtmp, qws, s);
    if (!rc) rc = launch_zero(st->buf[0], (size_t)(nx - 1), s);      // nothing before the stream's start
    if (!rc) rc = launch_zero(st->blk, 2 * sizeof(tde_peak), s);
    if (!rc) rc = stream_plan_fast(st, s);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = set_error(TDE_ERR_HIP, "tde_stream_create: sync failed");
    (void)hipFree(qtmp);
    if (rc) {
        tde_stream_destroy(st);
        return rc;
    }
    *out = st;
    return TDE_OK;
}

int tde_stream_push(tde_stream* st, const float* y, int64_t n, void* r_out, int r_dtype, tde_peak* block_peak,
                    tde_peak* running_peak, void* stream) {
    if (!st) return set_error(TDE_ERR_ARG, "tde_stream_push: null stream");
    if (st->finished) return set_error(TDE_ERR_ARG, "tde_stream_push: the stream is finished");
    if (!y) return set_error(TDE_ERR_ARG, "tde_stream_push: null y");
    if (n < 1 || n > st->max_block)
        return set_error(TDE_ERR_ARG, "tde_stream_push: n = %lld not in [1, %lld]", (long long)n,
                         (long long)st->max_block);
    if (r_out) {
        if (r_dtype != TDE_I32 && r_dtype != TDE_I64) return set_error(TDE_ERR_ARG, "tde_stream_push: bad r_dtype");
        if (((uintptr_t)r_out) & (r_dtype == TDE_I32 ? 3 : 7))
            return set_error(TDE_ERR_ARG, "tde_stream_push: r_out is not aligned to its element size");
        if (r_dtype == TDE_I32 && (__int128)st->nx * st->kmax * st->kmax >= ((__int128)1 << 31))
            return set_error(TDE_ERR_RANGE, "tde_stream_push: int32 r cannot hold the exact values");
    }
    Dev dv(st->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = tde_quantize(st->ctx, y, n, st->bits, st->inv_y, st->buf[st->cur] + (st->nx - 1), nullptr, nullptr, 0,
                          s);
    if (rc) return rc;
    rc = (st->fast && n == st->max_block && !r_out) ? stream_step_fast(st, block_peak, running_peak, s)
                                                    : stream_step(st, n, r_out, r_dtype, block_peak, running_peak, s);
    if (rc) return rc;
    st->pos += n;
    return TDE_OK;
}

int tde_stream_finish(tde_stream* st, void* r_out, int r_dtype, tde_peak* block_peak, tde_peak* running_peak,
                      void* stream) {
    if (!st) return set_error(TDE_ERR_ARG, "tde_stream_finish: null stream");
    if (st->finished) return set_error(TDE_ERR_ARG, "tde_stream_finish: the stream is finished");
    if (r_out) {
        if (r_dtype != TDE_I32 && r_dtype != TDE_I64) return set_error(TDE_ERR_ARG, "tde_stream_finish: bad r_dtype");
        if (((uintptr_t)r_out) & (r_dtype == TDE_I32 ? 3 : 7))
            return set_error(TDE_ERR_ARG, "tde_stream_finish: r_out is not aligned to its element size");
        if (r_dtype == TDE_I32 && (__int128)st->nx * st->kmax * st->kmax >= ((__int128)1 << 31))
            return set_error(TDE_ERR_RANGE, "tde_stream_finish: int32 r cannot hold the exact values");
    }
    Dev dv(st->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = st->nx - 1;
    if (n > 0) {
        // zeros after the stream's end
        int rc = launch_zero(st->buf[st->cur] + (st->nx - 1), (size_t)n, s);
        if (rc) return rc;
        rc = stream_step(st, n, r_out, r_dtype, block_peak, running_peak, s);
        if (rc) return rc;
    } else if (running_peak) {
        hipLaunchKernelGGL(k_peak_copy, dim3(1), dim3(64), 0, s, st->run, running_peak);
        TDE_HIP_CHECK(hipGetLastError());
    }
    st->finished = true;
    return TDE_OK;
}

int64_t tde_stream_position(const tde_stream* st) { return st ? st->pos : -1; }

void tde_stream_destroy(tde_stream* st) {
    if (!st) return;
    Dev dv(st->device);
    (void)hipDeviceSynchronize();
    for (void* q : {(void*)st->u, (void*)st->buf[0], (void*)st->buf[1], (void*)st->r, (void*)st->ws, (void*)st->blk,
                    (void*)st->fdev})
        if (q) (void)hipFree(q);
    delete st;
}

}  // extern "C"
