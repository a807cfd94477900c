// Model object of the learned lag-window proposer: parameters, Adam state,
// activation buffers, and the C ABI calls that drive the CNN kernels.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "tde_internal.h"

struct tde_model {
    int device;
    tde::CnnNet net;
    float* p = nullptr;        // fp32 masters
    float* wc = nullptr;       // bf16-rounded copies used by the kernels
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    void* frag = nullptr;      // packed bf16 fragments of the matrix-core layers
    int step = 0;
    // training buffers, sized for up to cap pairs
    int cap = 0;
    void* buf = nullptr;
    tde::CnnActs acts{};
    tde::CnnGrad g{};
    float* raw = nullptr;
    float* logits = nullptr;
    int32_t* labels_tmp = nullptr;
    std::mutex mu;
};

namespace tde {

namespace {

struct Guard {
    int prev = -1;
    explicit Guard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~Guard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// He-normal initial weights from a seeded generator (splitmix64 + Box-Muller),
// zero biases, alpha = 1 / (C F) so that initial logits are O(1).
void init_host(const CnnNet& net, uint64_t seed, std::vector<float>& out) {
    out.assign(net.nparams, 0.f);
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 0x2509199740ull;
    auto next = [&]() {
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    for (int l = 0; l < kCnnLayers; ++l) {
        const int cin = l == 0 ? 1 : kCnnC;
        const double sd = sqrt(2.0 / (cin * kCnnK));
        const size_t o = cnn_param_offset(l);
        for (int e = 0; e < kCnnC * cin * kCnnK; e += 2) {
            const double u1 = next(), u2 = next();
            const double r = sqrt(-2.0 * log(u1));
            out[o + e] = (float)(sd * r * cos(6.283185307179586 * u2));
            if (e + 1 < kCnnC * cin * kCnnK) out[o + e + 1] = (float)(sd * r * sin(6.283185307179586 * u2));
        }
    }
    const int F = net.ld >> kCnnLayers;
    out[net.nparams - 1] = 1.f / (float)(kCnnC * F);
}

size_t act_bytes(const CnnNet& net, int B, bool train) {
    const size_t nsig = 2 * (size_t)B;
    size_t tot = align_bytes(nsig * net.ld * 2);                 // x[0]
    for (int l = 0; l < kCnnLayers; ++l) {
        const size_t L = (size_t)net.ld >> l;
        tot += align_bytes(nsig * (L / 2) * kCnnC * 2);          // x[l+1]
        if (train) tot += align_bytes(nsig * L * kCnnC * 2);     // z[l]
    }
    tot += 2 * align_bytes((size_t)B * net.nb * 4);             // raw, logits
    return tot;
}

// Carves the activations (and, for training, the gradient buffers) of B pairs.
void carve_acts(const CnnNet& net, int B, bool train, uint8_t* base, CnnActs& A, float*& raw, float*& logits,
                size_t& off) {
    const size_t nsig = 2 * (size_t)B;
    auto take = [&](size_t bytes) {
        uint8_t* p = base + off;
        off += align_bytes(bytes);
        return p;
    };
    A.x[0] = reinterpret_cast<uint16_t*>(take(nsig * net.ld * 2));
    for (int l = 0; l < kCnnLayers; ++l) {
        const size_t L = (size_t)net.ld >> l;
        A.x[l + 1] = reinterpret_cast<uint16_t*>(take(nsig * (L / 2) * kCnnC * 2));
        A.z[l] = train ? reinterpret_cast<uint16_t*>(take(nsig * L * kCnnC * 2)) : nullptr;
    }
    raw = reinterpret_cast<float*>(take((size_t)B * net.nb * 4));
    logits = reinterpret_cast<float*>(take((size_t)B * net.nb * 4));
}

size_t grad_bytes(const CnnNet& net, int B) {
    const size_t nsig = 2 * (size_t)B;
    size_t tot = 0;
    for (int l = 1; l <= kCnnLayers; ++l) tot += align_bytes(nsig * ((size_t)net.ld >> l) * kCnnC * 4);
    // partials: largest layer count of workgroups x values per layer
    size_t part = 0;
    for (int l = 0; l < kCnnLayers; ++l) {
        const size_t L = (size_t)net.ld >> l;
        const size_t nchunk = (L + 511) / 512;
        const size_t n = kCnnC * (l == 0 ? 1 : kCnnC) * kCnnK + kCnnC;
        part = part > nchunk * nsig * n ? part : nchunk * nsig * n;
    }
    tot += align_bytes(part * 4);
    tot += align_bytes((size_t)B * net.nb * 4) + 2 * align_bytes((size_t)B * 4) + align_bytes(4 * B);
    return tot;
}

int ensure_train(tde_model* M, int B) {
    if (B <= M->cap) return TDE_OK;
    if (M->buf) TDE_HIP_CHECK(hipFree(M->buf));
    M->buf = nullptr;
    M->cap = 0;
    const size_t bytes = act_bytes(M->net, B, true) + grad_bytes(M->net, B);
    TDE_HIP_CHECK(hipMalloc(&M->buf, bytes));
    size_t off = 0;
    uint8_t* base = static_cast<uint8_t*>(M->buf);
    carve_acts(M->net, B, true, base, M->acts, M->raw, M->logits, off);
    const size_t nsig = 2 * (size_t)B;
    auto take = [&](size_t b) {
        uint8_t* p = base + off;
        off += align_bytes(b);
        return p;
    };
    M->g.dx[0] = nullptr;
    for (int l = 1; l <= kCnnLayers; ++l)
        M->g.dx[l] = reinterpret_cast<float*>(take(nsig * ((size_t)M->net.ld >> l) * kCnnC * 4));
    size_t part = 0;
    for (int l = 0; l < kCnnLayers; ++l) {
        const size_t L = (size_t)M->net.ld >> l;
        const size_t nchunk = (L + 511) / 512;
        const size_t n = kCnnC * (l == 0 ? 1 : kCnnC) * kCnnK + kCnnC;
        part = part > nchunk * nsig * n ? part : nchunk * nsig * n;
    }
    M->g.part = reinterpret_cast<float*>(take(part * 4));
    M->g.dlog = reinterpret_cast<float*>(take((size_t)B * M->net.nb * 4));
    M->g.dalpha = reinterpret_cast<float*>(take((size_t)B * 4));
    M->g.loss = reinterpret_cast<float*>(take((size_t)B * 4));
    M->labels_tmp = reinterpret_cast<int32_t*>(take(4 * (size_t)B));
    M->g.grad = M->grad;
    M->cap = B;
    return TDE_OK;
}

}  // namespace

size_t cnn_infer_bytes(const CnnNet& net, int B) { return act_bytes(net, B, false); }

int cnn_infer(const tde_model* M, const uint16_t* xdec_or_null, int B, uint8_t* ws, int topk, int32_t* top,
              float* margin, float* logits_out, hipStream_t s, const CnnSig* sigs_dev) {
    CnnActs A{};
    float *raw, *logits;
    size_t off = 0;
    carve_acts(M->net, B, false, ws, A, raw, logits, off);
    if (sigs_dev) {
        int rc = launch_cnn_decimate(sigs_dev, 2 * B, M->net.ld, A.x[0], s);
        if (rc) return rc;
    } else {
        A.x[0] = const_cast<uint16_t*>(xdec_or_null);
    }
    int rc = launch_cnn_forward(M->net, M->wc, A.x[0], B, A, raw, logits_out ? logits_out : logits, s);
    if (rc) return rc;
    if (top) return launch_cnn_topk(logits_out ? logits_out : logits, B, M->net.nb, topk, top, margin, s);
    return TDE_OK;
}

const CnnNet& model_net(const tde_model* M) { return M->net; }
int model_device(const tde_model* M) { return M->device; }

}  // namespace tde

using namespace tde;

extern "C" {

int tde_model_create(tde_ctx* ctx, int ld, int nbins, uint64_t seed, tde_model** out) {
    if (!out) return set_error(TDE_ERR_ARG, "tde_model_create: null output");
    *out = nullptr;
    if (ld < 256 || ld % 256 != 0 || ld > (1 << 20))
        return set_error(TDE_ERR_ARG, "tde_model_create: ld must be a multiple of 256 in [256, 2^20]");
    const int F = ld >> kCnnLayers;
    if (nbins < 64 || nbins % 64 != 0 || nbins > 2 * F || nbins > 1024)
        return set_error(TDE_ERR_ARG, "tde_model_create: nbins must be a multiple of 64, at most 2 ld / 16 and 1024");
    if (!ctx) return set_error(TDE_ERR_ARG, "tde_model_create: null context");
    tde_model* M = new tde_model();
    M->device = ctx_device(ctx);
    M->net.ld = ld;
    M->net.nb = nbins;
    M->net.nparams = cnn_param_count(kCnnLayers);
    M->net.frag = nullptr;
    Guard gd(M->device);
    const size_t n = (size_t)M->net.nparams * 4;
    if (hipMalloc(&M->p, n) != hipSuccess || hipMalloc(&M->wc, n) != hipSuccess || hipMalloc(&M->m, n) != hipSuccess ||
        hipMalloc(&M->v, n) != hipSuccess || hipMalloc(&M->grad, n) != hipSuccess ||
        hipMalloc(&M->frag, kCnnFragBytes) != hipSuccess) {
        tde_model_destroy(M);
        return set_error(TDE_ERR_HIP, "tde_model_create: allocation failed");
    }
    std::vector<float> h;
    init_host(M->net, seed, h);
    const int rc = tde_model_set_params(M, h.data(), M->net.nparams);
    if (rc) {
        tde_model_destroy(M);
        return rc;
    }
    *out = M;
    return TDE_OK;
}

void tde_model_destroy(tde_model* M) {
    if (!M) return;
    Guard gd(M->device);
    (void)hipDeviceSynchronize();
    for (void* q : {(void*)M->p, (void*)M->wc, (void*)M->m, (void*)M->v, (void*)M->grad, M->buf, M->frag})
        if (q) (void)hipFree(q);
    delete M;
}

int64_t tde_model_num_params(const tde_model* M) { return M ? M->net.nparams : (int64_t)set_error(TDE_ERR_ARG, "null model"); }

int tde_model_get_params(tde_model* M, float* host, int64_t n) {
    if (!M || !host) return set_error(TDE_ERR_ARG, "tde_model_get_params: null pointer");
    if (n != M->net.nparams) return set_error(TDE_ERR_ARG, "tde_model_get_params: %lld != %d values", (long long)n, M->net.nparams);
    std::lock_guard<std::mutex> lock(M->mu);
    Guard gd(M->device);
    TDE_HIP_CHECK(hipDeviceSynchronize());
    TDE_HIP_CHECK(hipMemcpy(host, M->p, (size_t)n * 4, hipMemcpyDeviceToHost));
    return TDE_OK;
}

int tde_model_set_params(tde_model* M, const float* host, int64_t n) {
    if (!M || !host) return set_error(TDE_ERR_ARG, "tde_model_set_params: null pointer");
    if (n != M->net.nparams) return set_error(TDE_ERR_ARG, "tde_model_set_params: %lld != %d values", (long long)n, M->net.nparams);
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(host[i])) return set_error(TDE_ERR_ARG, "tde_model_set_params: non-finite value %lld", (long long)i);
    std::lock_guard<std::mutex> lock(M->mu);
    Guard gd(M->device);
    TDE_HIP_CHECK(hipDeviceSynchronize());
    TDE_HIP_CHECK(hipMemcpy(M->p, host, (size_t)n * 4, hipMemcpyHostToDevice));
    TDE_HIP_CHECK(hipMemset(M->m, 0, (size_t)n * 4));
    TDE_HIP_CHECK(hipMemset(M->v, 0, (size_t)n * 4));
    M->step = 0;
    int rc = launch_round_copy(M->p, M->wc, (int)n, nullptr);
    if (rc) return rc;
    M->net.frag = M->frag;
    rc = launch_pack_frags(M->wc, M->frag, nullptr);
    if (rc) return rc;
    TDE_HIP_CHECK(hipDeviceSynchronize());
    return TDE_OK;
}

// Checkpoint: a header {magic "TDE2", ld, nbins, nparams, Adam step}, then
// the float32 parameters and the Adam moments m and v, so a run resumed from
// it continues bit for bit. Files with magic "TDE1" (parameters only) load
// with the Adam state reset.
int tde_model_save(tde_model* M, const char* path) {
    if (!M || !path) return set_error(TDE_ERR_ARG, "tde_model_save: null pointer");
    const size_t n = (size_t)M->net.nparams;
    std::vector<float> h(3 * n);
    int32_t step;
    {
        std::lock_guard<std::mutex> lock(M->mu);
        Guard gd(M->device);
        TDE_HIP_CHECK(hipDeviceSynchronize());
        TDE_HIP_CHECK(hipMemcpy(h.data(), M->p, n * 4, hipMemcpyDeviceToHost));
        TDE_HIP_CHECK(hipMemcpy(h.data() + n, M->m, n * 4, hipMemcpyDeviceToHost));
        TDE_HIP_CHECK(hipMemcpy(h.data() + 2 * n, M->v, n * 4, hipMemcpyDeviceToHost));
        step = M->step;
    }
    FILE* f = fopen(path, "wb");
    if (!f) return set_error(TDE_ERR_IO, "tde_model_save: cannot open %s", path);
    const int32_t head[5] = {0x32454454, M->net.ld, M->net.nb, M->net.nparams, step};   // "TDE2"
    bool ok = fwrite(head, sizeof(head), 1, f) == 1 && fwrite(h.data(), 4, h.size(), f) == h.size();
    ok = (fclose(f) == 0) && ok;
    return ok ? TDE_OK : set_error(TDE_ERR_IO, "tde_model_save: write to %s failed", path);
}

int tde_model_load(tde_model* M, const char* path) {
    if (!M || !path) return set_error(TDE_ERR_ARG, "tde_model_load: null pointer");
    FILE* f = fopen(path, "rb");
    if (!f) return set_error(TDE_ERR_IO, "tde_model_load: cannot open %s", path);
    const size_t n = (size_t)M->net.nparams;
    int32_t head[4], step = 0;
    std::vector<float> h(3 * n);
    bool ok = fread(head, sizeof(head), 1, f) == 1 && (head[0] == 0x31454454 || head[0] == 0x32454454) &&
              head[1] == M->net.ld && head[2] == M->net.nb && head[3] == M->net.nparams;
    const bool full = ok && head[0] == 0x32454454;
    if (full) ok = fread(&step, 4, 1, f) == 1 && step >= 0;
    if (ok) ok = fread(h.data(), 4, full ? 3 * n : n, f) == (full ? 3 * n : n);
    if (ok) ok = fgetc(f) == EOF;        // nothing after the last value
    fclose(f);
    if (!ok) return set_error(TDE_ERR_IO, "tde_model_load: %s is not a model of this shape", path);
    if (full)
        for (size_t i = n; i < 3 * n; ++i)
            if (!isfinite(h[i]) || (i >= 2 * n && h[i] < 0.f))
                return set_error(TDE_ERR_IO, "tde_model_load: %s holds an invalid Adam moment", path);
    int rc = tde_model_set_params(M, h.data(), M->net.nparams);     // resets m, v and the step
    if (rc || !full) return rc;
    std::lock_guard<std::mutex> lock(M->mu);
    Guard gd(M->device);
    TDE_HIP_CHECK(hipMemcpy(M->m, h.data() + n, n * 4, hipMemcpyHostToDevice));
    TDE_HIP_CHECK(hipMemcpy(M->v, h.data() + 2 * n, n * 4, hipMemcpyHostToDevice));
    M->step = step;
    return TDE_OK;
}

int tde_model_forward(tde_ctx* ctx, tde_model* M, const uint16_t* xdec, int64_t B, float* logits, int topk,
                      int32_t* top, float* margin, void* stream) {
    if (!ctx || !M || !xdec || !logits) return set_error(TDE_ERR_ARG, "tde_model_forward: null pointer");
    if (B < 1 || B > 65535) return set_error(TDE_ERR_ARG, "tde_model_forward: B out of range");
    if ((top || margin) && (!top || !margin || topk < 1 || topk > kCnnMaxTop || topk >= M->net.nb))
        return set_error(TDE_ERR_ARG, "tde_model_forward: top-k needs top, margin and 1 <= topk <= %d", kCnnMaxTop);
    std::lock_guard<std::mutex> lock(M->mu);
    Guard gd(M->device);
    int rc = ensure_train(M, (int)B);     // reuses the training activations (no Z kept)
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    CnnActs A = M->acts;
    for (int l = 0; l < kCnnLayers; ++l) A.z[l] = nullptr;
    rc = launch_cnn_forward(M->net, M->wc, xdec, (int)B, A, M->raw, logits, s);
    if (rc) return rc;
    if (top) return launch_cnn_topk(logits, (int)B, M->net.nb, topk, top, margin, s);
    return TDE_OK;
}

int tde_train_step(tde_ctx* ctx, tde_model* M, const uint16_t* xdec, const int32_t* labels, int64_t B, float lr,
                   float* loss_out, void* stream) {
    if (!ctx || !M || !xdec || !labels) return set_error(TDE_ERR_ARG, "tde_train_step: null pointer");
    if (B < 1 || B > 65535) return set_error(TDE_ERR_ARG, "tde_train_step: B out of range");
    if (!(lr >= 0.f) || !isfinite(lr)) return set_error(TDE_ERR_ARG, "tde_train_step: bad learning rate");
    std::lock_guard<std::mutex> lock(M->mu);
    Guard gd(M->device);
    int rc = ensure_train(M, (int)B);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    CnnActs A = M->acts;
    A.x[0] = const_cast<uint16_t*>(xdec);       // the layer-0 input is the caller's array
    rc = launch_cnn_forward(M->net, M->wc, xdec, (int)B, A, M->raw, M->logits, s);
    if (rc) return rc;
    rc = launch_cnn_backward(M->net, M->wc, (int)B, labels, A, M->raw, M->logits, M->g, s);
    if (rc) return rc;
    M->step += 1;
    rc = launch_adam(M->p, M->grad, M->m, M->v, M->wc, M->net.nparams, lr, M->step, s);
    if (rc) return rc;
    rc = launch_pack_frags(M->wc, M->frag, s);
    if (rc) return rc;
    if (loss_out) {
        std::vector<float> l(B);
        TDE_HIP_CHECK(hipMemcpyAsync(l.data(), M->g.loss, (size_t)B * 4, hipMemcpyDeviceToHost, s));
        TDE_HIP_CHECK(hipStreamSynchronize(s));
        double acc = 0.0;
        for (float x : l) acc += x;
        *loss_out = (float)(acc / (double)B);
    }
    return TDE_OK;
}

int tde_model_gradients(tde_model* M, float* host, int64_t n) {
    if (!M || !host) return set_error(TDE_ERR_ARG, "tde_model_gradients: null pointer");
    if (n != M->net.nparams) return set_error(TDE_ERR_ARG, "tde_model_gradients: %lld != %d values", (long long)n, M->net.nparams);
    std::lock_guard<std::mutex> lock(M->mu);
    Guard gd(M->device);
    TDE_HIP_CHECK(hipDeviceSynchronize());
    TDE_HIP_CHECK(hipMemcpy(host, M->grad, (size_t)n * 4, hipMemcpyDeviceToHost));
    return TDE_OK;
}

}  // extern "C"
