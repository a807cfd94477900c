/* Host paths of libtde (argument checks, planners, workspace sizes, tuning
 * files, quantizer tables) exercised under AddressSanitizer and
 * UndefinedBehaviorSanitizer: the library is built with the sanitizers on
 * its host code and loaded with dlopen (argv[1]); no GPU is needed, and
 * calls that reach the device are not made. Exit status 0 when every call
 * returned; the sanitizers abort on a fault. */
#include <dlfcn.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "tde.h"

/* every entry point used below, resolved from the loaded library */
#define TDE_FNS(X)                                                                                    \
    X(const char*, tde_status_string, (int))                                                          \
    X(const char*, tde_last_error, (void))                                                            \
    X(int, tde_quantizer_thresholds, (int, int, float*))                                              \
    X(size_t, tde_xcorr_workspace_size, (int64_t, int64_t, int, int, int64_t, int64_t, int))         \
    X(int, tde_mfma_tile_lags, (int64_t, int64_t, int, int, int64_t, int64_t, int))                   \
    X(int, tde_mfma_operand_bits, (int, int, int))                                                    \
    X(size_t, tde_argmax_workspace_size, (int64_t))                                                   \
    X(size_t, tde_quantize_workspace_size, (int64_t))                                                 \
    X(size_t, tde_refine_workspace_size, (int))                                                       \
    X(size_t, tde_estimate_workspace_size, (const tde_pair*, int64_t, const tde_opts*))              \
    X(size_t, tde_model_prepare_workspace_size, (const tde_pair*, int64_t))                          \
    X(int, tde_tune_reset, (void))                                                                    \
    X(int, tde_tune_save, (const char*))                                                              \
    X(int, tde_tune_load, (const char*))                                                              \
    X(int, tde_tune_query, (int64_t, int64_t, int, int, int64_t, int64_t))                            \
    X(int, tde_xcorr_int, (tde_ctx*, const int8_t*, int64_t, const int8_t*, int64_t, int, int, int64_t, \
                           int64_t, void*, int, int, void*, size_t, void*))                           \
    X(int, tde_argmax_lag, (tde_ctx*, const void*, int, int64_t, int64_t, tde_peak*, void*, size_t, void*))
#define DECL(ret, name, args) static ret(*p_##name) args;
TDE_FNS(DECL)
#define LOAD(ret, name, args)                                                                         \
    if (!(*(void**)&p_##name = dlsym(lib, #name))) {                                                  \
        fprintf(stderr, "missing symbol %s\n", #name);                                                \
        return 2;                                                                                     \
    }

static int calls = 0;
#define CALL(x) do { (void)(x); ++calls; } while (0)

static void planner_cases(void) {
    const int paths[] = {TDE_PATH_AUTO, TDE_PATH_MFMA, TDE_PATH_MFMA_I8, TDE_PATH_POPC, TDE_PATH_NTT, 77};
    const int64_t ns[] = {0, 1, 2, 31, 4096, 65536, 133145, 1 << 20, 1 << 22, (int64_t)1 << 40, -5};
    const int ks[] = {0, 1, 3, 7, 127, 128};
    for (size_t a = 0; a < sizeof ns / sizeof ns[0]; ++a)
        for (size_t b = 0; b < sizeof ks / sizeof ks[0]; ++b)
            for (size_t c = 0; c < sizeof paths / sizeof paths[0]; ++c) {
                const int64_t n = ns[a];
                CALL(p_tde_xcorr_workspace_size(n, n, ks[b], ks[b], -(n - 1), n - 1, paths[c]));
                if (n < (int64_t)1 << 30)   /* larger: a valid request whose work list takes seconds to count */
                    CALL(p_tde_xcorr_workspace_size(n, n / 2 + 1, ks[b], 1, -n / 4, n / 4, paths[c]));
                CALL(p_tde_xcorr_workspace_size(n, n, ks[b], ks[b], 10, -10, paths[c]));
                CALL(p_tde_mfma_tile_lags(n, n, ks[b], ks[b], -n, n, paths[c]));
                CALL(p_tde_mfma_operand_bits(ks[b], ks[b], paths[c]));
            }
    for (int64_t n = 0; n < 70000; n = n * 3 + 1) {
        CALL(p_tde_argmax_workspace_size(n));
        CALL(p_tde_quantize_workspace_size(n));
    }
    const int ties[] = {-1, 0, 1, 2, 4096, 65536, 1 << 30};
    for (size_t i = 0; i < sizeof ties / sizeof ties[0]; ++i) CALL(p_tde_refine_workspace_size(ties[i]));
}

static void batch_cases(void) {
    enum { NP = 37 };
    tde_pair* p = calloc(NP, sizeof *p);
    const float* fake = (const float*)(uintptr_t)0x10000;   /* never dereferenced on the host */
    for (int i = 0; i < NP; ++i) {
        p[i].x = fake;
        p[i].y = fake;
        p[i].nx = 1000 + 977 * i;
        p[i].ny = 900 + 1013 * i;
        p[i].lag_lo = -(p[i].nx / 4);
        p[i].lag_hi = p[i].ny / 4;
        p[i].bits = (int[]){1, 2, 4, 8}[i % 4];
        p[i].r_dtype = TDE_I64;
    }
    for (int mode = 0; mode < 2; ++mode)
        for (int path = 0; path < 6; ++path)
            for (int q = 0; q < 4; ++q) {
                tde_opts o = {mode, path, path & 1, 8, NULL, 3.0f, q};
                CALL(p_tde_estimate_workspace_size(p, NP, &o));
                CALL(p_tde_estimate_workspace_size(p, 0, &o));
                CALL(p_tde_estimate_workspace_size(NULL, NP, &o));
            }
    /* invalid pairs, one at a time: each must be refused with a message */
    tde_opts o = {TDE_MODE_FULL, TDE_PATH_AUTO, 0, 8, NULL, 0.0f, 0};
    for (int k = 0; k < 8; ++k) {
        tde_pair b = p[3];
        switch (k) {
        case 0: b.bits = 3; break;
        case 1: b.nx = -1; break;
        case 2: b.lag_lo = 5; b.lag_hi = 4; break;
        case 3: b.x = NULL; break;
        case 4: b.r_dtype = 9; break;
        case 5: b.lag_lo = INT64_MIN / 2; break;
        case 6: b.inv_step_x = NAN; break;
        case 7: b.ny = (int64_t)1 << 50; break;
        }
        CALL(p_tde_estimate_workspace_size(&b, 1, &o));
        CALL(p_tde_last_error());
    }
    CALL(p_tde_model_prepare_workspace_size(p, NP));
    free(p);
}

static void tuning_files(const char* dir, const char* committed) {
    char path[4096];
    CALL(p_tde_tune_reset());
    snprintf(path, sizeof path, "%s/none.txt", dir);
    CALL(p_tde_tune_save(path));                     /* no table: refused */
    if (committed) CALL(p_tde_tune_load(committed));
    for (int lg = 8; lg < 24; ++lg)
        for (int k = 1; k <= 127; k = k * 2 + 1) {
            const int64_t n = (int64_t)1 << lg;
            CALL(p_tde_tune_query(n, n, k, k, -(n - 1), n - 1));
            CALL(p_tde_tune_query(n, n / 3 + 1, k, 1, -n / 4, n / 4));
        }
    snprintf(path, sizeof path, "%s/saved.txt", dir);
    CALL(p_tde_tune_save(path));
    CALL(p_tde_tune_load(path));
    const char* bad[] = {"", "tde-tune 2\n", "tde-tune 2\n0 0 10 1 4\n", "tde-tune 9\n0 0 10 1 4\n",
                         "tde-tune 2\n99 99 99 99 99\n", "tde-tune 2\n0 0 10 1\n", "garbage\x01\x02\n",
                         "tde-tune 1\n0 0 10 1\n1 1 11 2\n", "tde-tune 2\n-1 -1 -1 -1 -1\n",
                         "tde-tune 2\n0 0 100000000000000000000 1 4\n"};
    for (size_t i = 0; i < sizeof bad / sizeof bad[0]; ++i) {
        snprintf(path, sizeof path, "%s/bad%zu.txt", dir, i);
        FILE* f = fopen(path, "w");
        if (!f) continue;
        fputs(bad[i], f);
        fclose(f);
        CALL(p_tde_tune_load(path));
        CALL(p_tde_tune_query(4096, 4096, 7, 7, -1024, 1024));
    }
    snprintf(path, sizeof path, "%s/missing/none.txt", dir);
    CALL(p_tde_tune_load(path));
    CALL(p_tde_tune_reset());
}

int main(int argc, char** argv) {
    if (argc < 3) {
        fprintf(stderr, "usage: host_driver LIB TMPDIR [TUNING_FILE]\n");
        return 2;
    }
    void* lib = dlopen(argv[1], RTLD_NOW);
    if (!lib) {
        fprintf(stderr, "dlopen: %s\n", dlerror());
        return 2;
    }
    TDE_FNS(LOAD)
    for (int s = -20; s < 20; ++s) CALL(p_tde_status_string(s));
    CALL(p_tde_last_error());
    float th[7];
    for (int q = -1; q < 4; ++q)
        for (int b = 0; b < 10; ++b) {
            CALL(p_tde_quantizer_thresholds(q, b, th));
            CALL(p_tde_quantizer_thresholds(q, b, NULL));
        }
    planner_cases();
    batch_cases();
    tuning_files(argv[2], argc > 3 ? argv[3] : NULL);
    /* calls that need a context are refused without one */
    CALL(p_tde_xcorr_int(NULL, NULL, 10, NULL, 10, 1, 1, -3, 3, NULL, TDE_I64, TDE_PATH_AUTO, NULL, 0, NULL));
    CALL(p_tde_argmax_lag(NULL, NULL, TDE_I64, 0, 10, NULL, NULL, 0, NULL));
    printf("host driver: %d calls\n", calls);
    return 0;
}
