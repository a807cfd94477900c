"""The allocation-free correlation entry point (tde_xcorr_int_noalloc):
called through the C ABI, it must give exactly what tde_xcorr_int gives
with a caller workspace, on consecutive calls that reuse the device's
static scratch (a larger call, then a smaller one), for every engine."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(T, ctx, entry, u, v, ku, kv, lo, hi, dt, path):
    from paper_2509_19974_amd import tde
    lib = tde.load_library()
    tdt = T.int32 if dt == tde.TDE_I32 else T.int64
    r = T.full((hi - lo + 1,), -7, dtype=tdt, device="cuda")      # stale values must be overwritten
    if entry == "noalloc":
        rc = lib.tde_xcorr_int_noalloc(ctx.handle, u.data_ptr(), u.numel(), v.data_ptr(), v.numel(), ku, kv, lo, hi,
                                       r.data_ptr(), dt, path, None)
    else:
        wsb = int(lib.tde_xcorr_workspace_size(u.numel(), v.numel(), ku, kv, lo, hi, path))
        ws = T.empty(max(wsb, 1), dtype=T.uint8, device="cuda")
        rc = lib.tde_xcorr_int(ctx.handle, u.data_ptr(), u.numel(), v.data_ptr(), v.numel(), ku, kv, lo, hi,
                               r.data_ptr(), dt, path, ws.data_ptr(), wsb, None)
    assert rc == 0, tde.tde_last_error()
    T.cuda.synchronize()
    return r.cpu().numpy()


@pytest.mark.parametrize("path_name", ["MFMA", "MFMA_I8", "POPC", "NTT", "AUTO"])
def test_noalloc_matches_workspace_entry(path_name):
    import torch as T
    from paper_2509_19974_amd import tde
    assert T.cuda.is_available()
    ctx = tde.Context(0)
    path = getattr(tde, "TDE_PATH_" + path_name)
    k = 1 if path_name == "POPC" else 7
    rng = np.random.default_rng(11)
    cases = [(60000, 50017, -60000 + 1, 50016, tde.TDE_I64), (3001, 2000, -500, 1999, tde.TDE_I32)]
    for nu, nv, lo, hi, dt in cases:
        say(f"noalloc {path_name} nu={nu} nv={nv} lags [{lo}, {hi}]")
        u = T.from_numpy(synth.random_int_seq(rng, nu, k, 0.1)).cuda()
        v = T.from_numpy(synth.random_int_seq(rng, nv, k, 0.1)).cuda()
        a = _run(T, ctx, "noalloc", u, v, k, k, lo, hi, dt, path)
        b = _run(T, ctx, "ws", u, v, k, k, lo, hi, dt, path)
        np.testing.assert_array_equal(a, b)
    ctx.close()


def test_noalloc_refuses_beyond_its_scratch():
    import torch as T
    from paper_2509_19974_amd import tde
    ctx = tde.Context(0)
    lib = tde.load_library()
    n = 1 << 21                    # two-prime transform of 2^22 points: 64 MiB of residues
    u = T.zeros(n, dtype=T.int8, device="cuda")
    r = T.empty(1, dtype=T.int64, device="cuda")
    rc = lib.tde_xcorr_int_noalloc(ctx.handle, u.data_ptr(), n, u.data_ptr(), n, 127, 127, 0, 0, r.data_ptr(),
                                   tde.TDE_I64, tde.TDE_PATH_NTT, None)
    assert rc == tde.TDE_ERR_UNSUPPORTED and "static scratch" in tde.tde_last_error()
    ctx.close()
