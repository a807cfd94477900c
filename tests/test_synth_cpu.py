"""The seeded generators feed both the HIP path and the oracle; these CPU
checks pin what their recipes promise (shapes, delays, energy, SNR,
determinism), not any estimator arithmetic."""
import numpy as np
import pytest
import torch

import synth


def test_reverb_torch_generator_recipe():
    n, L = 8192, 1024
    a = synth.config5_reverb_torch(torch, 16, salt=3, n=n, max_lag=L, device="cpu", t60_range=(200, 600))
    b = synth.config5_reverb_torch(torch, 16, salt=3, n=n, max_lag=L, device="cpu", t60_range=(200, 600))
    c = synth.config5_reverb_torch(torch, 16, salt=4, n=n, max_lag=L, device="cpu", t60_range=(200, 600))
    for k in ("x", "y", "d", "t60"):
        assert torch.equal(a[k], b[k])            # same salt, same bytes
    assert not torch.equal(a["x"], c["x"])
    assert a["x"].shape == (16, n) and a["x"].dtype == torch.float32
    d = a["d"].numpy()
    assert d.min() >= -L and d.max() <= L - 1
    t60 = a["t60"].numpy()
    assert t60.min() >= 200 and t60.max() <= 600
    x, y = a["x"].numpy().astype(np.float64), a["y"].numpy().astype(np.float64)
    snr = a["snr_db"].numpy()
    assert snr.min() >= 0 and snr.max() <= 30
    for i in range(16):
        # the noise is the residual after the zero-fill delay; its power sets the SNR
        clean = synth.delay_zero_fill(x[i], int(d[i]))
        sup = clean != 0
        noise = y[i] - clean
        got = 10 * np.log10(np.mean(clean[sup] ** 2) / np.mean(noise ** 2))
        assert abs(got - snr[i]) < 0.5, (i, got, snr[i])
        # unit-energy response on white noise: x has unit variance
        assert 0.8 < np.var(x[i]) < 1.2
        # steady state: no start-up ramp (first and last quarters alike)
        q = n // 4
        assert 0.6 < np.var(x[i][:q]) / np.var(x[i][-q:]) < 1.6
    # the delayed copy is the noisy y's strongest correlate at lag d
    i = int(np.argmax(snr))
    r = np.correlate(y[i], x[i], mode="full")
    assert int(np.argmax(r)) - (n - 1) == int(d[i])
