"""The allocation-free inference entry point against the allocating one.

symhss_predictor_predict_noalloc takes device pointers and keeps the
network's activations in the library's fixed device scratch; it must give
what symhss_predictor_predict gives on the same features and weights (the
same FP32 layer kernels; normalisation and exp are both formed in FP64 and
rounded once, so the bar is a few FP32 ulps: relative 2e-6).  Two calls in a
row, the second with fewer samples, so that what the first left in the
scratch cannot leak into the second; sizes beyond the stated maximum are
refused without touching the outputs.
"""

import numpy as np
import pytest

from paper_2609_33216_amd import binding

pytestmark = pytest.mark.gpu


def _weights(rng):
    w = (0.15 * rng.standard_normal(binding.PREDICTOR_WEIGHTS)).astype(np.float32)
    nf = binding.N_FEATURES
    w[-2 * nf:-nf] = rng.uniform(-1.0, 1.0, nf)   # feature means
    w[-nf:] = rng.uniform(0.5, 2.0, nf)           # feature scales
    return w


def test_noalloc_matches_allocating_predict():
    import torch
    rng = np.random.default_rng(20)
    s = binding.Solver(0)
    s.predictor_load(_weights(rng))
    dev = torch.device("cuda:0")
    for n in (5000, 1237):
        feat = rng.uniform(-3.0, 3.0, (n, binding.N_FEATURES)).astype(np.float32)
        ref = s.predictor_predict(feat)
        fd = torch.from_numpy(feat).to(dev)
        out = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        s.predictor_predict_noalloc(fd.data_ptr(), n, out.data_ptr())
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        err = float(np.max(np.abs(got - ref) / np.abs(ref)))
        print(f"n={n}: max relative difference {err:.2e}")
        assert err <= 2e-6


def test_noalloc_rejects_oversized_batches():
    import torch
    rng = np.random.default_rng(21)
    s = binding.Solver(0)
    s.predictor_load(_weights(rng))
    n = binding.PREDICT_NOALLOC_MAX + 1
    fd = torch.zeros((n, binding.N_FEATURES), dtype=torch.float32, device="cuda:0")
    out = torch.full((n,), -1.0, dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    with pytest.raises(binding.SymhssError) as ei:
        s.predictor_predict_noalloc(fd.data_ptr(), n, out.data_ptr())
    assert ei.value.status == binding.EINVAL
    torch.cuda.synchronize()
    assert bool((out == -1.0).all())
    # the largest allowed batch works
    m = binding.PREDICT_NOALLOC_MAX
    s.predictor_predict_noalloc(fd.data_ptr(), m, out.data_ptr())
    torch.cuda.synchronize()
    ref = s.predictor_predict(np.zeros((m, binding.N_FEATURES), dtype=np.float32))
    assert np.allclose(out[:m].cpu().numpy(), ref, rtol=2e-6, atol=0)
