"""Rank predictor on the GPU against the FP64 oracle (oracle/mlp.py).

* Gradient of the asymmetric log-rank loss from the HIP kernels vs the
  oracle's analytic gradient (itself pinned by finite differences): FP32
  kernels with FP64 batch sums, bar 1e-4 relative on the whole vector.
* Inference of trained weights vs the oracle forward pass.
* Training on the GPU lowers the loss and fits a learnable rank law.
* The solver's box features equal the oracle's feature definition.
* Predictor-sized compression keeps the solution within 1e-8 of the dense
  oracle, uses fewer proxy rows than the rule, and falls back where the
  measured rank exceeds the prediction."""

import dataclasses

import numpy as np
import pytest

import workloads
from oracle import dense, geometry, mlp
from tests.gpu_common import make_solver, oracle_system, rel

pytestmark = pytest.mark.gpu


def _solver():
    from paper_2609_33216_amd import binding
    return binding.Solver(0)


def _weights(p, mu, sd):
    return np.concatenate([p, mu, sd]).astype(np.float32)


def test_gradient_vs_oracle():
    rng = np.random.default_rng(3)
    n = 700
    feat = rng.standard_normal((n, 6)) * [30, 45, 2, 5, 3, 2] + [60, 90, 3, 8, 4, -9]
    rank = rng.integers(4, 150, n).astype(np.float64)
    mu, sd = mlp.normalisation(feat)
    p = mlp.init_params(11).astype(np.float32).astype(np.float64)
    p[-1] = 3.0
    s = _solver()
    for alpha in (1.0, 4.0):
        loss, g = s.predictor_grad(_weights(p, mu, sd), feat, rank, alpha)
        # the oracle sees exactly the kernels' inputs: FP32 features, normalised in FP64
        x = ((feat.astype(np.float32).astype(np.float64) - mu.astype(np.float32)) / sd.astype(np.float32))
        Lo, go = mlp.loss_and_grad(p, x, rank.astype(np.float32), alpha)
        print("alpha", alpha, "loss", loss, Lo, "grad rel err", np.linalg.norm(g - go) / np.linalg.norm(go))
        assert abs(loss - Lo) <= 1e-5 * abs(Lo)
        assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


def _synthetic(n, seed):
    rng = np.random.default_rng(seed)
    feat = np.column_stack([rng.uniform(1, 200, n), rng.uniform(1, 300, n), rng.uniform(0, 5, n),
                            rng.uniform(0, 20, n), rng.integers(1, 10, n), rng.choice([-6, -8, -10, -12], n)])
    rank = np.round(8 + 0.35 * feat[:, 1] - 1.5 * feat[:, 5] + 2 * feat[:, 2])
    return feat, rank


def test_training_fits_and_inference_matches_oracle():
    feat, rank = _synthetic(6000, 1)
    s = _solver()
    hist = s.predictor_train(feat, rank, epochs=120, batch=512, lr=3e-3, alpha=4.0, seed=2)
    print("loss", hist[0], "->", hist[-1])
    assert hist[-1] < 0.05 * hist[0]
    ft, rt = _synthetic(500, 9)
    pred = s.predictor_predict(ft)
    err = np.abs(np.log(pred) - np.log(rt))
    print("median |log err|", np.median(err))
    assert np.median(err) < 0.1
    w = s.predictor_get().astype(np.float64)
    p, mu, sd = w[:8833], w[8833:8839], w[8839:]
    x = (ft.astype(np.float32).astype(np.float64) - mu) / sd
    yo, _ = mlp.forward(p, x)
    assert np.max(np.abs(np.log(pred) - yo)) < 1e-4 * max(1.0, np.max(np.abs(yo)))


def test_box_features_match_oracle_definition():
    wl = workloads.scaled_config(workloads.config2(), 2048, leaf=64)
    s = make_solver(wl)
    s.compress()
    feat, rank, info = s.box_table()
    x, dx, ddx = wl.boundary()
    g = geometry.discretize(x, dx, ddx)
    for i in range(0, len(feat), max(1, len(feat) // 25)):
        tree, level, lo, hi = info[i, :4]
        fo = mlp.box_features(x, g.kappa, lo, hi, wl.k0, wl.k1, level, wl.tol)
        assert np.allclose(feat[i], fo, rtol=2e-6, atol=1e-6), (i, feat[i], fo)
        assert rank[i] >= 1


def test_predictor_sized_compression():
    base = workloads.config2()
    train = [dataclasses.replace(base, name=f"t{i}", curve_params=(("amp", a), ("arms", m)), n=n, k0=k, k1=1.5 * k,
                                 leaf=64)
             for i, (a, m, n, k) in enumerate([(0.15, 3, 2048, 10.0), (0.25, 5, 3072, 25.0),
                                               (0.3, 4, 4096, 40.0), (0.2, 6, 2560, 18.0),
                                               (0.1, 7, 3584, 32.0), (0.28, 3, 1536, 45.0)])]
    from paper_2609_33216_amd import predictor
    feats, ranks = [], []
    for tol in (1e-8, 1e-10):
        f, r = predictor.measured_boxes([w.boundary() for w in train], [(w.k0, w.k1, w.eps0, w.eps1) for w in train],
                                        tol=tol, leaf=64)
        feats.append(f)
        ranks.append(r)
    feat, rank = np.concatenate(feats), np.concatenate(ranks)
    wl = dataclasses.replace(base, name="test", curve_params=(("amp", 0.22), ("arms", 5)), n=3000, k0=30.0, k1=45.0,
                             leaf=64)
    _, _, A, b = oracle_system(wl)
    xd = dense.solve_dense(A, b)
    s = make_solver(wl)
    hist = s.predictor_train(feat, rank, epochs=300, batch=256, lr=2e-3, alpha=4.0, seed=0)
    print("training samples", len(rank), "loss", hist[0], "->", hist[-1])
    s.configure(predictor=True)
    s.compress()
    s.factor()
    x = s.solve(b)
    st = s.stats()
    print("pred boxes", st["pred_boxes"], "fallbacks", st["pred_fallbacks"], "rows", st["proxy_rows"],
          "rule rows", st["proxy_rows_rule"], "err", rel(x, xd))
    assert st["pred_boxes"] > 0
    assert rel(x, xd) < 1e-8
    assert st["proxy_rows"] < st["proxy_rows_rule"]
