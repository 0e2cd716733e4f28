"""The FP64 sizing-network reference against central finite differences."""
import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.NPARAM == 11659


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, size=mlp.NPARAM)
    x = rng.normal(size=(5, mlp.NF))
    y = rng.normal(size=(5, mlp.NT))
    loss, g = mlp.loss_and_grad(p, x, y)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, y)[0] - mlp.loss_and_grad(pm, x, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_gelu_values():
    # GELU(0) = 0, GELU(x) -> x for large x, GELU(-x) -> 0
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    assert abs(mlp.gelu(np.array([-8.0]))[0]) < 1e-12
    # exact value at 1: 0.5 * (1 + erf(1/sqrt 2)) = Phi(1) = 0.8413447460685429
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_bf16_rounding():
    v = np.array([1.0, 1.00390625, 1.005859375, -3.14159], dtype=np.float32)
    r = mlp.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125
    assert abs(r[3] + 3.140625) < 1e-7
