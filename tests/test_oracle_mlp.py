"""Pins of the reference MLP (P16): float64 gradients against central finite
differences, bfloat16 rounding against its definition, Adam against its
closed form on a quadratic."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_definition():
    # exact bf16 values are fixed points; halfway cases go to even
    vals = np.array([1.0, -2.5, 1.5 * 2.0 ** -16, 65280.0])
    assert np.all(mlp.bf16(vals) == vals.astype(np.float32).astype(np.float64))
    one_ulp = 2.0 ** -7        # bf16 spacing at 1.0
    assert mlp.bf16(1.0 + one_ulp / 2) == 1.0                 # tie -> even (1.0)
    assert mlp.bf16(1.0 + 3 * one_ulp / 2) == 1.0 + 2 * one_ulp  # tie -> even
    assert mlp.bf16(1.0 + 0.6 * one_ulp) == 1.0 + one_ulp
    x = np.random.default_rng(0).standard_normal(1000)
    r = mlp.bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) + 1e-45)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init(3)
    X = rng.standard_normal((37, 16))
    t = rng.standard_normal(37)
    loss, g = mlp.loss_and_grad(p, X, t, emulate_bf16=False)
    idx = rng.choice(mlp.NPARAM, size=60, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(p[i]))
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, X, t, False)[0] - mlp.loss_and_grad(pm, X, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_closed_form_first_steps():
    """On f(w) = w^2/2 with constant-sign gradients the first Adam step moves
    each weight by exactly lr (bias-corrected m/sqrt(v) = sign(g))."""
    w = np.array([3.0, -2.0, 0.5])
    m = np.zeros(3)
    v = np.zeros(3)
    w1, m, v = mlp.adam(w, w.copy(), m, v, 1, lr=1e-2, eps=0.0)
    np.testing.assert_allclose(w1, w - 1e-2 * np.sign(w), rtol=0, atol=1e-15)
