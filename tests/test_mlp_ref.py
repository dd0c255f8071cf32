"""Pins of the FP64 MLP reference: finite differences, an independent
autograd evaluation, bfloat16 rounding on exact cases, Adam's first step."""
import numpy as np
import pytest

from oracle import mlp_ref as R


def _rand(seed, n=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.2, R.N_PARAMS)
    x = rng.normal(0, 1, (n, R.IN)).astype(np.float32)
    t = rng.normal(0, 1, (n, R.OUT))
    mean = rng.normal(0, 0.1, R.IN).astype(np.float32)
    std = (1 + rng.random(R.IN)).astype(np.float32)
    return p, x, t, mean, std


def test_bf16_rounding_exact_cases():
    one = np.float32(1.0)
    cases = {1.0: 1.0, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6, 1 + 2 ** -7: 1 + 2 ** -7,
             -2.5: -2.5, 1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7, 0.0: 0.0, 3.0e38: 2.9975e38}
    for a, b in cases.items():
        got = R.bf16(np.array([a], np.float32))[0]
        if a == 3.0e38:
            assert abs(got - 3.0e38) / 3.0e38 < 2 ** -8
        else:
            assert got == b, (a, got, b)
    assert one == 1


def test_gradients_match_finite_differences():
    p, x, t, mean, std = _rand(1)
    _, g = R.loss_and_grads(p, mean, std, x, t, quantized=False)
    rng = np.random.default_rng(2)
    h = 1e-6
    for i in rng.choice(R.N_PARAMS, 60, replace=False):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        lp, _ = R.loss_and_grads(pp, mean, std, x, t, quantized=False)
        lm, _ = R.loss_and_grads(pm, mean, std, x, t, quantized=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(g[i]), (i, fd, g[i])


def test_gradients_match_torch_autograd():
    torch = pytest.importorskip("torch")
    p, x, t, mean, std = _rand(3, n=5)
    loss, g = R.loss_and_grads(p, mean, std, x, t, quantized=False)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in R.unpack(p).items()}
    xn = torch.tensor(R.normalize(x, mean, std), dtype=torch.float64)
    h1 = torch.relu(xn @ P["W1"] + P["b1"])
    h2 = torch.relu(h1 @ P["W2"] + P["b2"])
    y = h2 @ P["W3"] + P["b3"]
    L = ((y - torch.tensor(t)) ** 2).mean()
    L.backward()
    tg = np.concatenate([P[k].grad.numpy().reshape(-1) for k, _ in R.SHAPES])
    assert abs(L.item() - loss) < 1e-12
    assert np.allclose(tg, g, rtol=1e-10, atol=1e-13)


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = R.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, 0.01)
    assert np.allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-4) and p[3] == 0.0
