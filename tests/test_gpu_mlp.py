"""GPU MLP kernels (BF16 MFMA, FP32 accumulation) against the FP64 reference
on the same bf16-rounded operands."""
import numpy as np
import pytest

from oracle import mlp_ref as R
from paper_2210_16998_amd import tpg
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

# Each product term is exact in fp32 (bf16 x bf16); the GPU's fp32 sums and
# its bf16 roundings of the hidden activations differ from the reference by
# at most a few bf16 units in the last place (2^-8 relative) of the
# propagated absolute-term sums; 2^-6 covers three layers.
FWD_TOL = 2.0 ** -6


def _setup(seed, n):
    rng = np.random.default_rng(seed)
    m = tpg.MLP(seed=seed)
    p = m.params().astype(np.float64)
    x = rng.normal(0, 1, (n, R.IN)).astype(np.float32) * 3 + 1
    mean = x.mean(0).astype(np.float32)
    std = x.std(0).astype(np.float32) + 0.1
    m.set_normalizer(mean, std)
    t = rng.normal(0, 1, (n, R.OUT)).astype(np.float32)
    return m, p, x, t, mean, std


@pytest.mark.parametrize("n", [1, 63, 64, 200, 1000])
def test_forward_within_bound(n):
    say("case mlp forward", n)
    m, p, x, t, mean, std = _setup(10 + n, n)
    y = m.forward(x)
    ref = R.forward(p, mean, std, x, True)["y"]
    bound = FWD_TOL * R.abs_terms_forward(p, mean, std, x) + 1e-6
    assert np.all(np.abs(y - ref) <= bound), np.max(np.abs(y - ref) / bound)


@pytest.mark.parametrize("n", [7, 256, 777])
def test_gradients_against_reference(n):
    say("case mlp gradients", n)
    m, p, x, t, mean, std = _setup(20 + n, n)
    g, loss = m.gradients(x, t)
    lref, gref = R.loss_and_grads(p, mean, std, x, t, True)
    assert abs(loss - lref) <= 2 ** -6 * lref
    q = 0
    for name, shape in R.SHAPES:
        k = int(np.prod(shape))
        a, b = g[q:q + k].astype(np.float64), gref[q:q + k]
        scale = np.max(np.abs(b)) + 1e-12
        assert np.max(np.abs(a - b)) <= 2 ** -5 * scale, (name, np.max(np.abs(a - b)) / scale)
        cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30)
        assert cos > 0.999, (name, cos)
        q += k


def test_adam_step_matches_reference_update():
    say("case mlp adam")
    m, p, x, t, mean, std = _setup(5, 300)
    g, _ = m.gradients(x, t)
    lr = 3e-3
    m.train_step(x, t, lr)
    p1 = m.params().astype(np.float64)
    ref, _, _ = R.adam(p, 0 * p, 0 * p, g.astype(np.float64), 1, lr)
    assert np.allclose(p1, ref, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss():
    say("case mlp training")
    rng = np.random.default_rng(0)
    x = rng.normal(0, 1, (2048, R.IN)).astype(np.float32)
    w = rng.normal(0, 1, (R.IN, R.OUT))
    t = np.tanh(x @ w / 6).astype(np.float32)
    m = tpg.MLP(seed=1)
    m.set_normalizer(np.zeros(R.IN, np.float32), np.ones(R.IN, np.float32))
    first = m.train_step(x[:512], t[:512], 1e-3)
    for it in range(300):
        b = (it * 512) % 2048
        last = m.train_step(x[b:b + 512], t[b:b + 512], 1e-3)
    assert last < 0.2 * first, (first, last)


def test_save_load_roundtrip(tmp_path):
    m, p, x, t, mean, std = _setup(3, 10)
    f = str(tmp_path / "m.tpgmlp")
    m.save(f)
    m2 = tpg.MLP.load(f)
    assert np.array_equal(m2.params(), m.params())
    assert np.array_equal(m2.forward(x), m.forward(x))
