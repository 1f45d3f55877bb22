"""CPU checks of the learned cost model: the float64 reference MLP against
central finite differences (the pin of its gradient), the library's host
forward pass against the reference, and the feature function."""
import numpy as np
import pytest

from oracle import mlp as ref


def _params(n_in, h, seed):
    rng = np.random.default_rng(seed)
    P = h * n_in + h + h * h + h + h + 1
    return rng.standard_normal(P) * 0.3


@pytest.mark.parametrize("n_in,h", [(3, 4), (16, 8)])
def test_reference_gradient_matches_finite_differences(n_in, h):
    rng = np.random.default_rng(1)
    p = _params(n_in, h, 2)
    x = rng.standard_normal((7, n_in))
    t = rng.standard_normal(7)
    g = ref.grad(p, n_in, h, x, t)
    eps = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = eps
        fd[i] = (ref.loss(p + e, n_in, h, x, t) - ref.loss(p - e, n_in, h, x, t)) / (2 * eps)
    assert np.max(np.abs(fd - g)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_reference_forward_closed_form():
    """With W1 = I (in = h), zero biases and positive inputs the net is
    y = W3 . relu(W2 x)."""
    n_in = h = 3
    W1 = np.eye(3)
    W2 = np.array([[1.0, -2, 0], [0, 1, 1], [2, 0, -1]])
    W3 = np.array([1.0, 2.0, -1.0])
    p = np.concatenate([W1.ravel(), np.zeros(3), W2.ravel(), np.zeros(3), W3, [0.5]])
    x = np.array([[1.0, 2.0, 3.0]])
    z2 = W2 @ x[0]
    want = W3 @ np.maximum(z2, 0) + 0.5
    y, _ = ref.forward(p, n_in, h, x)
    assert y[0] == pytest.approx(want, abs=1e-15)


def test_adam_reference_first_step():
    """Adam's first step moves each parameter by lr * sign(g) (bias-corrected)."""
    p = np.array([1.0, -1.0, 0.5])
    g = np.array([0.3, -2.0, 1e-3])
    p1, m, v = ref.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_host_forward_matches_reference():
    from paper_1704_01127_amd import qsim
    n_in, h = 16, 64
    p = _params(n_in, h, 3).astype(np.float32)
    x = np.random.default_rng(4).standard_normal((50, n_in)).astype(np.float32)
    y_host = qsim.mlp_predict_host(p, n_in, h, x)
    y_ref, _ = ref.forward(p.astype(np.float64), n_in, h, x.astype(np.float64))
    assert np.max(np.abs(y_host - y_ref)) <= 1e-4 * max(1.0, np.max(np.abs(y_ref)))


def test_cost_features():
    from paper_1704_01127_amd import qsim
    f = qsim.cost_features(30, qsim.C64, [13, 0, 1, 12, 18], n_epi=3)
    assert f.shape == (16,)
    assert f[0] == pytest.approx(5 / 6) and f[2] == 0 and f[5] == 0 and f[6] == pytest.approx(18 / 30)
    assert f[12] == 1 and f[10] == 1  # epilogue, matrix-core kernel
    g = qsim.cost_features(30, qsim.C128, [], 0)  # diagonal pass
    assert g[15] == 1 and g[2] == 1


def test_learned_scheduler_falls_back_without_model():
    from paper_1704_01127_amd import qsim
    from supremacy_inputs import supremacy_circuit
    qsim.set_cost_model(None)
    c = supremacy_circuit(4, 5, 20, 0)
    a = qsim.schedule(c.n, c.gates, kmax=5, scheduler="learned")
    b = qsim.schedule(c.n, c.gates, kmax=5, scheduler="greedy")
    assert a == b
