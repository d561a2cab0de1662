"""Pins of the FP64 surrogate oracle (oracle/mlp.py) against things other
than itself: central differences of the forward pass, the zero gradient at a
least-squares solution, closed forms of Adam's first steps and of the decay
curve of an exponential histogram."""
import numpy as np
import pytest

from oracle import mlp


def _net(seed, widths, batch):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.n_params(widths)) * 0.5
    x = rng.standard_normal((batch, widths[0]))
    t = rng.standard_normal((batch, widths[-1]))
    m = (rng.uniform(size=t.shape) < 0.7).astype(np.float64)
    return theta, x, t, m


def test_split_params_layout():
    w = (3, 2, 4)
    theta = np.arange(mlp.n_params(w), dtype=np.float64)
    (W0, b0), (W1, b1) = mlp.split_params(theta, w)
    assert W0.shape == (2, 3) and b0.tolist() == [6, 7]
    assert W1.shape == (4, 2) and W1[0].tolist() == [8, 9] and b1.tolist() == [16, 17, 18, 19]


def test_gradient_matches_central_differences():
    widths = (6, 5, 4, 3)
    theta, x, t, m = _net(0, widths, 9)
    acts = mlp.forward(theta, widths, x)
    for h in acts[1:-1]:                           # both ReLU regimes occur
        assert (h > 0).any() and (h == 0).any()
    L, g = mlp.backward(theta, widths, x, t, m)
    assert L == pytest.approx(mlp.loss(acts[-1], t, m), rel=1e-15)
    eps = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd[i] = (mlp.loss(mlp.forward(tp, widths, x)[-1], t, m)
                 - mlp.loss(mlp.forward(tm, widths, x)[-1], t, m)) / (2 * eps)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_zero_gradient_at_least_squares_solution():
    rng = np.random.default_rng(1)
    n, i, o = 40, 5, 3
    x = rng.standard_normal((n, i))
    t = rng.standard_normal((n, o))
    xa = np.concatenate([x, np.ones((n, 1))], axis=1)
    sol, *_ = np.linalg.lstsq(xa, t, rcond=None)    # [i+1, o]
    theta = np.concatenate([sol[:i].T.ravel(), sol[i]])
    _, g = mlp.backward(theta, (i, o), x, t, np.ones_like(t))
    assert np.abs(g).max() < 1e-12
    theta2 = theta.copy()
    theta2[0] += 0.1                                 # away from the optimum the gradient is not zero
    assert np.abs(mlp.backward(theta2, (i, o), x, t, np.ones_like(t))[1]).max() > 1e-3


def test_adam_steps_closed_form():
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10 ** rng.uniform(-3, 3, 50)
    lr, eps = 1e-3, 1e-8
    m = np.zeros(50)
    v = np.zeros(50)
    th = theta
    for t in range(1, 6):                            # constant gradient: m_hat = g, v_hat = g^2 exactly
        th, m, v = mlp.adam(th, g, m, v, t, lr, eps=eps)
        want = theta - t * lr * g / (np.abs(g) + eps)
        assert np.allclose(th, want, rtol=0, atol=1e-12)


def test_schroeder_curve_of_exponential_histogram():
    q, S = 0.93, 128
    h = q ** np.arange(S)
    edc = mlp.schroeder_edc_db(h[None, :])[0]
    want = 10 * np.log10((q ** np.arange(S) - q ** S) / (1 - q ** S))
    assert np.allclose(edc, want, rtol=0, atol=1e-9)
    one = np.zeros(S)
    one[17] = 3.0
    e1 = mlp.schroeder_edc_db(one)
    assert np.all(e1[:18] == 0.0) and np.all(e1[18:] == mlp.FEAT_FLOOR_DB)
    assert np.all(mlp.schroeder_edc_db(np.zeros(S)) == mlp.FEAT_FLOOR_DB)


def test_features_and_band_rms():
    f = mlp.hist_features(np.array([1e-3, 0.0, 1.0, 1e-30]))
    assert np.allclose(f, [(-30 + 75) / 25, -3.0, 3.0, -3.0])
    p = np.array([[0.0, -10, -20, -70]])
    full = np.array([[0.0, -11, -22, -90]])
    assert mlp.band_rms_db(p, full)[0] == pytest.approx(np.sqrt((0 + 1 + 4) / 3))
