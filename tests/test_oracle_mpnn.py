"""Pins for the warm-start network reference (oracle.mpnn): bf16 rounding,
closed forms, and gradients against central finite differences."""
import numpy as np
import pytest

import graphgen as gg
from oracle import mpnn as om


def test_bf16_round_nearest_even():
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-9, 1 + 2**-7 + 2**-8, -2.5, 0.0, 3.0e38])
    got = om.bf16_round(x)
    assert got[0] == 1.0
    assert got[1] == 1.0                      # halfway -> even (1.0)
    assert got[2] == 1 + 2**-7                # above halfway -> up
    assert got[3] == 1 + 2**-6                # halfway, odd neighbour -> up to even
    assert got[4] == -2.5 and got[5] == 0.0
    assert np.isfinite(got[6])
    # every result is representable in 8 mantissa bits
    r = om.bf16_round(gg.philox(1).standard_normal(1000))
    m, _ = np.frexp(r)
    assert np.all(np.abs(m * 2**8 - np.round(m * 2**8)) < 1e-12)


def test_zero_weights_give_uniform_guess():
    g = gg.random_connected(30, 4.0, seed=2)
    params = {k: np.zeros_like(v) for k, v in gg.mpnn_init(0).items()}
    x0, _ = om.mpnn_forward(g, params, source=3)
    assert np.allclose(x0, 1.0 / g.n, atol=1e-15)


def test_one_layer_closed_form():
    """With one layer and identity-like weights the output is an explicit
    function of degrees and the source indicator."""
    g = gg.star(5)
    p = gg.mpnn_init(0, layers=1, hidden=2)
    p["w_self0"] = np.eye(2, dtype=np.float32)
    p["w_nbr0"] = np.zeros((2, 2), dtype=np.float32)
    p["b0"] = np.zeros(2, dtype=np.float32)
    p["w_out"] = np.array([0.0, 1.0], dtype=np.float32)
    p["b_out"] = np.zeros(1, dtype=np.float32)
    x0, _ = om.mpnn_forward(g, p, source=2, layers=1)
    e = np.exp([0.0, 0.0, 1.0, 0.0, 0.0])
    assert np.allclose(x0, e / e.sum(), atol=1e-15)


def test_log_degree_score_gives_stationary_vector():
    """score = log d reproduces the stationary distribution d / vol exactly."""
    g = gg.random_connected(40, 5.0, seed=9)
    p = gg.mpnn_init(0, layers=1, hidden=2)
    p["w_self0"] = np.eye(2, dtype=np.float32)
    p["w_nbr0"] = np.zeros((2, 2), dtype=np.float32)
    p["b0"] = np.zeros(2, dtype=np.float32)
    p["w_out"] = np.array([1.0, 0.0], dtype=np.float32)
    p["b_out"] = np.zeros(1, dtype=np.float32)
    d = np.diff(g.row_ptr).astype(float)
    x0, _ = om.mpnn_forward(g, p, source=0, layers=1)
    assert np.allclose(x0, d / d.sum(), atol=1e-15)


def test_aggregation_is_transition_matrix():
    g = gg.random_connected(20, 4.0, seed=5)
    import oracle
    P = oracle.transition_dense(g)
    params = gg.mpnn_init(1, layers=1, hidden=4)
    _, cache = om.mpnn_forward(g, params, source=0, layers=1)
    assert np.allclose(cache["M"][0], P @ cache["H"][0], atol=1e-14)


@pytest.mark.parametrize("layers", [1, 3])
def test_gradients_match_finite_differences(layers):
    g = gg.random_connected(25, 4.0, seed=7)
    params = {k: v.astype(np.float64) for k, v in gg.mpnn_init(3, layers=layers, hidden=8).items()}
    params["b_out"] = np.array([0.1])
    import oracle
    target = oracle.pagerank_exact(g, gg.source_personalization(g.n, [4])[0], 0.85)
    x0, cache = om.mpnn_forward(g, params, 4, layers=layers)
    grads = om.mpnn_backward(params, cache, target, layers=layers)
    rng = gg.philox(11)
    h = 1e-6
    for name in om.param_names(layers):
        flat = params[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = om.mpnn_loss(om.mpnn_forward(g, params, 4, layers=layers)[0], target)
            flat[idx] = old - h
            lm = om.mpnn_loss(om.mpnn_forward(g, params, 4, layers=layers)[0], target)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, an)


def test_mutation_wrong_aggregation_transpose_is_caught(monkeypatch):
    """Planting D^{-1} A (the transpose) instead of A D^{-1} in the forward
    breaks the aggregation pin."""
    g = gg.random_connected(20, 4.0, seed=5)
    import oracle
    P = oracle.transition_dense(g)
    orig = om.mpnn_forward

    def wrong(g_, params, source, layers=3, bf16=False):
        x0, cache = orig(g_, params, source, layers, bf16)
        d = cache["d"]
        cache["M"][0] = (cache["A"] @ cache["H"][0]) / d[:, None]
        return x0, cache
    monkeypatch.setattr(om, "mpnn_forward", wrong)
    _, cache = om.mpnn_forward(g, gg.mpnn_init(1, layers=1, hidden=4), 0, layers=1)
    assert not np.allclose(cache["M"][0], P @ cache["H"][0], atol=1e-10)


def test_adam_first_step_is_signed_learning_rate():
    # with zero moments, the bias-corrected first update is lr * g / (|g| + eps)
    g = np.array([3.0, -2e-3, 0.0, 5e-9])
    w, m, v = om.adam_step(np.ones(4), g, np.zeros(4), np.zeros(4), 0, 0.1)
    assert np.allclose(w, 1.0 - 0.1 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert abs(w[0] - 0.9) < 1e-9 and abs(w[1] - 1.1) < 1e-6 and w[2] == 1.0
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_moves_lr_per_step():
    # bias correction makes m_hat = g and v_hat = g^2 exactly for a constant gradient
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    g = np.array([0.5, -4.0, 1e-3])
    for t in range(25):
        w, m, v = om.adam_step(w, g, m, v, t, 0.01)
    assert np.allclose(w, -25 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
