"""Pins of the oracle's learned-guess network (oracle/mlp.py): hand-evaluated
closed forms, central finite differences of the loss for every parameter and
input, Adam's closed-form first steps, the feature maps' round trip, a
training sanity check, and planted mistakes that the pins must catch."""
import math

import numpy as np
import pytest

from oracle import mlp as om

SMALL = (6, 5, 2, 4)      # n_in, n_hidden, n_layers, n_out


def _params(shape, seed):
    _, n = om.layout(*shape)
    return np.random.default_rng(seed).uniform(-0.6, 0.6, n)


def test_layout_counts_the_paper_sized_network():
    # 1250 -> 256 -> 256 -> 625 at order 4: 546,673 weights and biases
    _, n = om.layout(1250, 256, 2, 625)
    assert n == 1250 * 256 + 256 + 256 * 256 + 256 + 256 * 625 + 625


def test_forward_closed_form():
    # one hidden unit: y = w2 tanh(w1 x + b1) + b2
    shape = (1, 1, 1, 1)
    w = np.array([0.5, -0.25, 2.0, 0.1])          # W1, b1, W2, b2
    x = np.array([[3.0], [-1.0]])
    y, acts = om.forward(w, x, shape)
    np.testing.assert_allclose(y[:, 0], 2.0 * np.tanh(0.5 * x[:, 0] - 0.25) + 0.1, rtol=0, atol=1e-15)
    assert len(acts) == 2


def test_mse_closed_form():
    loss, dy = om.mse(np.array([[1.0, 2.0]]), np.array([[0.0, 4.0]]))
    assert loss == pytest.approx(2.5, abs=1e-15)
    np.testing.assert_allclose(dy, [[1.0, -2.0]], atol=1e-15)


def _loss(w, x, t, shape):
    y, _ = om.forward(w, x, shape)
    return om.mse(y, t)[0]


@pytest.mark.parametrize("shape", [SMALL, (3, 4, 1, 2), (5, 3, 3, 5)])
def test_gradients_match_central_differences(shape):
    rng = np.random.default_rng(2)
    w = _params(shape, 1)
    x = rng.standard_normal((3, shape[0]))
    t = rng.standard_normal((3, shape[3]))
    y, acts = om.forward(w, x, shape)
    _, dy = om.mse(y, t)
    dw, dx = om.backward(w, acts, dy, shape)
    h = 1e-6
    fd = np.array([(_loss(w + h * e, x, t, shape) - _loss(w - h * e, x, t, shape)) / (2 * h)
                   for e in np.eye(w.size)])
    assert np.abs(fd - dw).max() <= 1e-8 * max(1.0, np.abs(dw).max())
    fdx = np.zeros_like(x)
    for i in range(x.shape[0]):
        for j in range(x.shape[1]):
            e = np.zeros_like(x)
            e[i, j] = h
            fdx[i, j] = (_loss(w, x + e, t, shape) - _loss(w, x - e, t, shape)) / (2 * h)
    assert np.abs(fdx - dx).max() <= 1e-8 * max(1.0, np.abs(dx).max())


def test_adam_closed_form_first_steps():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m1 = np.zeros(3)
    m2 = np.zeros(3)
    # with bias correction, a constant gradient gives m_hat = g and v_hat = g^2,
    # so every step moves each weight by lr * g / (|g| + eps)
    w1, m1, m2 = om.adam(w, g, m1, m2, lr=0.01, step=1)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    w2, m1, m2 = om.adam(w1, g, m1, m2, lr=0.01, step=2)
    np.testing.assert_allclose(w2, w1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-13)


def test_field_stats_and_maps_round_trip():
    rng = np.random.default_rng(5)
    n_elem, dpe = 3, 5 * 8
    q = rng.standard_normal(n_elem * dpe) + np.tile([1.0, 0.0, 0.0, 0.0, 100.0], n_elem * dpe // 5)
    dq_prev = 1e-3 * rng.standard_normal(n_elem * dpe)
    dq = dq_prev + 1e-5 * rng.standard_normal(n_elem * dpe)
    r = 50.0 * rng.standard_normal(n_elem * dpe)
    stats = om.field_stats(q, dq_prev, dq, r)
    mean, std, rms, rc, rr = stats
    qv = q.reshape(-1, 5)
    # two-pass textbook formulas for comparison
    for v in range(5):
        col = qv[:, v]
        assert mean[v] == pytest.approx(sum(col) / len(col), rel=1e-14)
        assert std[v] == pytest.approx(math.sqrt(sum((c - mean[v]) ** 2 for c in col) / len(col)), rel=1e-12)
    cv = (dq - dq_prev).reshape(-1, 5)
    for v in range(5):
        assert rms[v] == pytest.approx(math.sqrt(sum(c * c for c in dq_prev.reshape(-1, 5)[:, v]) / len(cv)),
                                       rel=1e-13)
        assert rc[v] == pytest.approx(math.sqrt(sum(c * c for c in cv[:, v]) / len(cv)), rel=1e-13)
        assert rr[v] == pytest.approx(math.sqrt(sum(c * c for c in r.reshape(-1, 5)[:, v]) / len(cv)), rel=1e-13)
    x = om.features(q, dq_prev, stats, n_elem)
    assert x.shape == (n_elem, 2 * dpe)
    np.testing.assert_allclose(x[1, :5], (q[dpe:dpe + 5] - mean) / std, atol=1e-14)
    np.testing.assert_allclose(x[2, dpe:dpe + 5], dq_prev[2 * dpe:2 * dpe + 5] / rms, atol=1e-14)
    x3 = om.features(q, dq_prev, stats, n_elem, r)
    assert x3.shape == (n_elem, 3 * dpe)
    np.testing.assert_array_equal(x3[:, :2 * dpe], x)
    np.testing.assert_allclose(x3[1, 2 * dpe:2 * dpe + 5], r[dpe:dpe + 5] / rr, atol=1e-14)
    t = om.target(dq, dq_prev, stats, n_elem)
    np.testing.assert_allclose(t[0, :5], (dq[:5] - dq_prev[:5]) / rc, atol=1e-14)
    np.testing.assert_allclose(om.apply(dq_prev, t, stats, n_elem), dq, rtol=0, atol=1e-17)
    # a constant variable has no spread: std becomes 1
    qc = np.tile([1.0, 2.0, 3.0, 4.0, 5.0], 10)
    _, std_c, rms_c, rc_c, rr_c = om.field_stats(qc, np.zeros(50))
    np.testing.assert_array_equal(std_c, np.ones(5))
    np.testing.assert_array_equal(rms_c, np.ones(5))
    np.testing.assert_array_equal(rc_c, np.ones(5))
    np.testing.assert_array_equal(rr_c, np.ones(5))       # no residual given


def test_training_reduces_loss():
    rng = np.random.default_rng(7)
    shape = (4, 16, 2, 2)
    w = _params(shape, 3) * 0.5
    x = rng.standard_normal((64, 4))
    t = np.stack([np.sin(x[:, 0] + x[:, 1]), x[:, 2] * x[:, 3]], axis=1)
    m1, m2 = np.zeros_like(w), np.zeros_like(w)
    first = _loss(w, x, t, shape)
    for step in range(1, 301):
        y, acts = om.forward(w, x, shape)
        _, dy = om.mse(y, t)
        dw, _ = om.backward(w, acts, dy, shape)
        w, m1, m2 = om.adam(w, dw, m1, m2, lr=1e-2, step=step)
    assert _loss(w, x, t, shape) < 0.1 * first


def test_planted_mistakes_are_caught(monkeypatch):
    good = om.backward

    def dropped_bias_gradients(w, acts, dy, shape):
        dw, dx = good(w, acts, dy, shape)
        lay, _ = om.layout(*shape)
        for _, _, fo, bo in lay:
            dw[bo:bo + fo] = 0.0
        return dw, dx

    monkeypatch.setattr(om, "backward", dropped_bias_gradients)
    with pytest.raises(AssertionError):
        test_gradients_match_central_differences(SMALL)
    monkeypatch.setattr(om, "backward", good)

    good_adam = om.adam
    monkeypatch.setattr(om, "adam", lambda w, g, m1, m2, lr, step, beta1=0.9, beta2=0.999, eps=1e-8:
                        good_adam(w, g, m1, m2, lr, 1, beta1, beta2, eps))   # bias correction frozen at step 1
    with pytest.raises(AssertionError):
        test_adam_closed_form_first_steps()


# ---------------------------------------------------------------- bfloat16 mode

def test_bf16_round_hand_values():
    one = 1.0
    cases = [(one, one), (1 + 2 ** -8, one),                    # tie between 1 and 1 + 2^-7: even is 1
             (1 + 3 * 2 ** -8, 1 + 2 ** -6),                    # tie between odd 1 + 2^-7 and even 1 + 2^-6
             (1 + 2 ** -8 + 2 ** -20, 1 + 2 ** -7),             # just above the tie
             (-(1 + 2 ** -8), -one), (0.0, 0.0), (3.0, 3.0), (2.0 ** -126, 2.0 ** -126),
             (65535.0, 65536.0), (255.5, 256.0)]
    got = om.bf16_round(np.array([c for c, _ in cases]))
    assert got.tolist() == [r for _, r in cases]


def test_bf16_round_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * np.exp(rng.uniform(-40, 40, 20000))).astype(np.float32)
    ties = (np.arange(1, 2001, dtype=np.uint32) << 16 | 0x8000).view(np.float32)   # exact ties
    x = np.concatenate([x, ties, -ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(om.bf16_round(x), ref)


def test_bf16_forward_is_exact_on_representable_operands():
    shape = (8, 6, 0, 5)                        # one linear map: no tanh between products
    _, n = om.layout(*shape)
    rng = np.random.default_rng(4)
    # values with at most 8 significant bits are their own bfloat16
    w = rng.integers(-127, 128, n) / 128.0
    x = rng.integers(-127, 128, (3, 8)) / 64.0
    y0, a0 = om.forward(w, x, shape)
    y1, a1 = om.forward(w, x, shape, bf16=True)
    assert np.array_equal(y0, y1)
    dy = rng.integers(-127, 128, y0.shape) / 32.0
    d0 = om.backward(w, a0, dy, shape)
    d1 = om.backward(w, a1, dy, shape, bf16=True)
    assert np.array_equal(d0[0], d1[0]) and np.array_equal(d0[1], d1[1])


def test_bf16_forward_within_the_rounding_bound():
    shape = (40, 16, 0, 12)
    _, n = om.layout(*shape)
    rng = np.random.default_rng(5)
    w, x = rng.standard_normal(n), rng.standard_normal((7, 40))
    y, _ = om.forward(w, x, shape)
    yb, _ = om.forward(w, x, shape, bf16=True)
    wl = w[:40 * 12].reshape(40, 12)
    bound = (2 * 2.0 ** -8 + 2.0 ** -16) * (np.abs(x) @ np.abs(wl))
    assert np.all(np.abs(yb - y) <= bound)
    assert np.any(yb != y)                      # the rounding is not a no-op


def test_bf16_planted_truncation_is_caught(monkeypatch):
    def truncate(a):
        u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
        return u.view(np.float32).astype(np.float64)
    monkeypatch.setattr(om, "bf16_round", truncate)
    with pytest.raises(AssertionError):
        test_bf16_round_hand_values()


# ---- condensed-residual loss (om.condensed_loss) ----

def _loss_case(seed=5, orders=(2, 3)):
    import oracle
    _, bnode = oracle.dof_maps(np.array(orders))
    n_dof = sum(5 * (p + 1) ** 3 for p in orders)
    n1 = bnode.size
    rng = np.random.default_rng(seed)
    s = rng.standard_normal((n1, n1)) + 3.0 * np.eye(n1)     # not symmetric
    y, t = rng.standard_normal(n_dof), rng.standard_normal(n_dof)
    rc = rng.uniform(0.2, 3.0, 5)
    return s, bnode, y, t, rc


def test_condensed_loss_with_identity_is_the_weighted_boundary_sum():
    s, bnode, y, t, rc = _loss_case()
    loss, g = om.condensed_loss(np.eye(s.shape[0]), bnode, y, t, rc)
    # plain loops over boundary slots
    want, gw = 0.0, np.zeros_like(y)
    for node in range(bnode.shape[0]):
        for v in range(5):
            i = int(bnode[node, v])
            assert i % 5 == v
            d = rc[v] * (y[i] - t[i])
            want += d * d
            gw[i] = 2.0 * rc[v] * d
    assert loss == pytest.approx(want, rel=1e-13)
    np.testing.assert_allclose(g, gw, rtol=1e-13, atol=0)


def test_condensed_loss_zero_error_and_interior_blindness():
    s, bnode, y, t, rc = _loss_case()
    loss, g = om.condensed_loss(s, bnode, t, t, rc)
    assert loss == 0.0 and not g.any()
    interior = np.setdiff1d(np.arange(y.size), bnode.reshape(-1))
    assert interior.size > 0
    y2 = y.copy()
    y2[interior] += 7.0
    l1, g1 = om.condensed_loss(s, bnode, y, t, rc)
    l2, _ = om.condensed_loss(s, bnode, y2, t, rc)
    assert l1 == l2 and not g1[interior].any()


def test_condensed_loss_gradient_matches_central_differences():
    s, bnode, y, t, rc = _loss_case()
    loss, g = om.condensed_loss(s, bnode, y, t, rc)
    rng = np.random.default_rng(9)
    picks = np.concatenate([bnode.reshape(-1)[rng.choice(bnode.size, 12, replace=False)], [0, 13]])
    h = 1e-6
    for i in picks:
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        fd = (om.condensed_loss(s, bnode, yp, t, rc)[0] - om.condensed_loss(s, bnode, ym, t, rc)[0]) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-6 * loss)


def test_condensed_loss_planted_transpose_is_caught():
    # a gradient built with S S^T in place of S^T S misses the central differences
    s, bnode, y, t, rc = _loss_case()
    idx = bnode.reshape(-1)
    w = np.tile(rc, y.size // 5)
    e = (w * (y - t))[idx]
    wrong = np.zeros_like(y)
    wrong[idx] = 2.0 * (s @ (s.T @ e))
    wrong *= w
    _, g = om.condensed_loss(s, bnode, y, t, rc)
    i = int(idx[3])
    h = 1e-6
    yp, ym = y.copy(), y.copy()
    yp[i] += h
    ym[i] -= h
    fd = (om.condensed_loss(s, bnode, yp, t, rc)[0] - om.condensed_loss(s, bnode, ym, t, rc)[0]) / (2 * h)
    assert fd == pytest.approx(g[i], rel=1e-6)
    assert abs(wrong[i] - fd) > 1e-3 * abs(fd)
