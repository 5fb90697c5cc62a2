"""Pins of the CNN oracle: convolution against scipy's correlation,
gradients against finite differences, Adam's first step in closed form,
bfloat16 rounding on known values."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import cnn


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 0.0], np.float32)
    got = cnn.bf16(vals)
    # 1+2^-8 is a tie between 1 and 1+2^-7: even mantissa wins (1.0)
    want = [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5, 0.0]
    assert list(got) == want


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 7, 9, cnn.CH))
    W = rng.normal(size=(9, cnn.CH, cnn.CH))
    b = rng.normal(size=cnn.CH)
    out = cnn.conv3x3(x, W, b)
    K = W.reshape(3, 3, cnn.CH, cnn.CH)  # [dy][dx][co][ci]
    for n in range(2):
        for co in range(cnn.CH):
            ref = np.full((7, 9), b[co])
            for ci in range(cnn.CH):
                ref += correlate(x[n, :, :, ci], K[:, :, co, ci], mode="same", method="direct")
            np.testing.assert_allclose(out[n, :, :, co], ref, rtol=1e-10, atol=1e-10)


def _loss(params, x0, coarse, label):
    _, out = cnn.forward(params, x0, rounding=False)
    return cnn.loss_and_grad(out, coarse, label)[0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    H, W = 5, 6
    params = rng.normal(scale=0.3, size=cnn.NPARAMS)
    x0 = rng.normal(size=(1, H, W, cnn.CH))
    coarse = rng.uniform(0, 4, size=(1, H, W))
    label = coarse + rng.normal(scale=1.5, size=(1, H, W))
    acts, out = cnn.forward(params, x0, rounding=False)
    _, dout = cnn.loss_and_grad(out, coarse, label)
    g = cnn.backward(params, x0, acts, dout, rounding=False)
    idx = rng.choice(cnn.NPARAMS, size=40, replace=False)
    idx = np.concatenate([idx, [3 * cnn.PER_LAYER - 1, cnn.NPARAMS - 1]])  # biases too
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (_loss(pp, x0, coarse, label) - _loss(pm, x0, coarse, label)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = cnn.adam(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-6)
    assert p[3] == 0.0
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_window_map_fallback_and_clamps():
    coarse = np.array([[2.0, 10.25], [0.1, 47.9]], np.float32)
    out = np.zeros((1, 2, 2, cnn.CH), np.float32)
    out[0, :, :, 0] = [[1.0, -0.5], [0.0, 3.0]]
    out[0, :, :, 1] = [[5.0, -5.0], [5.0, 5.0]]
    lo, nfb, mask = cnn.window_map(coarse, out, 8, 8, 192, 16, 0.5)
    assert nfb == 4 * 4  # one coarse pixel of four falls back, 16 full pixels
    assert mask[:4, 4:].all() and mask.sum() == 16
    assert lo[0, 0] == 4 * 3 - 8           # confident: 4 * (2 + 1) = 12 -> 4
    assert lo[0, 4] == 41 - 8              # fallback: 4 * 10.25 = 41
    assert lo[4, 0] == 0                   # clamped below
    assert lo[4, 4] == 192 - 16            # 4 * 50.9 -> clamped above
    # tau = 1 sends every pixel to the fallback, tau = 0 none
    assert cnn.window_map(coarse, out, 8, 8, 192, 16, 1.0)[1] == 64
    assert cnn.window_map(coarse, out, 8, 8, 192, 16, 0.0)[1] == 0


def test_window_map_fallback_margin_by_hand():
    # one coarse pixel, not confident, 4 x 4 full pixels at x = 0..3
    # (and a copy at x = 4..7 through the clamp to the last coarse column)
    out = np.zeros((1, 1, 1, cnn.CH), np.float32)
    out[0, 0, 0, 1] = -1.0
    coarse = np.array([[0.5]], np.float32)  # match x - 2: left of the image for x < 2
    _, n_all, _ = cnn.window_map(coarse, out, 8, 4, 64, 16, 0.5)
    assert n_all == 32
    _, n0, m0 = cnn.window_map(coarse, out, 8, 4, 64, 16, 0.5, 0)
    assert n0 == 4 * 6 and not m0[:, :2].any() and m0[:, 2:].all()  # x - 2 >= 0 from x = 2 on
    _, n5, m5 = cnn.window_map(coarse, out, 8, 4, 64, 16, 0.5, 5)
    assert n5 == 4 * 1 and m5[:, 7].all()                             # only x = 7 has x - 2 >= 5
    _, nneg, _ = cnn.window_map(coarse, out, 8, 4, 64, 16, 0.5, -2)
    assert nneg == 32                                                  # x - 2 >= -2 everywhere
    # the margin never touches confident pixels or the window starts
    out[0, 0, 0, 1] = 1.0
    lo_a, n_a, _ = cnn.window_map(coarse, out, 8, 4, 64, 16, 0.5)
    lo_b, n_b, _ = cnn.window_map(coarse, out, 8, 4, 64, 16, 0.5, 0)
    assert n_a == n_b == 0 and (lo_a == lo_b).all()


def test_confidence_threshold_is_the_logit():
    for tau in (0.1, 0.5, 0.73, 0.99):
        t = float(cnn.confidence_threshold(tau))
        assert abs(1.0 / (1.0 + np.exp(-t)) - tau) < 1e-6
    assert cnn.confidence_threshold(0.5) == 0.0


def test_prepare_input_border_channel():
    cd = np.array([[0.0, 3.0, 1.5, 0.0]], np.float32)
    left = np.array([[0, 255, 51, 128]], np.uint8)
    x = cnn.prepare_input(cd, left)
    np.testing.assert_allclose(x[0, 0, :, 2], [0.0, -2.0 / 16, 0.5 / 16, 3.0 / 16])
    np.testing.assert_allclose(x[0, 0, :, 0], cd[0] / 16)
    np.testing.assert_allclose(x[0, 0, :, 1], left[0] / 255.0 - 0.5, atol=1e-7)
    assert not x[..., 3:].any()
    far = cnn.prepare_input(np.zeros((1, 40), np.float32), np.zeros((1, 40), np.uint8))
    assert far[0, 0, 39, 2] == 1.0  # saturates at 16 columns


def test_fallback_rects():
    H, W, D, r = 200, 600, 64, 3
    m = np.zeros((H, W), np.uint8)
    assert cnn.fallback_rects(m, 32, 0.75, D, r) == []
    m[100, 300] = 1
    # rows 68..132, columns 300 - 32 - 63 - 3 .. 300 + 32 + 3
    assert cnn.fallback_rects(m, 32, 0.75, D, r) == [(68, 133, 202, 336)]
    m[10, 5] = 1
    m[150, 320] = 1  # touches the band of row 100 once widened
    assert cnn.fallback_rects(m, 32, 0.75, D, r) == [(0, 43, 0, 41), (68, 183, 202, 356)]
    # area 43 * 41 + 115 * 154 = 19473 > 0.15 * H * W = 18000
    assert cnn.fallback_rects(m, 32, 0.15, D, r) == [(0, H, 0, W)]
    m[:] = 1
    assert cnn.fallback_rects(m, 32, 1.0, D, r) == [(0, H, 0, W)]
    m[:] = 0
    m[0, W - 1] = m[H - 1, 0] = 1
    assert cnn.fallback_rects(m, 10, 0.75, D, r) == [(0, 11, W - 1 - 10 - 63 - 3, W), (H - 11, H, 0, 14)]


def test_merge_fallback_takes_rect_results_on_masked_pixels():
    rng = np.random.default_rng(3)
    H, W = 12, 7
    wi = rng.integers(0, 50, (H, W)).astype(np.uint16)
    ws = wi.astype(np.float32) + 0.25
    mask = (rng.random((H, W)) < 0.3).astype(np.uint8)
    mask[:3] = 0
    mask[:, 5:] = 0
    mask[:, 0] = 0
    rects = [(2, 12, 1, 5)]
    bi = rng.integers(100, 150, (10, 4)).astype(np.uint16)
    bs = bi.astype(np.float32) - 0.25
    di, ds = cnn.merge_fallback(wi, ws, mask, rects, [(bi, bs)])
    m = mask.astype(bool)
    assert (di[m] >= 100).all() and (di[~m] < 50).all()
    np.testing.assert_array_equal(di[2:, 1:5][m[2:, 1:5]], bi[m[2:, 1:5]])
    np.testing.assert_array_equal(ds[~m], ws[~m])


def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "hand_cnn_loss_adam.json")) as f:
        return json.load(f)


def test_loss_value_and_gradient_on_hand_worked_pixels():
    """The loss value itself (not only its gradient): Huber delta 1, the
    strict |e| < 1 confidence target (pixel C sits exactly at |e| = 1) and
    the mean over pixels, worked by hand."""
    g = _golden()["loss"]
    out = np.zeros((1, 1, 3, cnn.CH))
    out[0, 0, :, 0] = g["offset"]
    out[0, 0, :, 1] = g["logit"]
    coarse = np.array(g["coarse"]).reshape(1, 1, 3)
    label = np.array(g["label"]).reshape(1, 1, 3)
    loss, grad = cnn.loss_and_grad(out, coarse, label)
    assert abs(loss - g["loss"]) <= 1e-14
    np.testing.assert_allclose(grad[0, 0, :, 0], g["d_offset"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(grad[0, 0, :, 1], g["d_logit"], rtol=0, atol=1e-15)
    assert not grad[..., 2:].any()


def test_adam_second_step_hand_worked():
    """Two bias-corrected steps with different gradients, worked by hand."""
    g = _golden()["adam"]
    p = np.array(g["p0"])
    m = np.zeros(2)
    v = np.zeros(2)
    p, m, v = cnn.adam(p, m, v, np.array(g["g"][0]), 1, lr=g["lr"], eps=0.0)
    np.testing.assert_allclose(p, g["p1"], rtol=0, atol=1e-15)
    p, m, v = cnn.adam(p, m, v, np.array(g["g"][1]), 2, lr=g["lr"], eps=0.0)
    np.testing.assert_allclose(m, g["m2"], rtol=1e-14)
    np.testing.assert_allclose(v, g["v2"], rtol=1e-13)
    assert abs(p[1] - g["p2_component2"]) <= 1e-14
    assert abs(p[0] - g["p2_component1_approx"]) <= g["p2_component1_tol"]


def test_adam_constant_gradient_moves_by_the_learning_rate_every_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each step moves
    by exactly lr * sign(g) when eps = 0 -- a property of the published
    update that fails for a bias correction taken at the wrong step."""
    g = np.array([0.7, -0.03, 5.0])
    p = np.array([0.0, 1.0, -2.0])
    m = np.zeros(3)
    v = np.zeros(3)
    for step in range(1, 8):
        before = p.copy()
        p, m, v = cnn.adam(p, m, v, g, step, lr=0.01, eps=0.0)
        np.testing.assert_allclose(before - p, 0.01 * np.sign(g), rtol=1e-9, err_msg="step %d" % step)
