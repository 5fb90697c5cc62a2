"""Search-window network kernels (forward, loss, backward, Adam, window map)
against the numpy oracle, plus the learned-window pipeline step by step.

Floating-point bar: the GPU rounds the same operands to bfloat16 as the
oracle and accumulates in float32, so a float32 result may differ from the
oracle's float64 sum by the accumulation error, bounded here by
K * 2^-22 * (the same sum over absolute values) for K = 144 products per
output; a bfloat16 result may in addition sit one bfloat16 step (2^-7
relative) away where the exact value lies near a rounding boundary.  Weight
gradients are sums over every pixel: bounded relative to their absolute
sums (2e-3, far below the O(1) error of any wrong index).  Integer results
(window starts, fallback counts, disparities) are exact.
"""
import numpy as np
import pytest

import oracle
from oracle import cnn as ocnn
from paper_2012_10802_amd import synth

pytestmark = pytest.mark.gpu

CH = 16


@pytest.fixture(scope="module")
def lw():
    import torch
    from paper_2012_10802_amd import learned_window as mod
    assert torch.cuda.is_available()
    return mod


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bf16_bits_to_f(t):
    a = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return a.view(np.float32).astype(np.float64)


def _params(seed):
    from paper_2012_10802_amd import learned_window as mod
    rng = np.random.default_rng(seed)
    p = mod.init_params(seed).astype(np.float64)
    per = ocnn.PER_LAYER
    for l in range(4):  # non-zero biases, last layer at full scale
        p[l * per + 9 * CH * CH: (l + 1) * per] = rng.normal(0, 0.1, CH)
    p[3 * per: 3 * per + 9 * CH * CH] *= 10
    return p.astype(np.float32)


def _input(n, H, W, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, H, W, CH))
    x[..., 0] = rng.uniform(0, 4, (n, H, W))
    x[..., 1] = rng.uniform(-0.5, 0.5, (n, H, W))
    return ocnn.bf16(x)


def _to_bf16_dev(x):
    u = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32) >> 16
    return _dev(u.astype(np.uint16).view(np.int16))


def _ulp_bf16(x):
    ax = np.maximum(np.abs(x), 1e-30)
    return 2.0 ** (np.floor(np.log2(ax)) - 7)


def _abs_conv(x, W, b):
    return ocnn.conv3x3(np.abs(x), np.abs(W), np.abs(b))


SHAPES = [(1, 5, 16), (2, 13, 37), (1, 9, 70)]  # several strips, ragged tails


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_forward_layerwise(lw, shape):
    """Each layer, fed the GPU's own previous activation, against the oracle."""
    import torch
    n, H, W = shape
    params = _params(n * 100 + W)
    x0 = _input(n, H, W, W)
    net = lw.WindowNet(params)
    acts, out = net.buffers(W, H, n)
    net.forward(_to_bf16_dev(x0), acts, out, W, H, n)
    torch.cuda.synchronize()
    Ws, bs = ocnn.unpack(params)
    x = x0
    for l in range(4):
        want = ocnn.conv3x3(x, ocnn.bf16(Ws[l]), bs[l])
        mag = _abs_conv(x, ocnn.bf16(Ws[l]), bs[l])
        tol = 144 * 2.0 ** -21 * mag + 1e-30
        if l < 3:
            got = _bf16_bits_to_f(acts[l])
            r = np.maximum(want, 0)
            err = np.abs(got - r)
            assert np.all(err <= tol + _ulp_bf16(r) * (r > 0)), "layer %d max err %g" % (l, err.max())
            assert np.mean(got == ocnn.bf16(r)) > 0.99
            x = got
        else:
            # the output keeps the two channels the window map reads
            got = out.cpu().numpy().astype(np.float64)
            assert got.shape[-1] == 2
            err = np.abs(got - want[..., :2])
            assert np.all(err <= tol[..., :2]), "output max err %g" % err.max()


@pytest.mark.parametrize("shape", SHAPES + [(2, 1, 1), (1, 3, 2), (3, 40, 61), (16, 270, 480)],
                         ids=lambda s: "x".join(map(str, s)))
def test_infer_equals_layer_by_layer_forward(lw, shape):
    """The one-launch inference (activations kept in LDS, tiles of 24 x 16
    with a 4-pixel halo) gives the layer-by-layer forward's output bit for
    bit: tiles in both directions, ragged right and bottom tiles, image
    borders inside tiles, several images."""
    import torch
    n, H, W = shape
    params = _params(n + H + W)
    x0 = _input(n, H, W, H)
    net = lw.WindowNet(params)
    acts, out = net.buffers(W, H, n)
    xd = _to_bf16_dev(x0)
    net.forward(xd, acts, out, W, H, n)
    out2 = torch.full_like(out, float("nan"))
    net.infer(xd, out2, W, H, n)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)


def test_forward_end_to_end_matches_oracle(lw):
    import torch
    n, H, W = 2, 11, 45
    params = _params(7)
    x0 = _input(n, H, W, 3)
    net = lw.WindowNet(params)
    acts, out = net.buffers(W, H, n)
    net.forward(_to_bf16_dev(x0), acts, out, W, H, n)
    torch.cuda.synchronize()
    _, want = ocnn.forward(params, x0)
    want = want[..., :2]
    got = out.cpu().numpy()
    scale = np.abs(want).max()
    assert np.abs(got - want).max() <= 0.02 * scale


def test_prepare_input_and_label_downsample(lw):
    import torch
    rng = np.random.default_rng(5)
    Hc, Wc = 9, 23
    cd = rng.uniform(0, 30, (2, Hc, Wc)).astype(np.float32)
    cl = rng.integers(0, 256, (2, Hc, Wc), dtype=np.uint8)
    x0 = lw.prepare_input(_dev(cd), _dev(cl), Wc, Hc, 2)  # two images in one call
    torch.cuda.synchronize()
    for i in range(2):
        np.testing.assert_array_equal(_bf16_bits_to_f(x0)[i], ocnn.bf16(ocnn.prepare_input(cd[i], cl[i]))[0])
    full = rng.uniform(0, 190, (4 * Hc + 2, 4 * Wc + 3)).astype(np.float32)
    got = lw.label_downsample4(_dev(full)).cpu().numpy()
    blocks = full[:4 * Hc, :4 * Wc].reshape(Hc, 4, Wc, 4).astype(np.float64)
    want = blocks.mean(axis=(1, 3)) / 4.0  # mean disparity in coarse pixels
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-5)


def test_loss_gradient(lw):
    import torch
    from paper_2012_10802_amd import sgm as S
    rng = np.random.default_rng(9)
    n, H, W = 1, 10, 33
    out = rng.normal(0, 2, (n, H, W, CH)).astype(np.float32)
    # multiples of 1/64: label - coarse is exact in float32 on both sides
    coarse = (rng.integers(0, 40 * 64, (H, W)) / 64.0).astype(np.float32)
    label = (coarse + rng.integers(-96, 97, (H, W)) / 64.0).astype(np.float32)
    dy = torch.empty((n, H, W, CH), dtype=torch.int16, device="cuda")
    loss = torch.zeros(2, dtype=torch.float32, device="cuda")
    # the GPU output holds the two channels the loss reads
    outd, cd, ld = _dev(np.ascontiguousarray(out[..., :2])), _dev(coarse), _dev(label)  # held until the call has run
    S._check(S.library().sgm_cnn_loss(lw._c(outd), lw._c(cd), lw._c(ld), W, H, n,
                                      lw._c(dy), lw._c(loss), S._stream()), "sgm_cnn_loss")
    torch.cuda.synchronize()
    want_loss, g = ocnn.loss_and_grad(out, coarse[None], label[None])
    got = _bf16_bits_to_f(dy)
    wb = ocnn.bf16(g)
    assert np.all(np.abs(got - wb) <= _ulp_bf16(g) + 1e-30)
    assert np.all(got[..., 2:] == 0)
    np.testing.assert_allclose(float(loss.sum()), want_loss, rtol=1e-4)


@pytest.mark.parametrize("shape", [(1, 6, 20), (2, 13, 37)], ids=lambda s: "x".join(map(str, s)))
def test_backward_gradients(lw, shape):
    """Parameter gradient for a given output gradient, with the GPU's own
    forward activations, against the oracle; and bitwise reproducible."""
    import torch
    n, H, W = shape
    params = _params(W + 1)
    x0 = _input(n, H, W, W + 2)
    rng = np.random.default_rng(W + 3)
    dout = np.zeros((n, H, W, CH))
    dout[..., :2] = rng.normal(0, 1e-3, (n, H, W, 2))
    dout = ocnn.bf16(dout)
    net = lw.WindowNet(params)
    bufs = net.train_buffers(W, H, n)
    acts, out, _, scratch, _ = bufs
    x0d, doutd = _to_bf16_dev(x0), _to_bf16_dev(dout)
    net.forward(x0d, acts, out, W, H, n)
    S = lw.S
    grads = []
    for _ in range(2):
        S._check(S.library().sgm_cnn_backward(lw._c(net.wb), lw._c(x0d), lw._c(acts), lw._c(doutd),
                                              W, H, n, lw._c(net.grad), lw._c(scratch), scratch.numel(),
                                              S._stream()), "sgm_cnn_backward")
        torch.cuda.synchronize()
        grads.append(net.grad.cpu().numpy().copy())
    np.testing.assert_array_equal(grads[0], grads[1])
    gacts = [_bf16_bits_to_f(acts[l]) for l in range(3)]
    want = ocnn.backward(params, x0, gacts, dout)
    mag = ocnn.backward(np.abs(params), np.abs(x0), gacts, np.abs(dout))
    err = np.abs(grads[0] - want)
    assert np.all(err <= 2e-3 * mag + 1e-30), "max rel err %g" % (err / np.maximum(mag, 1e-30)).max()
    # the unused input channels of layer 0 get exactly zero gradient
    W0 = grads[0][:9 * CH * CH].reshape(9, CH, CH)
    assert np.all(W0[:, :, 2:] == 0)


def test_adam_and_weight_packing(lw):
    import torch
    rng = np.random.default_rng(21)
    params = _params(3)
    net = lw.WindowNet(params)
    m = rng.normal(0, 1e-3, params.shape).astype(np.float32)
    v = rng.uniform(0, 1e-6, params.shape).astype(np.float32)
    g = rng.normal(0, 1e-3, params.shape).astype(np.float32)
    net.m.copy_(_dev(m))
    net.v.copy_(_dev(v))
    net.grad.copy_(_dev(g))
    S = lw.S
    step, lr = 7, 1e-3
    S._check(S.library().sgm_cnn_adam(lw._c(net.params), lw._c(net.m), lw._c(net.v), lw._c(net.grad), step, lr,
                                      0.9, 0.999, 1e-8, lw._c(net.wf), lw._c(net.wb), S._stream()), "adam")
    torch.cuda.synchronize()
    # the kernel receives the hyper-parameters as float32: the oracle takes
    # the same values
    f = lambda a: float(np.float32(a))  # noqa: E731
    wp, wm, wv = ocnn.adam(params.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                           g.astype(np.float64), step, f(lr), f(0.9), f(0.999), f(1e-8))
    # float32 rounding, bounded by the magnitudes of the terms that are added
    # (the moments can cancel), then carried through the update
    b1, b2, eps = f(0.9), f(0.999), f(1e-8)
    tm = 2.0 ** -21 * (b1 * np.abs(m) + (1 - b1) * np.abs(g))
    tv = 2.0 ** -21 * (b2 * v + (1 - b2) * g.astype(np.float64) ** 2)
    c1, c2 = 1 - b1 ** step, 1 - b2 ** step
    den = np.sqrt(wv / c2) + eps
    tp = 2.0 ** -22 * np.abs(wp) + lr * (tm / c1 / den + 2.0 ** -19 * np.abs(wm / c1) / den)
    assert np.all(np.abs(net.m.cpu().numpy() - wm) <= tm)
    assert np.all(np.abs(net.v.cpu().numpy() - wv) <= tv)
    assert np.all(np.abs(net.params.cpu().numpy() - wp) <= tp)
    # bfloat16 weight layouts: forward [tap][co][ci], transposed [tap][ci][co]
    p = net.params.cpu().numpy()
    Ws, _ = ocnn.unpack(p)
    wf = _bf16_bits_to_f(net.wf).reshape(4, 9, CH, CH)
    wb = _bf16_bits_to_f(net.wb).reshape(4, 9, CH, CH)
    for l in range(4):
        np.testing.assert_array_equal(wf[l], ocnn.bf16(Ws[l]))
        np.testing.assert_array_equal(wb[l], ocnn.bf16(Ws[l]).transpose(0, 2, 1))


def test_window_map_exact(lw):
    import torch
    rng = np.random.default_rng(4)
    Hc, Wc, D, w = 17, 29, 192, 16
    H, W = 4 * Hc + 3, 4 * Wc + 1  # ragged: last coarse row/column is reused
    cd = rng.uniform(0, 48, (Hc, Wc)).astype(np.float32)
    cd[0, :4] = [0.0, 47.9, 1.9, 2.125]  # clamps at both ends, a .5 tie
    out = rng.normal(0, 1.5, (1, Hc, Wc, CH)).astype(np.float32)
    out[0, 1, :3, 1] = 0.0  # logit exactly at the tau = 1/2 threshold: not confident
    cd[2, 5] = 5.0  # coarse match exactly at x = 20 - 4 * 5 = 0 for the pixel (8, 20): on the margin-0 edge
    for margin in (lw.ALWAYS_FALL_BACK, 0, 37):
        for tau in (0.0, 0.5, 0.8, 1.0):
            msg = f"tau {tau} margin {margin}"
            nfb = torch.zeros(1, dtype=torch.int32, device="cuda")
            stats = torch.full((3, H), 7, dtype=torch.int32, device="cuda")  # cleared by the call
            mask = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            lo = lw.window_map(_dev(cd), _dev(np.ascontiguousarray(out[..., :2])), W, H, D, w, tau, mask=mask,
                               row_stats=stats, nfallback=nfb, fallback_margin=margin)
            torch.cuda.synchronize()
            want, want_n, want_mask = ocnn.window_map(cd, out, W, H, D, w, tau,
                                                      None if margin == lw.ALWAYS_FALL_BACK else margin)
            np.testing.assert_array_equal(lo.cpu().numpy(), want, err_msg=msg)
            np.testing.assert_array_equal(mask.cpu().numpy(), want_mask, err_msg=msg)
            st = stats.cpu().numpy()
            cols = np.arange(W)
            np.testing.assert_array_equal(st[0], want_mask.sum(axis=1), err_msg=msg)
            np.testing.assert_array_equal(st[1], np.where(want_mask > 0, cols, W).min(axis=1), err_msg=msg)
            np.testing.assert_array_equal(st[2], np.where(want_mask > 0, cols, -1).max(axis=1), err_msg=msg)
            assert int(nfb.item()) == want_n
            if tau == 1.0 and margin == lw.ALWAYS_FALL_BACK:
                assert want_n == H * W  # every pixel falls back
            if tau == 1.0 and margin == 0:
                assert want_mask[8, 20] == 1 and 0 < want_n < H * W


def test_fallback_merge(lw):
    import torch
    rng = np.random.default_rng(12)
    H, W = 37, 300
    wi = rng.integers(0, 50, (H, W)).astype(np.int16)
    ws = rng.uniform(0, 50, (H, W)).astype(np.float32)
    mask = (rng.random((H, W)) < 0.4).astype(np.uint8)
    rects = [(0, 9, 0, 300), (20, 37, 41, 250), (9, 20, 299, 300)]
    res = [(rng.integers(100, 190, (b - a, x1 - x0)).astype(np.int16),
            rng.uniform(100, 190, (b - a, x1 - x0)).astype(np.float32)) for a, b, x0, x1 in rects]
    di, ds = _dev(wi), _dev(ws)
    md = _dev(mask)
    keep = []
    for (a, b, x0, x1), (bi, bs) in zip(rects, res):
        bid, bsd = _dev(bi), _dev(bs)
        keep += [bid, bsd]
        lw.fallback_merge(md, bid, bsd, a, x0, di, ds)
    torch.cuda.synchronize()
    want_i, want_s = ocnn.merge_fallback(wi, ws, mask, rects, res)
    np.testing.assert_array_equal(di.cpu().numpy(), want_i)
    np.testing.assert_array_equal(ds.cpu().numpy(), want_s)


def test_fallback_merge_rects_one_launch(lw):
    """Every rectangle of a two-frame batch merged by one launch equals the
    rectangle-by-rectangle merge of the oracle (rectangles of one frame do
    not overlap; a table row outside the frames is skipped)."""
    import torch
    rng = np.random.default_rng(13)
    n, H, W = 2, 37, 300
    wi = rng.integers(0, 50, (n, H, W)).astype(np.int16)
    ws = rng.uniform(0, 50, (n, H, W)).astype(np.float32)
    mask = (rng.random((n, H, W)) < 0.4).astype(np.uint8)
    rects = [(0, (0, 9, 0, 300)), (0, (20, 37, 41, 250)), (1, (9, 20, 299, 300)), (1, (0, 5, 7, 19))]
    res = [(rng.integers(100, 190, (b - a, x1 - x0)).astype(np.int16),
            rng.uniform(100, 190, (b - a, x1 - x0)).astype(np.float32)) for _, (a, b, x0, x1) in rects]
    table, off = [], 0
    for (f, (a, b, x0, x1)), (bi, _) in zip(rects, res):
        table.append((f, a, b - a, x0, x1 - x0, off))
        off += bi.size
    table.append((5, 0, 4, 0, 4, 0))  # frame outside the batch: skipped
    band_i = np.concatenate([bi.ravel() for bi, _ in res])
    band_s = np.concatenate([bs.ravel() for _, bs in res])
    di, ds = _dev(wi), _dev(ws)
    tab = _dev(np.array(table, np.int32))
    bid, bsd, md = _dev(band_i), _dev(band_s), _dev(mask)
    lw.fallback_merge_rects(md, tab, len(table), 17, 300, bid, bsd, di, ds)
    torch.cuda.synchronize()
    for f in range(n):
        sel = [k for k, (g, _) in enumerate(rects) if g == f]
        want_i, want_s = ocnn.merge_fallback(wi[f], ws[f], mask[f], [rects[k][1] for k in sel], [res[k] for k in sel])
        np.testing.assert_array_equal(di[f].cpu().numpy(), want_i)
        np.testing.assert_array_equal(ds[f].cpu().numpy(), want_s)


def test_training_resume_is_bitwise(lw, tmp_path):
    """N steps straight == N/2 steps, checkpoint, reload, N/2 steps; and
    the loss goes down on a fixed batch."""
    import torch
    n, H, W = 2, 12, 40
    rng = np.random.default_rng(8)
    coarse = rng.uniform(2, 40, (n, H, W)).astype(np.float32)
    label = (coarse + np.clip(rng.normal(0, 0.8, (n, H, W)), -3, 3)).astype(np.float32)
    left = rng.integers(0, 256, (n, H, W), dtype=np.uint8)
    x0 = torch.empty((n, H, W, CH), dtype=torch.int16, device="cuda")
    for i in range(n):
        lw.prepare_input(_dev(coarse[i]), _dev(left[i]), W, H, 1, x0[i])
    cdev, ldev = _dev(coarse), _dev(label)

    def run(net, steps):
        bufs = net.train_buffers(W, H, n)
        losses = []
        for _ in range(steps):
            loss = net.train_step(x0, cdev, ldev, W, H, n, 3e-3, bufs)
            losses.append(float(loss.sum()))
        return losses

    a = lw.WindowNet(seed=1)
    la = run(a, 20)
    b = lw.WindowNet(seed=1)
    run(b, 10)
    ck = str(tmp_path / "ck.npz")
    b.save(ck)
    c = lw.WindowNet.load(ck)
    assert c.step == 10
    run(c, 10)
    torch.cuda.synchronize()
    for name in ("params", "m", "v", "wf", "wb"):
        np.testing.assert_array_equal(getattr(a, name).cpu().numpy(), getattr(c, name).cpu().numpy(), err_msg=name)
    assert la[-1] < la[0]


def _road_pairs(name, seeds):
    ps = [synth.make_pair(synth.scene_for_config(name, sd), sd) for sd in seeds]
    return ps, np.stack([p.left for p in ps]), np.stack([p.right for p in ps])


@pytest.mark.parametrize("fallback", ["most", "few"])
def test_learned_window_pipeline_stepwise(lw, fallback):
    """Every stage of the learned-window matcher, for a batch of two pairs,
    checked against the oracle on the inputs that stage consumed; the
    fallback bands are the oracle's own, from its own mask.  'few' sets tau
    just above the lowest logits, so that only a few rows fall back."""
    import torch
    ps, L, R = _road_pairs("road320", [2, 3])
    n, H, W = L.shape
    D, w = 64, 16
    net = lw.WindowNet(_params(11))
    m = lw.LearnedWindowMatcher(W, H, batch=n, ndisp=D, window=w, census=7, npaths=8, p1=10, p2=120, net=net,
                                tau=0.5, margin=8, full_fraction=0.75)
    Ld, Rd = _dev(L), _dev(R)
    dint, dsub = m.match(Ld, Rd)
    torch.cuda.synchronize()
    if fallback == "few":
        logits = np.sort(m.out[..., 1].cpu().numpy().ravel())
        m.tau = float(1.0 / (1.0 + np.exp(-0.5 * (logits[3] + logits[4]))))
        dint, dsub = m.match(Ld, Rd)
        torch.cuda.synchronize()
        assert 0 < int(m.nfallback.sum()) <= 4 * 16
        assert any(rc and rc != [(0, H, 0, W)] for rc in m.last_rects)
    tau = m.tau
    nfb_total = 0
    for i in range(n):
        Lc, Rc = oracle.downsample4(L[i]), oracle.downsample4(R[i])
        np.testing.assert_array_equal(m.cl[i].cpu().numpy(), Lc)
        ci, cs = oracle.sgm(Lc, Rc, 7, D // 4, 8, 10, 120)
        np.testing.assert_array_equal(m.coarse.disp_int[i].cpu().numpy().astype(np.uint16), ci)
        gcs = m.coarse.disp_sub[i].cpu().numpy()
        assert np.abs(gcs - cs).max() <= 1e-4
        x0 = ocnn.prepare_input(gcs, Lc)
        np.testing.assert_array_equal(_bf16_bits_to_f(m.x0[i]), ocnn.bf16(x0)[0])
        _, want_out = ocnn.forward(net.params.cpu().numpy(), x0)
        want_out = want_out[..., :2]
        gout = m.out[i:i + 1].cpu().numpy()
        assert np.abs(gout - want_out).max() <= 0.02 * np.abs(want_out).max() + 1e-6
        want_lo, want_n, want_mask = ocnn.window_map(gcs, gout, W, H, D, w, tau, m.fallback_margin)
        np.testing.assert_array_equal(m.lo[i].cpu().numpy(), want_lo)
        np.testing.assert_array_equal(m.mask[i].cpu().numpy(), want_mask)
        nfb_total += want_n
        wi, ws = oracle.sgm_win(L[i], R[i], 7, w, 8, 10, 120, want_lo)
        rects = ocnn.fallback_rects(want_mask, 8, 0.75, D, 3)
        assert m.last_rects[i] == rects
        res = [oracle.sgm(L[i][a:b, x0:x1], R[i][a:b, x0:x1], 7, D, 8, 10, 120) for a, b, x0, x1 in rects]
        fi, fs = ocnn.merge_fallback(wi, ws, want_mask, rects, res)
        np.testing.assert_array_equal(dint[i].cpu().numpy().astype(np.uint16), fi)
        assert np.abs(dsub[i].cpu().numpy() - fs).max() <= 1e-4
    assert int(m.nfallback.sum()) == nfb_total


def test_full_fallback_is_plain_sgm(lw):
    """tau = 1 with every low-confidence pixel sent to the fallback: the
    learned-window form returns plain full-range SGM of each frame, exactly."""
    import torch
    from paper_2012_10802_amd import sgm as S
    ps, L, R = _road_pairs("road320", [5, 6])
    n, H, W = L.shape
    D = 64
    m = lw.LearnedWindowMatcher(W, H, batch=n, ndisp=D, window=16, net=lw.WindowNet(_params(2)), tau=1.0,
                                fallback_margin=lw.ALWAYS_FALL_BACK)
    Ld, Rd = _dev(L), _dev(R)
    dint, dsub = m.match(Ld, Rd)
    plain = S.Matcher(W, H, census=7, ndisp=D, npaths=8, p1=10, p2=120)
    for i in range(n):
        pi, pf = plain.match(Ld[i], Rd[i])
        torch.cuda.synchronize()
        assert m.last_rects[i] == [(0, H, 0, W)]
        np.testing.assert_array_equal(dint[i].cpu().numpy(), pi.cpu().numpy())
        np.testing.assert_array_equal(dsub[i].cpu().numpy(), pf.cpu().numpy())
        wi, _ = oracle.sgm(L[i], R[i], 7, D, 8, 10, 120)
        np.testing.assert_array_equal(dint[i].cpu().numpy().astype(np.uint16), wi)


def test_learned_window_full_size_batch16(lw):
    """The configuration the benchmark times: a batch of 16 1920x1080 road
    pairs (disparities 0..191, census 7x7, 8 paths) through the trained
    network.  Two pairs are checked stage by stage against the oracle; every
    pair's result equals the single-pair windowed path on the same windows,
    with the fallback rectangles' plain full-range SGM merged in."""
    import torch
    from paper_2012_10802_amd import sgm as S
    n, H, W, D, w = 16, 1080, 1920, 192, 16
    Ls, Rs = [], []
    for i in range(n):
        sd = 777 + i
        l, r, _, _ = synth.make_pair_torch(synth.scene_for_config("road1920", sd), sd, device="cuda")
        Ls.append(l)
        Rs.append(r)
    Ld, Rd = torch.stack(Ls).contiguous(), torch.stack(Rs).contiguous()
    m = lw.LearnedWindowMatcher(W, H, batch=n, ndisp=D, window=w)
    dint, dsub = m.match(Ld, Rd)
    torch.cuda.synchronize()
    single = S.Matcher(W, H, census=7, ndisp=w, npaths=8, p1=10, p2=120)
    for i in range(n):
        si, ss = single.match_win(Ld[i], Rd[i], m.lo[i])
        want_i, want_s = si.clone(), ss.clone()
        for (y0, y1, x0, x1) in m.last_rects[i]:
            full = S.Matcher(x1 - x0, y1 - y0, census=7, ndisp=D, npaths=8, p1=10, p2=120)
            fi, fs = full.match_at(Ld[i], Rd[i], y0, x0)
            msk = m.mask[i][y0:y1, x0:x1].bool()
            want_i[y0:y1, x0:x1][msk] = fi[msk]
            want_s[y0:y1, x0:x1][msk] = fs[msk]
        torch.cuda.synchronize()
        assert torch.equal(dint[i], want_i), i
        assert torch.equal(dsub[i], want_s), i
    params = m.net.params.cpu().numpy()
    for i in (0, 9):
        L, R = Ld[i].cpu().numpy(), Rd[i].cpu().numpy()
        Lc, Rc = oracle.downsample4(L), oracle.downsample4(R)
        ci, cs = oracle.sgm(Lc, Rc, 7, D // 4, 8, 10, 120)
        np.testing.assert_array_equal(m.coarse.disp_int[i].cpu().numpy().astype(np.uint16), ci)
        gcs = m.coarse.disp_sub[i].cpu().numpy()
        assert np.abs(gcs - cs).max() <= 1e-4
        x0 = ocnn.prepare_input(gcs, Lc)
        _, want_out = ocnn.forward(params, x0)
        want_out = want_out[..., :2]
        gout = m.out[i:i + 1].cpu().numpy()
        assert np.abs(gout - want_out).max() <= 0.02 * np.abs(want_out).max()
        want_lo, _, want_mask = ocnn.window_map(gcs, gout, W, H, D, w, m.tau, m.fallback_margin)
        np.testing.assert_array_equal(m.lo[i].cpu().numpy(), want_lo)
        rects = ocnn.fallback_rects(want_mask, m.margin, m.full_fraction, D, 3)
        assert m.last_rects[i] == rects
        wi, ws = oracle.sgm_win(L, R, 7, w, 8, 10, 120, want_lo)
        res = [oracle.sgm(L[a:b, x0:x1], R[a:b, x0:x1], 7, D, 8, 10, 120) for a, b, x0, x1 in rects]
        fi, fs = ocnn.merge_fallback(wi, ws, want_mask, rects, res)
        np.testing.assert_array_equal(dint[i].cpu().numpy().astype(np.uint16), fi)
        assert np.abs(dsub[i].cpu().numpy() - fs).max() <= 1e-4
