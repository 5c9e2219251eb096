"""Pins of the U-Net oracle (oracle/unet_oracle.py) against things other
than itself: scipy's n-d correlation, a brute-force loop, exact adjoint
identities, central finite differences, torch's bfloat16 rounding, and for
the optimiser the closed forms of Adam's steps and torch.optim.Adam."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import unet_oracle as U


def _rng(s):
    return np.random.default_rng(14090105 + s)


def test_conv_matches_scipy_correlate():
    rng = _rng(1)
    x = rng.standard_normal((5, 6, 7, 3))
    w = rng.standard_normal((2, 27, 3))
    b = rng.standard_normal(2)
    out = U.conv3_fwd(x, w, b)
    for o in range(2):
        ref = np.full(x.shape[:3], b[o])
        for i in range(3):
            ref += ndi.correlate(x[..., i], w[o, :, i].reshape(3, 3, 3), mode="constant", cval=0.0)
        np.testing.assert_allclose(out[..., o], ref, rtol=1e-13, atol=1e-13)


def test_conv_matches_brute_force_loops():
    rng = _rng(2)
    D, H, W, Ci, Co = 3, 4, 5, 2, 3
    x = rng.standard_normal((D, H, W, Ci))
    w = rng.standard_normal((Co, 27, Ci))
    out = U.conv3_fwd(x, w)
    for z in range(D):
        for y in range(H):
            for xx in range(W):
                for o in range(Co):
                    s = 0.0
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, x2 = z + dz, y + dy, xx + dx
                                if 0 <= zz < D and 0 <= yy < H and 0 <= x2 < W:
                                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    s += sum(x[zz, yy, x2, i] * w[o, t, i] for i in range(Ci))
                    assert abs(out[z, y, xx, o] - s) <= 1e-12 * (1 + abs(s))


def test_conv_gradients_are_exact_adjoints():
    rng = _rng(3)
    x = rng.standard_normal((4, 5, 6, 3))
    w = rng.standard_normal((4, 27, 3))
    b = rng.standard_normal(4)
    g = rng.standard_normal((4, 5, 6, 4))
    lhs = np.sum(U.conv3_fwd(x, w) * g)
    # <conv(x), g> = <x, dgrad(g)> = <w, wgrad(x, g)>
    assert abs(lhs - np.sum(x * U.conv3_dgrad(g, w))) <= 1e-11 * abs(lhs)
    dw, db = U.conv3_wgrad(x, g)
    assert abs(lhs - np.sum(w * dw)) <= 1e-11 * abs(lhs)
    # the bias enters as <b, sum_v g>
    assert abs(np.sum((U.conv3_fwd(x, w, b) - U.conv3_fwd(x, w)) * g) - b @ db) <= 1e-11 * np.abs(b @ db)


def test_pool_and_upsample():
    rng = _rng(4)
    x = rng.standard_normal((4, 6, 8, 2))
    g = rng.standard_normal((2, 3, 4, 2))
    np.testing.assert_allclose(U.avgpool2(U.up2(g)), g, rtol=1e-15, atol=0)
    np.testing.assert_allclose(U.avgpool2(np.full((4, 4, 4, 1), 3.5)), 3.5)
    lhs = np.sum(U.avgpool2(x) * g)
    assert abs(lhs - np.sum(x * U.avgpool2_bwd(g))) <= 1e-12 * (1 + abs(lhs))
    h = rng.standard_normal(x.shape)
    lhs = np.sum(U.up2(g) * h)
    assert abs(lhs - np.sum(g * U.up2_bwd(h))) <= 1e-12 * (1 + abs(lhs))


def test_untrained_net_is_identity():
    rng = _rng(5)
    P = U.init_params(rng, c=4)
    x = rng.random((8, 8, 8, 1))
    np.testing.assert_array_equal(U.unet_forward(x, P, c=4), x)


@pytest.mark.parametrize("c", [2, 4])
def test_net_gradient_matches_finite_differences(c):
    rng = _rng(6 + c)
    P = U.init_params(rng, c=c)
    for k in P:
        P[k] = (P[k][0], 0.1 * rng.standard_normal(np.shape(P[k][1])))
    P["head"] = (rng.standard_normal((1, c)), rng.standard_normal(1))
    x = rng.random((8, 8, 4, 1))
    t = rng.random((8, 8, 4, 1))
    loss, G = U.unet_loss_and_grads(x, t, P, c=c)
    assert abs(loss - np.mean((U.unet_forward(x, P, c=c) - t) ** 2)) <= 1e-14 * loss
    v = U.flatten_params(P, c)
    gv = U.flatten_params(G, c)

    def f(vv):
        return U.unet_loss_and_grads(x, t, U.unflatten_params(vv, c), c=c)[0]

    for _ in range(3):
        d = rng.standard_normal(v.size)
        h = 1e-6
        fd = (f(v + h * d) - f(v - h * d)) / (2 * h)
        assert abs(fd - gv @ d) <= 1e-6 * abs(gv @ d)
    # one coordinate per layer as well (catches a gradient dropped for a layer)
    o = 0
    for name, ci, co in U.unet_layers(c):
        i = o + 13 * ci  # w[0, 13, 0]: centre tap
        e = np.zeros(v.size)
        e[i] = 1.0
        h = 1e-6
        fd = (f(v + h * e) - f(v - h * e)) / (2 * h)
        assert abs(fd - gv[i]) <= 1e-6 * abs(gv[i]) + 1e-9, name
        o += co * 27 * ci + co


def test_flat_parameter_order_round_trips():
    rng = _rng(9)
    P = U.init_params(rng, c=16)
    v = U.flatten_params(P)
    assert v.size == 27 * 14352 + sum(co for _, _, co in U.unet_layers(16)) + 17
    np.testing.assert_array_equal(U.flatten_params(U.unflatten_params(v)), v)


def test_bf16_round():
    import torch
    # ties go to the even neighbour
    assert U.bf16_round(np.float32(1 + 2.0 ** -8)) == 1.0
    assert U.bf16_round(np.float32(1 + 3 * 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)
    a = _rng(10).standard_normal(100_000).astype(np.float32) * 1e3
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(U.bf16_round(a), ref)


def test_adam_closed_forms():
    """Adam's first step moves every parameter by lr g / (|g| + eps) (the bias
    corrections undo the zero start exactly), and so does every later step
    under a constant gradient; a zero gradient leaves the parameter alone."""
    rng = _rng(30)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.integers(-6, 3, 50)
    g[3] = 0.0
    lr = 3e-3
    p, m, v = U.adam_step(p0, g, np.zeros(50), np.zeros(50), 1, lr)
    np.testing.assert_allclose(p, p0 - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert p[3] == p0[3]
    for t in range(2, 6):
        q, m, v = U.adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(q - p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-17)
        p = q


def test_adam_matches_torch_optim():
    """Five steps with changing gradients against torch.optim.Adam (float64)."""
    import torch
    rng = _rng(31)
    p0 = rng.standard_normal(200)
    grads = [rng.standard_normal(200) * (0.1 + k) for k in range(5)]
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(200), np.zeros(200)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = U.adam_step(p, g, m, v, t, 1e-2)
        np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-13, atol=1e-15)
