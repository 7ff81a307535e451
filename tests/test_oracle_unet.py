"""Pins of the network oracle: its backward pass equals central finite
differences of its forward pass (fp64), and its pieces satisfy their
definitions (adjoint identities, bf16 rounding)."""
import numpy as np
import pytest

from oracle import unet_ref as U


def test_bf16_round_nearest_even():
    # 1 + 2^-8 is halfway between bf16 1.0 and 1 + 2^-7: ties to even (1.0)
    assert U.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert U.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert U.bf16_round(-2.5) == -2.5
    x = np.random.default_rng(0).normal(size=1000)
    r = U.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_pool_up_adjoints():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(2, 8, 6, 3))
    b = rng.normal(size=(2, 4, 3, 3))
    # <pool(a), b> = <a, pool_grad(b)>;  <up(b), a> = <b, up_grad(a)>
    assert abs(np.sum(U.pool2(a) * b) - np.sum(a * U.pool2_grad(b))) < 1e-12
    assert abs(np.sum(U.up2(b) * a) - np.sum(b * U.up2_grad(a))) < 1e-12


def test_conv_grads_adjoint():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 5, 7, 4))
    w = rng.normal(size=(3, 9, 4))
    dy = rng.normal(size=(2, 5, 7, 3))
    dx, dw, db = U.conv3x3_grads(x, w, dy)
    # <conv(x), dy> is linear in x and in w
    lin = np.sum((U.conv3x3(x, w, np.zeros(3))) * dy)
    assert abs(np.sum(dx * x) - lin) < 1e-9
    assert abs(np.sum(dw * w) - lin) < 1e-9
    assert np.allclose(db, dy.sum(axis=(0, 1, 2)))


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    p = U.init_params(5)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(0, 0.05, size=p[k].shape)
    x = np.zeros((1, 16, 16, 16))
    x[..., :2] = rng.uniform(0.2, 1.0, size=(1, 16, 16, 2))
    t = rng.uniform(0.0, 1.0, size=(1, 32, 32))
    out, cache = U.forward(p, x)
    g = U.backward(p, cache, out, t)
    names = [n for n, *_ in U.LAYERS]
    checked = 0
    for n in names:
        for kind in ("w", "b"):
            key = f"{n}.{kind}"
            arr = p[key]
            for _ in range(2):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                h = 1e-6 * max(1.0, abs(old))
                arr[idx] = old + h
                lp = U.mse(U.forward(p, x)[0], t)
                arr[idx] = old - h
                lm = U.mse(U.forward(p, x)[0], t)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                an = g[key][idx]
                scale = max(abs(fd), abs(an), 1e-8)
                assert abs(fd - an) <= 1e-5 * scale + 1e-11, (key, idx, fd, an)
                checked += 1
    assert checked == 64
