"""Network kernels (bf16 MFMA) against the fp64 network oracle.

Tolerances: fp32 outputs of a convolution accumulate <= 9*384 bf16 products
in fp32 (relative error ~1e-6 of the output scale), so |gpu - ref| <=
1e-4 * max|ref|; bf16 outputs add one rounding: <= 2^-8 relative plus 1e-4 of
the scale.  Whole-network comparisons round activations to bf16 on both
sides, but a value near a rounding boundary can round differently after the
fp32-vs-fp64 accumulation, so they are compared in relative L2 norm (forward
<= 1e-2; gradients, also stored in bf16, <= 5e-2 per layer).
"""
import numpy as np
import pytest

from oracle import unet_ref as U
from paper_2201_13191_amd import mcx, unet
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on the MI355X box")
    return torch, mcx.mc_create(0)


def to_bf16_bits(a):
    f = np.asarray(U.bf16_round(a), np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def from_bf16_bits(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


# The kernel splits each tile's reduction over 1, 2 or 4 waves by the layer's
# tile count: (2, 256, ...) takes the one-wave path, (1, 256, ...) and
# (2, 16, 32, ...) the two-wave one, the others the four-wave one (or two
# waves when the reduction is short).  Images whose width is a multiple of 64,
# or 16 or 32 wide, stage their input rows in LDS per 16-channel chunk (wide
# windows of 66 pixels, or 2 and 4 whole rows); the 8-, 9-, 12- and 5-pixel
# images read their operands directly.
@pytest.mark.parametrize("n,s,cin,cout,ldx,xoff,relu", [
    (1, 8, 16, 32, 16, 0, 1), (2, 16, 32, 64, 48, 16, 1), (1, 12, 48, 128, 48, 0, 0),
    (3, 9, 16, 16, 32, 16, 1), (1, 32, 384, 128, 384, 0, 1), (2, 5, 64, 1, 64, 0, 0),
    (2, 256, 16, 32, 32, 16, 1), (1, 256, 32, 32, 32, 0, 1),
    (2, 256, 32, 64, 32, 0, 1), (2, 256, 48, 32, 64, 16, 0),
    (1, 64, 64, 64, 64, 0, 1), (2, 16, 128, 64, 128, 0, 1)])
def test_conv_forward(env, n, s, cin, cout, ldx, xoff, relu):
    torch, ctx = env
    say("conv", n, s, cin, cout, ldx, xoff, relu)
    rng = np.random.default_rng(cin + cout)
    x = U.bf16_round(rng.normal(size=(n, s, s, ldx)))
    w = U.bf16_round(rng.normal(0, 0.2, size=(cout, 9, cin)))
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    ca = unet.cout_alloc(cout)
    wpad = np.zeros((ca, 9, cin))
    wpad[:cout] = w
    dx = torch.from_numpy(to_bf16_bits(x)).cuda()
    dw = torch.from_numpy(to_bf16_bits(wpad)).cuda()
    db = torch.from_numpy(b.astype(np.float32)).cuda()
    yb = torch.zeros((n, s, s, cout + 16), dtype=torch.int16, device="cuda")
    yf = torch.zeros((n * s * s, cout), dtype=torch.float32, device="cuda")
    mcx.mc_nn_conv3x3_async(ctx, dx, ldx, xoff, dw, db, yb, cout + 16, 16, n, s, s, cin, cout,
                            relu=relu, yf=yf)
    torch.cuda.synchronize()
    ref = U.conv3x3(x[..., xoff:xoff + cin], w, b)
    if relu:
        ref = np.maximum(ref, 0)
    got = yf.cpu().numpy().astype(np.float64).reshape(ref.shape)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-4 * scale
    gb = from_bf16_bits(yb)[..., 16:16 + cout]
    assert np.all(np.abs(gb - ref) <= np.abs(ref) * 2.0 ** -8 + 1e-4 * scale)
    assert np.all(from_bf16_bits(yb)[..., :16] == 0)     # outside the slice untouched


# The epilogue finishes 16-channel groups with 16-byte accesses when the
# channel count is a multiple of 16 and the output, mask and fp32 rows are
# 16-byte aligned, else element by element: aligned and unaligned output
# slices, half slabs (48 and 16 channels), 40 channels, and the one-, two-
# and four-wave reductions (2 x 256^2, 2 x 10^2 and 12^2 pixels), with the
# mask and accumulation options the network itself does not use.
@pytest.mark.parametrize("n,s,cin,cout,ypad,relu", [
    (1, 12, 32, 64, 16, 1), (1, 12, 32, 64, 3, 1), (2, 10, 16, 48, 8, 0), (1, 12, 16, 40, 8, 1),
    (2, 64, 32, 16, 16, 1),
    (2, 256, 16, 32, 16, 1), (2, 256, 16, 32, 5, 0)])
def test_conv_mask_and_accumulate(env, n, s, cin, cout, ypad, relu):
    torch, ctx = env
    say("conv mask/accumulate", n, s, cin, cout, ypad, relu)
    rng = np.random.default_rng(3 * cin + cout + ypad)
    x = U.bf16_round(rng.normal(size=(n, s, s, cin)))
    w = U.bf16_round(rng.normal(0, 0.2, size=(cout, 9, cin)))
    b = rng.normal(size=cout).astype(np.float32).astype(np.float64)
    ca = unet.cout_alloc(cout)
    wpad = np.zeros((ca, 9, cin))
    wpad[:cout] = w
    ldy, ldm = cout + ypad, cout + 8
    y0 = U.bf16_round(rng.normal(size=(n, s, s, ldy)))
    m = U.bf16_round(rng.normal(size=(n, s, s, ldm)))
    m[..., 8:][rng.random(size=(n, s, s, cout)) < 0.2] = 0.0     # exact zeros are masked too
    dx = torch.from_numpy(to_bf16_bits(x)).cuda()
    dw = torch.from_numpy(to_bf16_bits(wpad)).cuda()
    db = torch.from_numpy(b.astype(np.float32)).cuda()
    yb = torch.from_numpy(to_bf16_bits(y0)).cuda()
    dm = torch.from_numpy(to_bf16_bits(m)).cuda()
    yf = torch.zeros((n * s * s, cout), dtype=torch.float32, device="cuda")
    mcx.mc_nn_conv3x3_async(ctx, dx, cin, 0, dw, db, yb, ldy, ypad, n, s, s, cin, cout,
                            relu=relu, yf=yf, mask=dm, ldm=ldm, moff=8, accumulate=1)
    torch.cuda.synchronize()
    ref = U.conv3x3(x, w, b)
    if relu:
        ref = np.maximum(ref, 0)
    ref = np.where(m[..., 8:8 + cout] > 0, ref, 0.0)
    scale = np.abs(ref).max()
    got = yf.cpu().numpy().astype(np.float64).reshape(ref.shape)
    assert np.abs(got - ref).max() <= 1e-4 * scale
    want = ref + y0[..., ypad:ypad + cout]
    gb = from_bf16_bits(yb)
    assert np.all(np.abs(gb[..., ypad:ypad + cout] - want) <= np.abs(want) * 2.0 ** -8 + 1e-4 * scale)
    assert np.array_equal(gb[..., :ypad], y0[..., :ypad])     # outside the slice untouched


# Widths that are multiples of 16 take the nine-tap kernel (16-pixel row
# slices), the others the per-tap one; split ranges that are not whole slices,
# a 16-channel output and a partial input tile are included.
@pytest.mark.parametrize("n,s,cin,cout,splits", [(1, 8, 16, 32, 1), (2, 16, 32, 64, 3),
                                                 (1, 16, 96, 32, 4), (4, 8, 128, 256, 2),
                                                 (2, 32, 48, 16, 5), (1, 64, 16, 64, 7),
                                                 (3, 48, 64, 96, 1), (2, 32, 16, 32, 70)])
def test_conv_weight_and_input_gradients(env, n, s, cin, cout, splits):
    torch, ctx = env
    say("wgrad", n, s, cin, cout, splits)
    rng = np.random.default_rng(7 + cin)
    x = U.bf16_round(rng.normal(size=(n, s, s, cin)))
    gy = U.bf16_round(rng.normal(size=(n, s, s, cout)))
    w = U.bf16_round(rng.normal(0, 0.2, size=(cout, 9, cin)))
    rdx, rdw, rdb = U.conv3x3_grads(x, w, gy)
    dx = torch.from_numpy(to_bf16_bits(x)).cuda()
    dgy = torch.from_numpy(to_bf16_bits(gy)).cuda()
    ws = torch.zeros((splits + 1) * 9 * cout * cin, dtype=torch.float32, device="cuda")
    dw = torch.zeros((cout, 9, cin), dtype=torch.float32, device="cuda")
    mcx.mc_nn_conv3x3_wgrad_async(ctx, dx, cin, 0, dgy, cout, 0, n, s, s, cin, cout, splits, ws, dw)
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    bws = torch.zeros(16 * cout, dtype=torch.float32, device="cuda")
    mcx.mc_nn_bias_grad_async(ctx, dgy, cout, 0, n * s * s, cout, bws, 16, db)
    # input gradient through the flipped weights
    wb = np.zeros((unet.cout_alloc(cout), 9, cin))
    wb[:cout] = w
    dwb = torch.from_numpy(to_bf16_bits(wb)).cuda()
    wt = torch.zeros((unet.cout_alloc(cin), 9, cout), dtype=torch.int16, device="cuda")
    mcx.mc_nn_flip_weights_async(ctx, dwb, wt, cout, cin, cout, unet.cout_alloc(cin))
    gx = torch.zeros((n * s * s, cin), dtype=torch.float32, device="cuda")
    mcx.mc_nn_conv3x3_async(ctx, dgy, cout, 0, wt, None, None, 0, 0, n, s, s, cout, cin, yf=gx)
    torch.cuda.synchronize()
    assert np.abs(dw.cpu().numpy() - rdw).max() <= 1e-4 * np.abs(rdw).max()
    assert np.abs(db.cpu().numpy() - rdb).max() <= 1e-4 * np.abs(rdb).max()
    g = gx.cpu().numpy().reshape(rdx.shape)
    assert np.abs(g - rdx).max() <= 1e-4 * np.abs(rdx).max()


def test_pool_upsample_and_mask(env):
    torch, ctx = env
    say("pool/up/mask")
    rng = np.random.default_rng(11)
    x = U.bf16_round(rng.normal(size=(2, 8, 8, 48)))
    dx = torch.from_numpy(to_bf16_bits(x)).cuda()
    pooled = torch.zeros((2, 4, 4, 16), dtype=torch.int16, device="cuda")
    mcx.mc_nn_pool2_async(ctx, dx, 48, 16, pooled, 16, 0, 2, 8, 8, 16)
    up = torch.zeros((2, 16, 16, 32), dtype=torch.int16, device="cuda")
    mcx.mc_nn_upsample2_async(ctx, dx, 48, 32, up, 32, 16, 2, 8, 8, 16)
    back = torch.zeros((2, 8, 8, 16), dtype=torch.int16, device="cuda")
    mcx.mc_nn_upsample2_async(ctx, up, 32, 16, back, 16, 0, 2, 8, 8, 16, backward=1)
    torch.cuda.synchronize()
    ref = U.bf16_round(U.pool2(x[..., 16:32]))
    assert np.array_equal(from_bf16_bits(pooled), ref)
    assert np.array_equal(from_bf16_bits(up)[..., 16:], U.up2(x[..., 32:48]))
    assert np.array_equal(from_bf16_bits(back), U.bf16_round(4 * x[..., 32:48]))
    g = torch.from_numpy(to_bf16_bits(np.ones((2, 8, 8, 48)))).cuda()
    mcx.mc_nn_relu_mask_async(ctx, g, 48, 0, dx, 48, 0, 2 * 64, 48)
    torch.cuda.synchronize()
    assert np.array_equal(from_bf16_bits(g), (x > 0).astype(np.float64))


# Pooling and up-sampling run 8 channels per thread when the channel count,
# the slices and the sizes allow it, else element by element: both paths,
# forward and backward, with accumulation into the output.
@pytest.mark.parametrize("c,ldx,xoff,ldy,yoff,h,w", [
    (16, 32, 16, 24, 8, 8, 8),        # 16-byte path
    (12, 20, 4, 16, 2, 6, 10),        # element by element (12 channels, odd offsets)
    (32, 32, 0, 40, 8, 6, 14)])       # 16-byte path, non-square
def test_resample_paths(env, c, ldx, xoff, ldy, yoff, h, w):
    torch, ctx = env
    say("pool/up paths", c, ldx, xoff, ldy, yoff, h, w)
    rng = np.random.default_rng(c + h + w)
    n = 2
    cases = [  # (op, backward, input (n, hi, wi), output (n, ho, wo), reference)
        ("pool", 0, (h, w), (h // 2, w // 2), U.pool2),
        ("pool", 1, (h // 2, w // 2), (h, w), U.pool2_grad),
        ("up", 0, (h, w), (2 * h, 2 * w), U.up2),
        ("up", 1, (2 * h, 2 * w), (h, w), U.up2_grad)]
    for op, bw, (hi, wi), (ho, wo), ref_f in cases:
        x = U.bf16_round(rng.normal(size=(n, hi, wi, ldx)))
        y0 = U.bf16_round(rng.normal(size=(n, ho, wo, ldy)))
        dx = torch.from_numpy(to_bf16_bits(x)).cuda()
        dy = torch.from_numpy(to_bf16_bits(y0)).cuda()
        fn = mcx.mc_nn_pool2_async if op == "pool" else mcx.mc_nn_upsample2_async
        # sizes passed are the full-size image for pooling, the coarse one for up-sampling
        hh, ww = (h, w)
        fn(ctx, dx, ldx, xoff, dy, ldy, yoff, n, hh, ww, c, backward=bw, accumulate=1)
        torch.cuda.synchronize()
        want = ref_f(x[..., xoff:xoff + c]) + y0[..., yoff:yoff + c]
        got = from_bf16_bits(dy)
        assert np.all(np.abs(got[..., yoff:yoff + c] - want) <= np.abs(want) * 2.0 ** -8 + 1e-6), \
            (op, bw)
        assert np.array_equal(got[..., :yoff], y0[..., :yoff]), (op, bw)
        assert np.array_equal(got[..., yoff + c:], y0[..., yoff + c:]), (op, bw)


@pytest.mark.parametrize("c,ldg,goff,ldy,yoff", [(48, 48, 0, 64, 16), (12, 20, 4, 16, 2)])
def test_relu_mask_paths(env, c, ldg, goff, ldy, yoff):
    """ReLU derivative on a gradient slice: 8 channels per thread when aligned, else
    element by element; zeros (and negatives) of the activation mask."""
    torch, ctx = env
    say("relu mask paths", c, ldg, goff, ldy, yoff)
    rng = np.random.default_rng(c + ldy)
    npix = 3 * 50
    y = U.bf16_round(rng.normal(size=(npix, ldy)))
    y[rng.random(size=y.shape) < 0.1] = 0.0
    g0 = U.bf16_round(rng.normal(size=(npix, ldg)))
    dg = torch.from_numpy(to_bf16_bits(g0)).cuda()
    dy = torch.from_numpy(to_bf16_bits(y)).cuda()
    mcx.mc_nn_relu_mask_async(ctx, dg, ldg, goff, dy, ldy, yoff, npix, c)
    torch.cuda.synchronize()
    got = from_bf16_bits(dg)
    want = g0.copy()
    want[:, goff:goff + c] = np.where(y[:, yoff:yoff + c] > 0, g0[:, goff:goff + c], 0.0)
    assert np.array_equal(got, want)


def small_net(torch, ctx, n=2, s=32, seed=3):
    p = U.init_params(seed)
    rng = np.random.default_rng(seed)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(0, 0.05, size=p[k].shape)
    # the GPU keeps fp32 master weights and computes with their bf16 copies
    pb = {k: (U.bf16_round(v) if k.endswith(".w") else v.astype(np.float32).astype(np.float64))
          for k, v in p.items()}
    net = unet.UNet(ctx, n, s, params=pb)
    sc = rng.uniform(0.1, 1.0, size=(n, s, s))
    pr = rng.uniform(0.1, 1.0, size=(n, s, s))
    tg = rng.uniform(0.0, 1.0, size=(n, 2 * s, 2 * s))
    x = np.zeros((n, s, s, 16))
    x[..., 0] = U.bf16_round(sc)
    x[..., 1] = U.bf16_round(pr)
    return net, pb, sc, pr, tg, x


def test_network_forward_and_gradients(env):
    torch, ctx = env
    say("network fwd/bwd")
    net, pb, sc, pr, tg, x = small_net(torch, ctx)
    t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    net.set_input(t(sc), t(pr))
    out = net.forward().cpu().numpy().astype(np.float64)
    ref, cache = U.forward(pb, x, bf16=True)
    say("forward rel-L2", rel(out, ref))
    assert rel(out, ref) <= 1e-2
    net.target.copy_(t(tg).reshape(-1))
    net.loss_and_grad()
    net.backward()
    torch.cuda.synchronize()
    assert abs(net.loss_value() - U.mse(ref, tg)) <= 1e-2 * U.mse(ref, tg)
    g = U.backward(pb, cache, ref, tg)
    got = net.gradients()
    for name, *_ in U.LAYERS:
        ew, eb = rel(got[name][0], g[name + ".w"]), rel(got[name][1], g[name + ".b"])
        say("grad", name, f"{ew:.2e} {eb:.2e}")
        assert ew <= 5e-2 and eb <= 5e-2, name


def test_training_reduces_loss_and_resumes_bitwise(env, tmp_path):
    torch, ctx = env
    say("training")
    net, pb, sc, pr, tg, x = small_net(torch, ctx, n=4, s=16, seed=9)
    rng = np.random.default_rng(0)
    # learn a smooth up-sampling: target = 2x nearest of a blurred input
    t = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    base = rng.uniform(0.2, 1.0, size=(4, 16, 16))
    target = np.repeat(np.repeat(base, 2, axis=1), 2, axis=2)
    net.lr = 2e-3
    losses = []
    for it in range(60):
        net.train_step(t(base), t(base), t(target))
        losses.append(net.loss_value())
    say("loss", losses[0], losses[-1])
    assert losses[-1] < 0.2 * losses[0]
    path = str(tmp_path / "ck.npz")
    net.save(path)
    net.train_step(t(base), t(base), t(target))
    l1 = net.loss_value()
    w1 = net.L["d2a"]["w32"].clone()
    net.load(path)
    net.train_step(t(base), t(base), t(target))
    assert net.loss_value() == l1
    assert torch.equal(net.L["d2a"]["w32"], w1)
