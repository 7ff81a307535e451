"""fp64 oracle of the learned scatter denoiser / up-sampler (TEST INFRASTRUCTURE ONLY).

The network (a reading: the paper smooths and up-samples with fixed filters,
section II-C-3/4; the learned replacement is a 4-level U-Net with 32 base
channels):

    input  [N,128,128,16]  channel 0 scatter, 1 primary, 2..15 zero
    e1a conv 16->32 relu, e1b conv 32->32 relu            -> s1 (128^2)
    pool2, e2a 32->64 relu, e2b 64->64 relu              -> s2 (64^2)
    pool2, e3a 64->128 relu, e3b 128->128 relu           -> s3 (32^2)
    pool2, b_a 128->256 relu, b_b 256->256 relu          (16^2)
    up2, concat [up, s3] (384), d3a 384->128 relu, d3b 128->128 relu
    up2, concat [up, s2] (192), d2a 192->64 relu,  d2b 64->64 relu
    up2, concat [up, s1] (96),  d1a 96->32 relu,   d1b 32->32 relu
    up2 (256^2), h_a 32->16 relu, h_b 16->1 (linear)    -> output [N,256,256]

conv = 3x3, stride 1, zero padding, bias; pool2 = 2x2 average; up2 = nearest.
Loss: mean squared error against the target map.

`bf16=True` rounds every stored activation (each layer's output, pooled and
up-sampled maps) to bfloat16 (round to nearest even), as the GPU path stores
them; the arithmetic itself is fp64.  The backward pass is the exact gradient
of the fp64 forward (with bf16 rounding treated as identity, as training does).
"""
import numpy as np

# (name, cin, cout, relu)
LAYERS = [
    ("e1a", 16, 32, True), ("e1b", 32, 32, True),
    ("e2a", 32, 64, True), ("e2b", 64, 64, True),
    ("e3a", 64, 128, True), ("e3b", 128, 128, True),
    ("b_a", 128, 256, True), ("b_b", 256, 256, True),
    ("d3a", 384, 128, True), ("d3b", 128, 128, True),
    ("d2a", 192, 64, True), ("d2b", 64, 64, True),
    ("d1a", 96, 32, True), ("d1b", 32, 32, True),
    ("h_a", 32, 16, True), ("h_b", 16, 1, False),
]


def bf16_round(x):
    """Round to bfloat16, nearest even, through float32."""
    f = np.asarray(x, np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def conv3x3(x, w, b):
    """x [N,H,W,Ci], w [Co,9,Ci] (tap = 3*(dy+1)+(dx+1)), b [Co] -> [N,H,W,Co]."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1] = x
    out = np.zeros((N, H, W, w.shape[0]))
    for tap in range(9):
        dy, dx = tap // 3 - 1, tap % 3 - 1
        sl = xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
        out += sl @ w[:, tap, :].T
    return out + b


def conv3x3_grads(x, w, dy):
    """Gradients of conv3x3 wrt x, w, b for output gradient dy."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for tap in range(9):
        ddy, ddx = tap // 3 - 1, tap % 3 - 1
        sl = xp[:, 1 + ddy:1 + ddy + H, 1 + ddx:1 + ddx + W]
        dw[:, tap, :] = np.einsum("nhwo,nhwi->oi", dy, sl)
        dxp[:, 1 + ddy:1 + ddy + H, 1 + ddx:1 + ddx + W] += dy @ w[:, tap, :]
    return dxp[:, 1:-1, 1:-1], dw, dy.sum(axis=(0, 1, 2))


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_grad(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) * 0.25


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_grad(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def init_params(seed):
    """He-normal weights, zero biases (fp64), seeded."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _ in LAYERS:
        p[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, 9, ci))
        p[name + ".b"] = np.zeros(co)
    return p


def forward(p, x, bf16=False):
    """x [N,128,128,16] -> (out [N,256,256], cache)."""
    q = bf16_round if bf16 else (lambda a: a)
    cache = {}

    def layer(name, inp, relu):
        pre = conv3x3(inp, p[name + ".w"], p[name + ".b"])
        out = np.maximum(pre, 0.0) if relu else pre
        out = q(out) if relu else out
        cache[name] = (inp, out)
        return out

    h = layer("e1a", x, True)
    s1 = layer("e1b", h, True)
    h = q(pool2(s1))
    h = layer("e2a", h, True)
    s2 = layer("e2b", h, True)
    h = q(pool2(s2))
    h = layer("e3a", h, True)
    s3 = layer("e3b", h, True)
    h = q(pool2(s3))
    h = layer("b_a", h, True)
    h = layer("b_b", h, True)
    h = np.concatenate([up2(h), s3], axis=3)
    h = layer("d3a", h, True)
    h = layer("d3b", h, True)
    h = np.concatenate([up2(h), s2], axis=3)
    h = layer("d2a", h, True)
    h = layer("d2b", h, True)
    h = np.concatenate([up2(h), s1], axis=3)
    h = layer("d1a", h, True)
    h = layer("d1b", h, True)
    h = up2(h)
    h = layer("h_a", h, True)
    out = layer("h_b", h, False)
    return out[..., 0], cache


def mse(out, target):
    return float(np.mean((out - target) ** 2))


def backward(p, cache, out, target):
    """Gradients of mse(out, target) wrt every parameter."""
    g = {}
    n = out.size
    d = (2.0 * (out - target) / n)[..., None]         # d loss / d h_b output

    def layer_back(name, dout, relu):
        inp, o = cache[name]
        if relu:
            dout = dout * (o > 0)
        dx, dw, db = conv3x3_grads(inp, p[name + ".w"], dout)
        g[name + ".w"] = dw
        g[name + ".b"] = db
        return dx

    d = layer_back("h_b", d, False)
    d = layer_back("h_a", d, True)
    d = up2_grad(d)
    d = layer_back("d1b", d, True)
    d = layer_back("d1a", d, True)
    d_up, d_s1 = d[..., :64], d[..., 64:]
    d = up2_grad(d_up)
    d = layer_back("d2b", d, True)
    d = layer_back("d2a", d, True)
    d_up, d_s2 = d[..., :128], d[..., 128:]
    d = up2_grad(d_up)
    d = layer_back("d3b", d, True)
    d = layer_back("d3a", d, True)
    d_up, d_s3 = d[..., :256], d[..., 256:]
    d = up2_grad(d_up)
    d = layer_back("b_b", d, True)
    d = layer_back("b_a", d, True)
    d = pool2_grad(d) + d_s3
    d = layer_back("e3b", d, True)
    d = layer_back("e3a", d, True)
    d = pool2_grad(d) + d_s2
    d = layer_back("e2b", d, True)
    d = layer_back("e2a", d, True)
    d = pool2_grad(d) + d_s1
    d = layer_back("e1b", d, True)
    layer_back("e1a", d, True)
    return g
