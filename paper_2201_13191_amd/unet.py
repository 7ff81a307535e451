"""Learned scatter denoiser / up-sampler: a U-Net whose every operation is a
libmcx kernel (include/mcx.h, mc_nn_*).  This module only allocates device
buffers (PyTorch tensors used as memory) and sequences the kernels.

Architecture (4 levels, 32 base channels; 3x3 convs with bias and ReLU, 2x2
average pooling, nearest 2x up-sampling, skip connections concatenated as
channel slices of one NHWC buffer):

    in [N,S,S,16] (ch 0 scatter, ch 1 primary, rest zero)
    e1: 16->32->32 (s1) | pool | e2: 32->64->64 (s2) | pool | e3: 64->128->128 (s3)
    pool | bottleneck 128->256->256 | up, [up,s3] 384 -> 128 -> 128 | up, [up,s2] 192 -> 64
    -> 64 | up, [up,s1] 96 -> 32 -> 32 | up (2S) | head 32->16 relu -> 1 (linear, fp32)

It replaces the Savitzky-Golay smoothing and cubic up-sampling of the paper's
correction loop (section II-C-3/4): input a low-count scatter map at S x S
plus the primary image, output the scatter map at 2S x 2S.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mcx

# (name, cin, cout, relu); h_b has one real output channel, stored as 16
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
INTERNAL_COUT = {"h_b": 16}
# (input channels, stored output channels) per layer
LAYER_CH = {name: (ci, INTERNAL_COUT.get(name, co)) for name, ci, co, _ in LAYERS}
# pixel ranges of the bias-gradient sums (blocks per 64 channels): at most
# this many, and at least 256 pixels each
BIAS_ROWS = 512
# weight gradients: pixel splits chosen so that a layer's (32 x 32 tile,
# split) blocks number about this many, with at least 256 pixels per split
WGRAD_BLOCKS = 1024


def cout_alloc(c):
    """Weight rows the conv kernel reads for c output channels."""
    return 32 if c <= 32 else (c + 63) // 64 * 64


def he_init(seed):
    """He-normal weights [cout][9][cin] and zero biases (fp64 numpy), seeded."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, ci, co, _ in LAYERS:
        out[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(co, 9, ci))
        out[name + ".b"] = np.zeros(co)
    return out


class UNet:
    def __init__(self, ctx, batch, size=128, params=None, seed=0, device="cuda:0",
                 lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        if size % 8:
            raise ValueError("size must be a multiple of 8")
        self.ctx, self.N, self.S, self.dev = ctx, batch, size, torch.device(device)
        self.lr, self.b1, self.b2, self.eps = lr, betas[0], betas[1], eps
        self.step_count = 0
        self.stream = None
        params = params if params is not None else he_init(seed)
        f32 = dict(dtype=torch.float32, device=self.dev)
        bf = dict(dtype=torch.int16, device=self.dev)     # bf16 bit patterns
        self.L = {}
        for name, ci, co, relu in LAYERS:
            coi = INTERNAL_COUT.get(name, co)
            w = np.zeros((coi, 9, ci))
            w[:co] = params[name + ".w"]
            b = np.zeros(coi)
            b[:co] = params[name + ".b"]
            d = dict(ci=ci, co=co, coi=coi, relu=relu,
                     w32=torch.tensor(w, **f32).contiguous(),
                     b32=torch.tensor(b, **f32).contiguous(),
                     wb=torch.zeros((cout_alloc(coi), 9, ci), **bf),
                     wt=torch.zeros((cout_alloc(ci), 9, coi), **bf),
                     gw=torch.zeros((coi, 9, ci), **f32), gb=torch.zeros(coi, **f32))
            for k in ("mw", "vw"):
                d[k] = torch.zeros_like(d["w32"])
            for k in ("mb", "vb"):
                d[k] = torch.zeros_like(d["b32"])
            self.L[name] = d
        self._sync_bf16()
        N, S = batch, size
        shapes = {
            "x": (S, 16), "e1a": (S, 32), "cat1": (S, 96), "p1": (S // 2, 32),
            "e2a": (S // 2, 64), "cat2": (S // 2, 192), "p2": (S // 4, 64),
            "e3a": (S // 4, 128), "cat3": (S // 4, 384), "p3": (S // 8, 128),
            "b_a": (S // 8, 256), "b_b": (S // 8, 256),
            "d3a": (S // 4, 128), "d3b": (S // 4, 128), "d2a": (S // 2, 64), "d2b": (S // 2, 64),
            "d1a": (S, 32), "d1b": (S, 32), "u0": (2 * S, 32), "h_a": (2 * S, 16),
            "out": (2 * S, 16),
        }
        self.A, self.G, self.shape = {}, {}, shapes
        for k, (s, c) in shapes.items():
            self.A[k] = torch.zeros((N, s, s, c), **bf)
            if k != "x":
                self.G[k] = torch.zeros((N, s, s, c), **bf)
        self.out32 = torch.zeros((N * 4 * S * S, 16), **f32)
        self.target = torch.zeros(N * 4 * S * S, **f32)
        self.loss_partial = torch.zeros((N * 4 * S * S + 255) // 256, **f32)
        ws = 0
        for name, ci, co, _ in LAYERS:
            coi = INTERNAL_COUT.get(name, co)
            ws = max(ws, (self._splits(name) + 1) * 9 * coi * ci)
        self.ws = torch.zeros(ws, **f32)
        self.bias_ws = torch.zeros(BIAS_ROWS * 256, **f32)

    # ------------------------------------------------------------------ helpers
    def _splits(self, name):
        s = self._in_size(name)
        npix = self.N * s * s
        ci, coi = LAYER_CH[name]
        tiles = -(-coi // 32) * -(-ci // 32)
        return int(max(1, min(npix // 256, -(-WGRAD_BLOCKS // tiles))))

    def _bias_rows(self, name):
        s = self._in_size(name)
        return int(max(1, min(BIAS_ROWS, self.N * s * s // 256)))

    def _in_size(self, name):
        lvl = {"e1a": 1, "e1b": 1, "e2a": 2, "e2b": 2, "e3a": 4, "e3b": 4, "b_a": 8, "b_b": 8,
               "d3a": 4, "d3b": 4, "d2a": 2, "d2b": 2, "d1a": 1, "d1b": 1, "h_a": 0.5, "h_b": 0.5}
        return int(self.S / lvl[name])

    def _sync_bf16(self):
        """bf16 copies and flipped copies of every weight tensor."""
        for d in self.L.values():
            n = d["w32"].numel()
            mcx.mc_nn_cast_bf16_async(self.ctx, d["w32"], d["wb"], n, self.stream)
            self._flip(d)

    def _flip(self, d):
        mcx.mc_nn_flip_weights_async(self.ctx, d["wb"], d["wt"], d["coi"], d["ci"], d["coi"],
                                     cout_alloc(d["ci"]), self.stream)

    def _conv(self, name, x, xoff, y, yoff, relu=True, yf=None):
        d = self.L[name]
        n, s = x.shape[0], x.shape[1]
        mcx.mc_nn_conv3x3_async(self.ctx, x, x.shape[3], xoff, d["wb"], d["b32"],
                                y, y.shape[3] if y is not None else 0, yoff, n, s, s, d["ci"],
                                d["coi"], relu=relu, yf=yf, stream=self.stream)

    def _pool(self, x, xoff, y, yoff, c, backward=False, acc=False):
        n, s = (x.shape[0], x.shape[1]) if not backward else (y.shape[0], y.shape[1])
        mcx.mc_nn_pool2_async(self.ctx, x, x.shape[3], xoff, y, y.shape[3], yoff, n, s, s, c,
                              backward, acc, self.stream)

    def _up(self, x, xoff, y, yoff, c, backward=False, acc=False):
        n, s = (x.shape[0], x.shape[1]) if not backward else (y.shape[0], y.shape[1])
        mcx.mc_nn_upsample2_async(self.ctx, x, x.shape[3], xoff, y, y.shape[3], yoff, n, s, s, c,
                                  backward, acc, self.stream)

    # ------------------------------------------------------------------ forward
    def set_input(self, scatter, primary, scale_s=1.0, scale_p=1.0):
        """scatter, primary: fp32 device tensors [N,S,S]."""
        A = self.A["x"]
        npix = self.N * self.S * self.S
        mcx.mc_nn_pack_channel_async(self.ctx, scatter.contiguous(), npix, scale_s, A, 16, 0,
                                     self.stream)
        mcx.mc_nn_pack_channel_async(self.ctx, primary.contiguous(), npix, scale_p, A, 16, 1,
                                     self.stream)

    def set_input_samples(self, scatter, primary, scale_s=1.0, scale_p=1.0):
        """scatter, primary: sequences of N fp32 device tensors [S,S]; sample i
        is packed into batch slot i."""
        A = self.A["x"]
        npix = self.S * self.S
        for i in range(self.N):
            mcx.mc_nn_pack_channel_async(self.ctx, scatter[i], npix, scale_s, A[i], 16, 0,
                                         self.stream)
            mcx.mc_nn_pack_channel_async(self.ctx, primary[i], npix, scale_p, A[i], 16, 1,
                                         self.stream)

    def set_target_samples(self, targets):
        """targets: sequence of N fp32 device tensors [2S,2S] (copied into place)."""
        n = 4 * self.S * self.S
        for i in range(self.N):
            self.target[i * n:(i + 1) * n].copy_(targets[i].reshape(-1))

    def forward(self):
        A = self.A
        self._conv("e1a", A["x"], 0, A["e1a"], 0)
        self._conv("e1b", A["e1a"], 0, A["cat1"], 64)
        self._pool(A["cat1"], 64, A["p1"], 0, 32)
        self._conv("e2a", A["p1"], 0, A["e2a"], 0)
        self._conv("e2b", A["e2a"], 0, A["cat2"], 128)
        self._pool(A["cat2"], 128, A["p2"], 0, 64)
        self._conv("e3a", A["p2"], 0, A["e3a"], 0)
        self._conv("e3b", A["e3a"], 0, A["cat3"], 256)
        self._pool(A["cat3"], 256, A["p3"], 0, 128)
        self._conv("b_a", A["p3"], 0, A["b_a"], 0)
        self._conv("b_b", A["b_a"], 0, A["b_b"], 0)
        self._up(A["b_b"], 0, A["cat3"], 0, 256)
        self._conv("d3a", A["cat3"], 0, A["d3a"], 0)
        self._conv("d3b", A["d3a"], 0, A["d3b"], 0)
        self._up(A["d3b"], 0, A["cat2"], 0, 128)
        self._conv("d2a", A["cat2"], 0, A["d2a"], 0)
        self._conv("d2b", A["d2a"], 0, A["d2b"], 0)
        self._up(A["d2b"], 0, A["cat1"], 0, 64)
        self._conv("d1a", A["cat1"], 0, A["d1a"], 0)
        self._conv("d1b", A["d1a"], 0, A["d1b"], 0)
        self._up(A["d1b"], 0, A["u0"], 0, 32)
        self._conv("h_a", A["u0"], 0, A["h_a"], 0)
        self._conv("h_b", A["h_a"], 0, None, 0, relu=False, yf=self.out32)
        return self.out32[:, 0].view(self.N, 2 * self.S, 2 * self.S)

    # ------------------------------------------------------------------ backward
    def loss_and_grad(self):
        """MSE against self.target; writes the output gradient (channel 0 of G['out'])."""
        n = self.out32.shape[0]
        mcx.mc_nn_mse_async(self.ctx, self.out32, 16, self.target, n, self.G["out"], 16, 0, 1.0,
                            self.loss_partial, self.stream)

    def loss_value(self):
        torch.cuda.synchronize()
        return float(self.loss_partial.cpu().double().sum().item() / self.out32.shape[0])

    def _layer_back(self, name, x, xoff, gy, gyoff, gx=None, gxoff=0, relu_of=None):
        """Gradients of layer `name`: dW, db from its input x (slice) and the
        (already masked) output gradient gy (slice); input gradient into gx,
        zeroed where relu_of (the activation gx belongs to, same slice) is not
        positive when given (the previous ReLU's derivative, applied in the
        convolution's epilogue)."""
        d = self.L[name]
        n, s = x.shape[0], x.shape[1]
        mcx.mc_nn_conv3x3_wgrad_async(self.ctx, x, x.shape[3], xoff, gy, gy.shape[3], gyoff, n,
                                      s, s, d["ci"], d["coi"], self._splits(name), self.ws,
                                      d["gw"], self.stream)
        mcx.mc_nn_bias_grad_async(self.ctx, gy, gy.shape[3], gyoff, n * s * s, d["coi"],
                                  self.bias_ws, self._bias_rows(name), d["gb"], self.stream)
        if gx is not None:
            mask = dict(mask=relu_of, ldm=relu_of.shape[3], moff=gxoff) if relu_of is not None \
                else {}
            mcx.mc_nn_conv3x3_async(self.ctx, gy, gy.shape[3], gyoff, d["wt"], None, gx,
                                    gx.shape[3], gxoff, n, s, s, d["coi"], d["ci"], relu=0,
                                    stream=self.stream, **mask)

    def _mask(self, g, goff, a, aoff, c):
        n, s = g.shape[0], g.shape[1]
        mcx.mc_nn_relu_mask_async(self.ctx, g, g.shape[3], goff, a, a.shape[3], aoff, n * s * s, c,
                                  self.stream)

    def backward(self):
        A, G = self.A, self.G
        self._layer_back("h_b", A["h_a"], 0, G["out"], 0, G["h_a"], 0, relu_of=A["h_a"])
        self._layer_back("h_a", A["u0"], 0, G["h_a"], 0, G["u0"], 0)
        self._up(G["u0"], 0, G["d1b"], 0, 32, backward=True)
        self._mask(G["d1b"], 0, A["d1b"], 0, 32)
        self._layer_back("d1b", A["d1a"], 0, G["d1b"], 0, G["d1a"], 0, relu_of=A["d1a"])
        self._layer_back("d1a", A["cat1"], 0, G["d1a"], 0, G["cat1"], 0)
        self._up(G["cat1"], 0, G["d2b"], 0, 64, backward=True)
        self._mask(G["d2b"], 0, A["d2b"], 0, 64)
        self._layer_back("d2b", A["d2a"], 0, G["d2b"], 0, G["d2a"], 0, relu_of=A["d2a"])
        self._layer_back("d2a", A["cat2"], 0, G["d2a"], 0, G["cat2"], 0)
        self._up(G["cat2"], 0, G["d3b"], 0, 128, backward=True)
        self._mask(G["d3b"], 0, A["d3b"], 0, 128)
        self._layer_back("d3b", A["d3a"], 0, G["d3b"], 0, G["d3a"], 0, relu_of=A["d3a"])
        self._layer_back("d3a", A["cat3"], 0, G["d3a"], 0, G["cat3"], 0)
        self._up(G["cat3"], 0, G["b_b"], 0, 256, backward=True)
        self._mask(G["b_b"], 0, A["b_b"], 0, 256)
        self._layer_back("b_b", A["b_a"], 0, G["b_b"], 0, G["b_a"], 0, relu_of=A["b_a"])
        self._layer_back("b_a", A["p3"], 0, G["b_a"], 0, G["p3"], 0)
        self._pool(G["p3"], 0, G["cat3"], 256, 128, backward=True, acc=True)
        self._mask(G["cat3"], 256, A["cat3"], 256, 128)
        self._layer_back("e3b", A["e3a"], 0, G["cat3"], 256, G["e3a"], 0, relu_of=A["e3a"])
        self._layer_back("e3a", A["p2"], 0, G["e3a"], 0, G["p2"], 0)
        self._pool(G["p2"], 0, G["cat2"], 128, 64, backward=True, acc=True)
        self._mask(G["cat2"], 128, A["cat2"], 128, 64)
        self._layer_back("e2b", A["e2a"], 0, G["cat2"], 128, G["e2a"], 0, relu_of=A["e2a"])
        self._layer_back("e2a", A["p1"], 0, G["e2a"], 0, G["p1"], 0)
        self._pool(G["p1"], 0, G["cat1"], 64, 32, backward=True, acc=True)
        self._mask(G["cat1"], 64, A["cat1"], 64, 32)
        self._layer_back("e1b", A["e1a"], 0, G["cat1"], 64, G["e1a"], 0, relu_of=A["e1a"])
        self._layer_back("e1a", A["x"], 0, G["e1a"], 0, None)

    def adam_step(self):
        self.step_count += 1
        for d in self.L.values():
            mcx.mc_nn_adam_async(self.ctx, d["w32"], d["gw"], d["mw"], d["vw"], d["wb"],
                                 d["w32"].numel(), self.lr, self.b1, self.b2, self.eps,
                                 self.step_count, 1.0, self.stream)
            mcx.mc_nn_adam_async(self.ctx, d["b32"], d["gb"], d["mb"], d["vb"], None,
                                 d["b32"].numel(), self.lr, self.b1, self.b2, self.eps,
                                 self.step_count, 1.0, self.stream)
            self._flip(d)

    def train_step(self, scatter, primary, target, scale_s=1.0, scale_p=1.0):
        self.set_input(scatter, primary, scale_s, scale_p)
        self.target.copy_(target.reshape(-1))
        self._step()

    def train_step_samples(self, scatter, primary, targets):
        """One step on N samples given as sequences of per-sample tensors."""
        self.set_input_samples(scatter, primary)
        self.set_target_samples(targets)
        self._step()

    def _step(self):
        self.forward()
        self.loss_and_grad()
        self.backward()
        self.adam_step()

    # ------------------------------------------------------------------ state
    def gradients(self):
        return {n: (d["gw"][:d["co"]].double().cpu().numpy(), d["gb"][:d["co"]].double().cpu().numpy())
                for n, d in self.L.items()}

    def state(self):
        out = {"step": np.array(self.step_count)}
        for n, d in self.L.items():
            for k in ("w32", "b32", "mw", "vw", "mb", "vb"):
                out[f"{n}.{k}"] = d[k].cpu().numpy()
        return out

    def load_state(self, st):
        self.step_count = int(st["step"])
        for n, d in self.L.items():
            for k in ("w32", "b32", "mw", "vw", "mb", "vb"):
                d[k].copy_(torch.from_numpy(np.asarray(st[f"{n}.{k}"])).to(self.dev))
        self._sync_bf16()

    def save(self, path):
        np.savez(path, **self.state())

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.load_state({k: z[k] for k in z.files})


def flops_per_sample(size=128):
    """Multiply-adds x 2 of the 3x3 convolutions of one forward pass."""
    f = 0
    for name, ci, co, _ in LAYERS:
        s = {"e1": 1, "e2": 2, "e3": 4, "b_": 8, "d3": 4, "d2": 2, "d1": 1, "h_": 0.5}[name[:2]]
        f += 2 * 9 * ci * co * (size / s) ** 2
    return f


def _time(argv=None):
    """Forward and training-step time of a batch on random data (no checkpoint)."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--no-train", action="store_true",
                    help="forward passes only (one untimed, then --reps timed)")
    args = ap.parse_args(argv)
    g = mcx.Projector(0)
    N, S = args.batch, args.size
    net = UNet(g.ctx, N, S, seed=1)
    gen = torch.Generator(device="cuda").manual_seed(0)
    s = torch.rand((N, S, S), device="cuda", generator=gen)
    p = torch.rand((N, S, S), device="cuda", generator=gen)
    t = torch.rand((N, 2 * S, 2 * S), device="cuda", generator=gen)
    net.set_input(s, p)
    net.forward()
    if not args.no_train:
        net.train_step(s, p, t)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.reps):
        net.forward()
    e1.record()
    torch.cuda.synchronize()
    fwd = e0.elapsed_time(e1) / args.reps
    fl = flops_per_sample(S) * N
    msg = (f"[unet] batch {N} at {S}^2: forward {fwd:.3f} ms ({fwd / N:.3f} ms per sample, "
           f"{fl / (fwd * 1e-3) / 1e12:.1f} TFLOP/s of 3x3 convolutions)")
    if not args.no_train:
        e0.record()
        for _ in range(args.reps):
            net.train_step(s, p, t)
        e1.record()
        torch.cuda.synchronize()
        msg += f", training step {e0.elapsed_time(e1) / args.reps:.3f} ms"
    print(msg, flush=True)
    g.close()


if __name__ == "__main__":
    _time()
