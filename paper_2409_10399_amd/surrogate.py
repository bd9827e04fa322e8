"""Learned surrogate of the LBM step: a convolutional neural operator (U-Net
of 3x3 convolutions) that maps the macroscopic fields of a D2Q9 channel
(alpha_g, u_g, u_l, delta p_k) plus per-lattice conditioning values
(ln R, bubble diameter, inlet gas fraction) to the change of the fields over
`jump` LBM steps.

Every operation runs in the HIP kernels of csrc/cno_kernels.hip (matrix-core
BF16 convolutions with FP32 accumulation, forward and backward, Adam); this
module only allocates buffers with PyTorch and chains the C-ABI calls.  The
surrogate is not part of the paper: it is trained on trajectories of the
batched LBM and judged against it (rollout with re-anchoring on plain LBM).
"""
import ctypes
import math
from ctypes import c_void_p

import numpy as np

from .binding import _check, lib

FIELD_PLANES = ("alpha_g", "u_gx", "u_gy", "u_lx", "u_ly", "dp_k")


def _p(t):
    return c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _pad16(c):
    return 16 * ((c + 15) // 16)


class CNO:
    """U-Net: `widths` channels per level (each a multiple of 16), two
    convolution + leaky-ReLU layers per encoder level with 2x2 average pooling
    between levels, on the way up nearest 2x upsampling + convolution, a
    concatenation with the skip of that level and one more convolution, then a
    linear output convolution.  Layer order and weight layout W[tap][ci][co]
    are those of the CPU reference (oracle/cno.py, class UNet)."""

    def __init__(self, cin, cout, widths=(32, 48, 96, 192), slope=0.1, seed=0):
        import torch
        assert len(widths) >= 2 and all(w % 16 == 0 for w in widths)
        self.cin_used, self.cout_used = cin, cout
        self.cin, self.cout = _pad16(cin), _pad16(cout)
        self.widths, self.slope = list(widths), float(slope)
        nl = len(widths)
        shapes, c = [], self.cin
        for w in widths:
            shapes += [(c, w), (w, w)]
            c = w
        for k in range(nl - 2, -1, -1):
            shapes += [(c, widths[k]), (2 * widths[k], widths[k])]
            c = widths[k]
        shapes.append((c, self.cout))
        self.shapes = shapes
        rng = np.random.default_rng(seed)
        dev = "cuda"
        self.W, self.b = [], []
        for k, (ci, co) in enumerate(shapes):
            w = rng.normal(0.0, math.sqrt(2.0 / (9 * ci)), (9, ci, co))
            if k == len(shapes) - 1:
                w *= 0.1  # the output starts near zero change
            self.W.append(torch.tensor(w, dtype=torch.float32, device=dev))
            self.b.append(torch.zeros(co, dtype=torch.float32, device=dev))
        self.gW = [torch.zeros_like(w) for w in self.W]
        self.gb = [torch.zeros_like(b) for b in self.b]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.wf = [torch.empty(w.numel(), dtype=torch.int16, device=dev) for w in self.W]
        self.wd = [torch.empty(w.numel(), dtype=torch.int16, device=dev) for w in self.W]
        self.adam_steps = 0
        self._bufs = {}
        self.repack()

    @property
    def n_params(self):
        return sum(w.numel() + b.numel() for w, b in zip(self.W, self.b))

    def repack(self):
        L, st = lib(), _stream()
        for (ci, co), w, wf, wd in zip(self.shapes, self.W, self.wf, self.wd):
            _check(L.eelbm_cno_pack_weights(_p(w), ci, co, _p(wf), _p(wd), st))

    def set_params(self, params):
        """Load [(w, b), ...] (NumPy, W[tap][ci][co]) and repack."""
        import torch
        for k, (w, b) in enumerate(params):
            self.W[k].copy_(torch.as_tensor(w, dtype=torch.float32))
            self.b[k].copy_(torch.as_tensor(b, dtype=torch.float32))
        self.repack()

    def get_params(self):
        return [(w.double().cpu().numpy(), b.double().cpu().numpy()) for w, b in zip(self.W, self.b)]

    # ------------------------------------------------------------ buffers
    def _buf(self, name, shape, bf16=False):
        import torch
        key = (name, tuple(shape), bf16)
        t = self._bufs.get(key)
        if t is None:
            t = torch.empty(shape, dtype=torch.int16 if bf16 else torch.float32, device="cuda")
            self._bufs[key] = t
        return t

    # ------------------------------------------------------------- passes
    def _conv(self, x, li, out, act):
        B, H, W, ci = x.shape
        _check(lib().eelbm_cno_conv_fwd(_p(x), B, H, W, ci, _p(self.wf[li]), _p(self.b[li]), out.shape[3], _p(out),
                                        int(act), self.slope, _stream()))

    def infer(self, x):
        """Inference forward pass with BF16 activations between the layers
        (the first layer reads the FP32 input x, the last writes FP32): the
        products round their operands to BF16 anyway, so only the pooling
        sees rounded inputs; half the activation traffic of forward()."""
        L, st = lib(), _stream()
        B, H, W, _ = x.shape
        nl, wd = len(self.widths), self.widths
        conv = L.eelbm_cno_conv_fwd_cat_dt
        h, li, hb = x, 0, 0
        for k in range(nl):
            Hk, Wk = H >> k, W >> k
            for j in range(2):
                out = self._buf(f"e{k}_{j}", (B, Hk, Wk, wd[k]), True)
                _check(conv(_p(h), h.shape[3], 0, None, 0, B, Hk, Wk, _p(self.wf[li]), _p(self.b[li]), wd[k],
                            _p(out), 1, self.slope, hb, 1, st))
                h, li, hb = out, li + 1, 1
            if k < nl - 1:
                p = self._buf(f"p{k + 1}", (B, Hk // 2, Wk // 2, wd[k]), True)
                _check(L.eelbm_cno_pool_bf16(_p(h), B, Hk, Wk, wd[k], _p(p), st))
                h = p
        for k in range(nl - 2, -1, -1):
            Hk, Wk = H >> k, W >> k
            skip = self._buf(f"e{k}_1", (B, Hk, Wk, wd[k]), True)
            d1 = self._buf(f"d{k}_1", (B, Hk, Wk, wd[k]), True)
            _check(conv(_p(h), wd[k + 1], 1, None, 0, B, Hk, Wk, _p(self.wf[li]), _p(self.b[li]), wd[k], _p(d1), 1,
                        self.slope, 1, 1, st))
            d2 = self._buf(f"d{k}_2", (B, Hk, Wk, wd[k]), True)
            _check(conv(_p(d1), wd[k], 0, _p(skip), wd[k], B, Hk, Wk, _p(self.wf[li + 1]), _p(self.b[li + 1]), wd[k],
                        _p(d2), 1, self.slope, 1, 1, st))
            h, li = d2, li + 2
        out = self._buf("out", (B, H, W, self.cout))
        _check(conv(_p(h), wd[0], 0, None, 0, B, H, W, _p(self.wf[li]), _p(self.b[li]), self.cout, _p(out), 0,
                    self.slope, 1, 0, st))
        return out

    def forward(self, x, keep=True):
        """x: (B, H, W, cin) FP32 contiguous device tensor (H, W divisible by
        2^(levels-1)); returns (B, H, W, cout) (the first cout_used channels
        are the output).  The decoder's upsampling and skip concatenation are
        fused into the input loads of its convolutions; keep=True also
        materialises the upsampled and concatenated tensors, which backward()
        needs (inference passes keep=False)."""
        L, st = lib(), _stream()
        B, H, W, _ = x.shape
        nl, wd = len(self.widths), self.widths
        self._x = x
        h, li = x, 0
        for k in range(nl):
            Hk, Wk = H >> k, W >> k
            for j in range(2):
                out = self._buf(f"e{k}_{j}", (B, Hk, Wk, wd[k]))
                self._conv(h, li, out, True)
                h, li = out, li + 1
            if k < nl - 1:
                p = self._buf(f"p{k + 1}", (B, Hk // 2, Wk // 2, wd[k]))
                _check(L.eelbm_cno_pool(_p(h), B, Hk, Wk, wd[k], _p(p), 0, st))
                h = p
        for k in range(nl - 2, -1, -1):
            Hk, Wk = H >> k, W >> k
            skip = self._buf(f"e{k}_1", (B, Hk, Wk, wd[k]))
            d1 = self._buf(f"d{k}_1", (B, Hk, Wk, wd[k]))
            _check(L.eelbm_cno_conv_fwd_cat(_p(h), wd[k + 1], 1, None, 0, B, Hk, Wk, _p(self.wf[li]), _p(self.b[li]),
                                            wd[k], _p(d1), 1, self.slope, st))
            d2 = self._buf(f"d{k}_2", (B, Hk, Wk, wd[k]))
            _check(L.eelbm_cno_conv_fwd_cat(_p(d1), wd[k], 0, _p(skip), wd[k], B, Hk, Wk, _p(self.wf[li + 1]),
                                            _p(self.b[li + 1]), wd[k], _p(d2), 1, self.slope, st))
            if keep:
                u = self._buf(f"u{k}", (B, Hk, Wk, wd[k + 1]))
                _check(L.eelbm_cno_up(_p(h), B, Hk // 2, Wk // 2, wd[k + 1], _p(u), 0, st))
                cat = self._buf(f"c{k}", (B, Hk, Wk, 2 * wd[k]))
                _check(L.eelbm_cno_concat(_p(d1), wd[k], _p(skip), wd[k], B * Hk * Wk, _p(cat), st))
            h, li = d2, li + 2
        out = self._buf("out", (B, H, W, self.cout))
        self._conv(h, li, out, False)
        self._shape = (B, H, W)
        return out

    def _bwd(self, x, dpre, li, din):
        """weight/bias gradients of layer li from its input x and the
        pre-activation gradient dpre; input gradient into din (or skip)."""
        L, st = lib(), _stream()
        B, H, W, ci = x.shape
        co = dpre.shape[3]
        _check(L.eelbm_cno_conv_bwd_weight(_p(x), _p(dpre), B, H, W, ci, co, _p(self.gW[li]), _p(self.gb[li]), st))
        if din is not None:
            _check(L.eelbm_cno_conv_bwd_data(_p(dpre), B, H, W, co, _p(self.wd[li]), ci, _p(din), st))

    def _act_bwd(self, y, dy, name):
        d = self._buf(name, y.shape)
        _check(lib().eelbm_cno_act_bwd(_p(y), _p(dy), y.numel(), self.slope, _p(d), _stream()))
        return d

    def backward(self, dout):
        """Gradients of all parameters (into gW, gb) for the output gradient
        dout of the last forward()."""
        L, st = lib(), _stream()
        B, H, W = self._shape
        nl, wd = len(self.widths), self.widths
        for g in self.gW + self.gb:
            _check(L.eelbm_cno_fill(_p(g), g.numel(), 0.0, st))
        li = len(self.W) - 1
        top = self._buf("d0_2", (B, H, W, wd[0]))
        dh = self._buf("gh0", (B, H, W, wd[0]))
        self._bwd(top, dout, li, dh)
        dskip = {}
        for k in range(0, nl - 1):
            Hk, Wk = H >> k, W >> k
            li_cat = 2 * nl + 2 * (nl - 2 - k) + 1
            dpre = self._act_bwd(self._buf(f"d{k}_2", (B, Hk, Wk, wd[k])), dh, f"gp{k}_2")
            dcat = self._buf(f"gc{k}", (B, Hk, Wk, 2 * wd[k]))
            self._bwd(self._buf(f"c{k}", (B, Hk, Wk, 2 * wd[k])), dpre, li_cat, dcat)
            dd1 = self._buf(f"gd{k}_1", (B, Hk, Wk, wd[k]))
            ds = self._buf(f"gs{k}", (B, Hk, Wk, wd[k]))
            _check(L.eelbm_cno_fill(_p(ds), ds.numel(), 0.0, st))
            _check(L.eelbm_cno_split_add(_p(dcat), wd[k], wd[k], B * Hk * Wk, _p(dd1), _p(ds), st))
            dskip[k] = ds
            dpre = self._act_bwd(self._buf(f"d{k}_1", (B, Hk, Wk, wd[k])), dd1, f"gp{k}_1")
            du = self._buf(f"gu{k}", (B, Hk, Wk, wd[k + 1]))
            self._bwd(self._buf(f"u{k}", (B, Hk, Wk, wd[k + 1])), dpre, li_cat - 1, du)
            dh = self._buf(f"gh{k + 1}", (B, Hk // 2, Wk // 2, wd[k + 1]))
            _check(L.eelbm_cno_up(_p(du), B, Hk // 2, Wk // 2, wd[k + 1], _p(dh), 1, st))
        for k in range(nl - 1, -1, -1):
            Hk, Wk = H >> k, W >> k
            if k < nl - 1:
                full = self._buf(f"ge{k}", (B, Hk, Wk, wd[k]))
                _check(L.eelbm_cno_pool(_p(dh), B, Hk, Wk, wd[k], _p(full), 1, st))
                _check(L.eelbm_cno_axpy(_p(dskip[k]), full.numel(), 1.0, _p(full), st))
                dh = full
            y1 = self._buf(f"e{k}_1", (B, Hk, Wk, wd[k]))
            y0 = self._buf(f"e{k}_0", (B, Hk, Wk, wd[k]))
            dpre = self._act_bwd(y1, dh, f"gq{k}_1")
            dh0 = self._buf(f"gf{k}_0", (B, Hk, Wk, wd[k]))
            self._bwd(y0, dpre, 2 * k + 1, dh0)
            dpre = self._act_bwd(y0, dh0, f"gq{k}_0")
            xin = self._x if k == 0 else self._buf(f"p{k}", (B, Hk, Wk, wd[k - 1]))
            din = None if k == 0 else self._buf(f"gi{k}", (B, Hk, Wk, wd[k - 1]))
            self._bwd(xin, dpre, 2 * k, din)
            dh = din

    def loss(self, pred, target, grad=True):
        """Mean squared error over the first cout_used channels; returns the
        loss (a float, synchronises) and leaves its gradient in self.dloss."""
        import torch
        nb = 256
        part = self._bufs.get("mse_part")
        if part is None:
            part = torch.empty(nb, dtype=torch.float64, device="cuda")
            self._bufs["mse_part"] = part
        d = self._buf("dloss", pred.shape) if grad else None
        P = pred.shape[0] * pred.shape[1] * pred.shape[2]
        _check(lib().eelbm_cno_mse(_p(pred), _p(target), P, pred.shape[3], self.cout_used, _p(part), nb, _p(d),
                                   _stream()))
        self.dloss = d
        return part

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8, weight_decay=0.0):
        L, st = lib(), _stream()
        self.adam_steps += 1
        for w, g, m, v in zip(self.W + self.b, self.gW + self.gb, self.mW + self.mb, self.vW + self.vb):
            _check(L.eelbm_cno_adam(_p(w), _p(g), _p(m), _p(v), w.numel(), lr, b1, b2, eps, self.adam_steps,
                                    weight_decay, st))
        self.repack()


def pack_input(fields, mean, inv_scale, cond, C, clip=8.0):
    """fields: (B, 6, H, W) FP32 device tensor of FIELD_PLANES; cond (B, nc);
    returns the (B, H, W, C) network input (normalised fields clamped to
    +-clip)."""
    import torch
    B, nf, H, W = fields.shape
    out = torch.empty((B, H, W, C), dtype=torch.float32, device="cuda")
    _check(lib().eelbm_cno_pack(_p(fields), H * W, nf, _p(mean), _p(inv_scale), _p(cond), cond.shape[1], B, C,
                                float(clip), _p(out), _stream()))
    return out


def apply_output(fields, net_out, dscale):
    """fields + the network's normalised change, (B, 6, H, W)."""
    import torch
    B, nf, H, W = fields.shape
    out = torch.empty_like(fields)
    _check(lib().eelbm_cno_unpack(_p(fields), _p(net_out), H * W, nf, net_out.shape[3], _p(dscale), B, _p(out),
                                  _stream()))
    return out


def _time_forward():
    """Time the forward pass of a randomly initialised network on a random
    NHWC input with HIP events: python -m paper_2409_10399_amd.surrogate
    [--widths 32,48,96,192] [--batch 8] [--grid 256] [--reps 20] [--fp32]
    (the inference pass with BF16 activations; --fp32: forward() with FP32
    activations, as in training)."""
    import argparse
    import json

    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--widths", default="32,48,96,192")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--fp32", action="store_true")
    a = ap.parse_args()
    net = CNO(9, 6, [int(w) for w in a.widths.split(",")], seed=0)
    x = torch.randn(a.batch, a.grid, a.grid, net.cin, device="cuda")
    run = (lambda: net.forward(x, keep=False)) if a.fp32 else (lambda: net.infer(x))
    for _ in range(3):
        run()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(a.reps):
        run()
    e1.record(st)
    torch.cuda.synchronize()
    print(json.dumps({"widths": net.widths, "params": net.n_params, "batch": a.batch, "grid": a.grid,
                      "activations": "fp32" if a.fp32 else "bf16", "ms_per_forward": e0.elapsed_time(e1) / a.reps}),
          flush=True)


if __name__ == "__main__":
    _time_forward()
