"""Plain FP64 NumPy reference of the learned surrogate's operations (test
infrastructure, like the rest of this package): the building blocks of a
convolutional neural operator -- 3x3 convolution with zero padding, 2x2
average pooling, nearest 2x upsampling, leaky-ReLU, channel concatenation,
mean squared error and the Adam update -- with hand-written backward passes,
and the U-Net they form.  Tensors are NHWC; convolution weights W[tap][ci][co]
with tap = 3 (dy + 1) + (dx + 1).

The surrogate is not part of the paper; its reference is pinned by finite
differences of the forward functions (tests/test_oracle_cno.py), not by
recomputing these formulas.
"""
import numpy as np

TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dy, dx):
    """s[b, y, x] = x[b, y + dy, x + dx], zero outside."""
    B, H, W, C = x.shape
    s = np.zeros_like(x)
    ys0, ys1 = max(0, -dy), min(H, H - dy)
    xs0, xs1 = max(0, -dx), min(W, W - dx)
    s[:, ys0:ys1, xs0:xs1] = x[:, ys0 + dy:ys1 + dy, xs0 + dx:xs1 + dx]
    return s


def conv3x3(x, w, b=None):
    """out[b, y, x, co] = sum_tap sum_ci x[b, y + dy, x + dx, ci] w[tap, ci, co] (+ bias)."""
    out = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, (dy, dx) in enumerate(TAPS):
        out += _shift(x, dy, dx) @ w[t]
    if b is not None:
        out += b
    return out


def conv3x3_backward(x, w, dout):
    """Gradients of conv3x3 wrt x, w and the bias."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dy, ddx) in enumerate(TAPS):
        dx += _shift(dout @ w[t].T, -dy, -ddx)
        dw[t] = _shift(x, dy, ddx).reshape(-1, x.shape[3]).T @ dout.reshape(-1, dout.shape[3])
    return dx, dw, dout.sum(axis=(0, 1, 2))


def leaky(x, slope):
    return np.where(x > 0, x, slope * x)


def leaky_backward(y, dy, slope):
    return np.where(y > 0, dy, slope * dy)


def pool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(dout):
    return 0.25 * np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2)


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dout):
    B, H2, W2, C = dout.shape
    return dout.reshape(B, H2 // 2, 2, W2 // 2, 2, C).sum(axis=(2, 4))


def mse(pred, target, cused):
    d = pred[..., :cused] - target[..., :cused]
    loss = float(np.mean(d * d))
    g = np.zeros_like(pred)
    g[..., :cused] = 2.0 * d / d.size
    return loss, g


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * ((m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps) + wd * w)
    return w, m, v


class UNet:
    """U-Net of the surrogate: `widths` channels per level (levels - 1 2x2
    poolings), two 3x3 convolutions + leaky-ReLU per encoder level, on the way
    up a nearest 2x upsampling + convolution + activation, concatenation with
    the skip of that level and one convolution + activation, then a linear
    3x3 output convolution.  Parameters: a list of (w, b) in layer order."""

    def __init__(self, cin, cout, widths, slope=0.1, rng=None):
        self.cin, self.cout, self.widths, self.slope = cin, cout, list(widths), slope
        self.shapes = []
        c = cin
        for k, wdt in enumerate(widths):
            self.shapes += [(c, wdt), (wdt, wdt)]
            c = wdt
        for k in range(len(widths) - 2, -1, -1):
            self.shapes += [(c, widths[k]), (2 * widths[k], widths[k])]
            c = widths[k]
        self.shapes.append((c, cout))
        rng = rng or np.random.default_rng(0)
        self.params = [(rng.normal(0, np.sqrt(2.0 / (9 * ci)), (9, ci, co)), np.zeros(co)) for ci, co in self.shapes]

    def forward(self, x):
        P, s = self.params, self.slope
        tape = []
        h, i, skips = x, 0, []
        for k in range(len(self.widths)):
            for _ in range(2):
                hin = h
                h = leaky(conv3x3(hin, *P[i]), s)
                tape.append(("conv", i, hin, h))
                i += 1
            if k < len(self.widths) - 1:
                skips.append(h)
                h = pool2(h)
        for k in range(len(self.widths) - 2, -1, -1):
            u = up2(h)
            h = leaky(conv3x3(u, *P[i]), s)
            tape.append(("conv", i, u, h))
            i += 1
            cat = np.concatenate([h, skips[k]], axis=3)
            h = leaky(conv3x3(cat, *P[i]), s)
            tape.append(("conv", i, cat, h))
            i += 1
        out = conv3x3(h, *P[i])
        tape.append(("out", i, h, out))
        self._tape = tape
        return out

    def backward(self, dout):
        """Parameter gradients (same structure as params) after forward()."""
        P, s, tape = self.params, self.slope, self._tape
        grads = [None] * len(P)
        nl = len(self.widths)
        _, i, hin, _ = tape[-1]
        dh, dw, db = conv3x3_backward(hin, P[i][0], dout)
        grads[i] = (dw, db)
        t = len(tape) - 2
        dskips = [None] * (nl - 1)
        for k in range(0, nl - 1):
            # up level k (processed here in reverse of the forward order)
            _, i, cat, y = tape[t]
            dpre = leaky_backward(y, dh, s)
            dcat, dw, db = conv3x3_backward(cat, P[i][0], dpre)
            grads[i] = (dw, db)
            c = P[i][0].shape[1] // 2
            dh, dskips[k] = dcat[..., :c], dcat[..., c:]
            t -= 1
            _, i, u, y = tape[t]
            dpre = leaky_backward(y, dh, s)
            du, dw, db = conv3x3_backward(u, P[i][0], dpre)
            grads[i] = (dw, db)
            dh = up2_backward(du)
            t -= 1
        # encoder, from the bottom level up; dskips[k] is the gradient of the
        # skip of level k
        for k in range(nl - 1, -1, -1):
            if k < nl - 1:
                dh = pool2_backward(dh) + dskips[k]
            for _ in range(2):
                _, i, hin, y = tape[t]
                dpre = leaky_backward(y, dh, s)
                dh, dw, db = conv3x3_backward(hin, P[i][0], dpre)
                grads[i] = (dw, db)
                t -= 1
        return grads, dh


def volume_defect(f0, f1, jump, chi):
    """Gas-volume defect of a jump f0 -> f1 of a channel (the surrogate's
    acceptance test), per lattice.  f: (N, 6, ny, nx) field planes (alpha_g,
    u_g,x, u_g,y, u_l,x, u_l,y, dp_k), rows y = 0 (inlet) .. ny - 1 (outlet);
    chi: (N,) diffusivity of the volume-fraction scheme.  The gas entering per
    step is the flux through the inlet row minus that through the outlet row,
    each advective alpha_g u_g,y plus diffusive -chi d(alpha_g)/dy (one-sided
    differences between the end row and its neighbour), summed over x; the
    budget of the jump is jump x the mean of that net inflow at its two ends
    (trapezoid in time).  Defect = |V(f1) - V(f0) - budget| / |V(f0)|, V the
    sum of alpha_g over the lattice.  Plain loops over rows and columns in
    FP64."""
    f0 = np.asarray(f0, dtype=np.float64)
    f1 = np.asarray(f1, dtype=np.float64)
    N, _, ny, nx = f0.shape
    out = np.zeros(N)
    for n in range(N):
        c = float(chi[n])

        def net_inflow(f):
            a, v = f[n, 0], f[n, 2]
            s = 0.0
            for x in range(nx):
                fin = a[0, x] * v[0, x] - c * (a[1, x] - a[0, x])
                fout = a[ny - 1, x] * v[ny - 1, x] - c * (a[ny - 1, x] - a[ny - 2, x])
                s += fin - fout
            return s

        v0 = f0[n, 0].sum()
        v1 = f1[n, 0].sum()
        budget = 0.5 * jump * (net_inflow(f0) + net_inflow(f1))
        out[n] = abs(v1 - v0 - budget) / abs(v0)
    return out
