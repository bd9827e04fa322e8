"""Pins of the surrogate's CPU reference (oracle/cno.py): every hand-written
backward pass against central finite differences of its forward function,
and the blocks against their definitions on small inputs (a direct loop
convolution, pooling/upsampling adjointness)."""
import numpy as np

from oracle import cno


def _fd(f, x, idx, h=1e-6):
    xp, xm = x.copy(), x.copy()
    xp[idx] += h
    xm[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def test_conv3x3_matches_direct_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 3))
    w = rng.normal(size=(9, 3, 4))
    b = rng.normal(size=4)
    out = cno.conv3x3(x, w, b)
    ref = np.zeros_like(out)
    for bb in range(2):
        for y in range(5):
            for xx in range(6):
                for t, (dy, dx) in enumerate(cno.TAPS):
                    yy, xs = y + dy, xx + dx
                    if 0 <= yy < 5 and 0 <= xs < 6:
                        ref[bb, y, xx] += x[bb, yy, xs] @ w[t]
                ref[bb, y, xx] += b
    assert np.max(np.abs(out - ref)) < 1e-12


def test_conv3x3_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 4, 5, 3))
    w = rng.normal(size=(9, 3, 2))
    b = rng.normal(size=2)
    r = rng.normal(size=(1, 4, 5, 2))
    dx, dw, db = cno.conv3x3_backward(x, w, r)
    for idx in [(0, 0, 0, 0), (0, 3, 4, 2), (0, 2, 1, 1)]:
        assert abs(_fd(lambda z: np.sum(cno.conv3x3(z, w, b) * r), x, idx) - dx[idx]) < 1e-7
    for idx in [(0, 0, 0), (4, 2, 1), (8, 1, 0)]:
        assert abs(_fd(lambda z: np.sum(cno.conv3x3(x, z, b) * r), w, idx) - dw[idx]) < 1e-7
    assert np.max(np.abs(db - r.sum(axis=(0, 1, 2)))) < 1e-12


def test_pool_and_up_backward_are_adjoints():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 6, 4, 3))
    y = rng.normal(size=(2, 3, 2, 3))
    assert abs(np.sum(cno.pool2(x) * y) - np.sum(x * cno.pool2_backward(y))) < 1e-12
    z = rng.normal(size=(2, 6, 4, 3))
    assert abs(np.sum(cno.up2(y) * z) - np.sum(y * cno.up2_backward(z))) < 1e-12


def test_unet_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    net = cno.UNet(cin=2, cout=2, widths=[3, 4, 5], slope=0.1, rng=rng)
    x = rng.normal(size=(1, 8, 8, 2))
    target = rng.normal(size=(1, 8, 8, 2))

    def loss_of(params):
        keep = net.params
        net.params = params
        l, _ = cno.mse(net.forward(x), target, 2)
        net.params = keep
        return l

    loss, g = cno.mse(net.forward(x), target, 2)
    grads, dx = net.backward(g)
    for li in [0, 3, 5, len(net.params) - 3, len(net.params) - 1]:
        w, b = net.params[li]
        for idx in [(0, 0, 0), (8, w.shape[1] - 1, w.shape[2] - 1)]:
            def f(z, li=li, idx=idx):
                ps = list(net.params)
                ps[li] = (z, ps[li][1])
                return loss_of(ps)
            assert abs(_fd(f, w, idx) - grads[li][0][idx]) < 1e-6 * max(1.0, abs(grads[li][0][idx])), (li, idx)
        fb = lambda z, li=li: loss_of([p if k != li else (p[0], z) for k, p in enumerate(net.params)])
        assert abs(_fd(fb, b, (0,)) - grads[li][1][0]) < 1e-6
    # gradient wrt the input as well
    def fx(z):
        l, _ = cno.mse(net.forward(z), target, 2)
        return l
    for idx in [(0, 0, 0, 0), (0, 7, 3, 1)]:
        assert abs(_fd(fx, x, idx) - dx[idx]) < 1e-6


def test_adam_first_step_moves_by_lr():
    w = np.array([1.0, -2.0]); g = np.array([0.5, -3.0])
    w1, m, v = cno.adam(w, g, np.zeros(2), np.zeros(2), 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * np.sign(g), atol=1e-7)


def _channel_fields(rng, N, ny, nx):
    f = np.zeros((N, 6, ny, nx))
    f[:, 0] = rng.uniform(0.01, 0.2, size=(N, ny, nx))
    f[:, 1:5] = rng.normal(0.0, 0.01, size=(N, 4, ny, nx))
    return f


def test_volume_defect_pins():
    """volume_defect against what the definition fixes: (1) a uniform, still
    field has no flux and no change, defect 0; (2) gas added uniformly with
    no flux: defect = added volume / initial volume exactly; (3) a discrete
    advection-diffusion update of alpha_g along y (upwind flux alpha u_y plus
    -chi (a[y+1] - a[y]) between rows, zero flux at the side columns) conserves
    the total up to the fluxes through the end faces, and with u_y, chi
    constant in time and the end rows unchanged the defect measures only the
    fluxes through its end rows: a step built from those fluxes has defect 0
    as a jump of 1 and one step's net inflow as a jump of 2."""
    rng = np.random.default_rng(3)
    # (1)
    f = np.zeros((2, 6, 8, 5))
    f[:, 0] = 0.1
    assert np.all(cno.volume_defect(f, f.copy(), 100, [0.1, 0.2]) == 0.0)
    # (2)
    g = f.copy()
    g[:, 0] += 1e-3
    np.testing.assert_allclose(cno.volume_defect(f, g, 100, [0.1, 0.2]), 1e-3 / 0.1, rtol=1e-12)
    # (3) one explicit step with face fluxes F[y] between row y-1 and y; the
    # inflow through the inlet face and the outflow through the outlet face
    # are set to the same one-sided expressions the defect uses, so the
    # defect of the step is 0 to rounding when f0 and f1 share end rows
    ny, nx, chi = 12, 7, 0.05
    f0 = _channel_fields(rng, 1, ny, nx)
    a, v = f0[0, 0], f0[0, 2]
    fin = a[0] * v[0] - chi * (a[1] - a[0])
    fout = a[-1] * v[-1] - chi * (a[-1] - a[-2])
    f1 = f0.copy()
    # move gas between interior rows 2..ny-3 only (no net change), then add
    # the end fluxes to rows 2 and ny - 3 (not read by the flux estimate)
    for y in range(2, ny - 3):
        flux = a[y] * v[y] - chi * (a[y + 1] - a[y])
        f1[0, 0, y] -= flux
        f1[0, 0, y + 1] += flux
    f1[0, 0, 2] += fin
    f1[0, 0, ny - 3] -= fout
    d = cno.volume_defect(f0, f1, 1, [chi])
    assert d[0] < 1e-14
    # the same step taken as a jump of 2 is off by exactly one step's net inflow
    d2 = cno.volume_defect(f0, f1, 2, [chi])
    np.testing.assert_allclose(d2[0], abs((fin - fout).sum()) / a.sum(), rtol=1e-9)
