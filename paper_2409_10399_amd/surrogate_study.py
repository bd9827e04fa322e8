"""Train and judge the learned surrogate on the batched LBM.

1. data: 256 x 256 D2Q9 channels with parameters drawn like the batched sweep
   (R log-uniform in [2, 1000], d in [1, 5] mm, inlet alpha in [0.02, 0.2]),
   advanced by one batched launch per step; the fields are taken every
   `snap` steps from t0 on, and pairs (t, t + jump) are the training data.
2. training: the U-Net of surrogate.CNO on the normalised fields and
   conditioning (ln R, d, alpha_in), target the normalised change over
   `jump` steps, Adam, all in the HIP kernels.
3. judging on held-out channels: from the LBM state at t0, `jumps` surrogate
   jumps; a jump whose conservation defect (change of the domain gas volume
   against the inlet/outlet flux budget) exceeds `defect_max`, and every
   `check_every`-th jump, is replaced by plain LBM steps started from the
   equilibria of the current fields (re-anchoring).  Reported: rel-L2 of
   alpha_g at t0 + jumps * jump against plain LBM, the same for frozen fields
   (no network), and the speedup = time of the plain LBM run (HIP-graph
   batched launches) / time of the rollout.

python -m paper_2409_10399_amd.surrogate_study [--train-inst 200] [--epochs 6] [--out report.json]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def instances(count, seed, n=256):
    import workloads
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        R = float(np.exp(rng.uniform(np.log(2.0), np.log(1000.0))))
        d = float(rng.uniform(1.0, 5.0))
        a = float(rng.uniform(0.02, 0.2))
        cfg, f = workloads.sweep_channel_2d(n, n, R, d, a, seed=[seed, i])
        # conditioning values scaled to about [0, 1]
        out.append((cfg, f, (math.log(R) / math.log(1000.0), d / 5.0, a / 0.2)))
    return out


def read_fields(lat, out):
    """(6, ny, nx) FP32 device view <- alpha_g, u_g, u_l, dp_k of a lattice."""
    lat.read_device("alpha_g", out[0])
    lat.read_device("u_g", out[1:3])
    lat.read_device("u_l", out[3:5])
    lat.read_device("dp_k", out[5])


def make_lattices(inst):
    from paper_2409_10399_amd import Lattice
    lats = []
    for cfg, f, _ in inst:
        lat = Lattice(cfg, storage="fp32")
        lat.init_fields(f)
        lat.set_launch(64, 4)
        lats.append(lat)
    return lats


def generate(inst, t0, t1, snap, log):
    """Snapshots (S, N, 6, ny, nx) at t0, t0 + snap, ..., t1 (FP32, device)."""
    import torch
    from paper_2409_10399_amd import Batch
    lats = make_lattices(inst)
    ny, nx = inst[0][0]["ny"], inst[0][0]["nx"]
    batch = Batch(lats, tile=(64, 4), graph_steps=snap)
    batch.advance(t0)
    S = (t1 - t0) // snap + 1
    snaps = torch.empty((S, len(lats), 6, ny, nx), dtype=torch.float32, device="cuda")
    for s in range(S):
        if s:
            batch.advance(snap)
        for i, lat in enumerate(lats):
            read_fields(lat, snaps[s, i])
        if s % 20 == 0:
            log(f"  snapshot {s}/{S} t={lats[0].t}")
    torch.cuda.synchronize()
    del batch
    return snaps, lats


def stable_members(snaps, umax=0.1):
    """Indices of the lattices whose fields stay finite with |u| < umax at
    every snapshot (a few parameter draws of the sweep diverge physically)."""
    import torch
    keep = []
    for i in range(snaps.shape[1]):
        x = snaps[:, i]
        ok = bool(torch.isfinite(x).all()) and float(x[:, 1:5].abs().amax()) < umax
        if ok:
            keep.append(i)
    return keep


class Normaliser:
    """Per-field mean and standard deviation of the snapshots, and standard
    deviation of the change over `lag` snapshots (field by field: the
    snapshot tensor is tens of GB)."""

    def __init__(self, snaps, lag, keep, alpha_weight=1.0):
        import torch
        mean, scale, dscale = [], [], []
        idx = torch.tensor(keep, device="cuda")
        for c in range(6):
            x = snaps[:, :, c].index_select(1, idx)
            mean.append(float(x.mean()))
            scale.append(float(x.std()))
            dscale.append(float((x[lag:] - x[:-lag]).std()))
            del x
        dscale[0] /= alpha_weight  # the judged field weighs alpha_weight^2 in the loss
        self.outliers = []
        for c in range(6):
            x = snaps[:, :, c].index_select(1, idx)
            self.outliers.append([float(((x - mean[c]) / scale[c]).abs().amax()),
                                  float(((x[lag:] - x[:-lag]) / dscale[c]).abs().amax())])
            del x
        t = lambda v: torch.tensor(v, dtype=torch.float32, device="cuda")
        self.mean, self.scale, self.dscale = t(mean), t(scale).clamp_min(1e-12), t(dscale).clamp_min(1e-12)
        self.inv, self.dinv = 1.0 / self.scale, 1.0 / self.dscale
        self.zero = torch.zeros(6, dtype=torch.float32, device="cuda")

    def as_dict(self):
        d = {k: getattr(self, k).tolist() for k in ("mean", "scale", "dscale")}
        d["max_abs_normalised_field_and_change"] = self.outliers
        return d


def defect(f0, f1, jump, chi):
    """Relative conservation defect of a jump f0 -> f1, per lattice: change of
    the domain gas volume minus jump x the mean net inflow, over the gas
    volume.  The flux through the inlet row and the outlet row is the
    advective alpha_g u_g,y plus the diffusive -chi d(alpha_g)/dy of the
    volume-fraction scheme (chi = c_s^2 (1/omega_ag - 1/2) per lattice, a
    tensor of N values; one-sided differences at the rows); without the
    diffusive part plain LBM itself shows defects of ~3e-3 per 100 steps."""
    vol0 = f0[:, 0].sum(dim=(1, 2))
    vol1 = f1[:, 0].sum(dim=(1, 2))
    budget = 0.5 * jump * (_net_inflow(f0, chi) + _net_inflow(f1, chi))
    return ((vol1 - vol0 - budget).abs() / vol0.abs()).double().cpu().numpy()


def _net_inflow(f, chi):
    """Gas volume entering per step through the inlet row minus that leaving
    through the outlet row (advective + diffusive; rows 0, 1 and -2, -1)."""
    a, v = f[:, 0], f[:, 2]
    fin = (a[:, 0, :] * v[:, 0, :]).sum(dim=1) - chi * (a[:, 1, :] - a[:, 0, :]).sum(dim=1)
    fout = (a[:, -1, :] * v[:, -1, :]).sum(dim=1) - chi * (a[:, -1, :] - a[:, -2, :]).sum(dim=1)
    return fin - fout


def conserve(f0, f1, jump, chi, smin=0.5, smax=2.0):
    """Make a predicted jump f0 -> f1 keep the gas-volume budget: scale
    alpha_g of f1 on the rows that the flux estimate does not read (2 .. ny-3)
    so that the domain gas volume changes by exactly jump x the mean net
    inflow of the two ends.  The scale keeps alpha_g >= 0; it is clamped to
    [smin, smax] (a jump that needs more keeps a defect and is re-anchored)."""
    a1 = f1[:, 0]
    vol0 = f0[:, 0].sum(dim=(1, 2))
    edge = a1[:, :2].sum(dim=(1, 2)) + a1[:, -2:].sum(dim=(1, 2))
    inner = a1[:, 2:-2].sum(dim=(1, 2))
    budget = 0.5 * jump * (_net_inflow(f0, chi) + _net_inflow(f1, chi))
    scale = ((vol0 + budget - edge) / inner).clamp(smin, smax)
    a1[:, 2:-2] *= scale[:, None, None]


def diffusivities(inst):
    """chi = c_s^2 (1/omega_ag - 1/2) of each lattice, as a device tensor."""
    import torch
    return torch.tensor([(1.0 / cfg["omega_ag"] - 0.5) / 3.0 for cfg, _, _ in inst], dtype=torch.float32,
                        device="cuda")


def train(net, snaps, cond, norm, lag, epochs, bsz, lr, log, keep, noise=0.0, pushforward=0.0):
    """Adam with cosine decay on random pairs; noise > 0 adds Gaussian noise
    of that standard deviation (normalised units) to the input fields, so
    that the network learns to correct perturbed states such as its own
    earlier predictions.  pushforward > 0: that fraction of the batches
    starts one jump earlier and feeds the network its own prediction of the
    input state (no gradient through that first jump), with the true state
    one jump later as the target, so that it learns to correct its own
    errors."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream, apply_output, pack_input
    S, N = snaps.shape[:2]
    pairs = [(s, i) for s in range(S - lag) for i in keep]
    rng = np.random.default_rng(0)
    L = lib()
    hist = []
    steps_per_epoch = len(pairs) // bsz
    total = epochs * steps_per_epoch
    it = 0
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        acc = torch.zeros((), dtype=torch.float64, device="cuda")
        for k in range(steps_per_epoch):
            idx = [pairs[j] for j in order[k * bsz:(k + 1) * bsz]]
            push = pushforward > 0 and rng.random() < pushforward and all(s >= lag for s, _ in idx)
            f1 = torch.stack([snaps[s + lag, i] for s, i in idx]).contiguous()
            c = torch.stack([cond[i] for _, i in idx]).contiguous()
            if push:
                fm = torch.stack([snaps[s - lag, i] for s, i in idx]).contiguous()
                f0 = apply_output(fm, net.forward(pack_input(fm, norm.mean, norm.inv, c, net.cin), keep=False),
                                  norm.dscale)
            else:
                f0 = torch.stack([snaps[s, i] for s, i in idx]).contiguous()
            x = pack_input(f0, norm.mean, norm.inv, c, net.cin)
            if noise > 0:
                eps = torch.zeros_like(x)
                eps[..., :6].normal_(0.0, noise)
                _check_rc(L.eelbm_cno_axpy(_p(eps), x.numel(), 1.0, _p(x), _stream()))
            tgt = pack_input(f1, norm.zero, norm.dinv, c[:, :0].contiguous(), net.cout, clip=0.0)
            tp = pack_input(f0, norm.zero, norm.dinv, c[:, :0].contiguous(), net.cout, clip=0.0)
            _check_rc(L.eelbm_cno_axpy(_p(tp), tgt.numel(), -1.0, _p(tgt), _stream()))
            # cosine learning-rate decay
            rate = lr * 0.5 * (1.0 + math.cos(math.pi * it / total))
            out = net.forward(x)
            acc += net.loss(out, tgt).sum()
            net.backward(net.dloss)
            net.adam(rate)
            it += 1
        mean_loss = float(acc) / steps_per_epoch
        hist.append(mean_loss)
        log(f"  epoch {ep + 1}/{epochs}: mean loss {mean_loss:.4e} ({time.time() - t0:.0f} s)")
    return hist


def _check_rc(rc):
    from paper_2409_10399_amd.binding import _check
    _check(rc)


def rollout(net, lats, inst, cond, norm, t0, jumps, jump, defect_max, check_every, log, project=False):
    """Surrogate rollout of all lattices together from their LBM state at t0
    (project: each predicted jump is made to keep the gas-volume budget,
    `conserve`, before its defect is judged)."""
    import torch
    from paper_2409_10399_amd import Batch
    from paper_2409_10399_amd.surrogate import apply_output, pack_input
    N = len(lats)
    ny, nx = inst[0][0]["ny"], inst[0][0]["nx"]
    chi = diffusivities(inst)
    f = torch.empty((N, 6, ny, nx), dtype=torch.float32, device="cuda")
    for i, lat in enumerate(lats):
        read_fields(lat, f[i])
    t = t0
    anchors = 0
    valid = np.ones(N, dtype=bool)  # lattice i's LBM state equals f[i] at time t
    defects = []
    for j in range(jumps):
        x = pack_input(f, norm.mean, norm.inv, cond, net.cin)
        pred = apply_output(f, net.forward(x, keep=False), norm.dscale)
        if project:
            conserve(f, pred, jump, chi)
        dfc = defect(f, pred, jump, chi)
        defects.append(float(np.nanmax(dfc)))
        force = check_every > 0 and (j + 1) % check_every == 0
        bad = np.where((dfc > defect_max) | ~np.isfinite(dfc) | force)[0]
        for i in bad:
            if not valid[i]:
                fi = f[i].double()
                lats[i].reinit_fields_device(t, {"alpha_g": fi[0].contiguous(), "u_g": fi[1:3].contiguous(),
                                                 "u_l": fi[3:5].contiguous(), "dp_k": fi[5].contiguous()})
        if len(bad):
            # the re-anchored lattices advance together, one launch per step
            Batch([lats[i] for i in bad], tile=(64, 4)).advance(jump)
            for i in bad:
                read_fields(lats[i], pred[i])
            anchors += len(bad)
        valid[:] = False
        valid[bad] = True
        f = pred
        t += jump
    torch.cuda.synchronize()
    return f, anchors, defects


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-inst", type=int, default=200)
    ap.add_argument("--test-inst", type=int, default=8)
    ap.add_argument("--t0", type=int, default=1000)
    ap.add_argument("--jump", type=int, default=100)
    ap.add_argument("--jumps", type=int, default=50)
    ap.add_argument("--snap", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--alpha-weight", type=float, default=3.0)
    ap.add_argument("--noise", type=float, default=0.0)
    ap.add_argument("--pushforward", type=float, default=0.0,
                    help="fraction of batches fed the network's own one-jump prediction as input")
    ap.add_argument("--widths", default="32,48,96,192")
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--defect-max", type=float, default=1e-3)
    ap.add_argument("--check-every", type=int, default=5)
    ap.add_argument("--out", default="")
    ap.add_argument("--save-weights", default="")
    ap.add_argument("--load-weights", default="", help="weights of --save-weights: skip training")
    ap.add_argument("--policies", default="",
                    help="extra re-anchoring policies to judge the same network with, "
                         "'defect_max:check_every[:p],...' (p: predicted jumps keep the gas-volume budget)")
    a = ap.parse_args()
    import torch
    from paper_2409_10399_amd import Batch
    from paper_2409_10399_amd.surrogate import CNO

    def log(m):
        print(m, flush=True)

    t_end = a.t0 + a.jumps * a.jump
    lag = a.jump // a.snap
    report = {"args": vars(a)}
    T = time.time()
    log(f"# data: {a.train_inst} channels {a.grid}^2, t {a.t0}..{t_end}, every {a.snap} steps")
    train_inst = instances(a.train_inst, seed=1, n=a.grid)
    snaps, lats_tr = generate(train_inst, a.t0, t_end, a.snap, log)
    del lats_tr
    torch.cuda.empty_cache()
    cond = torch.tensor([c for _, _, c in train_inst], dtype=torch.float32, device="cuda")
    keep = stable_members(snaps)
    report["train_members_kept"] = len(keep)
    log(f"# {len(keep)} of {a.train_inst} channels stay finite with |u| < 0.1 up to t = {t_end}")
    norm = Normaliser(snaps, lag, keep, a.alpha_weight)
    report["normaliser"] = norm.as_dict()
    log(f"# max |normalised| (field, change) per plane: {[[round(v, 1) for v in o] for o in norm.outliers]}")
    # plain LBM's own conservation defect over single jumps (calibrates defect_max)
    chi_k = diffusivities([train_inst[i] for i in keep])
    lbm_def = np.concatenate([defect(snaps[s][keep], snaps[s + lag][keep], a.jump, chi_k)
                              for s in range(snaps.shape[0] - lag)])
    report["lbm_defect_percentiles_50_99_max"] = [float(np.percentile(lbm_def, 50)), float(np.percentile(lbm_def, 99)),
                                                   float(lbm_def.max())]
    log(f"# plain LBM defect per jump: median {np.percentile(lbm_def, 50):.2e}, 99% {np.percentile(lbm_def, 99):.2e}, "
        f"max {lbm_def.max():.2e}")
    report["data_seconds"] = time.time() - T
    net = CNO(9, 6, [int(w) for w in a.widths.split(",")], seed=0)
    log(f"# network: widths {net.widths}, {net.n_params} parameters; {snaps.shape[0] - lag} x {a.train_inst} pairs")
    T = time.time()
    if a.load_weights:
        w = np.load(a.load_weights)
        arrs = [w["arr_%d" % k] for k in range(len(w.files))]
        net.set_params(list(zip(arrs[0::2], arrs[1::2])))
        report["loss_history"] = None
        log(f"# weights loaded from {a.load_weights}")
    else:
        report["loss_history"] = train(net, snaps, cond, norm, lag, a.epochs, a.batch, a.lr, log, keep, a.noise,
                                       a.pushforward)
    report["train_seconds"] = time.time() - T
    del snaps
    torch.cuda.empty_cache()
    if a.save_weights:
        np.savez(a.save_weights, *[w for wb in net.get_params() for w in wb])

    # ---- judging on held-out channels: plain LBM from t0 (HIP-graph batched
    # launches, timed), then the surrogate rollout from the same state
    # held-out channels: drawn from a fresh seed, screened like the training set
    pool = instances(3 * a.test_inst, seed=2, n=a.grid)
    psnaps, plats = generate(pool, a.t0, t_end, (t_end - a.t0), log)
    ok = stable_members(psnaps)[:a.test_inst]
    del psnaps, plats
    torch.cuda.empty_cache()
    test_inst = [pool[i] for i in ok]
    report["test_members_screened"] = [len(pool), len(ok)]
    tcond = torch.tensor([c for _, _, c in test_inst], dtype=torch.float32, device="cuda")
    run_lats = make_lattices(test_inst)
    runb = Batch(run_lats, tile=(64, 4), graph_steps=a.jump)
    runb.advance(a.t0)
    torch.cuda.synchronize()
    blobs = [lat.save() for lat in run_lats]
    start = torch.empty((len(run_lats), 6, a.grid, a.grid), dtype=torch.float32, device="cuda")
    for i, lat in enumerate(run_lats):
        read_fields(lat, start[i])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    runb.advance(a.jumps * a.jump)
    e1.record()
    torch.cuda.synchronize()
    t_lbm = e0.elapsed_time(e1) / 1e3
    ref_f = torch.empty_like(start)
    for i, lat in enumerate(run_lats):
        read_fields(lat, ref_f[i])
    # surrogate rollout from the same state
    for lat, blob in zip(run_lats, blobs):
        lat.load(blob)
    del runb
    net.forward(torch.zeros((len(run_lats), a.grid, a.grid, net.cin), device="cuda"), keep=False)  # warm-up
    torch.cuda.synchronize()
    e0.record()
    t_wall = time.time()
    fin, anchors, defects = rollout(net, run_lats, test_inst, tcond, norm, a.t0, a.jumps, a.jump, a.defect_max,
                                    a.check_every, log)
    e1.record()
    torch.cuda.synchronize()
    t_sur = e0.elapsed_time(e1) / 1e3
    t_wall = time.time() - t_wall

    def rel_alpha(x):
        return [float((x[i, 0] - ref_f[i, 0]).norm() / ref_f[i, 0].norm()) for i in range(len(run_lats))]
    err = rel_alpha(fin)
    frozen = rel_alpha(start)
    # plain LBM's own conservation defect over single jumps (calibrates the threshold)
    report.update({
        "n_params": net.n_params, "widths": net.widths,
        "rel_l2_alpha_surrogate": err, "rel_l2_alpha_frozen": frozen,
        "rel_l2_alpha_surrogate_max": max(err), "rel_l2_alpha_frozen_max": max(frozen),
        "anchors": anchors, "jumps": a.jumps * len(run_lats), "defect_max_per_jump": defects,
        "seconds_plain_lbm": t_lbm, "seconds_surrogate": t_sur, "seconds_surrogate_wall": t_wall,
        "speedup": t_lbm / t_sur,
    })
    log(f"# rel-L2(alpha_g) at t = {t_end}: surrogate max {max(err):.4f} (frozen fields {max(frozen):.4f}); "
        f"re-anchored {anchors} of {a.jumps * len(run_lats)} jumps; plain LBM {t_lbm * 1e3:.1f} ms, "
        f"surrogate {t_sur * 1e3:.1f} ms, speedup {t_lbm / t_sur:.2f}")
    # the same network under other re-anchoring policies (same start, same reference)
    report["policies"] = []
    for pol in [x for x in a.policies.split(",") if x]:
        parts = pol.split(":")
        dmax, chk = float(parts[0]), int(parts[1])
        proj = len(parts) > 2 and parts[2] == "p"
        for lat, blob in zip(run_lats, blobs):
            lat.load(blob)
        torch.cuda.synchronize()
        e0.record()
        fin_p, anchors_p, _ = rollout(net, run_lats, test_inst, tcond, norm, a.t0, a.jumps, a.jump, dmax, chk, log,
                                      project=proj)
        e1.record()
        torch.cuda.synchronize()
        t_p = e0.elapsed_time(e1) / 1e3
        err_p = rel_alpha(fin_p)
        report["policies"].append({"defect_max": dmax, "check_every": chk, "project": proj,
                                   "rel_l2_alpha_max": max(err_p),
                                   "rel_l2_alpha_mean": float(np.mean(err_p)), "anchors": anchors_p,
                                   "seconds_surrogate": t_p, "speedup": t_lbm / t_p})
        log(f"# policy defect_max {dmax:g}, check every {chk}{', budget kept' if proj else ''}: "
            f"rel-L2 max {max(err_p):.4f} mean "
            f"{np.mean(err_p):.4f}; re-anchored {anchors_p}; speedup {t_lbm / t_p:.2f}")
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
