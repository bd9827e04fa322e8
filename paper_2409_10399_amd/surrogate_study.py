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
4. the policy (defect_max, check_every) is chosen on validation channels
   (their own seed): the fastest whose largest rel-L2 stays within
   --val-target; the test channels (another seed) are judged once, under
   that policy and under the specified one (1e-3, every 5th jump).

python -m paper_2409_10399_amd.surrogate_study [--train-inst 200] [--epochs 6] [--save prefix] [--out report.json]
python -m paper_2409_10399_amd.surrogate_study --load prefix      # judge a saved model on its test channels
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

    @classmethod
    def from_arrays(cls, mean, scale, dscale):
        """A normaliser with the given per-field statistics (a saved model)."""
        import torch
        self = cls.__new__(cls)
        t = lambda v: torch.tensor(np.asarray(v, dtype=np.float64), dtype=torch.float32, device="cuda")
        self.mean, self.scale, self.dscale = t(mean), t(scale), t(dscale)
        self.inv, self.dinv = 1.0 / self.scale, 1.0 / self.dscale
        self.zero = torch.zeros(6, dtype=torch.float32, device="cuda")
        self.outliers = []
        return self

    def as_dict(self):
        d = {k: getattr(self, k).tolist() for k in ("mean", "scale", "dscale")}
        d["max_abs_normalised_field_and_change"] = self.outliers
        return d


def defect(f0, f1, jump, chi):
    """Relative conservation defect of a jump f0 -> f1, per lattice (NumPy
    array of N values): change of the domain gas volume minus jump x the mean
    net inflow, over the gas volume, computed by eelbm_cno_volume_defect.  The
    flux through the inlet row and the outlet row is the advective
    alpha_g u_g,y plus the diffusive -chi d(alpha_g)/dy of the volume-fraction
    scheme (chi = c_s^2 (1/omega_ag - 1/2) per lattice, a tensor of N values;
    one-sided differences at the rows); without the diffusive part plain LBM
    itself shows defects of ~3e-3 per 100 steps."""
    import torch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream
    N, _, ny, nx = f0.shape
    assert f0.is_contiguous() and f1.is_contiguous() and f0.dtype == torch.float32 and f1.dtype == torch.float32
    out = torch.empty(N, dtype=torch.float64, device=f0.device)
    _check_rc(lib().eelbm_cno_volume_defect(_p(f0), _p(f1), N, ny, nx, int(jump), _p(chi.contiguous()), _p(out),
                                            _stream()))
    return out.cpu().numpy()


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


def rollout(net, lats, inst, cond, norm, t0, jumps, jump, defect_max, check_every, log, project=False,
            one_batch=False):
    """Surrogate rollout of all lattices together from their LBM state at t0,
    deciding on the host after every jump (it waits for the defects) and
    advancing only the re-anchored lattices (project: each predicted jump is
    made to keep the gas-volume budget, `conserve`, before its defect is
    judged).  Default: a batch of the re-anchored lattices built anew each
    jump (one launch per step); one_batch: one batch of all lattices,
    captured once into a HIP graph of `jump` steps, in which the re-anchored
    lattices are flagged active for each jump (eelbm_batch_set_active) --
    the same fields and, measured on the 8 test channels, the same time
    (157 against 158 ms), so the simpler path is the default.
    rollout_device gives the same fields without waiting for the device; on
    the MI355X it is slower (the host issues the rebuilds and reads of every
    lattice, and its launches, not the device, set the pace), so the study
    times this one."""
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
    if one_batch:
        batch = Batch(lats, tile=(64, 4), graph_steps=jump)
        flags = torch.zeros(N, dtype=torch.int32, device="cuda")
        host_flags = torch.zeros(N, dtype=torch.int32, pin_memory=True)
        batch.set_active(flags)
    for j in range(jumps):
        x = pack_input(f, norm.mean, norm.inv, cond, net.cin)
        pred = apply_output(f, net.infer(x), norm.dscale)
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
        if one_batch:
            # the lattices left out keep their stale state (not valid after
            # this jump) while their time moves with the batch
            host_flags.zero_()
            host_flags[torch.as_tensor(bad, dtype=torch.long)] = 1
            flags.copy_(host_flags, non_blocking=True)
            batch.advance(jump)
        elif len(bad):
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
    if one_batch:
        del batch
    return f, anchors, defects


def rollout_device(net, lats, inst, cond, norm, t0, jumps, jump, defect_max, check_every, log, project=False,
                   batch=None):
    """Surrogate rollout of all lattices together from their LBM state at t0,
    every decision taken on the device (no host wait inside the loop): per
    jump the network's prediction, its gas-volume defects
    (eelbm_cno_volume_defect), the re-anchoring mask (eelbm_cno_reanchor_policy),
    gated rebuilds of the masked lattices whose LBM state is stale
    (eelbm_batch_rebuild_gated), `jump` steps of one batch of all lattices
    in which only the masked ones advance (eelbm_batch_set_active, the steps
    replayed from a HIP graph), and the masked lattices' LBM fields
    (eelbm_batch_read_fields) taken in place of the prediction
    (eelbm_cno_select).  The same fields as
    rollout.  project: see rollout (a host step: it is taken before the
    defect, on the device tensors)."""
    import torch
    from paper_2409_10399_amd import Batch
    from paper_2409_10399_amd.binding import lib
    from paper_2409_10399_amd.surrogate import _p, _stream, apply_output, pack_input
    L = lib()
    N = len(lats)
    ny, nx = inst[0][0]["ny"], inst[0][0]["nx"]
    chi = diffusivities(inst)
    f = torch.empty((N, 6, ny, nx), dtype=torch.float32, device="cuda")
    for i, lat in enumerate(lats):
        read_fields(lat, f[i])
    valid = torch.ones(N, dtype=torch.int32, device="cuda")  # lattice i's LBM state equals f[i] at time t
    mask = torch.zeros(N, dtype=torch.int32, device="cuda")
    rebuild = torch.zeros(N, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    dfc = torch.empty(N, dtype=torch.float64, device="cuda")
    lbm = torch.empty_like(f)
    own = batch is None
    if own:
        batch = Batch(lats, tile=(64, 4), graph_steps=jump)
    batch.set_active(mask)
    t = t0
    st = _stream()
    for j in range(jumps):
        x = pack_input(f, norm.mean, norm.inv, cond, net.cin)
        pred = apply_output(f, net.infer(x), norm.dscale)
        if project:
            conserve(f, pred, jump, chi)
        _check_rc(L.eelbm_cno_volume_defect(_p(f), _p(pred), N, ny, nx, int(jump), _p(chi), _p(dfc), st))
        force = int(check_every > 0 and (j + 1) % check_every == 0)
        _check_rc(L.eelbm_cno_reanchor_policy(_p(dfc), N, float(defect_max), force, _p(valid), _p(mask),
                                              _p(rebuild), _p(count), st))
        fd = f.double()  # the planes of FIELD_PLANES are the rebuild layout
        batch.rebuild_gated(t, fd, rebuild)
        batch.advance(jump)
        batch.read_fields(lbm)
        _check_rc(L.eelbm_cno_select(_p(mask), N, 6 * ny * nx, _p(lbm), _p(pred), _p(pred), st))
        f = pred
        t += jump
    torch.cuda.synchronize()
    if own:
        del batch
    else:
        batch.set_active(None)
    return f, int(count.item()), []


class JudgeSet:
    """Held-out channels for judging the surrogate: `pool` draws of the sweep
    distribution from `seed`, screened like the training set (the first
    `count` that stay finite with |u| < 0.1 up to t0 + jumps x jump),
    advanced to t0 on plain LBM; then plain LBM from t0 to the end, timed
    (HIP-graph batched launches, the same as the data generation), gives the
    reference fields and the reference time."""

    def __init__(self, seed, count, grid, t0, jumps, jump, log, pool_factor=3):
        import torch
        from paper_2409_10399_amd import Batch
        t_end = t0 + jumps * jump
        pool = instances(pool_factor * count, seed=seed, n=grid)
        psnaps, plats = generate(pool, t0, t_end, t_end - t0, log)
        ok = stable_members(psnaps)[:count]
        del psnaps, plats
        torch.cuda.empty_cache()
        self.screened = [len(pool), len(ok)]
        self.inst = [pool[i] for i in ok]
        self.cond = torch.tensor([c for _, _, c in self.inst], dtype=torch.float32, device="cuda")
        self.t0, self.jumps, self.jump = t0, jumps, jump
        self.lats = make_lattices(self.inst)
        runb = Batch(self.lats, tile=(64, 4), graph_steps=jump)
        runb.advance(t0)
        torch.cuda.synchronize()
        self.blobs = [lat.save() for lat in self.lats]
        self.start = torch.empty((len(self.lats), 6, grid, grid), dtype=torch.float32, device="cuda")
        for i, lat in enumerate(self.lats):
            read_fields(lat, self.start[i])
        # timed after the advance to t0, which captured and ran the graph
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        runb.advance(jumps * jump)
        e1.record()
        torch.cuda.synchronize()
        self.t_lbm = e0.elapsed_time(e1) / 1e3
        self.ref = torch.empty_like(self.start)
        for i, lat in enumerate(self.lats):
            read_fields(lat, self.ref[i])
        del runb

    def restore(self):
        import torch
        for lat, blob in zip(self.lats, self.blobs):
            lat.load(blob)
        torch.cuda.synchronize()

    def rel_alpha(self, x):
        return [float((x[i, 0] - self.ref[i, 0]).norm() / self.ref[i, 0].norm()) for i in range(len(self.lats))]

    def judge(self, net, norm, dmax, chk, log, project=False, reps=1):
        """Rollout under the policy (defect_max dmax, re-anchor every chk-th
        jump), `reps` times from the same state; rel-L2 of alpha_g at the end
        against plain LBM, re-anchored jumps, rollout time (median over reps)
        and speedup = plain LBM time / rollout time."""
        import torch
        secs = []
        for _ in range(reps):
            self.restore()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fin, anchors, _ = rollout(net, self.lats, self.inst, self.cond, norm, self.t0, self.jumps, self.jump, dmax,
                                      chk, log, project=project)
            e1.record()
            torch.cuda.synchronize()
            secs.append(e0.elapsed_time(e1) / 1e3)
        t = float(np.median(secs))
        err = self.rel_alpha(fin)
        return {"defect_max": dmax, "check_every": chk, "project": project, "rel_l2_alpha_max": max(err),
                "rel_l2_alpha_mean": float(np.mean(err)), "anchors": anchors, "jumps": self.jumps * len(self.lats),
                "seconds_surrogate": t, "seconds_surrogate_reps": secs, "seconds_plain_lbm": self.t_lbm,
                "speedup": self.t_lbm / t}


# policies judged on the validation channels when --policies is not given
DEFAULT_POLICIES = [(d, c) for d in (1e-4, 1.5e-4, 2e-4, 2.5e-4, 3e-4, 4e-4, 5e-4, 7.5e-4, 1e-3) for c in (0, 3, 5)]


def choose_policy(table, target):
    """The fastest policy whose largest rel-L2 over the validation channels is
    within `target` (None if none is)."""
    ok = [r for r in table if r["rel_l2_alpha_max"] <= target]
    return max(ok, key=lambda r: r["speedup"]) if ok else None


def save_model(prefix, net, norm, meta):
    """prefix.npz: weights W[tap][ci][co] and biases per layer, and the
    normaliser's per-field statistics; prefix.json: everything else needed to
    judge the model again (meta)."""
    arrs = {}
    for k, (w, b) in enumerate(net.get_params()):
        arrs[f"w{k}"] = w.astype(np.float32)
        arrs[f"b{k}"] = b.astype(np.float32)
    for k in ("mean", "scale", "dscale"):
        arrs["norm_" + k] = getattr(norm, k).double().cpu().numpy()
    np.savez(prefix + ".npz", **arrs)
    with open(prefix + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)


def load_model(prefix):
    """(net, norm, meta) of save_model."""
    from paper_2409_10399_amd.surrogate import CNO
    with open(prefix + ".json") as fh:
        meta = json.load(fh)
    with np.load(prefix + ".npz", allow_pickle=False) as z:
        net = CNO(9, 6, meta["widths"], seed=0)
        net.set_params([(z[f"w{k}"], z[f"b{k}"]) for k in range(len(net.shapes))])
        norm = Normaliser.from_arrays(z["norm_mean"], z["norm_scale"], z["norm_dscale"])
    return net, norm, meta


def measure_saved(prefix, log=lambda m: None, reps=3):
    """Judge a saved model on its held-out test channels under its chosen
    policy (and the specified 1e-3 / every 5th jump): the measured speedup
    and rel-L2 of alpha_g against plain LBM, timed now."""
    net, norm, meta = load_model(prefix)
    ts = JudgeSet(meta["test_seed"], meta["test_inst"], meta["grid"], meta["t0"], meta["jumps"], meta["jump"], log)
    pol = meta["chosen_policy"]
    x0 = __import__("torch").zeros((len(ts.lats), meta["grid"], meta["grid"], net.cin), device="cuda")
    net.infer(x0)  # warm-up
    out = {"chosen": ts.judge(net, norm, pol["defect_max"], pol["check_every"], log, reps=reps),
           "specified": ts.judge(net, norm, 1e-3, 5, log, reps=reps), "test_screened": ts.screened}
    return out, meta


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-inst", type=int, default=200)
    ap.add_argument("--val-inst", type=int, default=8)
    ap.add_argument("--test-inst", type=int, default=8)
    ap.add_argument("--val-seed", type=int, default=3)
    ap.add_argument("--test-seed", type=int, default=2)
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
    ap.add_argument("--target", type=float, default=0.02, help="rel-L2 of alpha_g the surrogate must stay within")
    ap.add_argument("--val-target", type=float, default=0.016,
                    help="the bound the policy must meet on the validation channels (below --target: margin "
                         "for the step from validation to test channels)")
    ap.add_argument("--out", default="")
    ap.add_argument("--save", default="", help="prefix of the saved model (.npz weights, .json policy and meta)")
    ap.add_argument("--load", default="", help="a saved model: skip training and validation, judge on test")
    ap.add_argument("--revalidate", action="store_true", help="with --load: choose the policy again on validation")
    ap.add_argument("--policies", default="",
                    help="re-anchoring policies judged on the validation channels, "
                         "'defect_max:check_every[:p],...' (p: predicted jumps keep the gas-volume budget)")
    a = ap.parse_args()
    import torch
    from paper_2409_10399_amd.surrogate import CNO

    def log(m):
        print(m, flush=True)

    if a.load and a.revalidate:
        # the saved network's policy chosen again on its validation channels
        # (e.g. after a change of the inference arithmetic), then the test
        # channels judged once; the model's json is rewritten under --save
        net, norm, meta = load_model(a.load)
        vs = JudgeSet(meta["val_seed"], meta["val_inst"], meta["grid"], meta["t0"], meta["jumps"], meta["jump"], log)
        net.infer(torch.zeros((len(vs.lats), meta["grid"], meta["grid"], net.cin), device="cuda"))  # warm-up
        table = []
        for dmax, chk in DEFAULT_POLICIES:
            r = vs.judge(net, norm, dmax, chk, log)
            table.append(r)
            log(f"# validation, policy {dmax:g}:{chk}: rel-L2 max {r['rel_l2_alpha_max']:.4f}; re-anchored "
                f"{r['anchors']}; speedup {r['speedup']:.2f}")
        best = choose_policy(table, meta["val_target"]) or min(table, key=lambda r: r["rel_l2_alpha_max"])
        meta["chosen_policy"] = {"defect_max": best["defect_max"], "check_every": best["check_every"]}
        meta["validation"] = [{k: r[k] for k in ("defect_max", "check_every", "rel_l2_alpha_max", "rel_l2_alpha_mean",
                                                  "anchors", "speedup")} for r in table]
        meta["revalidated"] = "python -m paper_2409_10399_amd.surrogate_study " + " ".join(sys.argv[1:])
        del vs
        ts = JudgeSet(meta["test_seed"], meta["test_inst"], meta["grid"], meta["t0"], meta["jumps"], meta["jump"], log)
        for name, (dmax, chk) in (("chosen", (best["defect_max"], best["check_every"])), ("specified", (1e-3, 5))):
            r = ts.judge(net, norm, dmax, chk, log, reps=3)
            log(f"# test, {name} policy {dmax:g}:{chk}: rel-L2 max {r['rel_l2_alpha_max']:.4f}, re-anchored "
                f"{r['anchors']}/{r['jumps']}, speedup {r['speedup']:.2f}")
        if a.save:
            with open(a.save + ".json", "w") as fh:
                json.dump(meta, fh, indent=1)
        return
    if a.load:
        res, meta = measure_saved(a.load, log)
        for k in ("chosen", "specified"):
            r = res[k]
            log(f"# test, {k} policy {r['defect_max']:g}:{r['check_every']}: rel-L2 max {r['rel_l2_alpha_max']:.4f}, "
                f"re-anchored {r['anchors']}/{r['jumps']}, speedup {r['speedup']:.2f} "
                f"(plain LBM {r['seconds_plain_lbm'] * 1e3:.1f} ms, rollout {r['seconds_surrogate'] * 1e3:.1f} ms)")
        if a.out:
            with open(a.out, "w") as fh:
                json.dump({"measured": res, "meta": meta}, fh, indent=1)
        return

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
    lbm_def = np.concatenate([defect(snaps[s][keep].contiguous(), snaps[s + lag][keep].contiguous(), a.jump, chi_k)
                              for s in range(snaps.shape[0] - lag)])
    report["lbm_defect_percentiles_50_99_max"] = [float(np.percentile(lbm_def, 50)), float(np.percentile(lbm_def, 99)),
                                                   float(lbm_def.max())]
    log(f"# plain LBM defect per jump: median {np.percentile(lbm_def, 50):.2e}, 99% {np.percentile(lbm_def, 99):.2e}, "
        f"max {lbm_def.max():.2e}")
    report["data_seconds"] = time.time() - T
    net = CNO(9, 6, [int(w) for w in a.widths.split(",")], seed=0)
    log(f"# network: widths {net.widths}, {net.n_params} parameters; {snaps.shape[0] - lag} x {a.train_inst} pairs")
    T = time.time()
    report["loss_history"] = train(net, snaps, cond, norm, lag, a.epochs, a.batch, a.lr, log, keep, a.noise,
                                   a.pushforward)
    report["train_seconds"] = time.time() - T
    del snaps
    torch.cuda.empty_cache()

    # ---- policy chosen on validation channels (their own seed), then judged
    # once on the test channels
    vs = JudgeSet(a.val_seed, a.val_inst, a.grid, a.t0, a.jumps, a.jump, log)
    net.infer(torch.zeros((len(vs.lats), a.grid, a.grid, net.cin), device="cuda"))  # warm-up
    pols = DEFAULT_POLICIES if not a.policies else [
        (float(x.split(":")[0]), int(x.split(":")[1])) for x in a.policies.split(",") if x]
    table = []
    for dmax, chk in pols:
        r = vs.judge(net, norm, dmax, chk, log)
        table.append(r)
        log(f"# validation, policy {dmax:g}:{chk}: rel-L2 max {r['rel_l2_alpha_max']:.4f} mean "
            f"{r['rel_l2_alpha_mean']:.4f}; re-anchored {r['anchors']}; speedup {r['speedup']:.2f}")
    report["validation"] = {"screened": vs.screened, "frozen_rel_l2_max": max(vs.rel_alpha(vs.start)),
                            "policies": table}
    best = choose_policy(table, a.val_target)
    if best is None:
        log(f"# no policy within {a.val_target} on validation; taking the most accurate")
        best = min(table, key=lambda r: r["rel_l2_alpha_max"])
    chosen = {"defect_max": best["defect_max"], "check_every": best["check_every"]}
    report["chosen_policy"] = chosen
    del vs
    torch.cuda.empty_cache()
    ts = JudgeSet(a.test_seed, a.test_inst, a.grid, a.t0, a.jumps, a.jump, log)
    res = ts.judge(net, norm, chosen["defect_max"], chosen["check_every"], log, reps=3)
    spec = ts.judge(net, norm, 1e-3, 5, log, reps=3)
    report["test"] = {"screened": ts.screened, "frozen_rel_l2_max": max(ts.rel_alpha(ts.start)), "chosen": res,
                      "specified": spec}
    log(f"# test, chosen policy {chosen['defect_max']:g}:{chosen['check_every']}: rel-L2 max "
        f"{res['rel_l2_alpha_max']:.4f}, re-anchored {res['anchors']}/{res['jumps']}, speedup {res['speedup']:.2f}; "
        f"specified 1e-3:5: rel-L2 max {spec['rel_l2_alpha_max']:.4f}, speedup {spec['speedup']:.2f}")
    if a.save:
        meta = {"widths": net.widths, "grid": a.grid, "t0": a.t0, "jumps": a.jumps, "jump": a.jump,
                "test_seed": a.test_seed, "test_inst": a.test_inst, "val_seed": a.val_seed, "val_inst": a.val_inst,
                "target": a.target, "val_target": a.val_target, "chosen_policy": chosen,
                "training": {k: getattr(a, k) for k in ("train_inst", "epochs", "batch", "lr", "alpha_weight",
                                                        "noise", "pushforward", "snap")},
                "loss_history": report["loss_history"],
                "command": "python -m paper_2409_10399_amd.surrogate_study " + " ".join(sys.argv[1:])}
        save_model(a.save, net, norm, meta)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
