"""Batched lattices: one launch per step over the tiles of every member, also
replayed from captured HIP graphs, must give every member exactly the fields
it gets when advanced on its own (each node is computed by one thread from the
same inputs in the same order); one member is checked against the oracle.
The autotuner must leave the state untouched."""
import numpy as np
import pytest

import workloads
from parity import FIELDS, check, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


def members(storage="fp32"):
    """Five uneven channels of the sweep (ragged sizes, R from 2 to 900)."""
    spec = [(64, 40, 900.0, 3.0, 0.05), (130, 70, 2.0, 1.0, 0.2), (70, 129, 37.0, 5.0, 0.02),
            (200, 64, 150.0, 2.0, 0.1), (96, 96, 8.0, 4.0, 0.15)]
    return [workloads.sweep_channel_2d(nx, ny, R, d, a, seed=i, n_ramp=30.0)
            for i, (nx, ny, R, d, a) in enumerate(spec)]


def _lattices(ws, storage):
    from paper_2409_10399_amd import Lattice
    out = []
    for cfg, f in ws:
        lat = Lattice(cfg, storage=storage)
        lat.init_fields(f)
        out.append(lat)
    return out


def members_3d():
    """Three uneven D3Q19 channels (walls on x and y, inlet z = 0)."""
    out = []
    for i, (nx, ny, nz) in enumerate([(70, 9, 12), (130, 6, 8), (40, 12, 10)]):
        cfg = workloads._base("D3Q19", nx=nx, ny=ny, nz=nz, rho_l=100.0, drag="cgw", kappa_I=1e-3,
                              g_hat=1e-6 / 99.0, up_axis=2, gamma=1.0, n_gamma=4,
                              bc={"x-": "wall", "x+": "wall", "y-": "wall", "y+": "wall", "z-": "inlet",
                                  "z+": "outlet"},
                              alpha_in_max=0.1, alpha_in_min=0.01, ug_in_max=3e-3, ug_in_min=3e-4,
                              ul_in_max=5e-4, ul_in_min=0.0, n_ramp=20.0)
        f = workloads.smooth_random_3d(max(nx, ny, nz), seed=30 + i, alpha0=0.05, amp_a=0.02)
        f = {k: np.ascontiguousarray(v[..., :nz, :ny, :nx]) for k, v in f.items()}
        f["inlet_noise"] = 1.0 + 0.1 * np.random.default_rng(40 + i).uniform(-1, 1, (ny, nx))
        out.append((cfg, f))
    return out


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16", "fp64"])
@pytest.mark.parametrize("graph_steps", [0, 8])
def test_batch_equals_members_alone(graph_steps, storage):
    from paper_2409_10399_amd import Batch
    ws = members()
    alone = _lattices(ws, storage)
    batched = _lattices(ws, storage)
    batch = Batch(batched, tile=(64, 4), graph_steps=graph_steps)
    # several advances (graph replays, remainders), with reads in between
    for n in (8, 3, 16, 5):
        batch.advance(n)
        for lat in alone:
            lat.set_launch(64, 4)
            lat.advance(n)
        for a, b in zip(alone, batched):
            assert a.t == b.t
            for k in FIELDS:
                assert np.array_equal(a.read(k), b.read(k)), (graph_steps, n, k)
            da, db = a.diag(), b.diag()
            assert da["nonfinite"] == 0 and db["nonfinite"] == 0
            assert abs(da["alpha_g"] - db["alpha_g"]) < 1e-9


def reversed_channel():
    """A small D2Q9 channel with the flow along -x (outlet at x = 0, inlet at
    the last column, walls on y): not the standard column, so its steps take
    the step instantiation that reads the boundary types at run time."""
    cfg = workloads._base("D2Q9", nx=30, ny=20, rho_l=20.0, drag="cgw", kappa_I=2e-3, g_hat=1e-6, up_axis=0,
                          gamma=1.0, n_gamma=5, bc={"x-": "outlet", "x+": "inlet", "y-": "wall", "y+": "wall"},
                          alpha_in_max=0.2, alpha_in_min=0.02, ug_in_max=4e-3, ug_in_min=4e-4, ul_in_max=1e-3,
                          ul_in_min=1e-4, n_ramp=30.0)
    f = workloads.smooth_random_2d(30, 20, seed=12, alpha0=0.1, amp_a=0.05)
    f["inlet_noise"] = 1.0 + 0.1 * np.random.default_rng(3).uniform(-1, 1, 20)
    return cfg, f


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16", "bf16", "fp32x", "mixed"])
@pytest.mark.parametrize("dim", [2, 3])
def test_trajectory_does_not_depend_on_read_outs(dim, storage):
    """A step that also writes the read-out fields (the last step of every
    advance) must leave the same state as one that does not: 27 steps in one
    advance and 19 + 8 with a read in between end bit-identical.  (Found with
    FP64 storage on the R = 2 channel, where the two step variants once fused
    multiplies and adds differently and ended 3e-20 apart after 27 steps.)"""
    ws = members() if dim == 2 else members_3d()
    a, b = _lattices(ws, storage), _lattices(ws, storage)
    for lat in a:
        lat.advance(27)
    for lat in b:
        lat.advance(19)
        lat.read("u_g")
        lat.advance(8)
    for x, y in zip(a, b):
        for k in FIELDS:
            assert np.array_equal(x.read(k), y.read(k)), (storage, k)


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_batch_of_mixed_boundary_layouts(storage):
    # standard columns batched with a reversed channel: the batch runs the
    # run-time boundary instantiation for every member, the members alone
    # run their own (compile-time column / run-time), and in 2D the two give
    # the same bits
    from paper_2409_10399_amd import Batch
    ws = members()[:3] + [reversed_channel()]
    alone = _lattices(ws, storage)
    batched = _lattices(ws, storage)
    batch = Batch(batched, tile=(64, 4))
    for n in (7, 12):
        batch.advance(n)
        for lat in alone:
            lat.set_launch(64, 4)
            lat.advance(n)
        for i, (a, b) in enumerate(zip(alone, batched)):
            for k in FIELDS:
                assert np.array_equal(a.read(k), b.read(k)), (i, n, k)
            assert b.diag()["nonfinite"] == 0


def test_batch_follows_members_rebuilt_at_another_time():
    # members rebuilt from their own fields at t = 41 (odd, while the batch's
    # device clock stood at 6): the next advance must run steps 42.. on the
    # right ping-pong buffers with the inlet ramp at the new time, exactly as
    # the lattices rebuilt and advanced alone
    import torch
    from paper_2409_10399_amd import Batch
    ws = members()[:3]
    alone = _lattices(ws, "fp32")
    batched = _lattices(ws, "fp32")
    batch = Batch(batched, tile=(64, 4))
    batch.advance(6)
    for a in alone:
        a.set_launch(64, 4)
        a.advance(6)
    for lat in alone + batched:
        f = {k: torch.tensor(lat.read(k), dtype=torch.float64, device="cuda") for k in ("alpha_g", "u_g", "u_l", "dp_k")}
        lat.reinit_fields_device(41, f)
    batch.advance(9)
    for a in alone:
        a.advance(9)
    for i, (a, b) in enumerate(zip(alone, batched)):
        assert a.t == b.t == 50
        for k in FIELDS:
            assert np.array_equal(a.read(k), b.read(k)), (i, k)
        assert b.diag()["nonfinite"] == 0


@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
def test_batch_equals_members_alone_d3q19(storage):
    from paper_2409_10399_amd import Batch
    ws = members_3d()
    alone = _lattices(ws, storage)
    batched = _lattices(ws, storage)
    batch = Batch(batched, tile=(64, 2), graph_steps=6)
    for n in (6, 5, 12):
        batch.advance(n)
        for lat in alone:
            lat.set_launch(64, 2)
            lat.advance(n)
        for a, b in zip(alone, batched):
            for k in FIELDS:
                assert np.array_equal(a.read(k), b.read(k)), (storage, n, k)


def test_batch_equals_members_alone_d3q19_periodic_fp16():
    """Periodic D3Q19 columns in FP16 (the step instantiation compiled for
    three waves per SIMD, alone and batched): identical bits."""
    from paper_2409_10399_amd import Batch
    ws = [workloads.column_3d(n=n, nblobs=2, seed=50 + n, background=0.01) for n in (16, 24)]
    alone = _lattices(ws, "fp16")
    batched = _lattices(ws, "fp16")
    batch = Batch(batched, tile=(64, 2), graph_steps=4)
    for n in (4, 7):
        batch.advance(n)
        for lat in alone:
            lat.set_launch(64, 2)
            lat.advance(n)
        for a, b in zip(alone, batched):
            for k in FIELDS:
                assert np.array_equal(a.read(k), b.read(k)), (n, k)
            assert b.diag()["nonfinite"] == 0


def test_batch_member_matches_oracle():
    from paper_2409_10399_amd import Batch
    ws = members()[:3]
    lats = _lattices(ws, "fp64")
    batch = Batch(lats, tile=(128, 2), graph_steps=10)
    batch.advance(60)
    for (cfg, f), lat in zip(ws, lats):
        check(lat.read_all(), run_oracle(cfg, f, 60).read(), "fp64", None, f"batch member {cfg['nx']}x{cfg['ny']}")


def test_batch_rejects_mixed_members():
    from paper_2409_10399_amd import Batch, EelbmError
    ws = members()[:2]
    with pytest.raises(EelbmError):  # FP32 storage with FP64 arithmetic runs single lattices only
        Batch(_lattices(ws, "fp32x"), tile=(64, 4))
    a = _lattices(ws[:1], "fp32") + _lattices(ws[1:], "fp64")
    with pytest.raises(EelbmError):
        Batch(a)
    b = _lattices(ws, "fp32")
    b[0].advance(1)
    with pytest.raises(EelbmError):
        Batch(b)


def test_autotune_keeps_state_and_results():
    cfg, f = workloads.channel_2d(nx=200, ny=72, n_ramp=30.0)
    a = run_gpu(cfg, f, 10, "fp32")
    before = {k: a.read(k) for k in FIELDS}
    shape = a.autotune(steps=5, force=True)
    assert shape[0] % 64 == 0 and shape[0] * shape[1] <= 256 and shape[2] in (0, 1)
    assert a.get_launch() == shape
    assert a.t == 10
    for k in FIELDS:
        assert np.array_equal(a.read(k), before[k]), k
    a.advance(15)
    b = run_gpu(cfg, f, 25, "fp32")
    for k in FIELDS:
        assert np.array_equal(a.read(k), b.read(k)), k
    # cached for the size class: a second lattice of the class gets it without timing
    c = run_gpu(cfg, f, 0, "fp32")
    assert c.autotune(steps=5) == shape


def test_batch_with_autotuned_tile():
    # tile None: the batch takes the tile the autotuner picks for its largest
    # member (timed on that member, its state restored); every member then
    # runs with it and the results equal the members advanced alone with it
    from paper_2409_10399_amd import Batch
    ws = members()
    alone = _lattices(ws, "fp32")
    batched = _lattices(ws, "fp32")
    batch = Batch(batched, graph_steps=8)
    tiles = {lat.get_launch()[:2] for lat in batched}
    assert len(tiles) == 1
    tx, ty = tiles.pop()
    assert tx % 64 == 0 and tx * ty <= 256
    for n in (8, 5):
        batch.advance(n)
        for lat in alone:
            lat.set_launch(tx, ty)
            lat.advance(n)
        for a, b in zip(alone, batched):
            for k in FIELDS:
                assert np.array_equal(a.read(k), b.read(k)), (n, k)


def test_batch_active_flags_and_gated_rebuilds():
    # members advance only where their device flag is set (also under graph
    # replay, with the flags changed on the device between replays); a gated
    # rebuild happens only where its device flag is set
    import torch
    from paper_2409_10399_amd import Batch
    ws = members()
    alone = _lattices(ws, "fp32")
    batched = _lattices(ws, "fp32")
    batch = Batch(batched, tile=(64, 4), graph_steps=4)
    flags = torch.tensor([1, 0, 1, 0, 1], dtype=torch.int32, device="cuda")
    batch.set_active(flags)
    before = [{k: b.read(k) for k in FIELDS} for b in batched]
    batch.advance(8)
    def state(lat):
        # what a failure needs to be read: time, tile, diagnostics, field ranges
        d = lat.diag()
        rng = {k: (float(np.min(v)), float(np.max(v))) for k, v in ((k, lat.read(k)) for k in FIELDS)}
        return dict(t=lat.t, tile=lat.get_launch(), nonfinite=d["nonfinite"], alpha_g=d["alpha_g"],
                    a_g=d["a_g"], ranges=rng)

    for i, (a, b) in enumerate(zip(alone, batched)):
        for k in FIELDS:
            if flags[i]:
                if k == FIELDS[0]:
                    a.set_launch(64, 4)
                    a.advance(8)
                ra, rb = a.read(k), b.read(k)
                if not np.array_equal(ra, rb):
                    raise AssertionError((i, k, "alone", state(a), "batched", state(b)))
            else:
                assert np.array_equal(before[i][k], b.read(k)), (i, k)  # left as it was
    # rebuild every member at t = 8 from other fields (the same channels
    # advanced 3 steps), gated: the flag of members 1 and 3 is set, members
    # 0, 2, 4 keep their state
    t = batched[0].t
    gate = torch.tensor([0, 1, 0, 1, 0], dtype=torch.int32, device="cuda")
    src = _lattices(ws, "fp32")
    for s_ in src:
        s_.set_launch(64, 4)
        s_.advance(3)  # other fields than the members hold
    for i, (s_, b) in enumerate(zip(src, batched)):
        f = {k: torch.tensor(s_.read(k), dtype=torch.float64, device="cuda") for k in ("alpha_g", "u_g", "u_l", "dp_k")}
        b.reinit_fields_device(t, f, gate=gate[i:i + 1])
        if gate[i]:
            alone[i].reinit_fields_device(t, f)
    flags.copy_(gate)  # now only the rebuilt members advance (graph replayed with the new flags)
    batch.advance(4)
    for i in (1, 3):
        alone[i].advance(4)
        for k in FIELDS:
            assert np.array_equal(alone[i].read(k), batched[i].read(k)), (i, k)
    # the members whose rebuild was gated off and which were inactive since
    # still hold their fields of t = 8
    for i in (0, 2, 4):
        for k in FIELDS:
            assert np.array_equal(alone[i].read(k), batched[i].read(k)), (i, k)


def test_batch_rebuild_and_read_fields():
    # the batch-level gated rebuild and field read equal the per-member calls
    import torch
    from paper_2409_10399_amd import Batch
    ws = members()[:3]
    a = _lattices(ws, "fp32")
    b = _lattices(ws, "fp32")
    for x in a + b:
        x.set_launch(64, 4)
        x.advance(5)
    batch = Batch(b, tile=(64, 4))
    src = _lattices(ws, "fp32")
    planes = []
    for s_ in src:
        s_.set_launch(64, 4)
        s_.advance(2)
        planes.append(np.concatenate([s_.read("alpha_g")[None], s_.read("u_g"), s_.read("u_l"),
                                      s_.read("dp_k")[None]]).ravel())
    fields = torch.tensor(np.concatenate(planes), dtype=torch.float64, device="cuda")
    gate = torch.tensor([1, 0, 1], dtype=torch.int32, device="cuda")
    batch.rebuild_gated(5, fields, gate)
    off = 0
    for i, x in enumerate(a):
        n = ws[i][0]["nx"] * ws[i][0]["ny"]
        if gate[i]:
            f = fields[off:off + 6 * n].view(6, -1)
            x.reinit_fields_device(5, {"alpha_g": f[0], "u_g": f[1:3], "u_l": f[3:5], "dp_k": f[5]})
        off += 6 * n
    batch.advance(3)
    for x in a:
        x.advance(3)
    out = torch.empty(off, dtype=torch.float32, device="cuda")
    batch.read_fields(out)
    got = out.cpu().numpy()
    off = 0
    for i, (x, y) in enumerate(zip(a, b)):
        n = ws[i][0]["nx"] * ws[i][0]["ny"]
        for k in FIELDS:
            assert np.array_equal(x.read(k), y.read(k)), (i, k)
        ref = np.concatenate([y.read("alpha_g")[None], y.read("u_g"), y.read("u_l"), y.read("dp_k")[None]]).ravel()
        np.testing.assert_array_equal(got[off:off + 6 * n], ref.astype(np.float32))
        off += 6 * n
