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


@pytest.mark.parametrize("graph_steps", [0, 8])
def test_batch_equals_members_alone(graph_steps):
    from paper_2409_10399_amd import Batch
    ws = members()
    alone = _lattices(ws, "fp32")
    batched = _lattices(ws, "fp32")
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
