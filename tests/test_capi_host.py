"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/eelbm.h declares, mirrors its structs, validates
parameters and maps physical units as Sec. 3.3 prescribes."""
import ctypes
import json
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2409_10399_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libeelbm.so is not built (run python -m paper_2409_10399_amd.build)")
    return binding


def test_library_exports_every_declared_symbol():
    b = _lib()
    header = open(os.path.join(ROOT, "include", "eelbm.h")).read()
    names = set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(eelbm_\w+)\s*\(", header, flags=re.M))
    assert len(names) >= 14
    L = ctypes.CDLL(b.LIB_PATH)
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(b.SYMBOLS) == names


def test_struct_mirror_and_version():
    b = _lib()
    L = b.lib()
    assert L.eelbm_abi_version() == b.ABI_VERSION
    assert L.eelbm_params_size() == ctypes.sizeof(b.Params)


def test_state_bytes_and_validation():
    b = _lib()
    cfg, _ = workloads.channel_2d()
    n = 1024 * 1024
    nb = b.state_bytes(cfg, "fp32")
    assert nb >= 2 * 4 * 9 * 4 * n + 2 * 4 * 4 * n
    assert b.state_bytes(cfg, "fp16") < nb < b.state_bytes(cfg, "fp64")
    bad = [dict(omega_g=2.0), dict(omega_al=0.0), dict(rho_g=0.0), dict(n_gamma=0), dict(alpha_min=0.0),
           dict(up_axis=2), dict(bc={"x-": "wall", "x+": "periodic"}),
           dict(bc={"x-": "inlet", "x+": "outlet", "y-": "inlet", "y+": "outlet"}), dict(ny=3)]
    for kw in bad:
        c = dict(cfg)
        c.update(kw)
        with pytest.raises(b.EelbmError) as e:
            b.state_bytes(c)
        assert e.value.code == -1, kw
    c3 = workloads._base("D3Q19", nx=8, ny=8, nz=8)
    assert b.state_bytes(c3, "fp32") > 0


def test_map_physical_reproduces_test4_numbers():
    b = _lib()
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "test4_mapping.json")))
    i, pr = g["inputs"], g["printed"]
    m = b.map_physical(i["g"], i["kappa_I"], i["g_hat"], i["kappa_hat"])
    assert abs(m["c_over_tau"] / pr["c_over_tau"] - 1) < 1e-3
    assert abs(m["c_tau"] / pr["c_tau"] - 1) < 1e-3
    assert abs(m["c"] / pr["c"] - 1) < 1e-3
    with pytest.raises(b.EelbmError):
        b.map_physical(-1.0, 1.0, 1.0, 1.0)


def test_storage_sizes_of_every_mode():
    """State bytes follow the bytes per stored population value: FP64 8,
    FP32 and FP32-with-FP64-arithmetic 4 (the latter with FP64 records),
    mixed 3 (a 12-byte group per direction), FP16/BF16 2."""
    b = _lib()
    cfg, _ = workloads.channel_2d(nx=128, ny=64)
    sizes = {s: b.state_bytes(cfg, s) for s in ("fp64", "fp32", "fp32x", "mixed", "fp16", "bf16")}
    assert sizes["fp16"] == sizes["bf16"] < sizes["mixed"] < sizes["fp32"] < sizes["fp32x"] < sizes["fp64"]
    n = 128 * 64
    # population copies differ by 2 x 4 x 9 values x the byte difference per value
    assert sizes["fp32"] - sizes["mixed"] == 2 * 4 * 9 * n * (4 - 3)
    assert sizes["mixed"] - sizes["fp16"] == 2 * 4 * 9 * n * (3 - 2)
    # FP64 records instead of FP32 ones: a D2Q9 record holds 2 + 2D = 6
    # values (+ alpha_l) in each of two copies, the lag region S''_g, S''_l
    # and Lambda', and the side buffers 2 copies x 2 faces x 2 x (2D + 2)
    # values per face node add 4 bytes per value
    assert cfg["n_gamma"] > 1
    side = 2 * 2 * 2 * (2 * 2 + 2) * 128
    assert sizes["fp32x"] - sizes["fp32"] == 4 * (n * (2 * (6 + 1) + 3) + side)
    # D3Q19: records of 2 + 2D = 8 values; a periodic column has no side buffers
    cfg3, _ = workloads.column_3d(n=32, nblobs=1)
    s3 = {s: b.state_bytes(cfg3, s) for s in ("fp32", "fp32x")}
    assert s3["fp32x"] - s3["fp32"] == 4 * 32 ** 3 * (2 * (8 + 1) + 3)


def test_new_entry_points_validate_without_a_gpu():
    """Parameter checks that return before any device work."""
    b = _lib()
    L = b.lib()
    assert L.eelbm_cno_conv_set_tile(3, 1) != 0 and L.eelbm_cno_conv_set_tile(1, 5) != 0
    assert L.eelbm_cno_conv_set_tile(0, 0) == 0
    assert L.eelbm_batch_set_active(None, None) != 0
    assert L.eelbm_batch_rebuild_gated(None, 0, None, None) != 0
    assert L.eelbm_batch_read_fields(None, None) != 0
    assert L.eelbm_cno_reanchor_policy(None, 1, 1e-3, 0, None, None, None, None, None) != 0
    assert L.eelbm_cno_select(None, 1, 1, None, None, None, None) != 0
    assert L.eelbm_cno_volume_defect(None, None, 1, 3, 1, 1, None, None, None) != 0
    assert L.eelbm_cno_pool_bf16(None, 1, 2, 2, 16, None, None) != 0
    # a shape whose tensors hold 2^31 values or more is refused before launch
    big = ctypes.c_void_p(16)
    assert L.eelbm_cno_conv_fwd_cat_dt(big, 64, 0, None, 0, 16, 2048, 2048, big, None, 64, big, 0, 0.1, 0, 0,
                                       None) != 0
