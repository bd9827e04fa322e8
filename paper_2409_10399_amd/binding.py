"""ctypes binding of the C ABI in include/eelbm.h (argument marshalling only).

Every step of the method runs in the HIP library ``_lib/libeelbm.so``; this
module translates a parameter dict into ``eelbm_params``, takes device memory
and the current stream from PyTorch, and copies fields in and out.  It raises
if the library is missing: there is no fallback path.
"""
import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_size_t, c_uint32, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EELBM_LIB") or os.path.join(_HERE, "_lib", "libeelbm.so")

ABI_VERSION = 1
E_CODES = {-1: "EELBM_E_PARAM", -2: "EELBM_E_SIZE", -3: "EELBM_E_HIP", -4: "EELBM_E_NONFINITE", -5: "EELBM_E_STATE"}
LATTICE = {"D2Q9": 2, "D3Q19": 3}
# fp32x: FP32 populations, FP64 arithmetic; mixed: f_g FP32, f_l and f_alpha FP16
STORAGE = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp32x": 4, "mixed": 5}
BC = {"periodic": 0, "wall": 1, "inlet": 2, "outlet": 3}
DRAG = {"const": 0, "cgw": 1}
FIELD = {"alpha_g": 0, "alpha_l": 1, "u_g": 2, "u_l": 3, "p_k": 4, "dp_k": 5}
FLAG_NO_RENORM = 1
FLAG_NO_SIGMA_GRAD = 2


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", c_int32), ("lattice", c_int32), ("storage", c_int32),
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("bc", c_int32 * 6),
        ("up_axis", c_int32), ("drag_model", c_int32), ("rho_ref_mode", c_int32),
        ("n_gamma", c_int32), ("flags", c_uint32), ("reserved_i", c_int32),
        ("rho_g", c_double), ("rho_l", c_double), ("omega_g", c_double), ("omega_l", c_double),
        ("psi_g", c_double), ("psi_l", c_double), ("omega_ag", c_double), ("omega_al", c_double),
        ("K_I", c_double), ("kappa_I", c_double), ("K_W", c_double), ("g_hat", c_double),
        ("rho_ref", c_double), ("gamma", c_double), ("alpha_min", c_double),
        ("alpha_in_max", c_double), ("alpha_in_min", c_double), ("ug_in_max", c_double),
        ("ug_in_min", c_double), ("ul_in_max", c_double), ("ul_in_min", c_double), ("n_ramp", c_double),
    ]


class Diagnostics(ctypes.Structure):
    _fields_ = [
        ("t", c_int64), ("nonfinite", c_int64), ("a_g", c_double), ("a_l", c_double),
        ("alpha_g", c_double), ("alpha_l", c_double), ("deps_g", c_double), ("deps_l", c_double),
        ("u_g", c_double * 3), ("u_l", c_double * 3), ("momentum", c_double * 3), ("renorm_defect", c_double),
    ]


SYMBOLS = {
    "eelbm_abi_version": (c_int32, []),
    "eelbm_params_size": (c_size_t, []),
    "eelbm_state_bytes": (c_int, [POINTER(Params), POINTER(c_size_t)]),
    "eelbm_create": (c_int, [POINTER(Params), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "eelbm_init_fields": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "eelbm_advance": (c_int, [c_void_p, c_int64]),
    "eelbm_read": (c_int, [c_void_p, c_int32, c_void_p, c_int32, c_int]),
    "eelbm_diag": (c_int, [c_void_p, POINTER(Diagnostics)]),
    "eelbm_time": (c_int64, [c_void_p]),
    "eelbm_set_launch": (c_int, [c_void_p, c_int32, c_int32, c_int32]),
    "eelbm_get_launch": (c_int, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "eelbm_save": (c_int, [c_void_p, c_void_p, POINTER(c_size_t)]),
    "eelbm_load": (c_int, [c_void_p, c_void_p, c_size_t]),
    "eelbm_destroy": (None, [c_void_p]),
    "eelbm_last_error": (ctypes.c_char_p, []),
    "eelbm_map_physical": (c_int, [c_double, c_double, c_double, c_double, POINTER(c_double),
                                   POINTER(c_double), POINTER(c_double)]),
    "eelbm_batch_bytes": (c_int, [POINTER(c_void_p), c_int32, c_int32, c_int32, POINTER(c_size_t)]),
    "eelbm_batch_create": (c_int, [POINTER(c_void_p), c_int32, c_int32, c_int32, c_void_p, c_size_t, c_void_p,
                                   POINTER(c_void_p)]),
    "eelbm_batch_set_graph": (c_int, [c_void_p, c_int32]),
    "eelbm_batch_advance": (c_int, [c_void_p, c_int64]),
    "eelbm_batch_destroy": (None, [c_void_p]),
    "eelbm_autotune": (c_int, [c_void_p, c_int32, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "eelbm_reinit_fields": (c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    # learned surrogate kernels (device pointers, NHWC FP32)
    "eelbm_cno_conv_fwd_cat": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                       c_void_p, c_void_p, c_int32, c_void_p, c_int32, ctypes.c_float, c_void_p]),
    "eelbm_cno_conv_set_tile": (c_int, [c_int32, c_int32]),
    "eelbm_cno_conv_fwd_cat_dt": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                          c_void_p, c_void_p, c_int32, c_void_p, c_int32, ctypes.c_float, c_int32,
                                          c_int32, c_void_p]),
    "eelbm_cno_pool_bf16": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    "eelbm_cno_volume_defect": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                        c_void_p]),
    "eelbm_cno_reanchor_policy": (c_int, [c_void_p, c_int32, ctypes.c_double, c_int32, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p]),
    "eelbm_cno_select": (c_int, [c_void_p, c_int32, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]),
    "eelbm_reinit_fields_gated": (c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "eelbm_batch_set_active": (c_int, [c_void_p, c_void_p]),
    "eelbm_batch_rebuild_gated": (c_int, [c_void_p, c_int64, c_void_p, c_void_p]),
    "eelbm_batch_read_fields": (c_int, [c_void_p, c_void_p]),
    "eelbm_cno_conv_fwd": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_int32,
                                   c_void_p, c_int32, ctypes.c_float, c_void_p]),
    "eelbm_cno_conv_bwd_data": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                        c_void_p]),
    "eelbm_cno_conv_bwd_weight": (c_int, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_int32, c_void_p,
                                          c_void_p, c_void_p]),
    "eelbm_cno_act_bwd": (c_int, [c_void_p, c_void_p, c_int64, ctypes.c_float, c_void_p, c_void_p]),
    "eelbm_cno_pool": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p]),
    "eelbm_cno_up": (c_int, [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p]),
    "eelbm_cno_concat": (c_int, [c_void_p, c_int32, c_void_p, c_int32, c_int64, c_void_p, c_void_p]),
    "eelbm_cno_split_add": (c_int, [c_void_p, c_int32, c_int32, c_int64, c_void_p, c_void_p, c_void_p]),
    "eelbm_cno_mse": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_void_p]),
    "eelbm_cno_mse_noalloc": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_int32, c_void_p, c_void_p,
                                      c_void_p]),
    "eelbm_cno_adam": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, ctypes.c_float, c_int64, ctypes.c_float, c_void_p]),
    "eelbm_cno_pack_weights": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "eelbm_cno_pack": (c_int, [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_int32,
                               ctypes.c_float, c_void_p, c_void_p]),
    "eelbm_cno_unpack": (c_int, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_int32, c_void_p,
                                 c_void_p]),
    "eelbm_cno_axpy": (c_int, [c_void_p, c_int64, ctypes.c_float, c_void_p, c_void_p]),
    "eelbm_cno_fill": (c_int, [c_void_p, c_int64, ctypes.c_float, c_void_p]),
}

_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2409_10399_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SYMBOLS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.eelbm_abi_version() != ABI_VERSION or L.eelbm_params_size() != ctypes.sizeof(Params):
        raise RuntimeError("libeelbm ABI does not match this binding")
    _lib = L
    return L


class EelbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{E_CODES.get(code, code)}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise EelbmError(rc, lib().eelbm_last_error().decode())
    return rc


def params_from_cfg(cfg, storage="fp32"):
    """Translate a parameter dict (keys of the workloads module) into eelbm_params."""
    p = Params()
    p.abi_version = ABI_VERSION
    p.lattice = LATTICE[cfg["lattice"]]
    D = 2 if p.lattice == 2 else 3
    p.storage = STORAGE[storage]
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    p.nz = int(cfg.get("nz", 1)) if D == 3 else 1
    bc = cfg.get("bc", {})
    for i, face in enumerate(("x-", "x+", "y-", "y+", "z-", "z+")):
        p.bc[i] = BC[bc.get(face, "periodic")]
    p.up_axis = int(cfg.get("up_axis", D - 1))
    p.drag_model = DRAG[cfg.get("drag", "const")]
    rr = cfg.get("rho_ref", "liquid")
    if rr == "liquid":
        p.rho_ref_mode = 0
    elif rr == "mixture_mean":
        p.rho_ref_mode = 1
    else:
        p.rho_ref_mode, p.rho_ref = 2, float(rr)
    p.n_gamma = int(cfg.get("n_gamma", 1))
    p.flags = (0 if cfg.get("renormalize", True) else FLAG_NO_RENORM) | \
              (0 if cfg.get("sigma_grad", True) else FLAG_NO_SIGMA_GRAD)
    for k in ("rho_g", "rho_l", "omega_g", "omega_l", "omega_ag", "omega_al"):
        setattr(p, k, float(cfg[k]))
    for k in ("psi_g", "psi_l", "K_I", "kappa_I", "K_W", "g_hat", "gamma",
              "alpha_in_max", "alpha_in_min", "ug_in_max", "ug_in_min", "ul_in_max", "ul_in_min", "n_ramp"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    p.alpha_min = float(cfg.get("alpha_min", 1e-6))
    return p


def state_bytes(cfg, storage="fp32"):
    n = c_size_t()
    p = params_from_cfg(cfg, storage)
    _check(lib().eelbm_state_bytes(byref(p), byref(n)))
    return n.value


def map_physical(g, kappa_I, g_hat, kappa_hat):
    a, b, c = c_double(), c_double(), c_double()
    _check(lib().eelbm_map_physical(g, kappa_I, g_hat, kappa_hat, byref(a), byref(b), byref(c)))
    return {"c_over_tau": a.value, "c_tau": b.value, "c": c.value}


def _ptr(a):
    return c_void_p(a.ctypes.data) if a is not None else None


class Lattice:
    """One lattice on the current CUDA (HIP) device, bound to torch's current stream."""

    def __init__(self, cfg, storage="fp32", stream=None):
        import torch
        L = lib()
        self.cfg = cfg
        self.params = params_from_cfg(cfg, storage)
        self.D = 2 if self.params.lattice == 2 else 3
        self.shape = ((self.params.nz,) if self.D == 3 else ()) + (self.params.ny, self.params.nx)
        nbytes = c_size_t()
        _check(L.eelbm_state_bytes(byref(self.params), byref(nbytes)))
        self.nbytes = nbytes.value
        self.mem = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = c_void_p()
        _check(L.eelbm_create(byref(self.params), c_void_p(self.mem.data_ptr()), nbytes,
                              c_void_p(self.stream.cuda_stream), byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.eelbm_destroy(h)
            self.h = None

    # -- fields ------------------------------------------------------------
    def _arr(self, a, shape):
        if a is None:
            return None
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(shape))
        return a

    def init_fields(self, fields):
        """Host (NumPy) initial fields in the layout of include/eelbm.h."""
        D, sh = self.D, self.shape
        keep = [self._arr(fields["alpha_g"], sh), self._arr(fields.get("u_g"), (D,) + sh),
                self._arr(fields.get("u_l"), (D,) + sh), self._arr(fields.get("dp_k"), sh),
                None if fields.get("inlet_noise") is None else
                np.ascontiguousarray(np.asarray(fields["inlet_noise"], dtype=np.float64))]
        _check(lib().eelbm_init_fields(self.h, *[_ptr(a) for a in keep], 0))

    def init_fields_device(self, tensors):
        """Device (torch float64, contiguous) initial fields."""
        ptr = lambda k: c_void_p(tensors[k].data_ptr()) if tensors.get(k) is not None else None
        _check(lib().eelbm_init_fields(self.h, ptr("alpha_g"), ptr("u_g"), ptr("u_l"), ptr("dp_k"),
                                       ptr("inlet_noise"), 1))

    def reinit_fields_device(self, t, tensors, gate=None):
        """Rebuild the state at time t from device (torch float64) fields;
        gate: a device int32 tensor element (a one-element view): rebuild
        only if it is nonzero when the rebuild runs."""
        ptr = lambda k: c_void_p(tensors[k].data_ptr()) if tensors.get(k) is not None else None
        if gate is None:
            _check(lib().eelbm_reinit_fields(self.h, int(t), ptr("alpha_g"), ptr("u_g"), ptr("u_l"), ptr("dp_k"), 1))
        else:
            _check(lib().eelbm_reinit_fields_gated(self.h, int(t), ptr("alpha_g"), ptr("u_g"), ptr("u_l"),
                                                   ptr("dp_k"), c_void_p(gate.data_ptr())))

    def advance(self, nsteps):
        _check(lib().eelbm_advance(self.h, int(nsteps)))

    def set_launch(self, tile_x, tile_y, xcd_remap=1):
        _check(lib().eelbm_set_launch(self.h, int(tile_x), int(tile_y), int(xcd_remap)))

    def get_launch(self):
        a, b, c = c_int32(), c_int32(), c_int32()
        _check(lib().eelbm_get_launch(self.h, byref(a), byref(b), byref(c)))
        return a.value, b.value, c.value

    def autotune(self, steps=50, force=False):
        """Time every launch shape on this lattice's own state (restored
        afterwards), apply the fastest; cached per size class."""
        a, b, c = c_int32(), c_int32(), c_int32()
        _check(lib().eelbm_autotune(self.h, int(steps), int(bool(force)), byref(a), byref(b), byref(c)))
        return a.value, b.value, c.value

    @property
    def t(self):
        return lib().eelbm_time(self.h)

    def read(self, name, dtype=np.float64):
        vec = name in ("u_g", "u_l")
        shape = ((self.D,) if vec else ()) + self.shape
        out = np.empty(shape, dtype=dtype)
        _check(lib().eelbm_read(self.h, FIELD[name], c_void_p(out.ctypes.data),
                                0 if dtype == np.float64 else 1, 0))
        return out

    def read_device(self, name, out):
        """Into a contiguous torch float64/float32 device tensor (asynchronous)."""
        import torch
        dt = 0 if out.dtype == torch.float64 else 1
        _check(lib().eelbm_read(self.h, FIELD[name], c_void_p(out.data_ptr()), dt, 1))
        return out

    def read_all(self):
        return {k: self.read(k) for k in ("alpha_g", "alpha_l", "u_g", "u_l", "p_k", "dp_k")}

    def diag(self):
        d = Diagnostics()
        rc = lib().eelbm_diag(self.h, byref(d))
        if rc not in (0, -4):
            _check(rc)
        out = {k: getattr(d, k) for k in ("t", "nonfinite", "a_g", "a_l", "alpha_g", "alpha_l",
                                          "deps_g", "deps_l", "renorm_defect")}
        for k in ("u_g", "u_l", "momentum"):
            out[k] = np.array(list(getattr(d, k))[: self.D])
        return out

    def save(self):
        n = c_size_t()
        _check(lib().eelbm_save(self.h, None, byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().eelbm_save(self.h, buf, byref(n)))
        return buf.raw

    def load(self, blob):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().eelbm_load(self.h, buf, len(blob)))


class Batch:
    """Lattices advanced together: one launch per step over all their tiles,
    optionally captured in HIP graphs of `graph_steps` steps.  tile=None: the
    autotuned tile of the largest member."""

    def __init__(self, members, tile=None, graph_steps=0, stream=None):
        import torch
        L = lib()
        tile = (0, 0) if tile is None else tile
        self.members = list(members)
        arr = (c_void_p * len(self.members))(*[m.h for m in self.members])
        self._arr = arr
        n = c_size_t()
        _check(L.eelbm_batch_bytes(arr, len(self.members), int(tile[0]), int(tile[1]), byref(n)))
        self.mem = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        b = c_void_p()
        _check(L.eelbm_batch_create(arr, len(self.members), int(tile[0]), int(tile[1]),
                                    c_void_p(self.mem.data_ptr()), n, c_void_p(self.stream.cuda_stream), byref(b)))
        self.b = b
        if graph_steps:
            _check(L.eelbm_batch_set_graph(self.b, int(graph_steps)))

    def set_graph(self, steps):
        _check(lib().eelbm_batch_set_graph(self.b, int(steps)))

    def rebuild_gated(self, t, fields, gate):
        """Rebuild member i at time t from fields[i] (device float64, the
        members' [2 + 2D][n] field planes one after the other) where gate[i]
        (device int32) is nonzero when the rebuild runs."""
        _check(lib().eelbm_batch_rebuild_gated(self.b, int(t), c_void_p(fields.data_ptr()),
                                               c_void_p(gate.data_ptr())))

    def read_fields(self, out):
        """Every member's output fields into out (device float32, the layout
        of rebuild_gated)."""
        _check(lib().eelbm_batch_read_fields(self.b, c_void_p(out.data_ptr())))

    def set_active(self, flags):
        """flags: device int32 tensor, one per member (kept alive by the
        batch), read at every step; None: every member advances."""
        self._active = flags
        _check(lib().eelbm_batch_set_active(self.b, c_void_p(flags.data_ptr()) if flags is not None else None))

    def advance(self, nsteps):
        _check(lib().eelbm_batch_advance(self.b, int(nsteps)))

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and _lib is not None:
            _lib.eelbm_batch_destroy(b)
            self.b = None

