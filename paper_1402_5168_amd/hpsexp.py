"""Python binding of the hpsexp C-ABI (include/hpsexp.h).

The functions hx_* mirror the C entry points one to one (argument
marshalling only).  ``Plan`` wraps them for PyTorch users: torch allocates
the device arena, the build workspace and the state buffers and provides
the stream; every step of the computation runs in the HIP library.

The library must have been built (``python -m paper_1402_5168_amd.build_lib``);
importing this module never falls back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_longlong, c_size_t, c_uint, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhpsexp.so")

HX_OK, HX_EINVAL, HX_ENOMEM, HX_ESINGULAR = 0, -1, -2, -3
HX_EUNSTABLE, HX_EDEVICE, HX_ESTATE, HX_ESTAGE = -4, -5, -6, -7
HX_WAVE_DIRICHLET, HX_SW_SLIP = 0, 1
HX_FP64, HX_FP32_REFINE = 0, 1
HX_FLAG_ALLOW_UNSTABLE, HX_FLAG_NO_GRAPH, HX_FLAG_CHECK_STATE, HX_FLAG_UNBATCHED = 0x1, 0x2, 0x4, 0x8
HX_FLAG_AUTOTUNE = 0x10
HX_FLAG_FUSED_MERGES = 0x20


class hx_mesh(ctypes.Structure):
    _fields_ = [("nex", c_int), ("ney", c_int), ("p", c_int),
                ("x0", c_double), ("x1", c_double), ("y0", c_double), ("y1", c_double)]


class hx_coeffs(ctypes.Structure):
    _fields_ = [("kind", c_int), ("c2", POINTER(c_double)), ("f", c_double), ("gH", c_double)]


class hx_rational(ctypes.Structure):
    _fields_ = [("npoles", c_int), ("alpha", POINTER(c_double)), ("b", POINTER(c_double))]


class hx_info(ctypes.Structure):
    _fields_ = [("arena_bytes", c_size_t), ("operator_bytes", c_size_t),
                ("workspace_bytes", c_size_t), ("workspace_min_bytes", c_size_t),
                ("dof_state", c_longlong), ("dof_nodes", c_longlong),
                ("folded_poles", c_int), ("n_instances", c_int),
                ("op_bytes_per_step", c_double), ("flops_per_step", c_double),
                ("max_abs_R", c_double), ("fit_X", c_double), ("sum_abs_b", c_double)]


(HX_K_LEAF_UP, HX_K_MERGE_UP, HX_K_MERGE_DOWN, HX_K_LEAF_DOWN, HX_K_POLE_SUM, HX_K_RESIDUAL,
 HX_K_SW_PREP, HX_K_SW_ROOT) = range(8)
HX_K_CLASSES = 8
KERNEL_NAMES = ("k_leaf_up", "k_merge_up", "k_merge_down", "k_leaf_down", "k_pole_sum",
                "k_residual", "k_sw_prep", "k_sw_root")

HX_STAGE_LEAF_UP, HX_STAGE_MERGE_UP, HX_STAGE_ROOT, HX_STAGE_MERGE_DOWN, HX_STAGE_LEAF_DOWN = range(5)
HX_STAGES = 5

EXPORTS = ("hx_plan_create", "hx_plan_add", "hx_plan_query", "hx_plan_bind",
           "hx_plan_build", "hx_step", "hx_step_profile", "hx_plan_tiles", "hx_plan_variants",
           "hx_status_str", "hx_last_error", "hx_plan_destroy")

_lib = None


def load() -> ctypes.CDLL:
    """Load libhpsexp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1402_5168_amd.build_lib`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.hx_plan_create.argtypes = [POINTER(c_void_p), c_int, c_int, c_uint]
    lib.hx_plan_add.argtypes = [c_void_p, POINTER(hx_mesh), POINTER(hx_coeffs), c_double,
                                c_double, POINTER(hx_rational), c_int, POINTER(c_int)]
    lib.hx_plan_query.argtypes = [c_void_p, POINTER(hx_info)]
    lib.hx_plan_bind.argtypes = [c_void_p, c_void_p, c_size_t]
    lib.hx_plan_build.argtypes = [c_void_p, c_void_p, c_size_t, c_void_p]
    lib.hx_step.argtypes = [c_void_p, POINTER(c_void_p), c_int, c_void_p]
    lib.hx_step_profile.argtypes = [c_void_p, POINTER(c_void_p), c_int, c_void_p,
                                    POINTER(c_double), POINTER(c_int), c_int]
    lib.hx_plan_tiles.argtypes = [c_void_p, c_int, POINTER(c_int), c_int]
    lib.hx_plan_variants.argtypes = [c_void_p, c_int, POINTER(c_int), c_int]
    lib.hx_status_str.argtypes = [c_int]
    lib.hx_status_str.restype = c_char_p
    lib.hx_last_error.argtypes = []
    lib.hx_last_error.restype = c_char_p
    lib.hx_plan_destroy.argtypes = [c_void_p]
    lib.hx_plan_destroy.restype = None
    for name in EXPORTS[:9]:
        getattr(lib, name).restype = c_int
    _lib = lib
    return lib


class HxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(message)
        self.status = status


def _check(status: int) -> int:
    if status != HX_OK:
        raise HxError(status, load().hx_last_error().decode())
    return status


# ---- one-to-one wrappers of the C entry points ------------------------------

def hx_plan_create(precision: int = HX_FP64, device: int = 0, flags: int = 0) -> c_void_p:
    plan = c_void_p()
    _check(load().hx_plan_create(byref(plan), precision, device, flags))
    return plan


def hx_plan_add(plan, mesh: hx_mesh, coeffs: hx_coeffs, tau: float, delta: float,
                rational: hx_rational, nrhs: int) -> int:
    inst = c_int(-1)
    _check(load().hx_plan_add(plan, byref(mesh), byref(coeffs), tau, delta,
                              byref(rational), nrhs, byref(inst)))
    return inst.value


def hx_plan_query(plan) -> hx_info:
    info = hx_info()
    _check(load().hx_plan_query(plan, byref(info)))
    return info


def hx_plan_bind(plan, arena_ptr: int, nbytes: int) -> None:
    _check(load().hx_plan_bind(plan, c_void_p(arena_ptr), nbytes))


def hx_plan_build(plan, ws_ptr: int, nbytes: int, stream: int = 0) -> None:
    _check(load().hx_plan_build(plan, c_void_p(ws_ptr), nbytes, c_void_p(stream)))


def hx_step(plan, state_ptrs, n_steps: int, stream: int = 0) -> None:
    arr = (c_void_p * len(state_ptrs))(*[c_void_p(p) for p in state_ptrs])
    _check(load().hx_step(plan, arr, n_steps, c_void_p(stream)))


def hx_step_profile(plan, state_ptrs, n_steps: int, stream: int = 0):
    """Returns (milliseconds, launches) per kernel class."""
    arr = (c_void_p * len(state_ptrs))(*[c_void_p(p) for p in state_ptrs])
    ms = (c_double * HX_K_CLASSES)()
    nl = (c_int * HX_K_CLASSES)()
    _check(load().hx_step_profile(plan, arr, n_steps, c_void_p(stream), ms, nl, HX_K_CLASSES))
    return list(ms), list(nl)


def hx_plan_tiles(plan, instance: int):
    t = (c_int * HX_STAGES)()
    _check(load().hx_plan_tiles(plan, instance, t, HX_STAGES))
    return list(t)


def hx_plan_variants(plan, instance: int):
    v = (c_int * HX_STAGES)()
    _check(load().hx_plan_variants(plan, instance, v, HX_STAGES))
    return list(v)


def hx_status_str(status: int) -> str:
    return load().hx_status_str(status).decode()


def hx_last_error() -> str:
    return load().hx_last_error().decode()


def hx_plan_destroy(plan) -> None:
    load().hx_plan_destroy(plan)


# ---- convenience wrapper for torch users ----------------------------------------

def _cplx_pairs(z) -> np.ndarray:
    z = np.asarray(z, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=-1).reshape(-1))


class Plan:
    """A plan whose device memory is owned by torch tensors."""

    def __init__(self, device: int = 0, flags: int = 0, precision: int = HX_FP64):
        self.device = device
        self.precision = precision
        self.handle = hx_plan_create(precision, device, flags)
        self._keep = []          # host arrays referenced by the C structs
        self.arena = None
        self.instances = []

    def add(self, nex: int, ney: int, p: int, c2: np.ndarray, tau: float, delta: float,
            alpha, b, nrhs: int = 1, domain=(0.0, 1.0, 0.0, 1.0)) -> int:
        mesh = hx_mesh(nex, ney, p, *[float(v) for v in domain])
        c2 = np.ascontiguousarray(np.asarray(c2, dtype=np.float64).reshape(-1))
        a2, b2 = _cplx_pairs(alpha), _cplx_pairs(b)
        coeffs = hx_coeffs(HX_WAVE_DIRICHLET, c2.ctypes.data_as(POINTER(c_double)), 0.0, 0.0)
        rat = hx_rational(len(a2) // 2, a2.ctypes.data_as(POINTER(c_double)),
                          b2.ctypes.data_as(POINTER(c_double)))
        k = hx_plan_add(self.handle, mesh, coeffs, tau, delta, rat, nrhs)
        self.instances.append(dict(nex=nex, ney=ney, p=p, nrhs=nrhs, fields=2))
        return k

    def add_sw(self, nex: int, ney: int, p: int, f: float, gH: float, tau: float,
               delta: float, alpha, b, nrhs: int = 1, domain=(0.0, 1.0, 0.0, 1.0)) -> int:
        """Shallow water with slip walls; state fields (v1, v2, eta)."""
        mesh = hx_mesh(nex, ney, p, *[float(v) for v in domain])
        a2, b2 = _cplx_pairs(alpha), _cplx_pairs(b)
        coeffs = hx_coeffs(HX_SW_SLIP, None, float(f), float(gH))
        rat = hx_rational(len(a2) // 2, a2.ctypes.data_as(POINTER(c_double)),
                          b2.ctypes.data_as(POINTER(c_double)))
        k = hx_plan_add(self.handle, mesh, coeffs, tau, delta, rat, nrhs)
        self.instances.append(dict(nex=nex, ney=ney, p=p, nrhs=nrhs, fields=3))
        return k

    def query(self) -> dict:
        info = hx_plan_query(self.handle)
        return {name: getattr(info, name) for name, _ in hx_info._fields_}

    def state_shape(self, k: int):
        d = self.instances[k]
        q = d["p"] - 2
        return (d["nrhs"], d["fields"], d["nex"] * d["ney"] * q * q)

    def bind(self):
        import torch
        n = self.query()["arena_bytes"]
        self.arena = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        hx_plan_bind(self.handle, self.arena.data_ptr(), n)

    def build(self, workspace_bytes: int | None = None, stream=None):
        import torch
        info = self.query()
        n = workspace_bytes or info["workspace_bytes"]
        ws = torch.empty(n, dtype=torch.uint8, device=f"cuda:{self.device}")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        hx_plan_build(self.handle, ws.data_ptr(), n, s.cuda_stream)
        del ws

    def step(self, states, n_steps: int, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        for k, x in enumerate(states):
            if x.dtype != torch.float64 or not x.is_contiguous() or not x.is_cuda:
                raise ValueError("states must be contiguous float64 CUDA tensors")
            if tuple(x.shape) != self.state_shape(k) and x.numel() != int(np.prod(self.state_shape(k))):
                raise ValueError(f"state {k} has shape {tuple(x.shape)}, "
                                 f"expected {self.state_shape(k)}")
        hx_step(self.handle, [x.data_ptr() for x in states], n_steps, s.cuda_stream)

    def tiles(self, k: int):
        """Right-hand-side tiles per block of instance k, per HX_STAGE_*."""
        return hx_plan_tiles(self.handle, k)

    def variants(self, k: int):
        """Kernel variant per HX_STAGE_* of instance k (staged upward sweep,
        one-wave merge blocks; 0 = the default shape)."""
        return hx_plan_variants(self.handle, k)

    def step_profile(self, states, n_steps: int, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        return hx_step_profile(self.handle, [x.data_ptr() for x in states], n_steps,
                               s.cuda_stream)

    def close(self):
        if self.handle is not None:
            hx_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
