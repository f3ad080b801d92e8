"""ctypes binding of librb (include/rb.h): argument marshalling only.

Every entry point keeps its C name.  Particle and acceleration arrays are
torch tensors on the GPU (float64, contiguous); their device pointers go
straight to the library, and the context works on the torch stream that is
current when it is created.  There is no fallback: if librb.so is missing or
cannot be loaded, importing this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librb.so")

RB_OK, RB_EINVAL, RB_ENOMEM, RB_EHIP, RB_ECAPACITY, RB_EOUTSIDE, RB_EUNSUPPORTED, RB_EIO = (
    0, -1, -2, -3, -4, -5, -6, -7)
RB_OPEN, RB_PERIODIC, RB_SHEAR = 0, 1, 2
RB_FP64, RB_FP32_MIXED = 0, 1
RB_SWEEP_X, RB_SWEEP_PHI = 0, 1
RB_DRIFT_LEAPFROG, RB_DRIFT_EPICYCLE = 0, 1

PHASES = ["keys", "sort", "permute", "topology", "moments", "walk", "kick_drift", "direct",
          "collide", "total", "coll_search"]


class rb_params(ctypes.Structure):
    _fields_ = [
        ("G", ctypes.c_double),
        ("softening", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("quadrupole", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("group_size", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("drift", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("box_size", ctypes.c_double),
        ("box_min", ctypes.c_double * 3),
        ("n_ghost", ctypes.c_int32 * 2),
        ("omega", ctypes.c_double),
        ("omega_z", ctypes.c_double),
        ("node_factor", ctypes.c_double),
        ("split_images", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("walk_waves", ctypes.c_int32),
        ("moments_level_log2", ctypes.c_int32),
        ("walk64_schedule", ctypes.c_int32),
        ("n_root", ctypes.c_int32 * 3),
        ("reuse_topology", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]


class rb_particles(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "y", "z", "vx", "vy", "vz", "m")]


class rb_tree_host(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in (
        "keys", "perm", "level", "prefix", "first", "count", "is_leaf", "n_child",
        "first_child", "skip", "M", "com", "Q")]


class rb_stats_t(ctypes.Structure):
    _fields_ = [("open_tests", ctypes.c_int64), ("cells", ctypes.c_int64),
                ("pp", ctypes.c_int64), ("list_cells", ctypes.c_int64),
                ("list_pp", ctypes.c_int64), ("ms", ctypes.c_double * 16),
                ("calls", ctypes.c_int64 * 16), ("reused_steps", ctypes.c_int64)]


class RBError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (code {code})")
        self.code = code


_lib = None

_SIGS = {
    "rb_params_default": (None, [ctypes.POINTER(rb_params)]),
    "rb_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(rb_params),
                                 ctypes.c_int64, ctypes.c_void_p]),
    "rb_batch_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(rb_params), ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "rb_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "rb_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_params)]),
    "rb_tree_build": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles),
                                     ctypes.c_int64, ctypes.c_int64]),
    "rb_tree_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64)]),
    "rb_tree_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(rb_tree_host)]),
    "rb_gravity": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles),
                                  ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rb_direct": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles), ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p]),
    "rb_direct_noalloc": (ctypes.c_int, [ctypes.POINTER(rb_params), ctypes.POINTER(rb_particles),
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                         ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "rb_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles), ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                               ctypes.c_int32]),
    "rb_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles),
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "rb_batch_gravity": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles),
                                        ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "rb_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "rb_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_stats_t)]),
    "rb_phase_name": (ctypes.c_char_p, [ctypes.c_int32]),
    "rb_state_save": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles),
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_char_p]),
    "rb_state_load": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles),
                                     ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_char_p]),
    "rb_collide": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles), ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                  ctypes.c_int64]),
    "rb_sweep": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(rb_particles), ctypes.c_void_p,
                                ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_double, ctypes.c_uint64,
                                ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                ctypes.c_int64]),
    "rb_peak_probe": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "rb_set_collisions": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.c_int32]),
    "rb_collision_counts": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "rb_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rb_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load librb.so (raises when it is absent: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1110_4876_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(code: int, where: str) -> None:
    if code != RB_OK:
        detail = lib().rb_last_error().decode(errors="replace")
        raise RBError(code, where, detail)


def params(**kw) -> rb_params:
    """rb_params with library defaults, then the given fields."""
    p = rb_params()
    lib().rb_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if k in ("box_min", "n_ghost", "n_root"):
            arr = getattr(p, k)
            for a, val in enumerate(v):
                arr[a] = val
        elif k in dict(rb_params._fields_):
            setattr(p, k, v)
        else:
            raise KeyError(k)
    return p


def params_from_problem(pp: dict, precision: int = RB_FP64, **kw) -> rb_params:
    """rb_params from a parameter dict of paper_1110_4876_amd.inputs."""
    d = dict(G=pp["G"], softening=pp["b"], theta=pp["theta"], quadrupole=int(bool(pp["quadrupole"])),
             leaf_size=int(pp.get("n_leaf", 1)), group_size=int(pp.get("group_size", 64)),
             boundary=int(pp["boundary"]), drift=int(pp["drift"]), precision=int(precision),
             box_size=float(pp["W"]), box_min=tuple(float(v) for v in pp["x0"]),
             n_ghost=tuple(int(v) for v in pp["ng"]), omega=float(pp["omega"]),
             omega_z=float(pp["omega_z"] if pp.get("omega_z") is not None else pp["omega"]),
             n_root=tuple(int(v) for v in pp.get("n_root", (1, 1, 1))))
    d.update(kw)
    return params(**d)


def _ptr(t) -> int:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or t.dtype not in (torch.float64, torch.int64) or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 / int64 CUDA tensor")
    return t.data_ptr()


def particles(x, y, z, m, vx=None, vy=None, vz=None) -> rb_particles:
    p = rb_particles()
    p.x, p.y, p.z, p.m = _ptr(x), _ptr(y), _ptr(z), _ptr(m)
    p.vx, p.vy, p.vz = _ptr(vx), _ptr(vy), _ptr(vz)
    return p


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def rb_create(p: rb_params, capacity: int):
    ctx = ctypes.c_void_p()
    check(lib().rb_create(ctypes.byref(ctx), ctypes.byref(p), int(capacity), _stream_handle()),
          "rb_create")
    return ctx


def rb_batch_create(p: rb_params, offsets, box_size, box_min):
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    box_size = np.ascontiguousarray(box_size, dtype=np.float64)
    box_min = np.ascontiguousarray(box_min, dtype=np.float64).reshape(-1)
    ctx = ctypes.c_void_p()
    check(lib().rb_batch_create(ctypes.byref(ctx), ctypes.byref(p), len(offsets) - 1,
                                offsets.ctypes.data, box_size.ctypes.data, box_min.ctypes.data,
                                _stream_handle()), "rb_batch_create")
    return ctx


def rb_destroy(ctx) -> None:
    check(lib().rb_destroy(ctx), "rb_destroy")


def rb_set_params(ctx, p: rb_params) -> None:
    check(lib().rb_set_params(ctx, ctypes.byref(p)), "rb_set_params")


def rb_tree_build(ctx, parts: rb_particles, n: int, n_active: int) -> None:
    check(lib().rb_tree_build(ctx, ctypes.byref(parts), int(n), int(n_active)), "rb_tree_build")


def rb_tree_info(ctx):
    nn, nl = ctypes.c_int64(), ctypes.c_int64()
    check(lib().rb_tree_info(ctx, ctypes.byref(nn), ctypes.byref(nl)), "rb_tree_info")
    return int(nn.value), int(nl.value)


def rb_tree_export(ctx, patch: int, n_nodes: int, n_live: int) -> dict:
    e = dict(keys=np.zeros(n_live, np.uint64), perm=np.zeros(n_live, np.int64),
             level=np.zeros(n_nodes, np.int8), prefix=np.zeros(n_nodes, np.uint64),
             first=np.zeros(n_nodes, np.int64), count=np.zeros(n_nodes, np.int64),
             is_leaf=np.zeros(n_nodes, np.int8), n_child=np.zeros(n_nodes, np.int32),
             first_child=np.zeros(n_nodes, np.int64), skip=np.zeros(n_nodes, np.int64),
             M=np.zeros(n_nodes), com=np.zeros((n_nodes, 3)), Q=np.zeros((n_nodes, 6)))
    h = rb_tree_host()
    for k, v in e.items():
        setattr(h, k, v.ctypes.data)
    check(lib().rb_tree_export(ctx, int(patch), ctypes.byref(h)), "rb_tree_export")
    return e


def rb_gravity(ctx, parts: rb_particles, n: int, n_active: int, t: float, ax, ay, az) -> None:
    check(lib().rb_gravity(ctx, ctypes.byref(parts), int(n), int(n_active), float(t), _ptr(ax),
                           _ptr(ay), _ptr(az)), "rb_gravity")


def rb_batch_gravity(ctx, parts: rb_particles, t: float, ax, ay, az) -> None:
    check(lib().rb_batch_gravity(ctx, ctypes.byref(parts), float(t), _ptr(ax), _ptr(ay),
                                 _ptr(az)), "rb_batch_gravity")


def rb_direct(ctx, parts: rb_particles, n: int, n_active: int, t: float, targets, ax, ay,
              az) -> None:
    check(lib().rb_direct(ctx, ctypes.byref(parts), int(n), int(n_active), float(t),
                          _ptr(targets), int(targets.numel()), _ptr(ax), _ptr(ay), _ptr(az)),
          "rb_direct")


def rb_direct_noalloc(p: rb_params, parts: rb_particles, n: int, n_active: int, t: float,
                      targets, ax, ay, az) -> None:
    """rb_direct without a context (rb.h), on the current torch stream."""
    check(lib().rb_direct_noalloc(ctypes.byref(p), ctypes.byref(parts), int(n), int(n_active),
                                  float(t), _ptr(targets), int(targets.numel()), _ptr(ax),
                                  _ptr(ay), _ptr(az), _stream_handle()), "rb_direct_noalloc")


def rb_step(ctx, parts: rb_particles, n: int, n_active: int, t: float, dt: float,
            nsteps: int) -> None:
    check(lib().rb_step(ctx, ctypes.byref(parts), int(n), int(n_active), float(t), float(dt),
                        int(nsteps)), "rb_step")


def rb_batch_step(ctx, parts: rb_particles, t: float, dt: float, nsteps: int) -> None:
    check(lib().rb_batch_step(ctx, ctypes.byref(parts), float(t), float(dt), int(nsteps)),
          "rb_batch_step")


def rb_sync(ctx) -> None:
    check(lib().rb_sync(ctx), "rb_sync")


def rb_stats(ctx) -> dict:
    s = rb_stats_t()
    check(lib().rb_stats(ctx, ctypes.byref(s)), "rb_stats")
    out = dict(open_tests=s.open_tests, cells=s.cells, pp=s.pp, list_cells=s.list_cells,
               list_pp=s.list_pp, reused_steps=s.reused_steps)
    out["ms"] = {name: s.ms[k] for k, name in enumerate(PHASES)}
    out["calls"] = {name: int(s.calls[k]) for k, name in enumerate(PHASES)}
    return out


def rb_state_save(ctx, parts: rb_particles, n: int, t: float, path: str) -> None:
    check(lib().rb_state_save(ctx, ctypes.byref(parts), int(n), float(t), path.encode()),
          "rb_state_save")


def rb_state_load(ctx, parts: rb_particles, n: int, path: str) -> float:
    t = ctypes.c_double()
    check(lib().rb_state_load(ctx, ctypes.byref(parts), int(n), ctypes.byref(t), path.encode()),
          "rb_state_load")
    return float(t.value)


def rb_error_string(code: int) -> str:
    return lib().rb_error_string(int(code)).decode()


def rb_last_error() -> str:
    return lib().rb_last_error().decode()


def rb_collide(ctx, parts, radius, n: int, t: float, epsilon: float, seed: int,
               codes=None):
    """Collisions at time t (rb.h); velocities of `parts` change in place.
    radius: device tensor (caller order).  codes: optional numpy uint64 array
    that receives the detected pair codes (unordered).  Returns
    (pairs, resolved)."""
    npairs, nres = ctypes.c_int64(0), ctypes.c_int64(0)
    cptr, ccap = None, 0
    if codes is not None:
        cptr, ccap = codes.ctypes.data_as(ctypes.c_void_p), len(codes)
    check(lib().rb_collide(ctx, ctypes.byref(parts), ctypes.c_void_p(_ptr(radius)), int(n),
                           float(t), float(epsilon), ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                           ctypes.byref(npairs), ctypes.byref(nres), cptr, ccap), "rb_collide")
    return int(npairs.value), int(nres.value)


def rb_sweep(ctx, parts, radius, n: int, t: float, dt: float, epsilon: float, seed: int,
             codes=None, axis: int = 0):
    """Collisions at time t found by the plane sweep over the past time-step
    dt (rb.h), along x (axis RB_SWEEP_X) or the azimuth (RB_SWEEP_PHI);
    velocities of `parts` change in place.  Returns (pairs, resolved)."""
    npairs, nres = ctypes.c_int64(0), ctypes.c_int64(0)
    cptr, ccap = None, 0
    if codes is not None:
        cptr, ccap = codes.ctypes.data_as(ctypes.c_void_p), len(codes)
    check(lib().rb_sweep(ctx, ctypes.byref(parts), ctypes.c_void_p(_ptr(radius)), int(n),
                         float(t), float(dt), int(axis), float(epsilon),
                         ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ctypes.byref(npairs),
                         ctypes.byref(nres), cptr, ccap), "rb_sweep")
    return int(npairs.value), int(nres.value)


def rb_peak_probe(kind: int) -> float:
    """Measured GPU ceiling (rb.h): 0 FP32 FMA flop/s (unpacked), 1 FP64 FMA
    flop/s, 2 HBM bytes/s of a streaming copy."""
    v = ctypes.c_double(0.0)
    check(lib().rb_peak_probe(int(kind), ctypes.byref(v)), "rb_peak_probe")
    return float(v.value)


def rb_set_collisions(ctx, radius, epsilon: float, seed: int, enable: bool = True) -> None:
    """Collisions at the end of every rb_step / rb_batch_step step (rb.h).
    radius: device tensor (caller order), kept alive by the caller."""
    check(lib().rb_set_collisions(ctx, ctypes.c_void_p(_ptr(radius) if enable else 0),
                                  float(epsilon), ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                                  int(bool(enable))), "rb_set_collisions")


def rb_collision_counts(ctx):
    """(pairs, resolved) of the steps since the last call (rb.h)."""
    a, b = ctypes.c_int64(0), ctypes.c_int64(0)
    check(lib().rb_collision_counts(ctx, ctypes.byref(a), ctypes.byref(b)),
          "rb_collision_counts")
    return int(a.value), int(b.value)
