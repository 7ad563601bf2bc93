"""ctypes binding of the HIP cloth library (include/cloth.h).

Argument marshalling only: every step of the simulation runs in the library's HIP kernels.
The functions keep the C names (cloth_create, cloth_step, ...); ``Cloth`` wraps a handle.
Loading fails loudly if libcloth.so cannot be built or loaded -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcloth.so")

CLOTH_OK, CLOTH_EINVAL, CLOTH_ENOMEM, CLOTH_EDEVICE = 0, -1, -2, -3
CLOTH_EUNSTABLE, CLOTH_ESTATE, CLOTH_ENAN = -4, -5, -6
CLOTH_F_CHECK_NAN, CLOTH_F_NO_STABILITY_CHECK, CLOTH_F_NARROW_MT = 0x1, 0x2, 0x4

_lib = None
_lock = threading.Lock()


class ClothError(RuntimeError):
    def __init__(self, status: int, text: str, detail: str):
        super().__init__(f"{text} ({status}): {detail}")
        self.status = status
        self.detail = detail


class cloth_launch(C.Structure):
    _fields_ = [("kernel", C.c_int), ("tile_nodes", C.c_int), ("substeps_per_launch", C.c_int),
                ("block_threads", C.c_int), ("use_graph", C.c_int), ("schedule", C.c_int),
                ("workgroups", C.c_int), ("hit_slots", C.c_int),
                ("xcd_runs", C.c_int), ("split_refs", C.c_int)]


CLOTH_KERNEL_TILE, CLOTH_KERNEL_DIRECT = 0, 1
CLOTH_KERNEL_SCATTER_F32, CLOTH_KERNEL_SCATTER_FIX = 2, 3
CLOTH_KERNEL_LANES2, CLOTH_KERNEL_LANES4, CLOTH_KERNEL_GRID = 4, 5, 6
CLOTH_SCHED_GRID, CLOTH_SCHED_LPT, CLOTH_SCHED_RR = 0, 1, 2


class cloth_sim_desc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("x0", C.c_void_p), ("v0", C.c_void_p),
                ("mass", C.c_void_p), ("pinned", C.c_void_p), ("n_springs", C.c_int),
                ("ends", C.c_void_p), ("rest", C.c_void_p), ("k", C.c_void_p), ("c", C.c_void_p),
                ("n_verts", C.c_int), ("verts", C.c_void_p), ("n_tris", C.c_int),
                ("tris", C.c_void_p)]


class cloth_params(C.Structure):
    _fields_ = [("gravity", C.c_float * 3), ("thickness", C.c_float), ("cell_size", C.c_float),
                ("restitution", C.c_float), ("flags", C.c_uint)]


_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int)
_u8p = C.POINTER(C.c_ubyte)
_llp = C.POINTER(C.c_longlong)
_vp = C.c_void_p

# (name, restype, argtypes)
_SIGNATURES = [
    ("cloth_create", C.c_int, [C.c_int, C.c_int, _fp, _fp, _fp, _u8p, C.c_int, _ip, _fp, _fp, _fp,
                               C.c_int, _fp, C.c_int, _ip, C.POINTER(cloth_params), _vp,
                               C.POINTER(_vp)]),
    ("cloth_step", C.c_int, [_vp, C.c_float, C.c_int, C.c_int]),
    ("cloth_read_state", C.c_int, [_vp, _fp, _fp]),
    ("cloth_write_state", C.c_int, [_vp, _fp, _fp]),
    ("cloth_device_state", C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp)]),
    ("cloth_node_order", C.c_int, [_vp, _ip]),
    ("cloth_info", C.c_int, [_vp, _llp]),
    ("cloth_destroy", C.c_int, [_vp]),
    ("cloth_debug_candidates", C.c_int, [_vp, C.c_int, _fp, _ip, C.c_longlong, _llp]),
    ("cloth_debug_candidates_noalloc", C.c_int, [_vp, C.c_int, _fp, _ip, C.c_longlong, _llp]),
    ("cloth_stability_bound", C.c_int, [C.c_int, _fp, _fp, _u8p, C.c_int, _ip, _fp, _fp,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("cloth_set_launch", C.c_int, [_vp, C.POINTER(cloth_launch)]),
    ("cloth_get_launch", C.c_int, [_vp, C.POINTER(cloth_launch)]),
    ("cloth_rollout_forward", C.c_int, [_vp, _vp, _vp, _vp, C.c_float, C.c_int, C.c_int, C.c_int,
                                        _ip, C.c_int, _vp]),
    ("cloth_rollout_backward", C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    ("cloth_autotune", C.c_int, [_vp, C.c_float, C.c_int, C.c_int, C.POINTER(cloth_launch)]),
    ("cloth_batch_create", C.c_int, [C.c_int, C.POINTER(cloth_sim_desc), C.POINTER(cloth_params),
                                     _vp, C.POINTER(_vp)]),
    ("cloth_batch_step", C.c_int, [_vp, C.c_float, C.c_int, C.c_int]),
    ("cloth_batch_read_state", C.c_int, [_vp, C.c_int, _fp, _fp]),
    ("cloth_batch_set_launch", C.c_int, [_vp, C.POINTER(cloth_launch)]),
    ("cloth_batch_get_launch", C.c_int, [_vp, C.POINTER(cloth_launch)]),
    ("cloth_batch_autotune", C.c_int, [_vp, C.c_float, C.c_int, C.c_int, C.POINTER(cloth_launch)]),
    ("cloth_batch_info", C.c_int, [_vp, _llp]),
    ("cloth_batch_destroy", C.c_int, [_vp]),
    ("cloth_debug_contacts", C.c_int, [_vp, C.c_float, _ip, _ip, C.c_int]),
    ("cloth_debug_query_volume", C.c_int, [_vp, C.c_float, _llp]),
    ("cloth_vertex_normals", C.c_int, [_vp, _vp]),
    ("cloth_update_surface", C.c_int, [_vp, _fp, C.c_int]),
    ("cloth_batch_update_surface", C.c_int, [_vp, C.c_int, _fp, C.c_int]),
    ("cloth_set_external_force", C.c_int, [_vp, _fp]),
    ("cloth_batch_set_external_force", C.c_int, [_vp, _fp]),
    ("cloth_batch_vertex_normals", C.c_int, [_vp, _vp]),
    ("cloth_status_str", C.c_char_p, [C.c_int]),
    ("cloth_last_error", C.c_char_p, []),
]


def load(path: str = LIB_PATH):
    """Load libcloth.so, building it first only if it does not exist."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            from . import build as _build
            _build.build()
        lib = C.CDLL(path)
        for name, res, args in _SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def _check(status: int):
    if status != CLOTH_OK:
        lib = load()
        raise ClothError(status, lib.cloth_status_str(status).decode(),
                         lib.cloth_last_error().decode())


def _f32(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _ptr(a, t):
    return None if a is None else a.ctypes.data_as(t)


def default_stream() -> int:
    """HIP stream handle of torch's current stream (0 if torch or a GPU is unavailable)."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return 0


def make_params(gravity=(0.0, -9.81, 0.0), thickness=0.0, cell_size=0.0, restitution=0.5,
                flags=0) -> cloth_params:
    p = cloth_params()
    for q in range(3):
        p.gravity[q] = float(gravity[q])
    p.thickness = float(thickness)
    p.cell_size = float(cell_size)
    p.restitution = float(restitution)
    p.flags = int(flags)
    return p


def cloth_create(nx, ny, x0, v0, mass, pinned, ends, rest, k, c, verts, tris, params,
                 stream=None):
    """Returns an opaque handle (int)."""
    lib = load()
    N = int(nx) * int(ny)
    x0 = _f32(x0).reshape(N, 3)
    v0 = None if v0 is None else _f32(v0).reshape(N, 3)
    mass = _f32(mass).reshape(N)
    pinned = None if pinned is None else np.ascontiguousarray(pinned, dtype=np.uint8).reshape(N)
    ends = np.ascontiguousarray(ends, dtype=np.int32).reshape(-1, 2)
    S = ends.shape[0]
    rest, k, c = _f32(rest).reshape(S), _f32(k).reshape(S), _f32(c).reshape(S)
    verts = _f32(np.zeros((0, 3)) if verts is None else verts).reshape(-1, 3)
    tris = np.ascontiguousarray(np.zeros((0, 3)) if tris is None else tris,
                                dtype=np.int32).reshape(-1, 3)
    out = _vp()
    st = lib.cloth_create(int(nx), int(ny), _ptr(x0, _fp), _ptr(v0, _fp), _ptr(mass, _fp),
                          _ptr(pinned, _u8p), S, _ptr(ends, _ip), _ptr(rest, _fp), _ptr(k, _fp),
                          _ptr(c, _fp), verts.shape[0], _ptr(verts, _fp), tris.shape[0],
                          _ptr(tris, _ip), C.byref(params),
                          _vp(default_stream() if stream is None else int(stream)), C.byref(out))
    _check(st)
    return out.value


def cloth_step(h, dt, n_substeps, n_steps):
    _check(load().cloth_step(_vp(h), float(dt), int(n_substeps), int(n_steps)))


def _state_out(a, n):
    """A caller-supplied output array for n nodes' state: float32, C-contiguous, [n, 3],
    writeable; None gives a new one."""
    if a is None:
        return np.empty((n, 3), dtype=np.float32)
    if (not isinstance(a, np.ndarray) or a.dtype != np.float32 or a.shape != (n, 3)
            or not a.flags.c_contiguous or not a.flags.writeable):
        raise ValueError(f"state output must be a writeable C-contiguous float32 array of "
                         f"shape ({n}, 3)")
    return a


def cloth_read_state(h, n, x=None, v=None):
    """The state (x, v), AoS [n, 3] in node-id order; x and v may be arrays to fill."""
    x = _state_out(x, n)
    v = _state_out(v, n)
    _check(load().cloth_read_state(_vp(h), _ptr(x, _fp), _ptr(v, _fp)))
    return x, v


def cloth_write_state(h, x, v=None):
    x = _f32(x)
    v = None if v is None else _f32(v)
    _check(load().cloth_write_state(_vp(h), _ptr(x, _fp), _ptr(v, _fp)))


def cloth_device_state(h):
    xp, vp = _vp(), _vp()
    _check(load().cloth_device_state(_vp(h), C.byref(xp), C.byref(vp)))
    return xp.value, vp.value


def cloth_node_order(h, n):
    order = np.zeros(n, dtype=np.int32)
    _check(load().cloth_node_order(_vp(h), _ptr(order, _ip)))
    return order


def cloth_info(h):
    out = np.zeros(8, dtype=np.int64)
    _check(load().cloth_info(_vp(h), _ptr(out, _llp)))
    keys = ("nodes", "springs", "tris", "cells", "refs", "dim_x", "dim_y", "dim_z")
    return dict(zip(keys, (int(x) for x in out)))


def cloth_destroy(h):
    if h:
        _check(load().cloth_destroy(_vp(h)))


def cloth_debug_candidates(h, points, noalloc=False):
    """Broad-phase (point, triangle) pairs of points [n, 3]; noalloc selects
    cloth_debug_candidates_noalloc (the library's fixed device scratch, no allocation)."""
    lib = load()
    fn = lib.cloth_debug_candidates_noalloc if noalloc else lib.cloth_debug_candidates
    P = _f32(points).reshape(-1, 3)
    n = C.c_longlong(0)
    _check(fn(_vp(h), P.shape[0], _ptr(P, _fp), None, 0, C.byref(n)))
    pairs = np.zeros((max(n.value, 1), 2), dtype=np.int32)
    n2 = C.c_longlong(0)
    _check(fn(_vp(h), P.shape[0], _ptr(P, _fp), _ptr(pairs, _ip), n.value, C.byref(n2)))
    return pairs[:n.value].copy()


def make_launch(kernel=CLOTH_KERNEL_DIRECT, tile_nodes=256, substeps_per_launch=1,
                block_threads=64, use_graph=1, schedule=CLOTH_SCHED_GRID, workgroups=0,
                hit_slots=32, xcd_runs=0, split_refs=0):
    return cloth_launch(int(kernel), int(tile_nodes), int(substeps_per_launch),
                        int(block_threads), int(use_graph), int(schedule), int(workgroups),
                        int(hit_slots), int(xcd_runs), int(split_refs))


def launch_dict(cfg: cloth_launch) -> dict:
    return {f: getattr(cfg, f) for f, _ in cloth_launch._fields_}


def cloth_set_launch(h, **kw):
    cfg = make_launch(**kw)
    _check(load().cloth_set_launch(_vp(h), C.byref(cfg)))


def cloth_get_launch(h) -> dict:
    cfg = cloth_launch()
    _check(load().cloth_get_launch(_vp(h), C.byref(cfg)))
    return launch_dict(cfg)


def cloth_autotune(h, dt, n_substeps, frames) -> dict:
    cfg = cloth_launch()
    _check(load().cloth_autotune(_vp(h), float(dt), int(n_substeps), int(frames), C.byref(cfg)))
    return launch_dict(cfg)


def cloth_rollout_forward(h, k_ptr, c_ptr, v0_ptr, dt, n_substeps, n_steps, ckpt_every,
                          out_steps, x_out_ptr):
    """Device pointers as ints (0 = NULL); out_steps is a host sequence of frame counts."""
    steps = np.ascontiguousarray(out_steps, dtype=np.int32)
    _check(load().cloth_rollout_forward(_vp(h), _vp(k_ptr), _vp(c_ptr), _vp(v0_ptr), float(dt),
                                        int(n_substeps), int(n_steps), int(ckpt_every),
                                        _ptr(steps, _ip), int(steps.shape[0]), _vp(x_out_ptr)))


def cloth_rollout_backward(h, gx_out_ptr, gk_ptr, gc_ptr, gv0_ptr):
    _check(load().cloth_rollout_backward(_vp(h), _vp(gx_out_ptr), _vp(gk_ptr), _vp(gc_ptr),
                                         _vp(gv0_ptr)))


def cloth_update_surface(h, verts):
    v = _f32(verts).reshape(-1, 3)
    _check(load().cloth_update_surface(_vp(h), _ptr(v, _fp), int(v.shape[0])))


def cloth_set_external_force(h, f):
    if f is None:
        _check(load().cloth_set_external_force(_vp(h), None))
    else:
        _check(load().cloth_set_external_force(_vp(h), _ptr(_f32(f).reshape(-1), _fp)))


def cloth_vertex_normals(h, n_out_ptr):
    """n_out_ptr: device pointer (int) to float[3 * N]; written on the handle's stream."""
    _check(load().cloth_vertex_normals(_vp(h), _vp(n_out_ptr)))


def cloth_batch_vertex_normals(h, n_out_ptr):
    _check(load().cloth_batch_vertex_normals(_vp(h), _vp(n_out_ptr)))


def _normals_tensor(n, out):
    import torch
    if out is None:
        out = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous() or out.numel() != 3 * n:
        raise ValueError("out must be a contiguous float32 CUDA tensor of 3*N elements")
    return out


def cloth_stability_bound(x0, mass, pinned, ends, k, c):
    """Host-only (omega2, gamma) bounds; see include/cloth.h."""
    lib = load()
    x0 = _f32(x0).reshape(-1, 3)
    n = x0.shape[0]
    mass = _f32(mass).reshape(n)
    pinned = None if pinned is None else np.ascontiguousarray(pinned, dtype=np.uint8).reshape(n)
    ends = np.ascontiguousarray(ends, dtype=np.int32).reshape(-1, 2)
    S = ends.shape[0]
    k, c = _f32(k).reshape(S), _f32(c).reshape(S)
    w2, g = C.c_double(0), C.c_double(0)
    _check(lib.cloth_stability_bound(n, _ptr(x0, _fp), _ptr(mass, _fp), _ptr(pinned, _u8p), S,
                                     _ptr(ends, _ip), _ptr(k, _fp), _ptr(c, _fp), C.byref(w2),
                                     C.byref(g)))
    return w2.value, g.value


class Cloth:
    """One simulation handle built from a ClothInputs-like object."""

    def __init__(self, inp, flags=0, stream=None):
        self.inp = inp
        self.n = int(inp.nx * inp.ny)
        self.params = make_params(inp.gravity, inp.thickness, inp.cell_size, inp.restitution,
                                  flags)
        self.h = cloth_create(inp.nx, inp.ny, inp.x0, inp.v0, inp.mass, inp.pinned, inp.ends,
                              inp.rest, inp.k, inp.c, inp.verts, inp.tris, self.params, stream)

    def step(self, dt=None, n_substeps=None, n_steps=1):
        cloth_step(self.h, self.inp.dt if dt is None else dt,
                   self.inp.n_substeps if n_substeps is None else n_substeps, n_steps)

    def read_state(self, x=None, v=None):
        return cloth_read_state(self.h, self.n, x, v)

    def write_state(self, x, v=None):
        cloth_write_state(self.h, x, v)

    def device_state(self):
        return cloth_device_state(self.h)

    def node_order(self):
        return cloth_node_order(self.h, self.n)

    def info(self):
        return cloth_info(self.h)

    def set_launch(self, **kw):
        cfg = dict(self.get_launch())
        cfg.update(kw)
        cloth_set_launch(self.h, **cfg)

    def get_launch(self):
        return cloth_get_launch(self.h)

    def debug_candidates(self, points, noalloc=False):
        return cloth_debug_candidates(self.h, points, noalloc=noalloc)

    def update_surface(self, verts):
        """Move the collision surface: new vertex positions [V, 3], same triangles."""
        cloth_update_surface(self.h, verts)

    def set_external_force(self, f=None):
        """Per-node external forces [N, 3] in newtons (None removes them)."""
        if f is not None and np.asarray(f).size != 3 * self.n:
            raise ValueError("f must hold N x 3 values")
        cloth_set_external_force(self.h, f)

    def vertex_normals(self, out=None):
        """Per-vertex normals [N, 3] of the current state as a CUDA tensor, written on the
        handle's stream (torch's current stream when the handle was made)."""
        out = _normals_tensor(self.n, out)
        cloth_vertex_normals(self.h, out.data_ptr())
        return out

    def debug_contacts(self, h, cap=16, csr=False):
        """Per node, the ascending triangle ids of its contacts in a substep of length h (a
        list of lists; with csr=True, (off [N+1], ids) int32 arrays)."""
        counts = np.zeros(self.n, dtype=np.int32)
        ids = np.zeros(self.n * cap, dtype=np.int32)
        _check(load().cloth_debug_contacts(_vp(self.h), float(h), _ptr(counts, _ip),
                                           _ptr(ids, _ip), int(cap)))
        assert counts.max(initial=0) <= cap, "raise cap"
        if csr:
            off = np.zeros(self.n + 1, dtype=np.int32)
            np.cumsum(counts, out=off[1:])
            keep = np.arange(cap)[None, :] < counts[:, None]
            return off, ids.reshape(self.n, cap)[keep].astype(np.int32)
        return [ids[i * cap:i * cap + counts[i]].tolist() for i in range(self.n)]

    def query_volume(self, h=None):
        """Surface data the next substep's collision query touches (cloth_debug_query_volume):
        dict of distinct non-empty cells queried, their references, distinct box-hit
        triangles, node queries, references tested and box hits over all nodes."""
        if h is None:
            h = float(np.float32(np.float32(self.inp.dt) / np.float32(self.inp.n_substeps)))
        out = np.zeros(6, dtype=np.int64)
        _check(load().cloth_debug_query_volume(_vp(self.h), float(h), _ptr(out, _llp)))
        keys = ("cells", "cell_refs", "candidate_tris", "node_queries", "refs_tested",
                "box_hits")
        return {k: int(v) for k, v in zip(keys, out)}

    def autotune(self, frames=10, dt=None, n_substeps=None):
        return cloth_autotune(self.h, self.inp.dt if dt is None else dt,
                              self.inp.n_substeps if n_substeps is None else n_substeps, frames)

    def close(self):
        if getattr(self, "h", None):
            cloth_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ClothBatch:
    """Many independent cloths (ClothInputs-like objects) stepped together.

    Every cloth shares dt, n_substeps, gravity, thickness and restitution (taken from the
    first); each keeps its own springs, surface and (with cell_size <= 0 in the shared
    parameters) its own grid cell."""

    def __init__(self, inputs, flags=0, stream=None, cell_size=0.0):
        lib = load()
        self.inputs = list(inputs)
        first = self.inputs[0]
        self.params = make_params(first.gravity, first.thickness, cell_size, first.restitution,
                                  flags)
        self._keep = []
        descs = (cloth_sim_desc * len(self.inputs))()
        for d, inp in zip(descs, self.inputs):
            arrs = dict(
                x0=_f32(inp.x0), v0=_f32(inp.v0), mass=_f32(inp.mass),
                pinned=np.ascontiguousarray(inp.pinned, dtype=np.uint8),
                ends=np.ascontiguousarray(inp.ends, dtype=np.int32), rest=_f32(inp.rest),
                k=_f32(inp.k), c=_f32(inp.c), verts=_f32(inp.verts),
                tris=np.ascontiguousarray(inp.tris, dtype=np.int32))
            self._keep.append(arrs)
            d.nx, d.ny = int(inp.nx), int(inp.ny)
            for f in ("x0", "v0", "mass", "pinned", "ends", "rest", "k", "c", "verts", "tris"):
                setattr(d, f, arrs[f].ctypes.data)
            d.n_springs = int(arrs["ends"].shape[0])
            d.n_verts = int(arrs["verts"].reshape(-1, 3).shape[0])
            d.n_tris = int(arrs["tris"].reshape(-1, 3).shape[0])
        out = _vp()
        st = lib.cloth_batch_create(len(self.inputs), descs, C.byref(self.params),
                                    _vp(default_stream() if stream is None else int(stream)),
                                    C.byref(out))
        self._keep = None
        _check(st)
        self.h = out.value

    def step(self, n_steps=1, dt=None, n_substeps=None):
        first = self.inputs[0]
        _check(load().cloth_batch_step(_vp(self.h), float(first.dt if dt is None else dt),
                                       int(first.n_substeps if n_substeps is None else n_substeps),
                                       int(n_steps)))

    def read_state(self, i):
        n = int(self.inputs[i].nx * self.inputs[i].ny)
        x = np.zeros((n, 3), dtype=np.float32)
        v = np.zeros((n, 3), dtype=np.float32)
        _check(load().cloth_batch_read_state(_vp(self.h), int(i), _ptr(x, _fp), _ptr(v, _fp)))
        return x, v

    def update_surface(self, i, verts):
        v = _f32(verts).reshape(-1, 3)
        _check(load().cloth_batch_update_surface(_vp(self.h), int(i), _ptr(v, _fp),
                                                 int(v.shape[0])))

    def set_external_force(self, f=None):
        """Per-node external forces [sum N_i, 3] (cloth after cloth; None removes them)."""
        n = sum(int(i.nx * i.ny) for i in self.inputs)
        if f is None:
            _check(load().cloth_batch_set_external_force(_vp(self.h), None))
            return
        f = _f32(f).reshape(-1)
        if f.size != 3 * n:
            raise ValueError("f must hold sum(N_i) x 3 values")
        _check(load().cloth_batch_set_external_force(_vp(self.h), _ptr(f, _fp)))

    def vertex_normals(self, out=None):
        """Per-vertex normals [sum N_i, 3] of every cloth, cloth after cloth (CUDA tensor)."""
        out = _normals_tensor(sum(int(i.nx * i.ny) for i in self.inputs), out)
        cloth_batch_vertex_normals(self.h, out.data_ptr())
        return out

    def set_launch(self, **kw):
        cfg = self.get_launch()
        cfg.update(kw)
        c = make_launch(**cfg)
        _check(load().cloth_batch_set_launch(_vp(self.h), C.byref(c)))

    def get_launch(self):
        cfg = cloth_launch()
        _check(load().cloth_batch_get_launch(_vp(self.h), C.byref(cfg)))
        return launch_dict(cfg)

    def autotune(self, frames=3, dt=None, n_substeps=None):
        first = self.inputs[0]
        cfg = cloth_launch()
        _check(load().cloth_batch_autotune(
            _vp(self.h), float(first.dt if dt is None else dt),
            int(first.n_substeps if n_substeps is None else n_substeps), int(frames),
            C.byref(cfg)))
        return launch_dict(cfg)

    def info(self):
        out = np.zeros(6, dtype=np.int64)
        _check(load().cloth_batch_info(_vp(self.h), _ptr(out, _llp)))
        keys = ("cloths", "nodes", "springs", "tris", "tiles", "workgroups")
        return dict(zip(keys, (int(x) for x in out)))

    def close(self):
        if getattr(self, "h", None):
            _check(load().cloth_batch_destroy(_vp(self.h)))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
