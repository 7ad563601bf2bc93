"""FP64 CPU oracle for the mass-spring cloth step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package.
The product path (the HIP library and its binding) never imports it and shares no code with
it.  The arithmetic lives in ``cloth_oracle.c`` (plain C, FP64, single-threaded); this file
only builds that library, marshals numpy arrays into it, and adds a complex-step tangent
(``substep_jvp_cs``) written independently in numpy for checking the hand-written adjoint.

Every function takes plain arrays (positions [N,3], spring ends [S,2], ...); FP32 inputs are
upcast exactly to FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cloth_oracle.c")
_LIB = os.path.join(_HERE, "libcloth_oracle.so")
_lib = None


def build() -> str:
    """Compile cloth_oracle.c with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    fp = C.POINTER(C.c_float)
    lib.orc_model_new.restype = P
    lib.orc_model_new.argtypes = [C.c_int, dp, C.c_int, ip, dp, dp, dp, dp, C.c_int, dp, C.c_int,
                                  ip, C.c_double, C.c_double, C.c_double]
    lib.orc_model_free.argtypes = [P]
    lib.orc_model_set_params.argtypes = [P, dp, dp]
    lib.orc_forces.argtypes = [P, dp, dp, dp]
    lib.orc_substep.argtypes = [P, dp, dp, C.c_double, ip, dp]
    lib.orc_run.argtypes = [P, dp, dp, C.c_double, C.c_int]
    lib.orc_predict.argtypes = [P, dp, dp, C.c_double]
    lib.orc_respond.argtypes = [P, dp, dp, ip, C.c_int]
    lib.orc_box_candidates.restype = C.c_int
    lib.orc_box_candidates.argtypes = [P, dp, ip, dp, C.c_int]
    lib.orc_contacts.restype = C.c_int
    lib.orc_contacts.argtypes = [P, dp, ip, C.c_int]
    lib.orc_point_tri_dist2.restype = C.c_double
    lib.orc_point_tri_dist2.argtypes = [dp, dp, dp, dp]
    lib.orc_candidates_f32.restype = C.c_longlong
    lib.orc_candidates_f32.argtypes = [C.c_int, fp, C.c_int, fp, ip, C.c_float, ip, C.c_longlong]
    lib.orc_substep_vjp.argtypes = [P, dp, dp, C.c_double, dp, dp, dp, dp, dp, dp]
    lib.orc_substep_vjp_given.argtypes = [P, dp, dp, C.c_double, ip, ip, dp, dp, dp, dp, dp, dp]
    lib.orc_substep_given.argtypes = [P, dp, dp, C.c_double, ip, ip]
    lib.orc_run_given.argtypes = [P, dp, dp, C.c_double, C.c_int, ip, ip]
    lib.orc_check_contacts.restype = C.c_int
    lib.orc_check_contacts.argtypes = [P, dp, C.c_double, ip, ip, ip, C.POINTER(C.c_longlong)]
    lib.orc_rollout_grad.argtypes = [P, dp, dp, C.c_double, C.c_int, C.c_int, ip, dp, C.c_int,
                                     dp, dp, dp, dp, dp]
    lib.orc_model_triangle.argtypes = [P, C.c_int, dp, dp, dp, dp]
    lib.orc_vertex_normals.argtypes = [C.c_int, C.c_int, dp, dp]
    lib.orc_model_set_surface.argtypes = [P, dp]
    lib.orc_mt.restype = C.c_int
    lib.orc_mt.argtypes = [dp, dp, dp, dp, dp, C.c_double, dp, dp]
    lib.orc_mt_contacts.restype = C.c_int
    lib.orc_mt_contacts.argtypes = [P, C.c_int, C.c_int, dp, dp, C.c_int, ip, C.c_int, dp]
    lib.orc_substep_mt.argtypes = [P, C.c_int, C.c_int, dp, dp, C.c_double, ip, dp]
    lib.orc_mt_candidates.restype = C.c_int
    lib.orc_mt_candidates.argtypes = [P, C.c_int, C.c_int, dp, dp, C.c_int, ip, ip, dp, C.c_int]
    lib.orc_model_set_external.argtypes = [P, dp]
    _lib = lib
    return lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int))


class Model:
    """A cloth plus its static surface, held by the C oracle.

    inv_mass: [N] (0 marks a pinned node); ends [S,2]; rest/k/c [S]; verts [V,3];
    tris [T,3]; thickness (0 disables collision); cell: bucket size of the oracle's own
    acceleration grid (any positive value gives the same results).
    """

    def __init__(self, inv_mass, ends, rest, k, c, gravity=(0.0, -9.81, 0.0), verts=None,
                 tris=None, thickness=0.0, restitution=0.5, cell=0.0):
        self._lib = _load()
        self.w = _d(inv_mass)
        self.N = int(self.w.shape[0])
        self.ends = _i(ends).reshape(-1, 2)
        self.S = int(self.ends.shape[0])
        self.rest, self.k, self.c = _d(rest), _d(k), _d(c)
        self.g = _d(gravity)
        self.verts = _d(np.zeros((0, 3)) if verts is None else verts).reshape(-1, 3)
        self.tris = _i(np.zeros((0, 3)) if tris is None else tris).reshape(-1, 3)
        self.thickness = float(thickness)
        self.restitution = float(restitution)
        self._h = self._lib.orc_model_new(
            self.N, _dp(self.w), self.S, _ip(self.ends), _dp(self.rest), _dp(self.k),
            _dp(self.c), _dp(self.g), self.verts.shape[0], _dp(self.verts), self.tris.shape[0],
            _ip(self.tris), self.thickness, self.restitution, float(cell))

    @classmethod
    def from_inputs(cls, inp, k=None, c=None):
        """Build from any object with the ClothInputs fields."""
        m = np.asarray(inp.mass, dtype=np.float64)
        pinned = np.asarray(inp.pinned).astype(bool)
        w = np.where(pinned, 0.0, 1.0 / m)
        return cls(w, inp.ends, inp.rest, inp.k if k is None else k, inp.c if c is None else c,
                   inp.gravity, inp.verts, inp.tris, inp.thickness, inp.restitution,
                   inp.cell_size)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_model_free(h)
            self._h = None

    def set_params(self, k=None, c=None):
        if k is not None:
            self.k = _d(k)
        if c is not None:
            self.c = _d(c)
        self._lib.orc_model_set_params(self._h, _dp(self.k), _dp(self.c))

    def set_surface(self, verts):
        """Move the surface: new vertex positions [V,3] for the same triangles."""
        v = _d(verts).reshape(-1, 3)
        assert v.shape == self.verts.shape
        self.verts = v
        self._lib.orc_model_set_surface(self._h, _dp(self.verts))

    def set_external_force(self, f=None):
        """Per-node external forces [N,3] added before integration (None removes them)."""
        self.fext = None if f is None else _d(f).reshape(self.N, 3)
        self._lib.orc_model_set_external(self._h, None if f is None else _dp(self.fext))

    def mt_contacts(self, nx, ny, xs, xp, i):
        """Node i's contact set under the triangle-triangle narrow phase (ascending triangle
        ids) and the smallest decision margin of its tests."""
        xs, xp = _d(xs).reshape(-1, 3), _d(xp).reshape(-1, 3)
        out = np.zeros(512, dtype=np.int32)
        mg = np.zeros(1)
        n = self._lib.orc_mt_contacts(self._h, int(nx), int(ny), _dp(xs), _dp(xp), int(i),
                                      _ip(out), 512, _dp(mg))
        return out[:min(n, 512)].tolist(), float(mg[0])

    def mt_candidates(self, nx, ny, xs, xp, i):
        """Node i's candidate triangles (ascending) with hit flags and decision margins."""
        xs, xp = _d(xs).reshape(-1, 3), _d(xp).reshape(-1, 3)
        n = self._lib.orc_mt_candidates(self._h, int(nx), int(ny), _dp(xs), _dp(xp), int(i),
                                        None, None, None, 0)
        ids = np.zeros(max(n, 1), dtype=np.int32)
        hits = np.zeros(max(n, 1), dtype=np.int32)
        mg = np.zeros(max(n, 1))
        self._lib.orc_mt_candidates(self._h, int(nx), int(ny), _dp(xs), _dp(xp), int(i),
                                    _ip(ids), _ip(hits), _dp(mg), n)
        return ids[:n], hits[:n].astype(bool), mg[:n]

    def substep_mt(self, nx, ny, x, v, h):
        """One substep with the triangle-triangle narrow phase: (x1, v1, counts, margins)."""
        x = _d(x).reshape(-1, 3).copy()
        v = _d(v).reshape(-1, 3).copy()
        cnt = np.zeros(self.N, dtype=np.int32)
        mg = np.zeros(self.N)
        self._lib.orc_substep_mt(self._h, int(nx), int(ny), _dp(x), _dp(v), float(h), _ip(cnt),
                                 _dp(mg))
        return x, v, cnt, mg

    def forces(self, x, v):
        x, v = _d(x).reshape(-1, 3), _d(v).reshape(-1, 3)
        F = np.zeros((self.N, 3))
        self._lib.orc_forces(self._h, _dp(x), _dp(v), _dp(F))
        return F

    def substep(self, x, v, h):
        """One substep; returns (x, v, contact_count [N], margin [N])."""
        x, v = _d(x).reshape(-1, 3).copy(), _d(v).reshape(-1, 3).copy()
        cnt = np.zeros(self.N, dtype=np.int32)
        mg = np.zeros(self.N)
        self._lib.orc_substep(self._h, _dp(x), _dp(v), float(h), _ip(cnt), _dp(mg))
        return x, v, cnt, mg

    def run(self, x, v, h, n_sub):
        x, v = _d(x).reshape(-1, 3).copy(), _d(v).reshape(-1, 3).copy()
        self._lib.orc_run(self._h, _dp(x), _dp(v), float(h), int(n_sub))
        return x, v

    def predict(self, x, v, h):
        """Forces and integration only: returns (x*, v*)."""
        x, v = _d(x).reshape(-1, 3).copy(), _d(v).reshape(-1, 3).copy()
        self._lib.orc_predict(self._h, _dp(x), _dp(v), float(h))
        return x, v

    def respond(self, p, v, ids):
        """Response of one node at predicted (p, v) to the contact triangles ids."""
        p, v = _d(p).reshape(3).copy(), _d(v).reshape(3).copy()
        ids = _i(np.sort(np.asarray(ids, dtype=np.int64)))
        self._lib.orc_respond(self._h, _dp(p), _dp(v), _ip(ids), int(ids.shape[0]))
        return p, v

    def box_candidates(self, p):
        """(ids, exact distances) of every triangle whose inflated box holds p."""
        ids = np.zeros(1024, dtype=np.int32)
        dist = np.zeros(1024)
        n = self._lib.orc_box_candidates(self._h, _dp(_d(p).reshape(3)), _ip(ids), _dp(dist),
                                         1024)
        n = min(n, 1024)
        return ids[:n].copy(), dist[:n].copy()

    def contacts(self, p):
        out = np.zeros(512, dtype=np.int32)
        n = self._lib.orc_contacts(self._h, _dp(_d(p)), _ip(out), 512)
        return out[:min(n, 512)].copy()

    def triangle(self, t):
        A, n, lo, hi = (np.zeros(3) for _ in range(4))
        self._lib.orc_model_triangle(self._h, int(t), _dp(A), _dp(n), _dp(lo), _dp(hi))
        return A, n, lo, hi

    def substep_vjp(self, x, v, h, xb_out, vb_out):
        """Adjoint of one substep at (x, v): returns (xb_in, vb_in, kb, cb)."""
        x, v = _d(x).reshape(-1, 3), _d(v).reshape(-1, 3)
        xbo, vbo = _d(xb_out).reshape(-1, 3), _d(vb_out).reshape(-1, 3)
        xbi, vbi = np.zeros((self.N, 3)), np.zeros((self.N, 3))
        kb, cb = np.zeros(self.S), np.zeros(self.S)
        self._lib.orc_substep_vjp(self._h, _dp(x), _dp(v), float(h), _dp(xbo), _dp(vbo),
                                  _dp(xbi), _dp(vbi), _dp(kb), _dp(cb))
        return xbi, vbi, kb, cb

    def substep_vjp_given(self, x, v, h, contacts, xb_out, vb_out):
        """Adjoint of one substep at (x, v) with node i's contact triangles given as
        contacts[i] (a sequence of ids, or a (off, ids) pair as from contact_csr);
        returns (xb_in, vb_in, kb, cb)."""
        x, v = _d(x).reshape(-1, 3), _d(v).reshape(-1, 3)
        off, ids = self.contact_csr(contacts)
        xbo, vbo = _d(xb_out).reshape(-1, 3), _d(vb_out).reshape(-1, 3)
        xbi, vbi = np.zeros((self.N, 3)), np.zeros((self.N, 3))
        kb, cb = np.zeros(self.S), np.zeros(self.S)
        self._lib.orc_substep_vjp_given(self._h, _dp(x), _dp(v), float(h), _ip(off), _ip(ids),
                                        _dp(xbo), _dp(vbo), _dp(xbi), _dp(vbi), _dp(kb),
                                        _dp(cb))
        return xbi, vbi, kb, cb

    def contact_csr(self, contacts):
        """Per-node contact sets as (off [N+1], ids) int32 arrays, each set ascending.
        contacts: a sequence of N id sequences, or an (off, ids) pair (returned as is)."""
        if isinstance(contacts, tuple):
            off, ids = contacts
            return _i(off), _i(ids if len(ids) else np.zeros(1))
        off = np.zeros(self.N + 1, dtype=np.int32)
        off[1:] = np.cumsum([len(c) for c in contacts])
        ids = _i(np.concatenate([np.sort(np.asarray(c, dtype=np.int64)) for c in contacts])
                 if off[-1] else np.zeros(1))
        return off, ids

    def substep_given(self, x, v, h, contacts):
        """One substep with the contact sets held fixed (contacts as for contact_csr):
        the prediction, then each unpinned node's response to its given triangles."""
        x, v = _d(x).reshape(-1, 3).copy(), _d(v).reshape(-1, 3).copy()
        off, ids = self.contact_csr(contacts)
        self._lib.orc_substep_given(self._h, _dp(x), _dp(v), float(h), _ip(off), _ip(ids))
        return x, v

    def run_given(self, x, v, h, sets):
        """len(sets) substeps of substep_given; sets[s] = (off, ids) of substep s."""
        x, v = _d(x).reshape(-1, 3).copy(), _d(v).reshape(-1, 3).copy()
        n = len(sets)
        if n == 0:
            return x, v
        offs, chunks, base = [], [], 0
        for off, ids in sets:
            off = np.asarray(off, dtype=np.int64)
            offs.append(off + base)
            chunks.append(np.asarray(ids[:off[-1]], dtype=np.int64))
            base += int(off[-1])
        off_all = _i(np.concatenate(offs))
        ids_all = _i(np.concatenate(chunks) if base else np.zeros(1))
        self._lib.orc_run_given(self._h, _dp(x), _dp(v), float(h), n, _ip(off_all),
                                _ip(ids_all))
        return x, v

    def check_contacts(self, xp, contacts, border):
        """Validity of another implementation's contact sets at predicted positions xp:
        (status [N] with 0 = valid, 1 = a listed triangle farther than th + border, 2 = a
        triangle closer than th - border missing, 3 = contacts on a pinned node; the number
        of listed triangles within border of th)."""
        xp = _d(xp).reshape(-1, 3)
        off, ids = self.contact_csr(contacts)
        st = np.zeros(self.N, dtype=np.int32)
        nb = C.c_longlong(0)
        self._lib.orc_check_contacts(self._h, _dp(xp), float(border), _ip(off), _ip(ids),
                                     _ip(st), C.byref(nb))
        return st, int(nb.value)

    def rollout_grad(self, x0, v0, h, n_sub, out_sub, xbar, ckpt=1):
        """Checkpointed rollout gradient.

        out_sub: ascending substep counts at which the loss reads positions; xbar:
        [len(out_sub), N, 3] = dL/dx there.  Returns dict(x_out, gk, gc, gv0, gx0)."""
        x0, v0 = _d(x0).reshape(-1, 3), _d(v0).reshape(-1, 3)
        out_sub = _i(out_sub)
        n_out = int(out_sub.shape[0])
        xbar = _d(xbar).reshape(n_out, self.N, 3)
        x_out = np.zeros((n_out, self.N, 3))
        gk, gc = np.zeros(self.S), np.zeros(self.S)
        gv0, gx0 = np.zeros((self.N, 3)), np.zeros((self.N, 3))
        self._lib.orc_rollout_grad(self._h, _dp(x0), _dp(v0), float(h), int(n_sub), n_out,
                                   _ip(out_sub), _dp(xbar), int(ckpt), _dp(x_out), _dp(gk),
                                   _dp(gc), _dp(gv0), _dp(gx0))
        return dict(x_out=x_out, gk=gk, gc=gc, gv0=gv0, gx0=gx0)


def point_tri_dist2(p, A, B, Cc):
    lib = _load()
    return lib.orc_point_tri_dist2(_dp(_d(p)), _dp(_d(A)), _dp(_d(B)), _dp(_d(Cc)))


MT_EPS = 1e-7


def mt(S, E, V0, V1, V2, eps=MT_EPS):
    """Extended Moller-Trumbore segment-triangle test: (hit, t, margin)."""
    lib = _load()
    t = np.zeros(1)
    mg = np.zeros(1)
    hit = lib.orc_mt(_dp(_d(S)), _dp(_d(E)), _dp(_d(V0)), _dp(_d(V1)), _dp(_d(V2)), float(eps),
                     _dp(t), _dp(mg))
    return bool(hit), float(t[0]) if hit else None, float(mg[0])


def vertex_normals(nx, ny, x):
    """Per-vertex normals of an nx-by-ny cloth grid (area-weighted, normalised)."""
    lib = _load()
    x = _d(x).reshape(-1, 3)
    n = np.zeros_like(x)
    lib.orc_vertex_normals(int(nx), int(ny), _dp(x), _dp(n))
    return n


def candidates_f32(x, verts, tris, thickness, cap=None):
    """FP32 brute-force broad-phase pairs (node, tri), sorted by node then triangle."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1, 3)
    verts = np.ascontiguousarray(verts, dtype=np.float32).reshape(-1, 3)
    tris = _i(tris).reshape(-1, 3)
    fp = C.POINTER(C.c_float)
    n = lib.orc_candidates_f32(x.shape[0], x.ctypes.data_as(fp), tris.shape[0],
                               verts.ctypes.data_as(fp), _ip(tris), float(np.float32(thickness)),
                               None, 0)
    pairs = np.zeros((max(n, 1), 2), dtype=np.int32)
    lib.orc_candidates_f32(x.shape[0], x.ctypes.data_as(fp), tris.shape[0],
                           verts.ctypes.data_as(fp), _ip(tris), float(np.float32(thickness)),
                           _ip(pairs), n)
    return pairs[:n].copy()


from .cstep import substep_jvp_cs  # noqa: E402,F401
