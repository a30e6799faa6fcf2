"""Thin ctypes binding of librpd (include/rpd.h): argument marshalling only; every step runs in the library.

Inputs may be numpy arrays (host) or torch tensors on a HIP device (passed as device pointers with
RPD_DEVICE_PTRS). The library must have been built (``paper_2403_18761_amd/build.py``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpd.so")

RPD_OK = 0
RPD_E_INVALID, RPD_E_MESH, RPD_E_DEGENERATE, RPD_E_NOMEM, RPD_E_DEVICE, RPD_E_INTERNAL = -1, -2, -3, -4, -5, -6
ERRORS = {-1: "RPD_E_INVALID", -2: "RPD_E_MESH", -3: "RPD_E_DEGENERATE", -4: "RPD_E_NOMEM", -5: "RPD_E_DEVICE",
          -6: "RPD_E_INTERNAL"}
RPD_FP32_FALLBACK = 0
RPD_FP64 = 1
RPD_CELL, RPD_FACE, RPD_EDGE, RPD_VERTEX = 1, 2, 3, 4
RPD_DEVICE_PTRS = 1 << 0
RPD_FORCE_FP64 = 1 << 1
RPD_FORCE_EXACT = 1 << 2
RPD_FORCE_SLOW_PATH = 1 << 3
RPD_TIMING = 1 << 4
RPD_KEEP_PIECES = 1 << 5
RPD_OWNER_WEIGHTS = 1 << 6
RPD_SHUFFLE_QUEUE = 1 << 7
RPD_ESTIMATED_ORDER = 1 << 8
RPD_NO_SPLIT = 1 << 9
RPD_NOALLOC_SCRATCH_BYTES = 64 << 20  # the no-allocation entry point's working memory per device

_f32p = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)


class _MeshDesc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("vx", _f32p), ("vy", _f32p), ("vz", _f32p), ("n_tets", C.c_int32),
                ("tv", _i32p)]


class _MeshInfo(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("n_edges", C.c_int32), ("n_faces", C.c_int32),
                ("euler", C.c_int32), ("components", C.c_int32), ("L", C.c_int64), ("volume", C.c_double),
                ("owner_weights", C.c_int32), ("n_blocks", C.c_int32)]


class _Sites(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("sx", _f32p), ("sy", _f32p), ("sz", _f32p), ("sr", _f32p)]


class _Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("clip_budget", C.c_int32), ("block", C.c_int32), ("flags", C.c_uint32),
                ("stream", C.c_void_p), ("slots", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_candidates", C.c_int64), ("n_deferred", C.c_int64),
                ("n_fp64", C.c_int64), ("n_exact", C.c_int64), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("n_edges", C.c_int64), ("n_rpv", C.c_int64), ("n_glue", C.c_int64), ("ms_clip", C.c_double),
                ("ms_deferred", C.c_double), ("ms_reduce", C.c_double), ("ms_total", C.c_double),
                ("n_defer_block", C.c_int64), ("n_defer_kmax", C.c_int64), ("n_defer_clip", C.c_int64), ("n_split", C.c_int64),
                ("n_items", C.c_int64), ("n_big", C.c_int64)]


class _SessionOpts(C.Structure):
    _fields_ = [("max_sites", C.c_int32), ("max_insert", C.c_int32), ("build", _Opts), ("insertion", C.c_int32)]


class _SessionInfo(C.Structure):
    _fields_ = [("n_sites", C.c_int32), ("rounds", C.c_int32), ("n_selected", C.c_int32), ("n_blocks", C.c_int32),
                ("n_inserted", C.c_int64), ("n_dirty_blocks", C.c_int64), ("n_clipped", C.c_int64),
                ("ms_last_run", C.c_double)]


class RPDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load librpd.so; raise if it has not been built (the product has no CPU path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2403_18761_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    lib.rpd_mesh_create.argtypes = [C.POINTER(_MeshDesc), C.c_uint32, C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rpd_mesh_get_info.argtypes = [C.c_void_p, C.POINTER(_MeshInfo)]
    lib.rpd_mesh_free.argtypes = [C.c_void_p]
    lib.rpd_mesh_free.restype = None
    lib.rpd_build.argtypes = [C.POINTER(C.c_void_p), C.POINTER(_Sites), C.c_int32, C.POINTER(_Opts),
                              C.POINTER(C.c_void_p)]
    lib.rpd_euler.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(_i32p),
                              C.POINTER(_i32p)]
    lib.rpd_components.argtypes = lib.rpd_euler.argtypes
    lib.rpd_geometry.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.POINTER(C.c_double)),
                                 C.POINTER(C.POINTER(C.c_double))]
    lib.rpd_adjacency.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(_i32p)]
    lib.rpd_get_stats.argtypes = [C.c_void_p, C.POINTER(_Stats)]
    lib.rpd_edge_geometry.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.POINTER(C.c_double)),
                                      C.POINTER(C.POINTER(C.c_double))]
    lib.rpd_medial_euler.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    lib.rpd_envelope_distance.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                          C.c_void_p, C.c_int64, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p,
                                          C.POINTER(C.c_float)]
    lib.rpd_envelope_distance_noalloc.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                                  C.c_int64, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                                  C.c_void_p]
    lib.rpd_shrink_spheres.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.c_uint32, C.c_void_p, C.c_void_p]
    lib.rpd_thin.argtypes = [C.c_int32, C.c_int64, _i32p, C.c_int64, _i32p, C.POINTER(C.c_double), C.c_int64, _i32p,
                             C.c_double, C.POINTER(C.c_uint8), C.POINTER(C.c_uint8), C.POINTER(C.c_uint8)]
    lib.rpd_pieces.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(_i32p), C.POINTER(_i32p),
                               C.POINTER(C.POINTER(C.c_double)), C.POINTER(C.POINTER(C.c_int64))]
    lib.rpd_piece_terms.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(_i32p),
                                    C.POINTER(_i32p), C.POINTER(C.POINTER(C.c_int64)), C.POINTER(_i32p)]
    lib.rpd_free.argtypes = [C.c_void_p]
    lib.rpd_free.restype = None
    lib.rpd_last_error.restype = C.c_char_p
    lib.rpd_version.restype = C.c_char_p
    lib.rpd_autotune.argtypes = [C.POINTER(C.c_void_p), C.POINTER(_Sites), C.c_int32, C.POINTER(_Opts),
                                 C.POINTER(_Opts)]
    lib.rpd_session_create.argtypes = [C.c_void_p, C.POINTER(_Sites), C.POINTER(_Sites), C.POINTER(_SessionOpts),
                                       C.POINTER(C.c_void_p)]
    lib.rpd_session_run.argtypes = [C.c_void_p, C.c_int32]
    lib.rpd_session_result.argtypes = [C.c_void_p, C.POINTER(C.c_void_p)]
    lib.rpd_session_get_info.argtypes = [C.c_void_p, C.POINTER(_SessionInfo)]
    lib.rpd_session_sites.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_int32)]
    lib.rpd_session_free.argtypes = [C.c_void_p]
    lib.rpd_session_free.restype = None
    for f in ("rpd_mesh_create", "rpd_mesh_get_info", "rpd_build", "rpd_euler", "rpd_components", "rpd_geometry",
              "rpd_adjacency", "rpd_get_stats", "rpd_pieces", "rpd_piece_terms", "rpd_session_create", "rpd_session_run",
              "rpd_session_result", "rpd_session_get_info", "rpd_session_sites", "rpd_autotune",
              "rpd_edge_geometry", "rpd_medial_euler", "rpd_thin", "rpd_envelope_distance",
              "rpd_envelope_distance_noalloc",
              "rpd_shrink_spheres"):
        getattr(lib, f).restype = C.c_int32
    _lib = lib
    return lib


def _check(code: int):
    if code != RPD_OK:
        raise RPDError(code, load().rpd_last_error().decode())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, ctype, keep: list):
    """Pointer to the data of a numpy array (host) or a contiguous torch tensor (device)."""
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return C.cast(C.c_void_p(x.data_ptr()), C.POINTER(ctype))
    a = np.ascontiguousarray(x, dtype={C.c_float: np.float32, C.c_int32: np.int32}[ctype])
    keep.append(a)
    return a.ctypes.data_as(C.POINTER(ctype))


def _stream_ptr(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


class Mesh:
    """A prepared tet mesh (rpd_mesh_create)."""

    def __init__(self, vx, vy, vz, tv, stream=None, owner_weights: bool = False):
        lib = load()
        keep = []
        dev = _is_torch(vx) and vx.is_cuda
        tv_flat = tv.reshape(-1) if hasattr(tv, "reshape") else tv
        d = _MeshDesc(int(vx.shape[0]), _ptr(vx, C.c_float, keep), _ptr(vy, C.c_float, keep),
                      _ptr(vz, C.c_float, keep), int(tv_flat.shape[0]) // 4, _ptr(tv_flat, C.c_int32, keep))
        h = C.c_void_p()
        fl = (RPD_DEVICE_PTRS if dev else 0) | (RPD_OWNER_WEIGHTS if owner_weights else 0)
        _check(lib.rpd_mesh_create(C.byref(d), fl, _stream_ptr(stream), C.byref(h)))
        self._h = h
        self._lib = lib

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = _MeshInfo()
        _check(self._lib.rpd_mesh_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in _MeshInfo._fields_}

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.rpd_mesh_free(self._h)
            self._h = C.c_void_p()


class Result:
    """Host-visible results of one rpd_build call."""

    def __init__(self, h, n_shapes):
        self._h = h
        self._lib = load()
        self.n_shapes = n_shapes

    def _elem(self, fn, shape, kind):
        n = C.c_int64()
        keys, vals = _i32p(), _i32p()
        _check(fn(self._h, shape, kind, C.byref(n), C.byref(keys), C.byref(vals)))
        width = {RPD_CELL: 1, RPD_FACE: 2, RPD_EDGE: 3}[kind]
        k = np.ctypeslib.as_array(keys, shape=(n.value * width,)).copy() if n.value else np.zeros(0, np.int32)
        v = np.ctypeslib.as_array(vals, shape=(n.value,)).copy() if n.value else np.zeros(0, np.int32)
        return k.reshape(-1, width) if kind != RPD_CELL else k, v

    def euler(self, shape: int, kind: int):
        """(keys, chi) for kind RPD_CELL / RPD_FACE / RPD_EDGE."""
        return self._elem(self._lib.rpd_euler, shape, kind)

    def components(self, shape: int, kind: int):
        """(keys, beta0) for kind RPD_CELL / RPD_FACE / RPD_EDGE."""
        return self._elem(self._lib.rpd_components, shape, kind)

    def geometry(self, shape: int):
        vol, cen = C.POINTER(C.c_double)(), C.POINTER(C.c_double)()
        _check(self._lib.rpd_geometry(self._h, shape, C.byref(vol), C.byref(cen)))
        n = self.euler(shape, RPD_CELL)[1].shape[0]
        return (np.ctypeslib.as_array(vol, shape=(n,)).copy(),
                np.ctypeslib.as_array(cen, shape=(3 * n,)).copy().reshape(n, 3))

    def adjacency(self, shape: int, kind: int):
        n = C.c_int64()
        keys = _i32p()
        _check(self._lib.rpd_adjacency(self._h, shape, kind, C.byref(n), C.byref(keys)))
        width = {RPD_FACE: 2, RPD_EDGE: 3, RPD_VERTEX: 4}[kind]
        if n.value == 0:
            return np.zeros((0, width), np.int32)
        return np.ctypeslib.as_array(keys, shape=(n.value * width,)).copy().reshape(-1, width)

    def edge_geometry(self, shape: int):
        """(length, alpha) of every RPE, in the order of euler(shape, RPD_EDGE)."""
        n = C.c_int64()
        ln, al = C.POINTER(C.c_double)(), C.POINTER(C.c_double)()
        _check(self._lib.rpd_edge_geometry(self._h, shape, C.byref(n), C.byref(ln), C.byref(al)))
        if n.value == 0:
            return np.zeros(0), np.zeros(0)
        return (np.ctypeslib.as_array(ln, shape=(n.value,)).copy(),
                np.ctypeslib.as_array(al, shape=(n.value,)).copy())

    def medial_euler(self, shape: int):
        """((V, E, F, T), chi) of the dual medial mesh."""
        counts = (C.c_int64 * 4)()
        chi = C.c_int64()
        _check(self._lib.rpd_medial_euler(self._h, shape, counts, C.byref(chi)))
        return tuple(int(c) for c in counts), int(chi.value)

    def medial_mesh(self, shape: int, xyzr, sigma: float | None = 0.3):
        """The dual medial mesh of one shape as enveloping elements: spheres (V, 4) of the sites whose cell is
        nonempty (xyzr: the shape's sites, (n, 4)), edges (E, 2) and triangles (F, 3) indexing those spheres, after
        rpd_thin with this sigma (None: unthinned; medial tets have no enveloping element and are dropped)."""
        xyzr = np.asarray(xyzr, np.float32).reshape(-1, 4)
        _, b0 = self.components(shape, RPD_CELL)
        e = self.adjacency(shape, RPD_FACE)
        f = self.adjacency(shape, RPD_EDGE)
        if sigma is not None:
            _, alpha = self.edge_geometry(shape)
            ke, kf, _ = thin(len(b0), e, f, alpha, self.adjacency(shape, RPD_VERTEX), sigma)
            e, f = e[ke], f[kf]
        live = np.flatnonzero(b0 > 0)
        remap = np.full(len(b0), -1, np.int32)
        remap[live] = np.arange(len(live), dtype=np.int32)
        return xyzr[live], remap[e], remap[f]

    def stats(self) -> dict:
        s = _Stats()
        _check(self._lib.rpd_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}

    def pieces(self, shape: int) -> dict:
        n = C.c_int64()
        t, i = _i32p(), _i32p()
        geo = C.POINTER(C.c_double)()
        chi = C.POINTER(C.c_int64)()
        _check(self._lib.rpd_pieces(self._h, shape, C.byref(n), C.byref(t), C.byref(i), C.byref(geo), C.byref(chi)))
        m = n.value
        if m == 0:
            return dict(t=np.zeros(0, np.int32), i=np.zeros(0, np.int32), geo=np.zeros((0, 4)),
                        chi=np.zeros(0, np.int64))
        return dict(t=np.ctypeslib.as_array(t, shape=(m,)).copy(), i=np.ctypeslib.as_array(i, shape=(m,)).copy(),
                    geo=np.ctypeslib.as_array(geo, shape=(4 * m,)).copy().reshape(m, 4),
                    chi=np.ctypeslib.as_array(chi, shape=(m,)).copy())

    def piece_terms(self, shape: int, kind: int) -> dict:
        """Per-piece element terms of one kind (RPD_KEEP_PIECES): t [m], sites [m, kind], num [m], glue [m]."""
        n = C.c_int64()
        t, sv, g = _i32p(), _i32p(), _i32p()
        num = C.POINTER(C.c_int64)()
        _check(self._lib.rpd_piece_terms(self._h, shape, kind, C.byref(n), C.byref(t), C.byref(sv), C.byref(num),
                                         C.byref(g)))
        m = n.value
        if m == 0:
            return dict(t=np.zeros(0, np.int32), sites=np.zeros((0, kind), np.int32), num=np.zeros(0, np.int64),
                        glue=np.zeros(0, np.int32))
        return dict(t=np.ctypeslib.as_array(t, shape=(m,)).copy(),
                    sites=np.ctypeslib.as_array(sv, shape=(m * kind,)).copy().reshape(m, kind),
                    num=np.ctypeslib.as_array(num, shape=(m,)).copy(),
                    glue=np.ctypeslib.as_array(g, shape=(m,)).copy())

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.rpd_free(self._h)
            self._h = C.c_void_p()


def build(meshes, sites, precision: int = RPD_FP32_FALLBACK, clip_budget: int = 0, block: int = 0,
          flags: int = 0, stream=None, slots: int = 0) -> Result:
    """rpd_build over shapes: ``meshes`` a list of Mesh, ``sites`` a list of (sx, sy, sz, sr) arrays or tensors."""
    lib = load()
    n = len(meshes)
    keep = []
    handles = (C.c_void_p * n)(*[m.handle.value for m in meshes])
    st = (_Sites * n)()
    dev = False
    for k, (sx, sy, sz, sr) in enumerate(sites):
        dev = dev or (_is_torch(sx) and sx.is_cuda)
        st[k] = _Sites(int(sx.shape[0]), _ptr(sx, C.c_float, keep), _ptr(sy, C.c_float, keep),
                       _ptr(sz, C.c_float, keep), _ptr(sr, C.c_float, keep))
    o = _Opts(precision, clip_budget, block, flags | (RPD_DEVICE_PTRS if dev else 0), _stream_ptr(stream), slots)
    h = C.c_void_p()
    _check(lib.rpd_build(handles, st, n, C.byref(o), C.byref(h)))
    return Result(h, n)


def autotune(meshes, sites, flags: int = 0, stream=None) -> dict:
    """rpd_autotune: time every launch shape on these inputs; returns the chosen {"block", "clip_budget", "slots"}
    (also cached in the library for rpd_build calls that leave them at 0)."""
    lib = load()
    n = len(meshes)
    keep = []
    handles = (C.c_void_p * n)(*[m.handle.value for m in meshes])
    st = (_Sites * n)()
    dev = False
    for k, (sx, sy, sz, sr) in enumerate(sites):
        dev = dev or (_is_torch(sx) and sx.is_cuda)
        st[k] = _Sites(int(sx.shape[0]), _ptr(sx, C.c_float, keep), _ptr(sy, C.c_float, keep),
                       _ptr(sz, C.c_float, keep), _ptr(sr, C.c_float, keep))
    o = _Opts(RPD_FP32_FALLBACK, 0, 0, flags | (RPD_DEVICE_PTRS if dev else 0), _stream_ptr(stream), 0)
    best = _Opts()
    _check(lib.rpd_autotune(handles, st, n, C.byref(o), C.byref(best)))
    return {"block": best.block, "clip_budget": best.clip_budget, "slots": best.slots}


def thin(n_vertices: int, edges, tris, alpha, tets, sigma: float):
    """rpd_thin on host arrays: returns the keep masks (edges, triangles, tets) as bool arrays."""
    lib = load()
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    f = np.ascontiguousarray(np.asarray(tris, np.int32).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(tets, np.int32).reshape(-1, 4))
    a = np.ascontiguousarray(np.asarray(alpha, np.float64).reshape(-1))
    if a.shape[0] != f.shape[0]:
        raise ValueError("alpha needs one value per triangle")
    ke, kf, kt = (np.zeros(max(x.shape[0], 1), np.uint8) for x in (e, f, t))
    i32 = lambda x: x.ctypes.data_as(_i32p)
    u8 = lambda x: x.ctypes.data_as(C.POINTER(C.c_uint8))
    _check(lib.rpd_thin(int(n_vertices), e.shape[0], i32(e), f.shape[0], i32(f),
                        a.ctypes.data_as(C.POINTER(C.c_double)), t.shape[0], i32(t), float(sigma), u8(ke), u8(kf),
                        u8(kt)))
    return ke[:e.shape[0]].astype(bool), kf[:f.shape[0]].astype(bool), kt[:t.shape[0]].astype(bool)


def envelope_distance(spheres, edges, tris, samples, stream=None, timing: bool = False, nearest: bool = True):
    """rpd_envelope_distance: distance from each sample to the enveloping volume of a medial mesh.

    spheres (n, 4) float32 (x, y, z, r); edges (m, 2) and tris (k, 3) int32 sphere ids; samples (s, 3) float32.
    CUDA tensors run on the device (outputs are tensors on that device); numpy arrays go through host memory.
    Returns (dist float32 [s], nearest int32 [s] or None when not asked for), plus the distance kernel's HIP-event
    ms when timing is set."""
    lib = load()
    kms = C.c_float(0.0)
    kptr = C.byref(kms) if timing else None
    if _is_torch(samples) and samples.is_cuda:
        import torch

        dev = samples.device
        sp = spheres.to(dev, torch.float32).contiguous().reshape(-1, 4)
        ed = edges.to(dev, torch.int32).contiguous().reshape(-1, 2)
        tr = tris.to(dev, torch.int32).contiguous().reshape(-1, 3)
        q = samples.to(torch.float32).contiguous().reshape(-1, 3)
        dist = torch.empty(q.shape[0], dtype=torch.float32, device=dev)
        near = torch.empty(q.shape[0], dtype=torch.int32, device=dev) if nearest else None
        ptr = lambda t: C.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)
        st = _stream_ptr(stream) if stream is not None else C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        _check(lib.rpd_envelope_distance(ptr(sp), sp.shape[0], ptr(ed), ed.shape[0], ptr(tr), tr.shape[0], ptr(q),
                                         q.shape[0], RPD_DEVICE_PTRS, st, ptr(dist), ptr(near), kptr))
        return (dist, near, kms.value) if timing else (dist, near)
    sp = np.ascontiguousarray(np.asarray(spheres, np.float32).reshape(-1, 4))
    ed = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    tr = np.ascontiguousarray(np.asarray(tris, np.int32).reshape(-1, 3))
    q = np.ascontiguousarray(np.asarray(samples, np.float32).reshape(-1, 3))
    dist = np.empty(q.shape[0], np.float32)
    near = np.empty(q.shape[0], np.int32) if nearest else None
    ptr = lambda a: C.c_void_p(a.ctypes.data if a is not None and a.size else 0)
    _check(lib.rpd_envelope_distance(ptr(sp), sp.shape[0], ptr(ed), ed.shape[0], ptr(tr), tr.shape[0], ptr(q),
                                     q.shape[0], 0, _stream_ptr(stream), ptr(dist), ptr(near), kptr))
    return (dist, near, kms.value) if timing else (dist, near)


def envelope_distance_noalloc(spheres, edges, tris, samples, dist, nearest=None, stream=None):
    """rpd_envelope_distance_noalloc: the same distances into caller-allocated device tensors (dist float32 [s],
    nearest int32 [s] or None). Every argument is a contiguous device tensor of the documented dtype and shape; the
    call allocates nothing (its working memory is the library's fixed scratch region on the device)."""
    lib = load()
    import torch

    for name, t, dt in (("spheres", spheres, torch.float32), ("edges", edges, torch.int32), ("tris", tris, torch.int32),
                        ("samples", samples, torch.float32), ("dist", dist, torch.float32),
                        ("nearest", nearest, torch.int32)):
        if t is None:
            continue
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dt} device tensor")
    ptr = lambda t: C.c_void_p(t.data_ptr() if t is not None and t.numel() else 0)
    dev = samples.device
    st = _stream_ptr(stream) if stream is not None else C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib.rpd_envelope_distance_noalloc(ptr(spheres), spheres.numel() // 4, ptr(edges), edges.numel() // 2,
                                             ptr(tris), tris.numel() // 3, ptr(samples), samples.numel() // 3, st,
                                             ptr(dist), ptr(nearest)))


def shrink_spheres(tris, pins, normals, own_tri=None, stream=None):
    """rpd_shrink_spheres: maximal empty balls tangent to the surface (triangles (m, 3, 3)) at the pins (s, 3) with
    inward unit normals (s, 3); own_tri (s,) the pin's triangle or None. CUDA tensors run on the device (output a
    tensor), numpy arrays through host memory. Returns (s, 4) float32 (centre, radius)."""
    lib = load()
    if _is_torch(pins) and pins.is_cuda:
        import torch

        dev = pins.device
        t = tris.to(dev, torch.float32).contiguous().reshape(-1, 9)
        p = pins.to(torch.float32).contiguous().reshape(-1, 3)
        n = normals.to(dev, torch.float32).contiguous().reshape(-1, 3)
        o = own_tri.to(dev, torch.int32).contiguous() if own_tri is not None else None
        out = torch.empty((p.shape[0], 4), dtype=torch.float32, device=dev)
        ptr = lambda x: C.c_void_p(x.data_ptr() if x is not None and x.numel() else 0)
        st = _stream_ptr(stream) if stream is not None else C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        _check(lib.rpd_shrink_spheres(ptr(t), t.shape[0], ptr(p), ptr(n), ptr(o), p.shape[0], RPD_DEVICE_PTRS, st,
                                      ptr(out)))
        return out
    t = np.ascontiguousarray(np.asarray(tris, np.float32).reshape(-1, 9))
    p = np.ascontiguousarray(np.asarray(pins, np.float32).reshape(-1, 3))
    n = np.ascontiguousarray(np.asarray(normals, np.float32).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(own_tri, np.int32)) if own_tri is not None else None
    out = np.empty((p.shape[0], 4), np.float32)
    ptr = lambda x: C.c_void_p(x.ctypes.data if x is not None and x.size else 0)
    _check(lib.rpd_shrink_spheres(ptr(t), t.shape[0], ptr(p), ptr(n), ptr(o), p.shape[0], 0, _stream_ptr(stream),
                                  ptr(out)))
    return out


def version() -> str:
    return load().rpd_version().decode()


RPD_INSERT_TABLE = 0
RPD_INSERT_SHRINK = 1


class Session:
    """Incremental sphere-insertion session over one mesh (rpd_session_*). ``sites`` and ``table`` are
    (x, y, z, r) arrays or tensors; ``table`` has one sphere per tet in the caller's tet order, or is None with
    insertion=RPD_INSERT_SHRINK (spheres shrunk at the furthest surface triangle of each violating cell)."""

    def __init__(self, mesh: Mesh, sites, table, max_sites: int, max_insert: int = 64,
                 precision: int = RPD_FP32_FALLBACK, clip_budget: int = 0, block: int = 0, flags: int = 0,
                 stream=None, insertion: int = RPD_INSERT_TABLE, slots: int = 0):
        lib = load()
        keep = []
        dev = _is_torch(sites[0]) and sites[0].is_cuda
        if table is not None and dev != (_is_torch(table[0]) and table[0].is_cuda):
            raise ValueError("sites and table must both be device tensors or both host arrays")

        def mk(q):
            return _Sites(int(q[0].shape[0]), *[_ptr(x, C.c_float, keep) for x in q])

        st = mk(sites)
        tb = mk(table) if table is not None else None
        o = _SessionOpts(max_sites, max_insert,
                         _Opts(precision, clip_budget, block, flags | (RPD_DEVICE_PTRS if dev else 0),
                               _stream_ptr(stream), slots), insertion)
        h = C.c_void_p()
        _check(lib.rpd_session_create(mesh.handle, C.byref(st), C.byref(tb) if tb is not None else None, C.byref(o),
                                      C.byref(h)))
        self._h = h
        self._lib = lib
        self.mesh = mesh  # the session borrows the mesh
        self.max_sites = max_sites

    def run(self, rounds: int = 1):
        _check(self._lib.rpd_session_run(self._h, rounds))

    def result(self) -> Result:
        h = C.c_void_p()
        _check(self._lib.rpd_session_result(self._h, C.byref(h)))
        return Result(h, 1)

    def info(self) -> dict:
        i = _SessionInfo()
        _check(self._lib.rpd_session_get_info(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in _SessionInfo._fields_}

    def sites(self) -> np.ndarray:
        """Current sites as an (n, 4) float32 array of (x, y, z, r)."""
        out = np.zeros((self.max_sites, 4), np.float32)
        n = C.c_int32()
        _check(self._lib.rpd_session_sites(self._h, self.max_sites, out.ctypes.data_as(C.POINTER(C.c_float)),
                                           C.byref(n)))
        return out[: n.value].copy()

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.rpd_session_free(self._h)
            self._h = C.c_void_p()
