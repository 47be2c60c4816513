"""CPU oracle of the RTSDF hot path -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It wraps `liboracle.so` (plain C, built by `oracle/build.py`) with numpy
arrays and shares nothing with the GPU library.  Each wrapper names the part of the
paper (arXiv 2210.06160) it follows; the C source documents the readings in full.
"""
import ctypes
import os

import numpy as np

from . import build as _build

EMPTY = -1

_lib = None


class Grid(ctypes.Structure):
    """Uniform grid: voxel (i, j, k) has centre org + h * (i + 1/2, j + 1/2, k + 1/2)."""
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("org", ctypes.c_float * 3), ("h", ctypes.c_float)]


class Shadow(ctypes.Structure):
    """Receiver plane y = const; pixel (a, b) at (x0 + (a+1/2) dx, y, z0 + (b+1/2) dz)."""
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("x0", ctypes.c_float),
                ("z0", ctypes.c_float), ("dx", ctypes.c_float), ("dz", ctypes.c_float), ("y", ctypes.c_float),
                ("light", ctypes.c_float * 3), ("k", ctypes.c_float), ("steps", ctypes.c_int32),
                ("smin", ctypes.c_float), ("smax", ctypes.c_float), ("t0", ctypes.c_float)]


def make_shadow(width, height, x0, z0, dx, dz, y, light, k, steps, smin, smax, t0):
    s = Shadow()
    s.width, s.height = int(width), int(height)
    s.x0, s.z0, s.dx, s.dz, s.y = float(x0), float(z0), float(dx), float(dz), float(y)
    for a in range(3):
        s.light[a] = float(light[a])
    s.k, s.steps, s.smin, s.smax, s.t0 = float(k), int(steps), float(smin), float(smax), float(t0)
    return s


MAX_LIGHTS = 8


class ShadowEx(ctypes.Structure):
    """The shadow pass with several lights, a jittered start and optional triangulation;
    base.light is not used."""
    _fields_ = [("base", Shadow), ("nlights", ctypes.c_int32), ("lights", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("triangulate", ctypes.c_int32), ("bounded", ctypes.c_int32), ("jitter", ctypes.c_float),
                ("frame", ctypes.c_uint32), ("key", ctypes.c_uint64)]


def make_shadow_ex(base, lights, triangulate=False, jitter=0.0, frame=0, key=0, bounded=False):
    s = ShadowEx()
    s.base = base
    s.nlights = len(lights)
    for i, l in enumerate(lights):
        for a in range(3):
            s.lights[i][a] = float(l[a])
    s.triangulate, s.jitter, s.frame, s.key = int(bool(triangulate)), float(jitter), int(frame), int(key)
    s.bounded = int(bool(bounded))
    return s


def make_grid(dims, org, h):
    g = Grid()
    g.nx, g.ny, g.nz = (int(d) for d in dims)
    for a in range(3):
        g.org[a] = float(org[a])
    g.h = float(h)
    return g


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        vp, i32, i64, u32, u64, f32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.c_uint32, ctypes.c_uint64, ctypes.c_float)
        L.orc_voxelize.argtypes = [vp, i32, vp, i32, Grid, vp]
        L.orc_voxelize.restype = ctypes.c_int
        L.orc_jfa_pass.argtypes = [vp, vp, Grid, i32]
        L.orc_jfa.argtypes = [vp, vp, Grid, vp, i32]
        L.orc_seed_d2.argtypes = [vp, Grid, vp]
        L.orc_band.argtypes = [vp, Grid, i32, i32, vp]
        L.orc_band.restype = i64
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_direction.argtypes = [u64, u32, u32, u32, u32, vp]
        L.orc_direction.restype = ctypes.c_int
        L.orc_ray_tri.argtypes = [vp, vp, vp, vp, vp, f32, vp, vp]
        L.orc_ray_tri.restype = ctypes.c_int
        L.orc_closest_brute.argtypes = [vp, vp, i32, vp, vp, f32, vp, vp, vp]
        L.orc_closest_brute.restype = ctypes.c_int
        L.orc_bvh_build.argtypes = [vp, vp, i32, f32]
        L.orc_bvh_build.restype = vp
        L.orc_bvh_free.argtypes = [vp]
        L.orc_bvh_closest.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_bvh_closest.restype = ctypes.c_int
        L.orc_voxel_centre.argtypes = [Grid, i64, vp]
        L.orc_raysample.argtypes = [vp, Grid, vp, i64, i32, u64, u32, u32, vp, vp, vp]
        L.orc_combine.argtypes = [vp, vp, vp, Grid, i32, vp, i64, i32, f32, f32, i32, f32, i32, vp, vp]
        L.orc_pack_id.argtypes = [i32, i32, i32]
        L.orc_pack_id.restype = i32
        L.orc_shadow_forward.argtypes = [vp, Grid, ctypes.POINTER(Shadow), vp]
        L.orc_shadow_backward.argtypes = [vp, Grid, ctypes.POINTER(Shadow), vp, vp]
        L.orc_sdf_backward.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, Grid, i32, u64, u32, vp]
        L.orc_sdf_backward.restype = ctypes.c_int
        L.orc_sample.argtypes = [vp, Grid, vp, i64, vp, vp]
        L.orc_shadow_margin.argtypes = [vp, Grid, ctypes.POINTER(Shadow), vp, vp, vp]
        L.orc_shadow_path.argtypes = [vp, Grid, ctypes.POINTER(Shadow), vp]
        L.orc_shadow_forward_ex.argtypes = [vp, Grid, ctypes.POINTER(ShadowEx), vp]
        L.orc_shadow_backward_ex.argtypes = [vp, Grid, ctypes.POINTER(ShadowEx), vp, vp]
        L.orc_shadow_margin_ex.argtypes = [vp, Grid, ctypes.POINTER(ShadowEx), vp, vp, vp, vp]
        L.orc_clipmap_sample.argtypes = [vp, vp, vp, i32, vp, i64, vp, vp]
        L.orc_shadow_forward_clip.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ShadowEx), vp]
        L.orc_shadow_backward_clip.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ShadowEx), vp, vp]
        L.orc_shadow_margin_clip.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ShadowEx), vp, vp, vp, vp]
        L.orc_shadow_triangulate.argtypes = [ctypes.c_double] * 5 + [vp]
        L.orc_shadow_triangulate.restype = ctypes.c_double
        _lib = L
    return _lib


def nvox(g):
    return g.nx * g.ny * g.nz


def refine_grid(g, ratio):
    """The grid with `ratio` times the points per axis over the same box."""
    return make_grid((g.nx * ratio, g.ny * ratio, g.nz * ratio), tuple(g.org), np.float32(g.h) / np.float32(ratio))


def pack_id(i, j, k):
    return int(lib().orc_pack_id(i, j, k))


def hit_pad(g):
    """Widening of a triangle's box used by the hit test: 1/256 of a voxel."""
    return np.float32(g.h) * np.float32(1.0 / 256.0)


def voxelize(verts, tris, g):
    """Section 2.2 voxelization: seed ids (own packed id) of overlapped voxels, else EMPTY."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.int32)
    seeds = np.empty(nvox(g), np.int32)
    rc = lib().orc_voxelize(_p(verts), len(verts), _p(tris), len(tris), g, _p(seeds))
    if rc != 0:
        raise ValueError("triangle index out of range")
    return seeds


def jfa_pass(seeds, g, k):
    """One section 2.2 jump-flooding pass with offset k."""
    seeds = np.ascontiguousarray(seeds, np.int32)
    out = np.empty_like(seeds)
    lib().orc_jfa_pass(_p(seeds), _p(out), g, int(k))
    return out


def jfa(seeds, g, steps):
    """Section 2.2 jump flooding over the given offsets, in order."""
    a = np.array(seeds, np.int32, copy=True)
    tmp = np.empty_like(a)
    st = np.ascontiguousarray(steps, np.int32)
    lib().orc_jfa(_p(a), _p(tmp), g, _p(st), len(st))
    return a


def jfa_steps(dims, extra=0):
    """Offsets n/2, n/4, ..., 1 (section 2.2) with n the next power of two of the largest
    side, followed by `extra` additional passes with offset 1."""
    n = max(dims)
    k = 1
    while k < n:
        k *= 2
    out = []
    k //= 2
    while k >= 1:
        out.append(k)
        k //= 2
    if not out:
        out = [1]
    return out + [1] * extra


def seed_d2(seeds, g):
    d2 = np.empty(nvox(g), np.int32)
    lib().orc_seed_d2(_p(np.ascontiguousarray(seeds, np.int32)), g, _p(d2))
    return d2


def band(seeds, g, band_vox, ratio=1):
    """Section 2.3 ray mask as an increasing list of voxel ids; with ratio > 1 the ids of the
    grid refined `ratio` times per axis whose coarse point is in the mask."""
    seeds = np.ascontiguousarray(seeds, np.int32)
    n = lib().orc_band(_p(seeds), g, int(ratio), int(band_vox), None)
    out = np.empty(n, np.int32)
    lib().orc_band(_p(seeds), g, int(ratio), int(band_vox), _p(out))
    return out


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.empty(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def direction(seed, vid, frame, ray, obj=0):
    """Section 2.1 uniform sphere direction; returns (w, philox calls used)."""
    w = np.empty(3, np.float32)
    n = lib().orc_direction(int(seed), int(vid), int(frame), int(ray), int(obj), _p(w))
    return w, n


def ray_tri(o, w, v0, v1, v2, pad):
    o, w, v0, v1, v2 = (np.ascontiguousarray(a, np.float32) for a in (o, w, v0, v1, v2))
    t = np.zeros(1, np.float32)
    fr = np.zeros(1, np.int32)
    hit = lib().orc_ray_tri(_p(o), _p(w), _p(v0), _p(v1), _p(v2), float(pad), _p(t), _p(fr))
    return bool(hit), float(t[0]), bool(fr[0])


def closest_brute(verts, tris, o, w, pad):
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.int32)
    o, w = np.ascontiguousarray(o, np.float32), np.ascontiguousarray(w, np.float32)
    t = np.zeros(1, np.float32)
    tri = np.zeros(1, np.int32)
    fr = np.zeros(1, np.int32)
    hit = lib().orc_closest_brute(_p(verts), _p(tris), len(tris), _p(o), _p(w), float(pad),
                                  _p(t), _p(tri), _p(fr))
    return bool(hit), t[0], int(tri[0]), bool(fr[0])


class BVH:
    """Median-split hierarchy whose closest hit equals brute force (tested)."""

    def __init__(self, verts, tris, pad):
        self.verts = np.ascontiguousarray(verts, np.float32)
        self.tris = np.ascontiguousarray(tris, np.int32)
        self.ptr = lib().orc_bvh_build(_p(self.verts), _p(self.tris), len(self.tris), float(pad))

    def closest(self, o, w):
        o, w = np.ascontiguousarray(o, np.float32), np.ascontiguousarray(w, np.float32)
        t = np.zeros(1, np.float32)
        tri = np.zeros(1, np.int32)
        fr = np.zeros(1, np.int32)
        hit = lib().orc_bvh_closest(self.ptr, _p(o), _p(w), _p(t), _p(tri), _p(fr))
        return bool(hit), t[0], int(tri[0]), bool(fr[0])

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.orc_bvh_free(self.ptr)
            self.ptr = None


def voxel_centre(g, vid):
    o = np.empty(3, np.float32)
    lib().orc_voxel_centre(g, int(vid), _p(o))
    return o


def new_accum(n):
    return (np.full(n, np.inf, np.float32), np.zeros(n, np.uint32),
            np.full(n, np.iinfo(np.uint64).max, np.uint64))


def raysample(bvh, g, vids, x, seed, frame, obj=0, acc=None):
    """Section 2.1 ray sampling of the listed voxels for one frame (accumulating)."""
    vids = np.ascontiguousarray(vids, np.int32)
    if acc is None:
        acc = new_accum(len(vids))
    dmin, hits, argmin = acc
    lib().orc_raysample(bvh.ptr, g, _p(vids), len(vids), int(x), int(seed), int(frame), int(obj),
                        _p(dmin), _p(hits), _p(argmin))
    return acc


def combine(seeds, dmin, hits, g, band_vox, beta, bias, mode, alpha=0.95, reset=True,
            state=None, vids=None, ratio=1):
    """Coarse/fine combination: mode 0 running minimum (section 2.1), mode 1 decay (Eq. 1).
    With ratio > 1, g is the jump-flooded (coarse) grid and dmin/hits/state/the result live
    on the grid refined `ratio` times per axis."""
    seeds = np.ascontiguousarray(seeds, np.int32)
    dmin = np.ascontiguousarray(dmin, np.float32)
    hits = np.ascontiguousarray(hits, np.uint32)
    n = len(vids) if vids is not None else nvox(g) * int(ratio) ** 3
    if vids is not None:
        vids = np.ascontiguousarray(vids, np.int32)
    if state is None:
        state = np.zeros(n, np.float32)
    fine = np.empty(n, np.float32)
    lib().orc_combine(_p(seeds), _p(dmin), _p(hits), g, int(ratio), _p(vids), n, int(band_vox),
                      float(beta), float(bias), int(mode), float(alpha), int(bool(reset)),
                      _p(state), _p(fine))
    return fine, state


def sample(fine, g, X):
    """Trilinear value and positional gradient of the fine field at points X [n, 3]."""
    f = np.ascontiguousarray(fine, np.float64)
    X = np.ascontiguousarray(X, np.float64)
    val = np.empty(len(X), np.float64)
    grad = np.empty((len(X), 3), np.float64)
    lib().orc_sample(_p(f), g, _p(X), len(X), _p(val), _p(grad))
    return val, grad


def shadow_forward(fine, g, s):
    """Section 2.4 soft shadow by sphere tracing the fine field (binary64)."""
    f = np.ascontiguousarray(fine, np.float64)
    img = np.empty(s.width * s.height, np.float64)
    lib().orc_shadow_forward(_p(f), g, ctypes.byref(s), _p(img))
    return img


def shadow_backward(fine, g, s, grad_img):
    """(d img / d fine)^T grad_img by reverse-mode differentiation of the march (binary64)."""
    f = np.ascontiguousarray(fine, np.float64)
    gi = np.ascontiguousarray(grad_img, np.float64)
    gf = np.zeros(len(f), np.float64)
    lib().orc_shadow_backward(_p(f), g, ctypes.byref(s), _p(gi), _p(gf))
    return gf


def shadow_path(fine, g, s):
    """Per-pixel hash of the march's discrete path (minimising step, clamped samples,
    trilinear cells): equal hashes mean the image is one smooth function of the field
    between the two fields (see orc_shadow_path)."""
    f = np.ascontiguousarray(fine, np.float64)
    sig = np.empty(s.width * s.height, np.uint64)
    lib().orc_shadow_path(_p(f), g, ctypes.byref(s), _p(sig))
    return sig


def shadow_margin(fine, g, s):
    """Per-pixel distances of the march's discrete decisions from flipping: (r_margin,
    s_margin, c_margin) -- see orc_shadow_margin."""
    f = np.ascontiguousarray(fine, np.float64)
    rm = np.empty(s.width * s.height, np.float64)
    sm = np.empty(s.width * s.height, np.float64)
    cm = np.empty(s.width * s.height, np.float64)
    lib().orc_shadow_margin(_p(f), g, ctypes.byref(s), _p(rm), _p(sm), _p(cm))
    return rm, sm, cm


def clipmap_levels(camera, h0, n, levels):
    """Grids of a clip map around `camera`: level l has n^3 points of size h0 * 2^l, its
    origin the camera's voxel of that level minus n/2 voxels on every axis (binary32:
    (floor(c / h) - n/2) * h), so that each level is fixed while the camera stays in one
    of its voxels, and each level's box lies inside the next one's (n >= 4, even)."""
    out = []
    for l in range(levels):
        h = np.float32(h0) * np.float32(2.0 ** l)
        org = [np.float32((np.floor(np.float32(c) / h) - np.float32(n // 2)) * h) for c in camera]
        out.append(make_grid((n, n, n), org, h))
    return out


def _levels(grids, fields):
    off = np.zeros(len(grids), np.int64)
    total = 0
    for l, g in enumerate(grids):
        off[l] = total
        total += nvox(g)
    f = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64).ravel() for x in fields]), np.float64)
    assert len(f) == total
    G = (Grid * len(grids))(*grids)
    return f, off, G


def clipmap_sample(grids, fields, X):
    """Values of a clip map (levels finest first, fields[l] on grids[l]) at points X [n, 3]:
    each point reads the finest level whose box of grid-point centres holds it, else the
    coarsest; returns (values, level of each point)."""
    f, off, G = _levels(grids, fields)
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 3)
    val = np.empty(len(X))
    lev = np.empty(len(X), np.int32)
    lib().orc_clipmap_sample(_p(f), _p(off), ctypes.cast(G, ctypes.c_void_p), len(grids), _p(X), len(X), _p(val),
                             _p(lev))
    return val, lev


def shadow_forward_clip(grids, fields, s):
    """shadow_forward_ex over a clip map (a bounded march ends at the coarsest level's box)."""
    f, off, G = _levels(grids, fields)
    img = np.empty(s.nlights * s.base.width * s.base.height)
    lib().orc_shadow_forward_clip(_p(f), _p(off), ctypes.cast(G, ctypes.c_void_p), len(grids), ctypes.byref(s),
                                  _p(img))
    return img


def shadow_backward_clip(grids, fields, s, grad_img):
    """(d img / d fields)^T grad_img over a clip map: the concatenated fields' gradient."""
    f, off, G = _levels(grids, fields)
    gi = np.ascontiguousarray(grad_img, np.float64)
    gf = np.zeros(len(f))
    lib().orc_shadow_backward_clip(_p(f), _p(off), ctypes.cast(G, ctypes.c_void_p), len(grids), ctypes.byref(s),
                                   _p(gi), _p(gf))
    return gf


def shadow_margin_clip(grids, fields, s):
    f, off, G = _levels(grids, fields)
    n = s.nlights * s.base.width * s.base.height
    rm, sm, cm, vm = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    lib().orc_shadow_margin_clip(_p(f), _p(off), ctypes.cast(G, ctypes.c_void_p), len(grids), ctypes.byref(s),
                                 _p(rm), _p(sm), _p(cm), _p(vm))
    return rm, sm, cm, vm


def shadow_triangulate(r1, r2, delta, t, k):
    """Two-sample estimate of the closest approach: (estimate, triangulated?)."""
    v = ctypes.c_int(0)
    e = lib().orc_shadow_triangulate(float(r1), float(r2), float(delta), float(t), float(k), ctypes.byref(v))
    return e, bool(v.value)


def shadow_forward_ex(fine, g, s):
    """Shadow images [nlights][height][width] (several lights, jitter, triangulation; binary64)."""
    f = np.ascontiguousarray(fine, np.float64)
    img = np.empty(s.nlights * s.base.width * s.base.height, np.float64)
    lib().orc_shadow_forward_ex(_p(f), g, ctypes.byref(s), _p(img))
    return img


def shadow_backward_ex(fine, g, s, grad_img):
    """(d img / d fine)^T grad_img for shadow_forward_ex (binary64)."""
    f = np.ascontiguousarray(fine, np.float64)
    gi = np.ascontiguousarray(grad_img, np.float64)
    gf = np.zeros(len(f), np.float64)
    lib().orc_shadow_backward_ex(_p(f), g, ctypes.byref(s), _p(gi), _p(gf))
    return gf


def shadow_margin_ex(fine, g, s):
    """Decision margins of shadow_forward_ex per pixel and light (r, s, c, v) -- see
    orc_shadow_margin_ex."""
    f = np.ascontiguousarray(fine, np.float64)
    n = s.nlights * s.base.width * s.base.height
    rm, sm, cm, vm = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    lib().orc_shadow_margin_ex(_p(f), g, ctypes.byref(s), _p(rm), _p(sm), _p(cm), _p(vm))
    return rm, sm, cm, vm


def sdf_backward(grad_fine, hits, argmin, vids, bvh, verts, tris, g, x, seed, obj=0):
    """Adjoint of the running-minimum fine field with respect to vertex positions
    (binary64); hits/argmin are indexed like vids, grad_fine by voxel."""
    gf = np.ascontiguousarray(grad_fine, np.float64)
    h = np.ascontiguousarray(hits, np.uint32)
    a = np.ascontiguousarray(argmin, np.uint64)
    v = np.ascontiguousarray(vids, np.int32)
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.int32)
    gv = np.zeros(3 * len(verts), np.float64)
    bad = lib().orc_sdf_backward(_p(gf), _p(h), _p(a), _p(v), len(v), bvh.ptr, _p(verts), _p(tris), g,
                                 int(x), int(seed), int(obj), _p(gv))
    if bad:
        raise RuntimeError("%d argmin rays found no hit" % bad)
    return gv.reshape(-1, 3)
