"""Thin ctypes binding of librtsdf.so (the C ABI in include/rtsdf.h).

Each `rtsdf_*` function marshals torch CUDA tensors into device pointers and the current
HIP stream and calls the C entry point of the same name; all computation happens in the
HIP kernels.  There is no fallback: if the library is missing or a call fails, an
exception is raised.  `StaticSDF` chains the calls into the paper's static pipeline
(voxelize -> jump flood -> mask -> BVH -> frames of ray sampling -> combine), `DeformSDF`
the per-frame chain of a deforming mesh, and `SDF` / `SoftShadow` are autograd Functions
whose backward passes call the adjoint entry points.
"""
import ctypes
import types
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librtsdf.so")
EMPTY = -1
MAX_RAYS = 65535  # rays accumulated into one 16-bit front or back hit count
ACCUM, DECAY = 0, 1
BVH_LBVH, BVH_PLOC = 0, 1
_lib = None


class RtsdfError(RuntimeError):
    pass


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("org", ctypes.c_float * 3), ("h", ctypes.c_float)]

    @property
    def n(self):
        return self.nx * self.ny * self.nz


class Shadow(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("x0", ctypes.c_float),
                ("z0", ctypes.c_float), ("dx", ctypes.c_float), ("dz", ctypes.c_float), ("y", ctypes.c_float),
                ("light", ctypes.c_float * 3), ("k", ctypes.c_float), ("steps", ctypes.c_int32),
                ("smin", ctypes.c_float), ("smax", ctypes.c_float), ("t0", ctypes.c_float)]


def make_shadow(width, height, x0, z0, dx, dz, y, light, k, steps, smin, smax, t0):
    s = Shadow()
    s.width, s.height, s.steps = int(width), int(height), int(steps)
    s.x0, s.z0, s.dx, s.dz, s.y = float(x0), float(z0), float(dx), float(dz), float(y)
    for a in range(3):
        s.light[a] = float(light[a])
    s.k, s.smin, s.smax, s.t0 = float(k), float(smin), float(smax), float(t0)
    return s


MAX_LIGHTS = 8


class ShadowEx(ctypes.Structure):
    _fields_ = [("base", Shadow), ("nlights", ctypes.c_int32), ("lights", (ctypes.c_float * 3) * MAX_LIGHTS),
                ("triangulate", ctypes.c_int32), ("bounded", ctypes.c_int32), ("jitter", ctypes.c_float),
                ("frame", ctypes.c_uint32), ("key", ctypes.c_uint64)]


def make_shadow_ex(base, lights, triangulate=False, jitter=0.0, frame=0, key=0, bounded=False):
    """The full shadow pass: `base` (a Shadow; its light is ignored) marched towards each of
    `lights` (unit directions), with a jittered start, optional triangulation, and
    (bounded) an end where the march leaves the grid's box."""
    if not 1 <= len(lights) <= MAX_LIGHTS:
        raise RtsdfError("1 to %d lights" % MAX_LIGHTS)
    s = ShadowEx()
    s.base = base
    s.nlights = len(lights)
    for i, l in enumerate(lights):
        for a in range(3):
            s.lights[i][a] = float(l[a])
    s.triangulate, s.jitter, s.frame, s.key = int(bool(triangulate)), float(jitter), int(frame), int(key)
    s.bounded = int(bool(bounded))
    return s


class Object(ctypes.Structure):
    _fields_ = [("g", Grid), ("nv", ctypes.c_int32), ("nt", ctypes.c_int32), ("band_vox", ctypes.c_int32),
                ("extra_passes", ctypes.c_int32), ("beta", ctypes.c_float), ("bias", ctypes.c_float)]


class BatchSizes(ctypes.Structure):
    _fields_ = [("voxels", ctypes.c_int64), ("verts", ctypes.c_int64), ("tris", ctypes.c_int64),
                ("bvh_bytes", ctypes.c_size_t), ("work_bytes", ctypes.c_size_t), ("max_passes", ctypes.c_int32)]


def make_grid(dims, org, h):
    g = Grid()
    g.nx, g.ny, g.nz = (int(d) for d in dims)
    for a in range(3):
        g.org[a] = float(org[a])
    g.h = float(h)
    return g


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RtsdfError("librtsdf.so is not built (run paper_2210_06160_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, f32, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                           ctypes.c_uint64, ctypes.c_float, ctypes.c_size_t)
        sig = {
            "rtsdf_last_error": ([], ctypes.c_char_p),
            "rtsdf_abi_version": ([], i32),
            "rtsdf_voxelize_work_bytes": ([i32], sz),
            "rtsdf_voxelize": ([vp, i32, vp, i32, Grid, vp, vp, sz, vp], i32),
            "rtsdf_jfa": ([vp, vp, Grid, vp, i32, vp, vp], i32),
            "rtsdf_band_work_bytes": ([Grid], sz),
            "rtsdf_band": ([vp, Grid, i32, vp, vp, vp, sz, vp], i32),
            "rtsdf_bvh_bytes": ([i32], sz),
            "rtsdf_bvh_work_bytes": ([i32], sz),
            "rtsdf_build_bvh": ([vp, i32, vp, i32, Grid, i32, vp, sz, vp, sz, vp], i32),
            "rtsdf_reset_accum": ([vp, vp, vp, i64, vp], i32),
            "rtsdf_raysample_work_bytes": ([i64, i32], sz),
            "rtsdf_raysample": ([vp, Grid, vp, vp, i64, i32, u64, u32, u32, vp, vp, vp, vp, sz, vp], i32),
            "rtsdf_raysample_noalloc": ([vp, Grid, vp, vp, i64, i32, u64, u32, u32, vp, vp, vp, vp], i32),
            "rtsdf_raysample_frame_device": ([vp, Grid, vp, vp, i64, i32, u64, vp, u32, vp, vp, vp, vp, sz, vp], i32),
            "rtsdf_combine": ([vp, vp, vp, Grid, i32, f32, f32, i32, f32, i32, i32, vp, vp, vp], i32),
            "rtsdf_refine_grid": ([Grid, i32, ctypes.POINTER(Grid)], i32),
            "rtsdf_band_refined_work_bytes": ([Grid, i32], sz),
            "rtsdf_band_refined": ([vp, Grid, i32, i32, vp, vp, vp, sz, vp], i32),
            "rtsdf_combine_refined": ([vp, vp, vp, Grid, i32, i32, f32, f32, i32, f32, i32, i32, vp, vp, vp], i32),
            "rtsdf_shadow_forward": ([vp, Grid, Shadow, vp, vp], i32),
            "rtsdf_shadow_backward": ([vp, Grid, Shadow, vp, vp, vp], i32),
            "rtsdf_shadow_forward_ex": ([vp, Grid, ctypes.POINTER(ShadowEx), vp, vp], i32),
            "rtsdf_clipmap_levels": ([vp, f32, i32, i32, vp], i32),
            "rtsdf_clipmap_sample": ([vp, vp, vp, i64, vp, vp, vp], i32),
            "rtsdf_shadow_forward_clip": ([vp, vp, ctypes.POINTER(ShadowEx), vp, vp], i32),
            "rtsdf_shadow_backward_clip": ([vp, vp, ctypes.POINTER(ShadowEx), vp, vp, vp], i32),
            "rtsdf_shadow_backward_ex": ([vp, Grid, ctypes.POINTER(ShadowEx), vp, vp, vp], i32),
            "rtsdf_backward": ([vp, vp, vp, vp, vp, i64, vp, vp, i32, i32, Grid, i32, u64, u32, vp, vp], i32),
            "rtsdf_batch_plan_bytes": ([i32], sz),
            "rtsdf_batch_plan": ([vp, i32, vp, vp, sz, vp], i32),
            "rtsdf_batch_upload": ([vp, vp], i32),
            "rtsdf_batch_offsets": ([vp, i32, vp, vp], i32),
            "rtsdf_voxelize_batched": ([vp, vp, vp, vp, vp, vp, sz, vp], i32),
            "rtsdf_jfa_batched": ([vp, vp, vp, vp], i32),
            "rtsdf_band_batched": ([vp, vp, vp, vp, vp, sz, vp], i32),
            "rtsdf_build_bvh_batched": ([vp, vp, vp, i32, vp, sz, vp, sz, vp], i32),
            "rtsdf_raysample_batched": ([vp, vp, vp, vp, i64, i32, u64, u32, vp, vp, vp, vp, sz, vp], i32),
            "rtsdf_combine_batched": ([vp, vp, vp, vp, vp, vp], i32),
            "rtsdf_backward_batched": ([vp, vp, vp, vp, vp, vp, i64, vp, vp, i32, u64, vp, vp], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


EXPORTED = ["rtsdf_last_error", "rtsdf_abi_version", "rtsdf_voxelize_work_bytes", "rtsdf_voxelize",
            "rtsdf_jfa", "rtsdf_band_work_bytes", "rtsdf_band", "rtsdf_bvh_bytes", "rtsdf_bvh_work_bytes",
            "rtsdf_build_bvh", "rtsdf_reset_accum", "rtsdf_raysample_work_bytes", "rtsdf_raysample",
            "rtsdf_raysample_noalloc", "rtsdf_raysample_frame_device",
            "rtsdf_combine", "rtsdf_refine_grid", "rtsdf_band_refined_work_bytes", "rtsdf_band_refined",
            "rtsdf_combine_refined", "rtsdf_shadow_forward", "rtsdf_shadow_backward", "rtsdf_shadow_forward_ex",
            "rtsdf_shadow_backward_ex", "rtsdf_clipmap_levels", "rtsdf_clipmap_sample", "rtsdf_shadow_forward_clip",
            "rtsdf_shadow_backward_clip", "rtsdf_backward",
            "rtsdf_batch_plan_bytes", "rtsdf_batch_plan", "rtsdf_batch_upload", "rtsdf_batch_offsets", "rtsdf_voxelize_batched",
            "rtsdf_jfa_batched", "rtsdf_band_batched", "rtsdf_build_bvh_batched", "rtsdf_raysample_batched",
            "rtsdf_combine_batched", "rtsdf_backward_batched"]


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise RtsdfError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise RtsdfError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise RtsdfError("expected %s, got %s" % (dtype, t.dtype))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(status, what):
    if status != 0:
        msg = lib().rtsdf_last_error().decode()
        raise RtsdfError("%s failed (status %d): %s" % (what, status, msg))


def workspace(nbytes, device="cuda"):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def rtsdf_abi_version():
    return lib().rtsdf_abi_version()


def rtsdf_voxelize_work_bytes(nt):
    return lib().rtsdf_voxelize_work_bytes(int(nt))


def rtsdf_voxelize(verts, tris, grid, seeds, work, stream=None):
    _check(lib().rtsdf_voxelize(_ptr(verts, torch.float32), verts.shape[0], _ptr(tris, torch.int32),
                                tris.shape[0], grid, _ptr(seeds, torch.int32), _ptr(work), work.numel(),
                                _stream(stream)), "rtsdf_voxelize")


def rtsdf_jfa(seeds, scratch, grid, steps, stream=None):
    """Returns the tensor holding the result (seeds or scratch)."""
    st = (ctypes.c_int32 * max(len(steps), 1))(*[int(k) for k in steps])
    flag = ctypes.c_int32(0)
    _check(lib().rtsdf_jfa(_ptr(seeds, torch.int32), _ptr(scratch, torch.int32), grid,
                           ctypes.cast(st, ctypes.c_void_p), len(steps), ctypes.byref(flag), _stream(stream)),
           "rtsdf_jfa")
    return scratch if flag.value else seeds


def rtsdf_band_work_bytes(grid):
    return lib().rtsdf_band_work_bytes(grid)


def rtsdf_band(seeds, grid, band_vox, band_list, band_count, work, stream=None):
    _check(lib().rtsdf_band(_ptr(seeds, torch.int32), grid, int(band_vox), _ptr(band_list, torch.int32),
                            _ptr(band_count, torch.int32), _ptr(work), work.numel(), _stream(stream)),
           "rtsdf_band")


def rtsdf_bvh_bytes(nt):
    return lib().rtsdf_bvh_bytes(int(nt))


def rtsdf_bvh_work_bytes(nt):
    return lib().rtsdf_bvh_work_bytes(int(nt))


def rtsdf_build_bvh(verts, tris, grid, bvh, work, method=BVH_PLOC, stream=None):
    _check(lib().rtsdf_build_bvh(_ptr(verts, torch.float32), verts.shape[0], _ptr(tris, torch.int32),
                                 tris.shape[0], grid, int(method), _ptr(bvh), bvh.numel(), _ptr(work), work.numel(),
                                 _stream(stream)), "rtsdf_build_bvh")


def rtsdf_reset_accum(dmin, hits, argmin=None, stream=None):
    _check(lib().rtsdf_reset_accum(_ptr(dmin, torch.float32), _ptr(hits, torch.int32),
                                   _ptr(argmin, torch.int64) if argmin is not None else None, dmin.numel(),
                                   _stream(stream)), "rtsdf_reset_accum")


def rtsdf_raysample_work_bytes(band_capacity, rays_per_voxel):
    return lib().rtsdf_raysample_work_bytes(int(band_capacity), int(rays_per_voxel))


def rtsdf_raysample(bvh, grid, band_list, band_count, rays_per_voxel, rng_key, frame, dmin, hits, work,
                    argmin=None, obj=0, band_capacity=None, stream=None):
    """hits is an int32 tensor holding the uint32 counters; argmin an int64 tensor holding
    the uint64 records (reinterpret with .view or `& 0xffffffff`).  band_capacity bounds the
    device-side count (default: the list length)."""
    cap = band_list.numel() if band_capacity is None else int(band_capacity)
    _check(lib().rtsdf_raysample(_ptr(bvh), grid, _ptr(band_list, torch.int32), _ptr(band_count, torch.int32),
                                 cap, int(rays_per_voxel), int(rng_key) & (2 ** 64 - 1),
                                 int(frame), int(obj), _ptr(dmin, torch.float32), _ptr(hits, torch.int32),
                                 _ptr(argmin, torch.int64) if argmin is not None else None, _ptr(work),
                                 work.numel(), _stream(stream)),
           "rtsdf_raysample")


def rtsdf_raysample_frame_device(bvh, grid, band_list, band_count, rays_per_voxel, rng_key, frame, dmin, hits, work,
                                 argmin=None, obj=0, band_capacity=None, stream=None):
    """rtsdf_raysample with the frame index read from `frame` (a one-element int32 device
    tensor) when the kernel runs."""
    cap = band_list.numel() if band_capacity is None else int(band_capacity)
    _check(lib().rtsdf_raysample_frame_device(_ptr(bvh), grid, _ptr(band_list, torch.int32),
                                              _ptr(band_count, torch.int32), cap, int(rays_per_voxel),
                                              int(rng_key) & (2 ** 64 - 1), _ptr(frame, torch.int32), int(obj),
                                              _ptr(dmin, torch.float32), _ptr(hits, torch.int32),
                                              _ptr(argmin, torch.int64) if argmin is not None else None, _ptr(work),
                                              work.numel(), _stream(stream)),
           "rtsdf_raysample_frame_device")


def rtsdf_raysample_noalloc(bvh, grid, band_list, band_count, rays_per_voxel, rng_key, frame, dmin, hits,
                            argmin=None, obj=0, band_capacity=None, stream=None):
    """rtsdf_raysample with the work cursors in the library's static per-GPU scratch (no
    work tensor; calls that overlap on one GPU race)."""
    cap = band_list.numel() if band_capacity is None else int(band_capacity)
    _check(lib().rtsdf_raysample_noalloc(_ptr(bvh), grid, _ptr(band_list, torch.int32),
                                         _ptr(band_count, torch.int32), cap, int(rays_per_voxel),
                                         int(rng_key) & (2 ** 64 - 1), int(frame), int(obj),
                                         _ptr(dmin, torch.float32), _ptr(hits, torch.int32),
                                         _ptr(argmin, torch.int64) if argmin is not None else None, _stream(stream)),
           "rtsdf_raysample_noalloc")


def rtsdf_combine(seeds, dmin, hits, grid, band_vox, beta, bias, mode, fine, alpha=0.95, first_frame=True,
                  consume=False, state=None, stream=None):
    _check(lib().rtsdf_combine(_ptr(seeds, torch.int32), _ptr(dmin, torch.float32), _ptr(hits, torch.int32),
                               grid, int(band_vox), float(beta), float(bias), int(mode), float(alpha),
                               int(bool(first_frame)), int(bool(consume)),
                               _ptr(state, torch.float32) if state is not None else None,
                               _ptr(fine, torch.float32), _stream(stream)), "rtsdf_combine")


def rtsdf_refine_grid(grid, ratio):
    fine = Grid()
    _check(lib().rtsdf_refine_grid(grid, int(ratio), ctypes.byref(fine)), "rtsdf_refine_grid")
    return fine


def rtsdf_band_refined_work_bytes(grid, ratio):
    return lib().rtsdf_band_refined_work_bytes(grid, int(ratio))


def rtsdf_band_refined(seeds, grid, ratio, band_vox, band_list, band_count, work, stream=None):
    """Mask of the grid refined by `ratio` over the coarse grid `grid`; lists fine indices."""
    _check(lib().rtsdf_band_refined(_ptr(seeds, torch.int32), grid, int(ratio), int(band_vox),
                                    _ptr(band_list, torch.int32), _ptr(band_count, torch.int32), _ptr(work),
                                    work.numel(), _stream(stream)), "rtsdf_band_refined")


def rtsdf_combine_refined(seeds, dmin, hits, grid, ratio, band_vox, beta, bias, mode, fine, alpha=0.95,
                          first_frame=True, consume=False, state=None, stream=None):
    """rtsdf_combine on the grid refined by `ratio` over the coarse grid `grid` (seeds are
    coarse; dmin, hits, state and fine are fine)."""
    _check(lib().rtsdf_combine_refined(_ptr(seeds, torch.int32), _ptr(dmin, torch.float32), _ptr(hits, torch.int32),
                                       grid, int(ratio), int(band_vox), float(beta), float(bias), int(mode),
                                       float(alpha), int(bool(first_frame)), int(bool(consume)),
                                       _ptr(state, torch.float32) if state is not None else None,
                                       _ptr(fine, torch.float32), _stream(stream)), "rtsdf_combine_refined")


def rtsdf_shadow_forward(fine, grid, shadow, img, stream=None):
    _check(lib().rtsdf_shadow_forward(_ptr(fine, torch.float32), grid, shadow, _ptr(img, torch.float32),
                                      _stream(stream)), "rtsdf_shadow_forward")


def rtsdf_shadow_backward(fine, grid, shadow, grad_img, grad_fine, stream=None):
    """grad_fine is accumulated into."""
    _check(lib().rtsdf_shadow_backward(_ptr(fine, torch.float32), grid, shadow, _ptr(grad_img, torch.float32),
                                       _ptr(grad_fine, torch.float32), _stream(stream)), "rtsdf_shadow_backward")


def rtsdf_shadow_forward_ex(fine, grid, shadow, img, stream=None):
    """img [nlights, height, width] float32."""
    _check(lib().rtsdf_shadow_forward_ex(_ptr(fine, torch.float32), grid, ctypes.byref(shadow),
                                         _ptr(img, torch.float32), _stream(stream)), "rtsdf_shadow_forward_ex")


def rtsdf_shadow_backward_ex(fine, grid, shadow, grad_img, grad_fine, stream=None):
    """grad_fine is accumulated into."""
    _check(lib().rtsdf_shadow_backward_ex(_ptr(fine, torch.float32), grid, ctypes.byref(shadow),
                                          _ptr(grad_img, torch.float32), _ptr(grad_fine, torch.float32),
                                          _stream(stream)), "rtsdf_shadow_backward_ex")


MAX_CLIP_LEVELS = 8


def rtsdf_clipmap_levels(camera, h0, n, levels):
    """Grids of a clip map around `camera` (level l: n^3 points of size h0 * 2^l)."""
    cam = (ctypes.c_float * 3)(*[float(c) for c in camera])
    out = (Grid * int(levels))()
    _check(lib().rtsdf_clipmap_levels(cam, float(h0), int(n), int(levels), out), "rtsdf_clipmap_levels")
    return list(out)


def rtsdf_clipmap_sample(plan, fine, points, values, levels=None, stream=None):
    """points [n, 3] float32, values [n] float32, levels [n] int32 or None."""
    _check(lib().rtsdf_clipmap_sample(plan.ptr, _ptr(fine, torch.float32), _ptr(points, torch.float32),
                                      points.shape[0], _ptr(values, torch.float32),
                                      _ptr(levels, torch.int32) if levels is not None else None, _stream(stream)),
           "rtsdf_clipmap_sample")


def rtsdf_shadow_forward_clip(plan, fine, shadow, img, stream=None):
    _check(lib().rtsdf_shadow_forward_clip(plan.ptr, _ptr(fine, torch.float32), ctypes.byref(shadow),
                                           _ptr(img, torch.float32), _stream(stream)), "rtsdf_shadow_forward_clip")


def rtsdf_shadow_backward_clip(plan, fine, shadow, grad_img, grad_fine, stream=None):
    """grad_fine (the clip map's concatenated levels) is accumulated into."""
    _check(lib().rtsdf_shadow_backward_clip(plan.ptr, _ptr(fine, torch.float32), ctypes.byref(shadow),
                                            _ptr(grad_img, torch.float32), _ptr(grad_fine, torch.float32),
                                            _stream(stream)), "rtsdf_shadow_backward_clip")


def rtsdf_backward(grad_fine, hits, argmin, band_list, band_count, bvh, tris, nv, grid, rays_per_voxel, rng_key,
                   grad_verts, obj=0, band_capacity=None, stream=None):
    """grad_verts [nv, 3] float32 is accumulated into."""
    cap = band_list.numel() if band_capacity is None else int(band_capacity)
    _check(lib().rtsdf_backward(_ptr(grad_fine, torch.float32), _ptr(hits, torch.int32),
                                _ptr(argmin, torch.int64), _ptr(band_list, torch.int32),
                                _ptr(band_count, torch.int32), cap, _ptr(bvh), _ptr(tris, torch.int32),
                                int(nv), tris.shape[0], grid, int(rays_per_voxel), int(rng_key) & (2 ** 64 - 1),
                                int(obj), _ptr(grad_verts, torch.float32), _stream(stream)), "rtsdf_backward")


class Plan:
    """A batch plan: the host copy (ctypes buffer), the device copy (uint8 tensor) and the
    sizes of the concatenated arrays."""

    def __init__(self, objects, device="cuda", stream=None, upload=True):
        n = len(objects)
        arr = (Object * n)(*objects)
        nbytes = lib().rtsdf_batch_plan_bytes(n)
        if nbytes == 0:
            raise RtsdfError("bad object count %d" % n)
        self.host = ctypes.create_string_buffer(nbytes)
        self.nbytes = nbytes
        self.sizes = BatchSizes()
        if upload:
            self.device = torch.empty(nbytes, dtype=torch.uint8, device=device)
            dev_ptr = _ptr(self.device)
        else:  # host-side inspection only: a placeholder device address, never dereferenced
            self.device = None
            dev_ptr = ctypes.c_void_p(0x1000)
        _check(lib().rtsdf_batch_plan(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.cast(self.host, ctypes.c_void_p),
                                      dev_ptr, nbytes, ctypes.byref(self.sizes)), "rtsdf_batch_plan")
        if upload:
            _check(lib().rtsdf_batch_upload(self.ptr, _stream(stream)), "rtsdf_batch_upload")
        self.nobj = n

    @property
    def ptr(self):
        return ctypes.cast(self.host, ctypes.c_void_p)

    def offsets(self, o):
        v, b = ctypes.c_int64(0), ctypes.c_size_t(0)
        _check(lib().rtsdf_batch_offsets(self.ptr, int(o), ctypes.byref(v), ctypes.byref(b)), "rtsdf_batch_offsets")
        return v.value, b.value


def make_object(dims, org, h, nv, nt, band_vox, extra_passes, beta, bias=0.0):
    o = Object()
    o.g = make_grid(dims, org, h)
    o.nv, o.nt, o.band_vox, o.extra_passes = int(nv), int(nt), int(band_vox), int(extra_passes)
    o.beta, o.bias = float(beta), float(bias)
    return o


def rtsdf_voxelize_batched(plan, verts, tris, seeds, scratch, work, stream=None):
    _check(lib().rtsdf_voxelize_batched(plan.ptr, _ptr(verts, torch.float32), _ptr(tris, torch.int32),
                                        _ptr(seeds, torch.int32), _ptr(scratch, torch.int32), _ptr(work), work.numel(),
                                        _stream(stream)), "rtsdf_voxelize_batched")


def rtsdf_jfa_batched(plan, seeds, scratch, stream=None):
    _check(lib().rtsdf_jfa_batched(plan.ptr, _ptr(seeds, torch.int32), _ptr(scratch, torch.int32), _stream(stream)),
           "rtsdf_jfa_batched")


def rtsdf_band_batched(plan, seeds, band_list, band_count, work, stream=None):
    _check(lib().rtsdf_band_batched(plan.ptr, _ptr(seeds, torch.int32), _ptr(band_list, torch.int32),
                                    _ptr(band_count, torch.int32), _ptr(work), work.numel(), _stream(stream)),
           "rtsdf_band_batched")


def rtsdf_build_bvh_batched(plan, verts, tris, bvh, work, method=BVH_PLOC, stream=None):
    _check(lib().rtsdf_build_bvh_batched(plan.ptr, _ptr(verts, torch.float32), _ptr(tris, torch.int32), int(method),
                                         _ptr(bvh), bvh.numel(), _ptr(work), work.numel(), _stream(stream)),
           "rtsdf_build_bvh_batched")


def rtsdf_raysample_batched(plan, bvh, band_list, band_count, rays_per_voxel, rng_key, frame, dmin, hits, work,
                            argmin=None, band_capacity=None, stream=None):
    cap = band_list.numel() if band_capacity is None else int(band_capacity)
    _check(lib().rtsdf_raysample_batched(plan.ptr, _ptr(bvh), _ptr(band_list, torch.int32),
                                         _ptr(band_count, torch.int32), cap, int(rays_per_voxel),
                                         int(rng_key) & (2 ** 64 - 1), int(frame), _ptr(dmin, torch.float32),
                                         _ptr(hits, torch.int32), _ptr(argmin, torch.int64) if argmin is not None
                                         else None, _ptr(work), work.numel(), _stream(stream)),
           "rtsdf_raysample_batched")


def rtsdf_combine_batched(plan, seeds, dmin, hits, fine, stream=None):
    _check(lib().rtsdf_combine_batched(plan.ptr, _ptr(seeds, torch.int32), _ptr(dmin, torch.float32),
                                       _ptr(hits, torch.int32), _ptr(fine, torch.float32), _stream(stream)),
           "rtsdf_combine_batched")


def rtsdf_backward_batched(plan, grad_fine, hits, argmin, band_list, band_count, bvh, tris, rays_per_voxel, rng_key,
                           grad_verts, band_capacity=None, stream=None):
    cap = band_list.numel() if band_capacity is None else int(band_capacity)
    _check(lib().rtsdf_backward_batched(plan.ptr, _ptr(grad_fine, torch.float32), _ptr(hits, torch.int32),
                                        _ptr(argmin, torch.int64), _ptr(band_list, torch.int32),
                                        _ptr(band_count, torch.int32), cap, _ptr(bvh), _ptr(tris, torch.int32),
                                        int(rays_per_voxel), int(rng_key) & (2 ** 64 - 1),
                                        _ptr(grad_verts, torch.float32), _stream(stream)), "rtsdf_backward_batched")


class BatchSDF:
    """Many static objects, each on its own grid, with one launch per stage (per JFA pass):
    voxelize, jump flood, mask, hierarchies, `frames` x ray sampling, combine (running
    minimum), and the vertex adjoint.  `objects` are (verts, tris, dims, org, h, steps, band)
    records such as synth.Scene; each object's JFA offsets must be the standard halving list
    plus trailing passes of 1.  Object o draws its rays with counter word obj = o, so its
    results equal StaticSDF(..., obj=o).  No call reads anything back to the host."""

    def __init__(self, objects, rays, frames=1, rng_key=0, beta=None, bias=0.0, bvh_method=BVH_PLOC, device="cuda"):
        check_hit_budget(rays, frames)
        recs = []
        for sc in objects:
            std = _halving_offsets(sc.dims)
            steps = list(sc.steps)
            extra = len(steps) - len(std)
            if steps[:len(std)] != std or any(k != 1 for k in steps[len(std):]):
                raise RtsdfError("batched objects use the halving offsets plus passes of 1, got %s" % steps)
            b = float(sc.h) / 2 if beta is None else float(beta)
            recs.append(make_object(sc.dims, sc.org, sc.h, len(sc.verts), len(sc.tris), sc.band, extra, b, bias))
        self.plan = Plan(recs, device)
        z = self.plan.sizes
        self.rays, self.frames, self.rng_key = int(rays), int(frames), int(rng_key)
        self.bvh_method = int(bvh_method)
        self.verts = torch.from_numpy(np.concatenate([np.asarray(sc.verts, np.float32).reshape(-1, 3)
                                                      for sc in objects])).to(device)
        self.tris = torch.from_numpy(np.concatenate([np.asarray(sc.tris, np.int32).reshape(-1, 3)
                                                     for sc in objects])).to(device)
        V = z.voxels
        self.seeds = torch.empty(V, dtype=torch.int32, device=device)
        self.scratch = torch.empty(V, dtype=torch.int32, device=device)
        self.band_list = torch.empty(V, dtype=torch.int32, device=device)
        self.band_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.dmin = torch.empty(V, dtype=torch.float32, device=device)
        self.hits = torch.empty(V, dtype=torch.int32, device=device)
        self.argmin = torch.empty(V, dtype=torch.int64, device=device)
        self.fine = torch.empty(V, dtype=torch.float32, device=device)
        self.bvh = torch.empty(max(int(z.bvh_bytes), 1), dtype=torch.uint8, device=device)
        self.work = workspace(z.work_bytes, device)
        self.offsets = [self.plan.offsets(o) for o in range(len(objects))]
        self.dims = [tuple(sc.dims) for sc in objects]

    def voxelize(self):
        rtsdf_voxelize_batched(self.plan, self.verts, self.tris, self.seeds, self.scratch, self.work)

    def jfa(self):
        rtsdf_jfa_batched(self.plan, self.seeds, self.scratch)

    def mask(self):
        rtsdf_band_batched(self.plan, self.seeds, self.band_list, self.band_count, self.work)

    def build_bvh(self):
        rtsdf_build_bvh_batched(self.plan, self.verts, self.tris, self.bvh, self.work, self.bvh_method)

    def trace(self, frame):
        rtsdf_raysample_batched(self.plan, self.bvh, self.band_list, self.band_count, self.rays, self.rng_key, frame,
                                self.dmin, self.hits, self.work, self.argmin)

    def combine(self):
        rtsdf_combine_batched(self.plan, self.seeds, self.dmin, self.hits, self.fine)

    def run(self):
        self.voxelize()
        self.jfa()
        self.mask()
        self.build_bvh()
        rtsdf_reset_accum(self.dmin, self.hits, self.argmin)
        for f in range(self.frames):
            self.trace(f)
        self.combine()
        return self.fine

    def capture(self):
        """Records the whole chain (run()) into one HIP graph; replay() runs it.  Nothing in
        the chain reads back to the host or allocates, so the graph replays it exactly."""
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()

    def replay(self):
        self.graph.replay()

    def backward(self, grad_fine, grad_verts=None):
        if grad_verts is None:
            grad_verts = torch.zeros_like(self.verts)
        rtsdf_backward_batched(self.plan, grad_fine.contiguous(), self.hits, self.argmin, self.band_list,
                               self.band_count, self.bvh, self.tris, self.rays, self.rng_key, grad_verts)
        return grad_verts

    def view(self, t, o):
        """Object o's part of a concatenated per-grid-point tensor."""
        off = self.offsets[o][0]
        n = int(np.prod(self.dims[o]))
        return t[off:off + n]


class ClipMapSDF:
    """A clip map around a camera: `levels` grids of n^3 points, level l of voxel size
    h0 * 2^l (rtsdf_clipmap_levels), each holding the same mesh, built with the batched chain
    (one launch per stage for all levels; level l draws its rays with object word l) and read
    by the clip-map sampler and shadow pass (each point reads the finest level holding it).
    `fine` is the levels' concatenated field (level l = view(fine, l))."""

    def __init__(self, verts, tris, camera, h0, n, levels, band, rays, frames=1, beta=None, bias=0.0, rng_key=0,
                 bvh_method=BVH_PLOC, device="cuda"):
        check_hit_budget(rays, frames)
        if not 1 <= int(levels) <= MAX_CLIP_LEVELS:
            raise RtsdfError("1 to %d levels" % MAX_CLIP_LEVELS)
        self.grids = rtsdf_clipmap_levels(camera, h0, n, levels)
        steps = _halving_offsets((n, n, n)) + [1]
        objs = [types.SimpleNamespace(verts=verts, tris=tris, dims=(n, n, n), org=tuple(g.org), h=g.h, steps=steps,
                                      band=band) for g in self.grids]
        self.batch = BatchSDF(objs, rays, frames=frames, rng_key=rng_key, beta=beta, bias=bias, bvh_method=bvh_method,
                              device=device)
        self.plan = self.batch.plan
        self.device = device

    @property
    def fine(self):
        return self.batch.fine

    def run(self):
        return self.batch.run()

    def view(self, t, level):
        return self.batch.view(t, level)

    def sample(self, points):
        """(values, levels) at points [n, 3] (float32, on the device)."""
        pts = points.contiguous()
        vals = torch.empty(pts.shape[0], dtype=torch.float32, device=pts.device)
        lev = torch.empty(pts.shape[0], dtype=torch.int32, device=pts.device)
        rtsdf_clipmap_sample(self.plan, self.fine, pts, vals, lev)
        return vals, lev

    def shadow(self, s):
        img = torch.empty(s.nlights, s.base.height, s.base.width, dtype=torch.float32, device=self.device)
        rtsdf_shadow_forward_clip(self.plan, self.fine, s, img)
        return img

    def shadow_backward(self, s, grad_img, grad_fine=None):
        if grad_fine is None:
            grad_fine = torch.zeros_like(self.fine)
        rtsdf_shadow_backward_clip(self.plan, self.fine, s, grad_img.contiguous(), grad_fine)
        return grad_fine


def check_hit_budget(rays, frames):
    """Raises unless rays x frames <= 65535: a voxel's hit word keeps front hits in its low
    and back hits in its high 16 bits (section 2.1 counts both), so one more front hit than
    that would carry into the back count and flip the majority sign."""
    if int(rays) < 1 or int(frames) < 1 or int(rays) * int(frames) > MAX_RAYS:
        raise RtsdfError("rays x frames accumulated into one hit buffer must lie in [1, %d], got %d x %d"
                         % (MAX_RAYS, int(rays), int(frames)))


def _halving_offsets(dims):
    n = max(dims)
    k = 1
    while k < n:
        k *= 2
    out = []
    k //= 2
    while k >= 1:
        out.append(k)
        k //= 2
    return out or [1]


class StaticSDF:
    """Device buffers and the call chain for one static scene (sections 2.1-2.3).

    run() = voxelize, jump flood, mask, BVH, `frames` x ray sampling (running minimum),
    combine.  Buffers are allocated in __init__ and no call reads anything back to the host
    (the mask count stays on the device; launches are bounded by the grid size).  `obj` is
    the object word of the ray counters.  set_verts() replaces the vertex positions in place
    (same triangle list) for optimisation loops.

    Two-level field (sections 2.3 and 2.5.1): with ratio r > 1, `dims` and `h` describe the
    coarse grid that is voxelized and jump-flooded (`g`); rays, the mask list, the
    accumulators and the field live on the grid refined by r over the same box (`gf`),
    each fine point taking its coarse parent's distance and band test.  With r = 1 both
    are the same grid and the single-level calls run.
    """

    def __init__(self, verts, tris, dims, org, h, steps, band, rays, frames, beta=None, bias=0.0,
                 rng_key=0, keep_argmin=True, obj=0, bvh_method=BVH_PLOC, ratio=1, device="cuda"):
        check_hit_budget(rays, frames)
        self.g = make_grid(dims, org, h)
        self.ratio = int(ratio)
        self.gf = rtsdf_refine_grid(self.g, self.ratio) if self.ratio != 1 else self.g
        N, Nf = self.g.n, self.gf.n
        self.verts = torch.as_tensor(verts, dtype=torch.float32).reshape(-1, 3).contiguous().to(device)
        self.tris = torch.as_tensor(tris, dtype=torch.int32).reshape(-1, 3).contiguous().to(device)
        nt = self.tris.shape[0]
        self.steps, self.band, self.rays, self.frames = list(steps), int(band), int(rays), int(frames)
        self.beta = float(h) / 2 if beta is None else float(beta)
        self.bias, self.rng_key, self.obj = float(bias), int(rng_key), int(obj)
        self.bvh_method = int(bvh_method)
        self.seeds = torch.empty(N, dtype=torch.int32, device=device)
        self.scratch = torch.empty(N, dtype=torch.int32, device=device)
        self.band_list = torch.empty(Nf, dtype=torch.int32, device=device)
        self.band_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.dmin = torch.empty(Nf, dtype=torch.float32, device=device)
        self.hits = torch.empty(Nf, dtype=torch.int32, device=device)
        self.argmin = torch.empty(Nf, dtype=torch.int64, device=device) if keep_argmin else None
        self.fine = torch.empty(Nf, dtype=torch.float32, device=device)
        self.bvh = torch.empty(rtsdf_bvh_bytes(nt), dtype=torch.uint8, device=device)
        wb = max(rtsdf_voxelize_work_bytes(nt), rtsdf_band_refined_work_bytes(self.g, self.ratio),
                 rtsdf_bvh_work_bytes(nt))
        self.work = workspace(wb, device)
        self.ray_work = workspace(rtsdf_raysample_work_bytes(Nf, self.rays), device)
        self.band_n = Nf  # launch bound for the mask list
        self.device = device
        self.jfa_out = None

    def set_verts(self, verts):
        self.verts.copy_(verts.reshape(-1, 3))

    def voxelize(self):
        rtsdf_voxelize(self.verts, self.tris, self.g, self.seeds, self.work)

    def jfa(self):
        self.jfa_out = rtsdf_jfa(self.seeds, self.scratch, self.g, self.steps)

    def mask(self):
        if self.ratio == 1:
            rtsdf_band(self.jfa_out, self.g, self.band, self.band_list, self.band_count, self.work)
        else:
            rtsdf_band_refined(self.jfa_out, self.g, self.ratio, self.band, self.band_list, self.band_count,
                               self.work)

    def build_bvh(self):
        rtsdf_build_bvh(self.verts, self.tris, self.gf, self.bvh, self.work, self.bvh_method)

    def trace(self, frame):
        rtsdf_raysample(self.bvh, self.gf, self.band_list, self.band_count, self.rays, self.rng_key, frame,
                        self.dmin, self.hits, self.ray_work, self.argmin, obj=self.obj, band_capacity=self.band_n)

    def combine(self):
        if self.ratio == 1:
            rtsdf_combine(self.jfa_out, self.dmin, self.hits, self.g, self.band, self.beta, self.bias, ACCUM,
                          self.fine)
        else:
            rtsdf_combine_refined(self.jfa_out, self.dmin, self.hits, self.g, self.ratio, self.band, self.beta,
                                  self.bias, ACCUM, self.fine)

    def run(self):
        self.voxelize()
        self.jfa()
        self.mask()
        self.build_bvh()
        rtsdf_reset_accum(self.dmin, self.hits, self.argmin)
        for f in range(self.frames):
            self.trace(f)
        self.combine()
        return self.fine

    def backward(self, grad_fine, grad_verts=None):
        """dL/dverts of the last run() given dL/dfine (running-minimum mode)."""
        if self.argmin is None:
            raise RtsdfError("the vertex adjoint needs the argmin records (keep_argmin=True)")
        if grad_verts is None:
            grad_verts = torch.zeros_like(self.verts)
        rtsdf_backward(grad_fine.contiguous(), self.hits, self.argmin, self.band_list, self.band_count, self.bvh,
                       self.tris, self.verts.shape[0], self.gf, self.rays, self.rng_key, grad_verts, obj=self.obj,
                       band_capacity=self.band_n)
        return grad_verts


class SDF(torch.autograd.Function):
    """fine = SDF.apply(verts, S): runs the static pipeline of StaticSDF `S` on `verts`
    ([nv, 3] float32, on the GPU) and returns a copy of the fine field.  The backward is
    the vertex adjoint through each grid point's argmin ray (rtsdf_backward)."""

    @staticmethod
    def forward(ctx, verts, S):
        S.set_verts(verts.detach())
        fine = S.run().clone()
        ctx.S = S
        return fine

    @staticmethod
    def backward(ctx, grad_fine):
        return ctx.S.backward(grad_fine), None


class SoftShadow(torch.autograd.Function):
    """img = SoftShadow.apply(fine, grid, shadow): the soft-shadow image of the fine field
    (section 2.4), [height, width] float32 for a Shadow, [nlights, height, width] for a
    ShadowEx (the full pass).  The backward is rtsdf_shadow_backward(_ex)."""

    @staticmethod
    def forward(ctx, fine, grid, shadow):
        fine = fine.detach().contiguous()
        if isinstance(shadow, ShadowEx):
            img = torch.empty(shadow.nlights, shadow.base.height, shadow.base.width, dtype=torch.float32,
                              device=fine.device)
            rtsdf_shadow_forward_ex(fine, grid, shadow, img)
        else:
            img = torch.empty(shadow.height, shadow.width, dtype=torch.float32, device=fine.device)
            rtsdf_shadow_forward(fine, grid, shadow, img)
        ctx.save_for_backward(fine)
        ctx.grid, ctx.shadow = grid, shadow
        return img

    @staticmethod
    def backward(ctx, grad_img):
        (fine,) = ctx.saved_tensors
        grad_fine = torch.zeros_like(fine)
        if isinstance(ctx.shadow, ShadowEx):
            rtsdf_shadow_backward_ex(fine, ctx.grid, ctx.shadow, grad_img.contiguous(), grad_fine)
        else:
            rtsdf_shadow_backward(fine, ctx.grid, ctx.shadow, grad_img.contiguous(), grad_fine)
        return grad_fine, None, None


class DeformSDF:
    """The per-frame chain for a deforming mesh (section 2.5.1): every frame re-voxelizes,
    re-floods, re-masks, rebuilds the hierarchy, ray-samples the mask and folds the frame
    into the field with the decay rule of Eq. 1 (RTSDF_DECAY, `consume` resets the frame's
    ray accumulators).  All frames' vertices are resident on the device.  frame(f) only
    enqueues kernels and never synchronizes; frame 0 also clears the accumulators and starts
    the decay from the coarse field.  capture() records the chain of frames >= 1 once into a
    HIP graph in which everything that depends on the frame reads a one-word frame index in
    device memory (the frame's vertices are gathered into a fixed buffer, ray sampling reads
    the counter word there), so replay(f) only writes f into that word and replays the same
    graph for every frame.
    ratio r > 1 is the paper's two-level configuration: `dims`/`h` are the coarse flooded
    grid `g`, rays and the field run on the grid `gf` refined by r (see StaticSDF).
    """

    def __init__(self, frame_verts, tris, dims, org, h, steps, band, rays, alpha=0.95, beta=None, bias=0.0,
                 rng_key=0, bvh_method=BVH_LBVH, ratio=1, device="cuda"):
        check_hit_budget(rays, 1)  # the combine consumes each frame's counts
        self.g = make_grid(dims, org, h)
        self.ratio = int(ratio)
        self.gf = rtsdf_refine_grid(self.g, self.ratio) if self.ratio != 1 else self.g
        N, Nf = self.g.n, self.gf.n
        self.verts = torch.as_tensor(frame_verts, dtype=torch.float32).contiguous().to(device)
        self.nframes = self.verts.shape[0]
        self.tris = torch.as_tensor(tris, dtype=torch.int32).reshape(-1, 3).contiguous().to(device)
        nt = self.tris.shape[0]
        self.steps, self.band, self.rays = list(steps), int(band), int(rays)
        self.alpha = float(alpha)
        self.bvh_method = int(bvh_method)
        self.beta = float(h) / 2 if beta is None else float(beta)
        self.bias, self.rng_key = float(bias), int(rng_key)
        self.seeds = torch.empty(N, dtype=torch.int32, device=device)
        self.scratch = torch.empty(N, dtype=torch.int32, device=device)
        self.band_list = torch.empty(Nf, dtype=torch.int32, device=device)
        self.band_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.dmin = torch.empty(Nf, dtype=torch.float32, device=device)
        self.hits = torch.empty(Nf, dtype=torch.int32, device=device)
        self.state = torch.zeros(Nf, dtype=torch.float32, device=device)
        self.fine = torch.empty(Nf, dtype=torch.float32, device=device)
        self.bvh = torch.empty(rtsdf_bvh_bytes(nt), dtype=torch.uint8, device=device)
        wb = max(rtsdf_voxelize_work_bytes(nt), rtsdf_band_refined_work_bytes(self.g, self.ratio),
                 rtsdf_bvh_work_bytes(nt))
        self.work = workspace(wb, device)
        self.ray_work = workspace(rtsdf_raysample_work_bytes(Nf, self.rays), device)
        self.graph = None
        self.frame_dev = torch.zeros(1, dtype=torch.int32, device=device)
        self.cur = torch.empty_like(self.verts[:1])  # the replayed graph's vertex buffer [1, V, 3]
        self.jfa_out = None

    def frame(self, f):
        self._chain(self.verts[f], f, None)

    def _chain(self, v, f, frame_dev):
        """One frame's chain on vertices v: frame f (frame_dev None) or the frame index held
        in frame_dev (a frame >= 1)."""
        if frame_dev is None and f == 0:
            rtsdf_reset_accum(self.dmin, self.hits)
        first = frame_dev is None and f == 0
        rtsdf_voxelize(v, self.tris, self.g, self.seeds, self.work)
        self.jfa_out = rtsdf_jfa(self.seeds, self.scratch, self.g, self.steps)
        if self.ratio == 1:
            rtsdf_band(self.jfa_out, self.g, self.band, self.band_list, self.band_count, self.work)
        else:
            rtsdf_band_refined(self.jfa_out, self.g, self.ratio, self.band, self.band_list, self.band_count,
                               self.work)
        rtsdf_build_bvh(v, self.tris, self.gf, self.bvh, self.work, self.bvh_method)
        if frame_dev is None:
            rtsdf_raysample(self.bvh, self.gf, self.band_list, self.band_count, self.rays, self.rng_key, f, self.dmin,
                            self.hits, self.ray_work)
        else:
            rtsdf_raysample_frame_device(self.bvh, self.gf, self.band_list, self.band_count, self.rays, self.rng_key,
                                         frame_dev, self.dmin, self.hits, self.ray_work)
        if self.ratio == 1:
            rtsdf_combine(self.jfa_out, self.dmin, self.hits, self.g, self.band, self.beta, self.bias, DECAY,
                          self.fine, alpha=self.alpha, first_frame=first, consume=True, state=self.state)
        else:
            rtsdf_combine_refined(self.jfa_out, self.dmin, self.hits, self.g, self.ratio, self.band, self.beta,
                                  self.bias, DECAY, self.fine, alpha=self.alpha, first_frame=first, consume=True,
                                  state=self.state)

    def capture(self):
        """Records the chain of a frame >= 1 once (vertices gathered by the device-side frame
        index, ray counters read from it)."""
        self.frame_dev.fill_(1)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            torch.index_select(self.verts, 0, self.frame_dev, out=self.cur)
            self._chain(self.cur[0], None, self.frame_dev)
        self.graph = gr

    def replay(self, f):
        """Frame f: frame 0 runs eagerly (it starts the decay); later frames replay the graph."""
        if f == 0 or self.graph is None:
            self.frame(f)
            return
        self.frame_dev.fill_(f)
        self.graph.replay()
