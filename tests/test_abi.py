"""The C ABI library loads without a GPU, exports every entry point the header declares,
and rejects bad arguments on the host before anything is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtsdf.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtsdf_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2210_06160_amd import rtsdf
    if not os.path.exists(rtsdf.LIB_PATH):
        pytest.skip("librtsdf.so not built")
    return rtsdf


def test_exports_every_declared_symbol(L):
    names = declared()
    assert len(names) >= 12
    raw = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(L.EXPORTED)
    assert L.rtsdf_abi_version() == 2


def fake(v=0x1000):
    return ctypes.c_void_p(v)


def test_host_validation(L):
    lib = L.lib()
    g = L.make_grid((8, 8, 8), (0, 0, 0), 0.1)
    bad = L.make_grid((0, 8, 8), (0, 0, 0), 0.1)
    big = L.make_grid((1025, 8, 8), (0, 0, 0), 0.1)
    nanh = L.make_grid((8, 8, 8), (0, 0, 0), float("nan"))
    E_ARG, E_RANGE, E_SIZE = -1, -2, -3
    st = (ctypes.c_int32 * 2)(4, 1)
    flag = ctypes.c_int32(0)
    assert lib.rtsdf_jfa(fake(), fake(), bad, st, 2, ctypes.byref(flag), None) == E_RANGE
    assert lib.rtsdf_jfa(fake(), fake(), big, st, 2, ctypes.byref(flag), None) == E_RANGE
    assert lib.rtsdf_jfa(fake(), fake(), nanh, st, 2, ctypes.byref(flag), None) == E_ARG
    assert lib.rtsdf_jfa(fake(), fake(), g, st, 2, ctypes.byref(flag), None) == E_ARG  # aliased
    assert b"alias" in lib.rtsdf_last_error()
    st0 = (ctypes.c_int32 * 2)(0, 1)
    assert lib.rtsdf_jfa(fake(), fake(0x2000), g, st0, 2, ctypes.byref(flag), None) == E_ARG
    assert lib.rtsdf_jfa(fake(), fake(0x2000), g, st, 65, ctypes.byref(flag), None) == E_RANGE
    assert lib.rtsdf_jfa(None, fake(0x2000), g, st, 2, ctypes.byref(flag), None) == E_ARG
    # voxelize
    assert lib.rtsdf_voxelize(fake(), 3, fake(), -1, g, fake(), fake(), 1 << 20, None) == E_RANGE
    assert lib.rtsdf_voxelize(fake(), 3, fake(), 1, g, fake(), fake(), 1, None) == E_SIZE
    assert lib.rtsdf_voxelize(fake(), 3, fake(), 1, g, None, fake(), 1 << 20, None) == E_ARG
    # band
    assert lib.rtsdf_band(fake(), g, -1, fake(), fake(), fake(), 1 << 20, None) == E_RANGE
    assert lib.rtsdf_band(fake(), g, 2, fake(), fake(), fake(), 0, None) == E_SIZE
    # bvh
    assert lib.rtsdf_build_bvh(fake(), 3, fake(), 1, g, 1, fake(), 10, fake(), 1 << 20, None) == E_SIZE
    assert lib.rtsdf_build_bvh(fake(), 3, fake(), (1 << 26) + 1, g, 1, fake(), 1 << 40, fake(), 1 << 40,
                               None) == E_RANGE
    assert lib.rtsdf_build_bvh(fake(), 3, fake(), 1, g, 2, fake(), 1 << 20, fake(), 1 << 20, None) == E_RANGE
    # raysample
    for rays in (0, 65536):
        assert lib.rtsdf_raysample(fake(), g, fake(), fake(), 10, rays, 0, 0, 0, fake(), fake(), None,
                                   fake(), 256, None) == E_RANGE
    assert lib.rtsdf_raysample(fake(), g, fake(), fake(), 10, 4, 0, 0, 1 << 24, fake(), fake(), None,
                               fake(), 256, None) == E_RANGE
    assert lib.rtsdf_raysample(fake(), g, fake(), fake(), 513, 4, 0, 0, 0, fake(), fake(), None,
                               fake(), 256, None) == E_RANGE
    assert lib.rtsdf_raysample(fake(), g, fake(), fake(), 10, 4, 0, 0, 0, fake(), fake(), None,
                               fake(), lib.rtsdf_raysample_work_bytes(10, 4) - 1, None) == E_SIZE
    assert lib.rtsdf_raysample(fake(), g, fake(), fake(), 10, 4, 0, 0, 0, fake(), fake(), None,
                               None, 256, None) == E_ARG
    # the device-side frame index variant: same checks, plus a NULL frame pointer
    assert lib.rtsdf_raysample_frame_device(fake(), g, fake(), fake(), 10, 4, 0, None, 0, fake(), fake(), None,
                                            fake(), 256, None) == E_ARG
    assert lib.rtsdf_raysample_frame_device(fake(), g, fake(), fake(), 10, 0, 0, fake(), 0, fake(), fake(), None,
                                            fake(), 256, None) == E_RANGE
    assert lib.rtsdf_raysample_frame_device(fake(), g, fake(), fake(), 10, 4, 0, fake(), 0, fake(), fake(), None,
                                            fake(), lib.rtsdf_raysample_work_bytes(10, 4) - 1, None) == E_SIZE
    # the allocation-free variant validates the same way, before it touches a device
    for rays in (0, 65536):
        assert lib.rtsdf_raysample_noalloc(fake(), g, fake(), fake(), 10, rays, 0, 0, 0, fake(), fake(), None,
                                           None) == E_RANGE
    assert lib.rtsdf_raysample_noalloc(fake(), g, fake(), fake(), 10, 4, 0, 0, 1 << 24, fake(), fake(), None,
                                       None) == E_RANGE
    assert lib.rtsdf_raysample_noalloc(fake(), g, fake(), fake(), 513, 4, 0, 0, 0, fake(), fake(), None,
                                       None) == E_RANGE
    assert lib.rtsdf_raysample_noalloc(fake(), bad, fake(), fake(), 10, 4, 0, 0, 0, fake(), fake(), None,
                                       None) == E_RANGE
    assert lib.rtsdf_raysample_noalloc(None, g, fake(), fake(), 10, 4, 0, 0, 0, fake(), fake(), None,
                                       None) == E_ARG
    assert lib.rtsdf_raysample_noalloc(fake(), g, fake(), fake(), 10, 4, 0, 0, 0, fake(), None, None,
                                       None) == E_ARG
    # combine
    assert lib.rtsdf_combine(fake(), fake(), fake(), g, 2, 0.0, 0.0, 7, 0.9, 1, 0, fake(), fake(),
                             None) == E_RANGE
    assert lib.rtsdf_combine(fake(), fake(), fake(), g, 2, 0.0, 0.0, 1, 1.5, 1, 0, fake(), fake(),
                             None) == E_ARG
    assert lib.rtsdf_combine(fake(), fake(), fake(), g, 2, 0.0, 0.0, 1, 0.9, 1, 0, None, fake(),
                             None) == E_ARG
    assert lib.rtsdf_combine(fake(), fake(), fake(), g, 2, float("inf"), 0.0, 0, 0.9, 1, 0, None,
                             fake(), None) == E_ARG
    assert lib.rtsdf_reset_accum(fake(), fake(), None, -1, None) == E_RANGE


def shadow_params(L, **kw):
    p = dict(width=16, height=16, x0=0.0, z0=0.0, dx=0.05, dz=0.05, y=0.1, light=(0.0, 1.0, 0.0), k=8.0,
             steps=64, smin=0.05, smax=0.05, t0=0.1)
    p.update(kw)
    return L.make_shadow(**p)


def test_host_validation_adjoints(L):
    lib = L.lib()
    g = L.make_grid((8, 8, 8), (0, 0, 0), 0.1)
    E_ARG, E_RANGE = -1, -2
    fwd, bwd = lib.rtsdf_shadow_forward, lib.rtsdf_shadow_backward
    for kw, code in [(dict(steps=0), E_RANGE), (dict(steps=257), E_RANGE), (dict(width=-1), E_RANGE),
                     (dict(height=16385), E_RANGE), (dict(k=0.0), E_ARG), (dict(t0=0.0), E_ARG),
                     (dict(smin=0.0), E_ARG), (dict(smax=0.01), E_ARG), (dict(x0=float("nan")), E_ARG),
                     (dict(light=(0.0, float("inf"), 0.0)), E_ARG)]:
        s = shadow_params(L, **kw)
        assert fwd(fake(), g, s, fake(0x2000), None) == code, kw
        assert bwd(fake(), g, s, fake(0x2000), fake(0x3000), None) == code, kw
    s = shadow_params(L)
    assert fwd(None, g, s, fake(0x2000), None) == E_ARG
    assert fwd(fake(), L.make_grid((0, 8, 8), (0, 0, 0), 0.1), s, fake(0x2000), None) == E_RANGE
    assert bwd(fake(), g, s, fake(0x2000), fake(), None) == E_ARG   # grad_fine aliases fine
    assert bwd(fake(), g, s, None, fake(0x3000), None) == E_ARG
    # vertex adjoint
    b = lib.rtsdf_backward
    args = lambda **kw: [kw.get("gf", fake()), fake(), fake(), fake(), fake(), kw.get("cap", 10), fake(),
                         kw.get("tris", fake()), kw.get("nv", 3), kw.get("nt", 1), g, kw.get("rays", 4), 0,
                         kw.get("obj", 0), kw.get("gv", fake()), None]
    assert b(*args(rays=0)) == E_RANGE
    assert b(*args(rays=65536)) == E_RANGE
    assert b(*args(obj=1 << 24)) == E_RANGE
    assert b(*args(cap=513)) == E_RANGE
    assert b(*args(nt=-1)) == E_RANGE
    assert b(*args(gf=None)) == E_ARG
    assert b(*args(gv=None)) == E_ARG
    assert b(*args(tris=None)) == E_ARG
    assert b(*args(nt=0, tris=None, gv=None)) == 0          # no triangles: nothing to do


def test_workspace_queries(L):
    lib = L.lib()
    g = L.make_grid((400, 200, 400), (0, 0, 0), 0.005)
    assert lib.rtsdf_voxelize_work_bytes(103000) >= 8 * 103001
    assert lib.rtsdf_band_work_bytes(g) > 0
    assert lib.rtsdf_bvh_bytes(103000) >= 256 + 64 * 102999 + 48 * 103000
    assert lib.rtsdf_bvh_work_bytes(103000) >= 16 * 103000
    assert lib.rtsdf_voxelize_work_bytes(-1) == 0
    assert lib.rtsdf_raysample_work_bytes(1000, 8) >= 32


def test_refined_grid_and_validation(L, orc):
    """rtsdf_refine_grid (host only) against the oracle's refinement, and host validation of
    the two-level entries."""
    lib = L.lib()
    E_ARG, E_RANGE, E_SIZE = -1, -2, -3
    for dims, org, h, r in [((200, 100, 200), (-1.0, 0.0, -1.0), 0.01, 2), ((16, 16, 16), (0, 0, 0), 1 / 16, 3),
                            ((7, 1, 5), (0.25, 0.5, 0.125), 0.3, 1), ((128, 128, 128), (0, 0, 0), 1 / 128, 8)]:
        g = L.make_grid(dims, org, h)
        f = L.rtsdf_refine_grid(g, r)
        o = orc.refine_grid(orc.make_grid(dims, org, h), r)
        assert (f.nx, f.ny, f.nz) == (o.nx, o.ny, o.nz)
        assert list(f.org) == list(o.org)
        assert ctypes.c_float(f.h).value == ctypes.c_float(o.h).value
        assert lib.rtsdf_band_refined_work_bytes(g, r) >= lib.rtsdf_band_work_bytes(f)
    g = L.make_grid((300, 8, 8), (0, 0, 0), 0.1)
    out = L.Grid()
    assert lib.rtsdf_refine_grid(g, 4, ctypes.byref(out)) == E_RANGE      # 1200 > 1024
    assert lib.rtsdf_refine_grid(g, 0, ctypes.byref(out)) == E_RANGE
    assert lib.rtsdf_refine_grid(g, 2, None) == E_ARG
    assert lib.rtsdf_band_refined_work_bytes(g, 4) == 0
    g = L.make_grid((8, 8, 8), (0, 0, 0), 0.1)
    need = lib.rtsdf_band_refined_work_bytes(g, 2)
    assert lib.rtsdf_band_refined(fake(), g, 2, 2, fake(), fake(), fake(), need - 1, None) == E_SIZE
    assert lib.rtsdf_band_refined(fake(), g, 2, -1, fake(), fake(), fake(), need, None) == E_RANGE
    assert lib.rtsdf_band_refined(fake(), g, 0, 2, fake(), fake(), fake(), need, None) == E_RANGE
    assert lib.rtsdf_band_refined(None, g, 2, 2, fake(), fake(), fake(), need, None) == E_ARG
    c = lib.rtsdf_combine_refined
    assert c(fake(), fake(), fake(), g, 2, 2, 0.0, 0.0, 7, 0.9, 1, 0, fake(), fake(), None) == E_RANGE
    assert c(fake(), fake(), fake(), g, 2, 2, 0.0, 0.0, 1, 0.9, 1, 0, None, fake(), None) == E_ARG
    assert c(fake(), fake(), fake(), g, 200, 2, 0.0, 0.0, 0, 0.9, 1, 0, None, fake(), None) == E_RANGE
    assert c(fake(), fake(), fake(), g, 2, 2, float("nan"), 0.0, 0, 0.9, 1, 0, None, fake(), None) == E_ARG


def test_host_validation_shadow_ex(L):
    """The full shadow pass rejects bad parameters on the host."""
    import ctypes as C
    lib = L.lib()
    g = L.make_grid((8, 8, 8), (0, 0, 0), 0.1)
    E_ARG, E_RANGE = -1, -2
    base = shadow_params(L)
    light = (0.0, 1.0, 0.0)

    def run(s, img=fake(0x2000)):
        return lib.rtsdf_shadow_forward_ex(fake(), g, C.byref(s), img, None)

    assert lib.rtsdf_shadow_forward_ex(fake(), g, None, fake(0x2000), None) == E_ARG
    s = L.make_shadow_ex(base, [light])
    s.nlights = 0
    assert run(s) == E_RANGE
    s.nlights = L.MAX_LIGHTS + 1
    assert run(s) == E_RANGE
    s = L.make_shadow_ex(base, [light, (float("nan"), 1.0, 0.0)])
    assert run(s) == E_ARG
    s = L.make_shadow_ex(base, [light], jitter=-0.1)
    assert run(s) == E_ARG
    s = L.make_shadow_ex(shadow_params(L, steps=0), [light])
    assert run(s) == E_RANGE
    s = L.make_shadow_ex(base, [light])
    assert lib.rtsdf_shadow_forward_ex(None, g, C.byref(s), fake(0x2000), None) == E_ARG
    assert lib.rtsdf_shadow_backward_ex(fake(), g, C.byref(s), fake(0x2000), fake(), None) == E_ARG  # aliases fine
    assert lib.rtsdf_shadow_backward_ex(fake(), g, C.byref(s), None, fake(0x3000), None) == E_ARG
    with pytest.raises(L.RtsdfError):
        L.make_shadow_ex(base, [])


def test_clipmap_levels_match_the_oracle(L, orc):
    """rtsdf_clipmap_levels (host only) places the levels as the oracle does, bit for bit,
    and rejects bad arguments."""
    import ctypes as C
    rng = np.random.default_rng(3)
    for _ in range(40):
        cam = rng.uniform(-5, 5, 3).astype(np.float32)
        h0 = float(np.float32(rng.uniform(0.001, 0.1)))
        n = int(rng.choice([4, 16, 64, 128]))
        lv = int(rng.integers(1, L.MAX_CLIP_LEVELS + 1))
        a = L.rtsdf_clipmap_levels(cam, h0, n, lv)
        b = orc.clipmap_levels(cam, h0, n, lv)
        for ga, gb in zip(a, b):
            assert (ga.nx, ga.ny, ga.nz) == (gb.nx, gb.ny, gb.nz)
            assert list(ga.org) == list(gb.org) and ga.h == gb.h
    lib = L.lib()
    cam = (C.c_float * 3)(0.0, 0.0, 0.0)
    out = (L.Grid * 9)()
    assert lib.rtsdf_clipmap_levels(cam, 0.1, 5, 2, out) == -2      # odd n
    assert lib.rtsdf_clipmap_levels(cam, 0.1, 2, 2, out) == -2      # n < 4
    assert lib.rtsdf_clipmap_levels(cam, 0.1, 8, 9, out) == -2      # too many levels
    assert lib.rtsdf_clipmap_levels(cam, 0.0, 8, 2, out) == -1      # h0
    assert lib.rtsdf_clipmap_levels(None, 0.1, 8, 2, out) == -1
    nan = (C.c_float * 3)(float("nan"), 0.0, 0.0)
    assert lib.rtsdf_clipmap_levels(nan, 0.1, 8, 2, out) == -1


def test_hit_budget_guard(L):
    """Front and back hits share one 32-bit word (16 bits each): the helpers refuse a
    configuration that could accumulate more than 65535 rays into one voxel's counts,
    before allocating or launching anything."""
    from paper_2210_06160_amd import synth
    L.check_hit_budget(8, 8191)
    L.check_hit_budget(65535, 1)
    for rays, frames in ((8, 8192), (65536, 1), (0, 1), (4, 0)):
        with pytest.raises(L.RtsdfError, match="rays x frames"):
            L.check_hit_budget(rays, frames)
    sc = synth.scene_tiny()
    with pytest.raises(L.RtsdfError, match="rays x frames"):
        L.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, 16, 4096)
    with pytest.raises(L.RtsdfError, match="rays x frames"):
        L.BatchSDF([sc], rays=256, frames=256)
    with pytest.raises(L.RtsdfError, match="rays x frames"):
        L.ClipMapSDF(sc.verts, sc.tris, (0.5, 0.5, 0.5), 1 / 32, 16, 2, 2, 300, frames=300)
    with pytest.raises(L.RtsdfError, match="rays x frames"):
        L.DeformSDF(np.stack([sc.verts] * 2), sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, 70000)
