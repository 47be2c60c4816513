"""The full shadow pass on the GPU (several lights, jittered start, two-sample
triangulation; sections 2.5.2 and 3.2) versus the binary64 oracle, through the C ABI.

Bars (as the single-light shadow tests): images within 1e-4 per pixel; the adjoint
element by element, |diff| <= 1e-3 |g| + 1e-4 max|g|, with the image gradient restricted
to pixels whose discrete decisions the oracle's margins show binary32 cannot flip
(r_margin > 1e-4, s_margin > 1e-5, c_margin > 2e-3 grid units, and v_margin > 1e-2: the
triangulated estimate's derivative carries 1/d and 1/(t - y), which amplify binary32
rounding by about r2^2/d^2 and t/(t - y), so the comparison keeps those below 100).
Triangulated images are compared where v_margin > 1e-4 (the validity tests -- samples in
grid units, d^2 and t - y relative -- about 100 times what binary32 rounding moves them):
a flipped validity test switches the estimate's formula, the other decisions move the
image continuously.
Cases: one light without jitter equals the single-light entry point bit for bit; a 48^3
sphere field with three lights, 128 steps and ragged 61 x 37 images, plain and
triangulated, with and without jitter, bounded or not; eight lights with 256 steps; an
empty image; and
the pass the benchmark times (the 128^3 ellipsoid field, 512^2 pixels, three lights, 128
steps, triangulated, jittered and bounded by the field's box).
"""
import sys

import numpy as np
import pytest

from paper_2210_06160_amd import synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2210_06160_amd import rtsdf
    rtsdf.lib()
    return rtsdf


def sphere_field(dims, h, C=(0.5, 0.3, 0.5), r=0.12):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    P = np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h, (k.ravel() + 0.5) * h], 1)
    return (np.linalg.norm(P - np.asarray(C), axis=1) - r).astype(np.float32)


def both(R, orc, p, lights, **kw):
    return (R.make_shadow_ex(R.make_shadow(**p), lights, **kw), orc.make_shadow_ex(orc.make_shadow(**p), lights, **kw))


def gpu_fwd(R, f, g, s):
    import torch
    img = torch.empty(s.nlights, s.base.height, s.base.width, dtype=torch.float32, device="cuda")
    R.rtsdf_shadow_forward_ex(torch.from_numpy(f).cuda(), g, s, img)
    torch.cuda.synchronize()
    return img.cpu().numpy().ravel()


def gpu_bwd(R, f, g, s, gi):
    import torch
    gf = torch.zeros(len(f), dtype=torch.float32, device="cuda")
    R.rtsdf_shadow_backward_ex(torch.from_numpy(f).cuda(), g, s, torch.from_numpy(gi.astype(np.float32)).cuda(), gf)
    torch.cuda.synchronize()
    return gf.cpu().numpy()


def close(a, b, rtol=1e-3, arel=1e-4):
    b = np.asarray(b, np.float64)
    tol = rtol * np.abs(b) + arel * np.abs(b).max()
    err = np.abs(np.asarray(a, np.float64) - b)
    bad = err > tol
    assert not bad.any(), "%d of %d elements differ; worst %g" % (bad.sum(), bad.size, err[bad].max())


def safe(orc, f, g, s, img):
    """(pixels whose image is comparable, penumbra pixels whose adjoint is comparable)"""
    rm, sm, cm, vm = orc.shadow_margin_ex(f, g, s)
    fwd = vm > 1e-4
    return fwd, (vm > 1e-2) & (img > 0) & (img < 1) & (rm > 1e-4) & (sm > 1e-5) & (cm > 2e-3)


def test_one_light_equals_single_light_entry(R):
    import torch
    dims, h = (48, 48, 48), 1.0 / 48
    g = R.make_grid(dims, (0, 0, 0), h)
    p = synth.shadow_setup(h, width=61, height=37, steps=128)
    f = torch.from_numpy(sphere_field(dims, h)).cuda()
    s1 = R.make_shadow(**p)
    sx = R.make_shadow_ex(R.make_shadow(**p), [p["light"]])
    a = torch.empty(37, 61, device="cuda")
    b = torch.empty(1, 37, 61, device="cuda")
    R.rtsdf_shadow_forward(f, g, s1, a)
    R.rtsdf_shadow_forward_ex(f, g, sx, b)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b[0].view(torch.int32))
    gi = torch.randn(37, 61, device="cuda")
    ga, gb = torch.zeros_like(f), torch.zeros_like(f)
    R.rtsdf_shadow_backward(f, g, s1, gi, ga)
    R.rtsdf_shadow_backward_ex(f, g, sx, gi[None], gb)
    torch.cuda.synchronize()
    close(gb.cpu().numpy(), ga.cpu().numpy().astype(np.float64), rtol=1e-5, arel=1e-6)


LIGHTS3 = [tuple(np.array(v) / np.linalg.norm(v)) for v in ((0.35, 1.0, 0.25), (-0.5, 1.0, 0.2), (0.15, 1.0, -0.45))]


@pytest.mark.parametrize("tri,jitter,bounded", [(False, 0.0, False), (False, 0.05, False), (True, 0.0, False),
                                                (True, 0.05, False), (True, 0.05, True), (False, 0.0, True)])
def test_three_lights_parity(R, orc, tri, jitter, bounded):
    dims, h = (48, 48, 48), 1.0 / 48
    log("case: 3 lights, 128 steps, 61x37, triangulate %s, jitter %g, bounded %s" % (tri, jitter, bounded))
    g_r, g_o = R.make_grid(dims, (0, 0, 0), h), orc.make_grid(dims, (0, 0, 0), h)
    p = synth.shadow_setup(h, width=61, height=37, steps=128)
    s_r, s_o = both(R, orc, p, LIGHTS3, triangulate=tri, jitter=jitter, frame=5, key=0xBEEF, bounded=bounded)
    f = sphere_field(dims, h)
    io = orc.shadow_forward_ex(f, g_o, s_o)
    ig = gpu_fwd(R, f, g_r, s_r)
    ok, use = safe(orc, f, g_o, s_o, io)
    pen = (io > 0) & (io < 1)
    err = np.abs(ig - io)
    log("  max |diff| (safe pixels)", err[ok].max(), "safe", ok.sum(), "of", io.size, "penumbra", pen.sum(),
        "adjoint pixels", use.sum())
    assert err[ok].max() <= 1e-4
    if not tri and not bounded:
        assert ok.all()
    # the oracle's margins keep >= 99.8 % of the pixels and 87-94 % of the penumbra adjoints
    assert ok.sum() >= 0.997 * io.size and pen.sum() > 0
    assert use.sum() >= 0.86 * pen.sum()
    gi = np.where(use, np.random.default_rng(7).normal(size=io.size), 0.0).astype(np.float32)
    go = orc.shadow_backward_ex(f, g_o, s_o, gi.astype(np.float64))
    gg = gpu_bwd(R, f, g_r, s_r, gi)
    assert np.abs(go).max() > 0
    close(gg, go)


def test_eight_lights_max_steps_and_empty(R, orc):
    import torch
    dims, h = (24, 20, 28), 1.0 / 28
    g_r, g_o = R.make_grid(dims, (0, 0, 0), h), orc.make_grid(dims, (0, 0, 0), h)
    rng = np.random.default_rng(3)
    lights = []
    for _ in range(8):
        v = np.array([rng.uniform(-0.6, 0.6), 1.0, rng.uniform(-0.6, 0.6)])
        lights.append(tuple(v / np.linalg.norm(v)))
    p = synth.shadow_setup(h, width=16, height=16, steps=256)
    s_r, s_o = both(R, orc, p, lights, triangulate=True, jitter=0.02, frame=1, key=9, bounded=True)
    f = sphere_field(dims, h, C=(0.4, 0.35, 0.5), r=0.1)
    io = orc.shadow_forward_ex(f, g_o, s_o)
    ig = gpu_fwd(R, f, g_r, s_r)
    ok, _ = safe(orc, f, g_o, s_o, io)
    assert np.abs(ig - io)[ok].max() <= 1e-4 and ok.sum() >= 0.99 * io.size  # the oracle keeps all
    # an empty image is a no-op (NULL image pointers allowed)
    pe = dict(p, width=0)
    se = R.make_shadow_ex(R.make_shadow(**pe), lights)
    fz = torch.from_numpy(f).cuda()
    assert R.lib().rtsdf_shadow_forward_ex(R._ptr(fz), g_r, R.ctypes.byref(se), None, None) == 0
    gz = torch.zeros_like(fz)
    assert R.lib().rtsdf_shadow_backward_ex(R._ptr(fz), g_r, R.ctypes.byref(se), None, R._ptr(gz), None) == 0
    torch.cuda.synchronize()
    assert (gz == 0).all()


def test_dl_workload_parity(R, orc):
    """The pass the benchmark times: the 128^3 ellipsoid field, 512^2 pixels, three lights,
    128 steps capped at 0.05, triangulated, start jittered by up to one step, bounded."""
    sc = synth.scene_grad()
    log("case: DL pass 512x512 x 3 lights x 128 steps over the 128^3 ellipsoid field")
    p, lights, kw = synth.dl_setup(sc.h)
    g_r, g_o = R.make_grid(sc.dims, sc.org, sc.h), orc.make_grid(sc.dims, sc.org, sc.h)
    s_r, s_o = both(R, orc, p, lights, **kw)
    f = sc.extra["target"].astype(np.float32)
    io = orc.shadow_forward_ex(f, g_o, s_o)
    ig = gpu_fwd(R, f, g_r, s_r)
    ok, use = safe(orc, f, g_o, s_o, io)
    pen = (io > 0) & (io < 1)
    log("  max |diff| (safe)", np.abs(ig - io)[ok].max(), "safe", ok.sum(), "penumbra", pen.sum(),
        "adjoint pixels", use.sum())
    # the oracle's margins keep 99.7 % of the pixels and 82.6 % of the penumbra adjoints
    assert np.abs(ig - io)[ok].max() <= 1e-4 and ok.sum() >= 0.996 * io.size
    assert use.sum() >= 0.82 * pen.sum()
    gi = np.where(use, 2.0 * (io - np.tile(sc.extra["target_img"], 3)), 0.0).astype(np.float32)
    go = orc.shadow_backward_ex(f, g_o, s_o, gi.astype(np.float64))
    gg = gpu_bwd(R, f, g_r, s_r, gi)
    close(gg, go)
