"""Pins of the oracle's ray/triangle hit, closest hit, ray sampling and combination.

Section 2.1: minimum hit distance per grid point; front/back from the dot product of the
ray direction with the triangle normal; negative if back hits are the majority.
Section 2.3: only grid points in the mask are traced.  Section 2.5.1 (Eq. 1): decay.
Pins: plane closed form, binary64 intersection away from edges, hierarchy == brute force,
any hit lies on the surface (dmin >= exact distance), convex-mesh sign counts exact,
convergence towards the exact distance as rays grow, Eq. 1 closed forms.
"""
import numpy as np
import pytest

from geom import point_mesh_distance, voxel_centres
from paper_2210_06160_amd import synth


def test_plane_closed_form(orc):
    v0, v1, v2 = np.array([-5, -5, 0.75]), np.array([5, -5, 0.75]), np.array([0, 6, 0.75])  # normal +z
    rng = np.random.default_rng(1)
    for _ in range(200):
        x, y = rng.uniform(-1, 1, 2)
        oz = rng.uniform(-2, 0.7)
        hit, t, front = orc.ray_tri([x, y, oz], [0, 0, 1], v0, v1, v2, 1e-4)
        assert hit and not front
        assert abs(t - (0.75 - np.float32(oz))) <= 2e-7 * 3
        hit, t, front = orc.ray_tri([x, y, 2.0 - oz], [0, 0, -1], v0, v1, v2, 1e-4)
        assert hit and front
        hit, _, _ = orc.ray_tri([x, y, oz], [0, 0, -1], v0, v1, v2, 1e-4)
        assert not hit          # behind the origin
    # a ray in the plane of the triangle never hits (det == 0)
    assert not orc.ray_tri([0, 0, 0.75], [1, 0, 0], v0, v1, v2, 1e-4)[0]


def test_random_rays_vs_binary64(orc):
    rng = np.random.default_rng(2)
    agree = 0
    for _ in range(3000):
        v = rng.uniform(-1, 1, (3, 3)).astype(np.float32)
        o = rng.uniform(-2, 2, 3).astype(np.float32)
        w = rng.normal(size=3)
        w = (w / np.linalg.norm(w)).astype(np.float32)
        a, b, c = (x.astype(np.float64) for x in v)
        e1, e2 = b - a, c - a
        n = np.cross(e1, e2)
        den = np.dot(w.astype(np.float64), n)
        if abs(den) < 1e-3:
            continue
        t = np.dot(a - o, n) / den
        p = o + t * w
        # barycentrics of p
        m = np.array([e1, e2]).T
        uv = np.linalg.lstsq(m, p - a, rcond=None)[0]
        bary = np.array([1 - uv.sum(), uv[0], uv[1]])
        if abs(min(bary.min(), t)) < 1e-4:
            continue
        hit, tt, front = orc.ray_tri(o, w, v[0], v[1], v[2], 1e-3)
        assert hit == (bary.min() > 0 and t > 0)
        if hit:
            assert abs(tt - t) <= 1e-5 * max(1.0, abs(t))
            assert front == (den < 0)
        agree += 1
    assert agree > 2000


@pytest.mark.parametrize("which", ["tiny", "static"])
def test_hierarchy_equals_brute_force(orc, which):
    if which == "tiny":
        sc = synth.scene_tiny()
    else:
        sc = synth.scene_static(dims=(80, 40, 80), nprims=25, seed=5)
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    pad = orc.hit_pad(g)
    bvh = orc.BVH(sc.verts, sc.tris, pad)
    rng = np.random.default_rng(3)
    N = sc.dims[0] * sc.dims[1] * sc.dims[2]
    vids = rng.choice(N, size=1500, replace=False)
    nhit = 0
    for q, vid in enumerate(vids):
        o = orc.voxel_centre(g, vid)
        w, _ = orc.direction(9, int(vid), 0, q % 7)
        a = orc.closest_brute(sc.verts, sc.tris, o, w, pad)
        b = bvh.closest(o, w)
        assert a[0] == b[0]
        if a[0]:
            nhit += 1
            assert (np.float32(a[1]).view(np.uint32), a[2], a[3]) == (np.float32(b[1]).view(np.uint32), b[2], b[3])
    assert nhit > 300


def tiny_band(orc):
    sc = synth.scene_tiny()
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    seeds = orc.jfa(orc.voxelize(sc.verts, sc.tris, g), g, sc.steps)
    return sc, g, seeds, orc.band(seeds, g, sc.band)


def convex_inside(verts, tris, pts):
    v = np.asarray(verts, np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    n = np.cross(b - a, c - a)
    s = np.einsum("ptk,tk->pt", pts[:, None, :] - a[None], n)
    return (s < 0).all(1), np.abs(s / np.linalg.norm(n, axis=1)).min(1)


def test_raysample_invariants(orc):
    sc, g, seeds, band = tiny_band(orc)
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    x = sc.rays
    dmin, hits, argmin = orc.raysample(bvh, g, band, x, 0, 0)
    front, back = hits & 0xFFFF, hits >> 16
    assert ((front + back) <= x).all()
    cen = voxel_centres(sc.dims, sc.org, sc.h, band)
    exact = point_mesh_distance(cen, sc.verts, sc.tris)
    hit = (front + back) > 0
    # R1: every hit point is on the surface, so dmin never undercuts the exact distance
    assert (dmin[hit] >= exact[hit] * (1 - 1e-6) - 1e-7).all()
    # convex closed mesh: inside -> only back faces, outside -> only front faces
    inside, margin = convex_inside(sc.verts, sc.tris, cen)
    clear = margin > 1e-5
    assert (front[inside & clear] == 0).all()
    assert (back[~inside & clear] == 0).all()
    assert (hits[inside & clear] >> 16 == x).all()   # every ray from inside hits
    # the argmin record names the ray that produced dmin
    for q in np.flatnonzero(hit)[:200]:
        tb = int(argmin[q]) >> 32
        assert tb == int(np.float32(dmin[q]).view(np.uint32))
        code = int(argmin[q]) & 0xFFFFFFFF
        w, _ = orc.direction(0, int(band[q]), code // x, code % x)
        ok, t, _, _ = orc.closest_brute(sc.verts, sc.tris, cen[q].astype(np.float32), w, orc.hit_pad(g))
        assert ok and np.float32(t) == dmin[q]


def test_raysample_converges(orc):
    sc, g, seeds, band = tiny_band(orc)
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    cen = voxel_centres(sc.dims, sc.org, sc.h, band)
    exact = point_mesh_distance(cen, sc.verts, sc.tris)
    acc = orc.new_accum(len(band))
    gaps = []
    frames = 0
    for total in (4, 16, 64):
        while frames * 4 < total:
            orc.raysample(bvh, g, band, 4, 21, frames, acc=acc)
            frames += 1
        d = acc[0]
        ok = np.isfinite(d)
        gaps.append(float(np.mean(d[ok] - exact[ok])))
    assert gaps[0] > gaps[1] > gaps[2] >= 0
    assert gaps[2] < 0.25 * sc.h


def test_combine_sign_and_band(orc):
    sc, g, seeds, band = tiny_band(orc)
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    dmin, hits, _ = orc.raysample(bvh, g, band, 32, 4, 0)
    N = len(seeds)
    D = np.full(N, np.inf, np.float32)
    H = np.zeros(N, np.uint32)
    D[band], H[band] = dmin, hits
    beta = sc.h / 2
    fine, _ = orc.combine(seeds, D, H, g, sc.band, beta, 0.0, 0)
    cen = voxel_centres(sc.dims, sc.org, sc.h)
    inside, margin = convex_inside(sc.verts, sc.tris, cen)
    inb = np.zeros(N, bool)
    inb[band] = True
    clear = margin > 1e-5
    # in the mask the sign is the majority vote: exact for a convex closed mesh
    assert (fine[inb & inside & clear] < 0).all()
    assert (fine[inb & ~inside & clear] > 0).all()
    # outside the mask the coarse field is used, whose interior is hollow (section 2.2)
    far_in = ~inb & inside
    assert far_in.any() and (fine[far_in] > 0).all()
    # the coarse magnitude is a distance to a seed voxel centre, and every seed centre is
    # within half a voxel diagonal of the mesh, so it cannot undercut the exact distance
    # by more than that
    exact = point_mesh_distance(cen[~inb], sc.verts, sc.tris)
    u = fine[~inb] + beta
    assert (u >= exact - np.sqrt(3) / 2 * sc.h - 1e-6).all()


def test_decay_closed_forms(orc):
    # Eq. 1 on magnitudes.  One seed at voxel 0 of a 6x1x1 grid, band 2 voxels.
    g = orc.make_grid((6, 1, 1), (0, 0, 0), 0.5)
    seeds = np.zeros(6, np.int32)                   # every voxel's seed is (0,0,0)
    u = 0.5 * np.arange(6, dtype=np.float32)        # coarse magnitude h*|p-s|
    inb = np.arange(6) <= 2
    state = np.zeros(6, np.float32)
    # constant r <= u: m_t = r from the first frame on
    r = np.float32(0.3)
    for t in range(5):
        dmin = np.full(6, r, np.float32)
        hits = np.full(6, 1 << 16, np.uint32)      # one back hit -> negative
        fine, state = orc.combine(seeds, dmin, hits, g, 2, 0.1, 0.0, 1, 0.95, reset=(t == 0), state=state)
        sel = inb & (u >= r)
        assert np.all(fine[sel] == -r)
        assert np.all(fine[~inb] == u[~inb] - np.float32(0.1))
    # no hits: m_t = alpha m_{t-1} + (1 - alpha) u_t -> stays u when started at u, sign kept
    state = np.zeros(6, np.float32)
    fine, state = orc.combine(seeds, np.full(6, np.inf, np.float32), np.zeros(6, np.uint32), g, 2, 0.1,
                              0.0, 1, 0.95, reset=True, state=state)
    assert np.all(np.abs(fine[inb] - u[inb]) <= 1e-6)
    # decay from a ray-traced value towards u: m_t - u = alpha^t (r - u)
    state = np.zeros(6, np.float32)
    one_front = np.ones(6, np.uint32)
    fine, state = orc.combine(seeds, np.full(6, 0.05, np.float32), one_front, g, 2, 0.1, 0.0, 1, 0.95,
                              reset=True, state=state)
    for t in range(1, 30):
        fine, state = orc.combine(seeds, np.full(6, np.inf, np.float32), np.zeros(6, np.uint32), g, 2, 0.1,
                                  0.0, 1, 0.95, reset=False, state=state)
        expect = u[2] + 0.95 ** t * (0.05 - u[2])
        assert abs(fine[2] - expect) < 1e-5
    # a tie keeps the previous sign
    st = np.full(6, -0.2, np.float32)
    tie = np.full(6, 1 | (1 << 16), np.uint32)
    fine, _ = orc.combine(seeds, np.full(6, 0.1, np.float32), tie, g, 2, 0.0, 0.0, 1, 0.95, reset=False, state=st)
    assert (fine[inb] < 0).all()
    # bias thickens: subtracted everywhere
    f0, _ = orc.combine(seeds, np.full(6, 0.1, np.float32), one_front, g, 2, 0.0, 0.0, 0)
    f1, _ = orc.combine(seeds, np.full(6, 0.1, np.float32), one_front, g, 2, 0.0, 0.01, 0)
    assert np.allclose(f0 - f1, 0.01, atol=1e-7)


def test_accum_in_band_closed_form(orc):
    """Running-minimum combine (section 2.1) value by value on a hand-built 7x1x1 grid whose
    points all hold the seed of point 0, so d2 = i^2 and u = h i exactly (dyadic values, so
    every expected value below is exact in binary32).  Mask width 3: points 0..3 are in it.
      in mask, one back hit         -> -dmin - bias   (back-face majority is negative)
      in mask, one front + one back -> +dmin - bias   (a tie is not a majority)
      in mask, no hits              -> u - beta - bias (the coarse value)
      in mask, two front + one back -> +dmin - bias
      outside the mask, back hits   -> u - beta - bias (hits outside the mask are ignored)
      outside the mask, no hits     -> u - beta - bias
      no seed                       -> +inf"""
    h, beta, bias = 0.25, 0.125, 0.0625
    g = orc.make_grid((7, 1, 1), (0, 0, 0), h)
    seeds = np.zeros(7, np.int32)
    seeds[6] = -1
    dmin = np.array([0.375, 0.5, 0.75, 0.625, 0.25, np.inf, 0.125], np.float32)
    back, front = 1 << 16, 1
    hits = np.array([back, front + back, 0, 2 * front + back, 3 * back, 0, back], np.uint32)
    fine, _ = orc.combine(seeds, dmin, hits, g, 3, beta, bias, 0)
    u = h * np.arange(7, dtype=np.float64)
    expect = np.array([-0.375 - bias, 0.5 - bias, u[2] - beta - bias, 0.625 - bias, u[4] - beta - bias,
                       u[5] - beta - bias, np.inf], np.float64)
    assert np.array_equal(fine.astype(np.float64), expect), (fine, expect)
    # mask width 0 keeps only the seed point itself
    fine0, _ = orc.combine(seeds, dmin, hits, g, 0, beta, bias, 0)
    assert fine0[0] == np.float32(-0.375 - bias) and fine0[1] == np.float32(u[1] - beta - bias)


def test_box_rule_keeps_closest_hits(orc):
    """The hit test's extra acceptance rule (the computed hit point must lie within h/256 of
    the triangle's box) changes no closest hit on 10,000 rays of a reduced static scene:
    the closest hit with the rule (the oracle's hierarchy, as ray sampling uses it) equals
    plain Moller-Trumbore by brute force over every triangle (an infinite widening)."""
    sc = synth.scene_static(dims=(100, 50, 100), nprims=40, seed=1)
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    band = orc.band(orc.jfa(orc.voxelize(sc.verts, sc.tris, g), g, sc.steps), g, sc.band)
    rng = np.random.default_rng(11)
    vids = rng.choice(band, 2500, replace=False)
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    n = hits = 0
    for vid in vids:
        o = orc.voxel_centre(g, int(vid))
        for j in range(4):
            w, _ = orc.direction(5, int(vid), 0, j)
            a = bvh.closest(o, w)
            b = orc.closest_brute(sc.verts, sc.tris, o, w, np.inf)
            assert a[0] == b[0] and a[2] == b[2] and a[3] == b[3], (vid, j, a, b)
            if a[0]:
                assert np.float32(a[1]).view(np.uint32) == np.float32(b[1]).view(np.uint32)
                hits += 1
            n += 1
    assert n == 10000 and hits > 0.5 * n  # upward rays leave the open scene
