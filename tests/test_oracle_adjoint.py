"""Pins of the oracle's soft-shadow march (section 2.4) and of its adjoints with respect
to the fine field and to vertex positions.

Pins: trilinear sampling reproduces affine fields (value and gradient); a far constant
field casts no shadow; a sphere's field shades the pixel straight under it along the light;
the shadow adjoint agrees with binary64 central differences of the forward pixel by pixel
along random directions; the vertex adjoint of one triangle agrees with central differences
of the exact ray/plane distance; and the whole chain (SDF term + shadow term) agrees with
central differences of the loss, with the discrete state (seeds, mask, argmin rays and
triangles, signs) held fixed and checked unchanged at both perturbed points.
"""
import numpy as np
import pytest

from paper_2210_06160_amd import synth


def grid_centres(dims, h):
    nx, ny, nz = dims
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([(i.ravel() + 0.5) * h, (j.ravel() + 0.5) * h, (k.ravel() + 0.5) * h], 1)


def shadow(orc, h, width, height):
    return orc.make_shadow(**synth.shadow_setup(h, width=width, height=height))


def test_trilinear_affine(orc):
    dims = (11, 7, 9)
    org = np.array([0.2, -0.3, 0.05], np.float32).astype(np.float64)   # the grid stores binary32
    h = float(np.float32(0.1))
    g = orc.make_grid(dims, org, h)
    c = grid_centres(dims, h) + org
    a = np.array([0.7, -1.3, 2.1])
    f = c @ a + 0.4
    rng = np.random.default_rng(0)
    lo = org + h / 2
    hi = lo + h * (np.array(dims) - 1)
    X = rng.uniform(lo + 1e-6, hi - 1e-6, size=(500, 3))
    v, gr = orc.sample(f, g, X)
    np.testing.assert_allclose(v, X @ a + 0.4, rtol=0, atol=1e-12)
    np.testing.assert_allclose(gr, np.broadcast_to(a, gr.shape), rtol=1e-9, atol=1e-9)


def test_shadow_far_field_and_sphere(orc):
    dims, h = (48, 48, 48), 1.0 / 48
    g = orc.make_grid(dims, (0, 0, 0), h)
    s = shadow(orc, h, 64, 64)
    img = orc.shadow_forward(np.full(48 ** 3, 10.0), g, s)
    assert (img == 1.0).all()          # k s / t >= 8 * 10 / t > 1 for every t on the march
    C, R = np.array([0.5, 0.5, 0.5]), 0.15
    f = np.linalg.norm(grid_centres(dims, h) - C, axis=1) - R
    img = orc.shadow_forward(f, g, s).reshape(64, 64)
    l = np.array(s.light[:])
    foot = C - (C[1] - s.y) / l[1] * l    # where the ray through the centre meets the receiver
    a, b = int(foot[0] * 64), int(foot[2] * 64)
    assert img[b, a] == 0.0
    assert img[0, 63] == 1.0 and img[63, 0] == 1.0
    assert 0.0 < img.mean() < 1.0


def test_shadow_adjoint_matches_central_differences(orc):
    dims, h = (40, 40, 40), 1.0 / 40
    g = orc.make_grid(dims, (0, 0, 0), h)
    s = shadow(orc, h, 48, 48)
    rng = np.random.default_rng(1)
    C = np.array([0.5, 0.45, 0.52])
    f = np.linalg.norm(grid_centres(dims, h) - C, axis=1) - 0.17
    delta = rng.normal(size=f.size)
    img = orc.shadow_forward(f, g, s)

    def fd(eps):
        return (orc.shadow_forward(f + eps * delta, g, s) - orc.shadow_forward(f - eps * delta, g, s)) / (2 * eps)

    d1, d2 = fd(1e-6), fd(5e-7)
    pix = rng.choice(np.flatnonzero((img > 0) & (img < 1)), 120, replace=False)
    checked = 0
    for p in pix:
        if abs(d1[p] - d2[p]) > 1e-6 * (1 + abs(d1[p])):
            continue                   # a discrete choice of the march flips within eps
        e = np.zeros(img.size)
        e[p] = 1.0
        adj = orc.shadow_backward(f, g, s, e) @ delta
        assert abs(adj - d1[p]) <= 1e-6 * (1 + abs(d1[p])), (p, adj, d1[p])
        checked += 1
    assert checked >= 90


def test_vertex_adjoint_single_triangle(orc):
    dims, h = (16, 16, 16), 1.0 / 16
    g = orc.make_grid(dims, (0, 0, 0), h)
    V = np.array([[0.1, 0.42, 0.15], [0.9, 0.47, 0.2], [0.45, 0.4, 0.88]], np.float32)
    T = np.array([[0, 1, 2]], np.int32)
    seeds = orc.jfa(orc.voxelize(V, T, g), g, orc.jfa_steps(dims))
    band = orc.band(seeds, g, 2)
    bvh = orc.BVH(V, T, orc.hit_pad(g))
    x = 8
    dmin, hits, argmin = orc.raysample(bvh, g, band, x, 7, 0)
    cen = grid_centres(dims, h)
    done = 0
    for q in np.flatnonzero(hits > 0)[:40]:
        p = band[q]
        gf = np.zeros(len(seeds))
        gf[p] = 1.0
        gv = orc.sdf_backward(gf, hits[q:q + 1], argmin[q:q + 1], band[q:q + 1], bvh, V, T, g, x, 7)
        code = int(argmin[q]) & 0xFFFFFFFF
        w, _ = orc.direction(7, int(p), code // x, code % x)
        o = orc.voxel_centre(g, p).astype(np.float64)
        w = w.astype(np.float64)
        sign = -1.0 if (hits[q] >> 16) > (hits[q] & 0xFFFF) else 1.0

        def t_of(Vd):
            n = np.cross(Vd[1] - Vd[0], Vd[2] - Vd[0])
            return np.dot(n, Vd[0] - o) / np.dot(n, w)

        Vd = V.astype(np.float64)
        for vtx in range(3):
            for ax in range(3):
                Vp, Vm = Vd.copy(), Vd.copy()
                Vp[vtx, ax] += 1e-6
                Vm[vtx, ax] -= 1e-6
                fdv = sign * (t_of(Vp) - t_of(Vm)) / 2e-6
                assert abs(gv[vtx, ax] - fdv) <= 1e-7 * (1 + abs(fdv))
        done += 1
    assert done >= 20


@pytest.mark.slow
def test_full_chain_central_differences(orc):
    """Loss = sum (fine - target)^2 + sum (img - target_img)^2 on a 48^3 icosphere."""
    dims, h = (48, 48, 48), 1.0 / 48
    g = orc.make_grid(dims, (0, 0, 0), h)
    V32, T = synth.icosphere(3, 0.3, (0.5, 0.5, 0.5))
    steps, bandw, x, key = orc.jfa_steps(dims), 2, 8, 11
    cen = grid_centres(dims, h)
    target = synth.ellipsoid_sdf(cen, (0.35, 0.3, 0.25), (0.5, 0.5, 0.5))
    s = shadow(orc, h, 48, 48)
    timg = np.random.default_rng(3).uniform(size=48 * 48)

    def discrete(Vf):
        seeds = orc.jfa(orc.voxelize(Vf, T, g), g, steps)
        band = orc.band(seeds, g, bandw)
        bvh = orc.BVH(Vf, T, orc.hit_pad(g))
        dmin, hits, argmin = orc.raysample(bvh, g, band, x, key, 0)
        fine, _ = orc.combine(seeds, np.full(len(seeds), np.inf, np.float32), np.zeros(len(seeds), np.uint32),
                              g, bandw, h / 2, 0.0, 0)   # the coarse field everywhere
        tri = np.full(len(band), -1)
        for q in np.flatnonzero(hits > 0):
            code = int(argmin[q]) & 0xFFFFFFFF
            w, _ = orc.direction(key, int(band[q]), code // x, code % x)
            ok, _, tri[q], _ = bvh.closest(orc.voxel_centre(g, band[q]), w)
        return dict(seeds=seeds, band=band, hits=hits, codes=argmin & 0xFFFFFFFF, tri=tri, coarse=fine, bvh=bvh,
                    argmin=argmin)

    base = discrete(V32)
    use = np.flatnonzero(base["hits"] > 0)
    # origins and directions of the argmin rays (fixed), binary64
    O = np.array([orc.voxel_centre(g, base["band"][q]) for q in use], np.float64)
    W = np.array([orc.direction(key, int(base["band"][q]), int(base["codes"][q]) // x,
                                int(base["codes"][q]) % x)[0] for q in use], np.float64)
    sign = np.where((base["hits"][use] >> 16) > (base["hits"][use] & 0xFFFF), -1.0, 1.0)
    tv = T[base["tri"][use]]

    def loss64(Vd):
        a, b, c = Vd[tv[:, 0]], Vd[tv[:, 1]], Vd[tv[:, 2]]
        n = np.cross(b - a, c - a)
        t = np.einsum("ij,ij->i", n, a - O) / np.einsum("ij,ij->i", n, W)
        fine = base["coarse"].astype(np.float64).copy()
        fine[base["band"][use]] = sign * t
        img = orc.shadow_forward(fine, g, s)
        return ((fine - target) ** 2).sum() + ((img - timg) ** 2).sum(), fine, img

    L0, fine0, img0 = loss64(V32.astype(np.float64))
    gfine = 2.0 * (fine0 - target) + orc.shadow_backward(fine0, g, s, 2.0 * (img0 - timg))
    gv = orc.sdf_backward(gfine, base["hits"], base["argmin"], base["band"], base["bvh"], V32, T, g, x, key)
    rng = np.random.default_rng(4)
    cand = np.argsort(-np.abs(gv).ravel())[:40]
    coords = list(cand[:8]) + list(rng.choice(cand[8:], 4, replace=False))
    checked = excluded = 0
    hstep = 2e-5
    for c in coords:
        vi, ax = divmod(int(c), 3)
        ok = True
        fds = []
        for hh in (hstep, hstep / 2):
            vals = []
            for sgn in (1, -1):
                Vd = V32.astype(np.float64)
                Vd[vi, ax] += sgn * hh
                d = discrete(Vd.astype(np.float32))
                if not (np.array_equal(d["seeds"], base["seeds"]) and np.array_equal(d["band"], base["band"])
                        and np.array_equal(d["hits"], base["hits"]) and np.array_equal(d["codes"], base["codes"])
                        and np.array_equal(d["tri"], base["tri"])):
                    ok = False
                    break
                vals.append(loss64(Vd)[0])
            if not ok:
                break
            fds.append((vals[0] - vals[1]) / (2 * hh))
        if not ok or abs(fds[0] - fds[1]) > 1e-4 * (1 + abs(fds[0])):
            excluded += 1
            continue
        rich = (4.0 * fds[1] - fds[0]) / 3.0      # Richardson: cancels the O(h^2) term
        assert abs(gv[vi, ax] - rich) <= 2e-6 * (1 + abs(rich)), (vi, ax, gv[vi, ax], fds)
        checked += 1
    print("checked", checked, "excluded", excluded)
    assert checked >= 6


@pytest.mark.slow
def test_gradient_workload_central_differences(orc):
    """The gradient workload itself (128^3, icosphere of 20,480 triangles, 2-voxel mask, 16
    rays, 512^2 shadow of 64 steps, loss against the ellipsoid field and a seeded image):
    the oracle's binary64 adjoint (SDF term + shadow term, through each masked point's argmin
    ray) against binary64 central differences of the loss with step 1e-4 on a dozen vertex
    coordinates drawn at random among those the loss depends on, refined by Richardson with
    step 5e-5.  A coordinate counts only where the
    discrete state is unchanged at every perturbed point (seeds, mask, hit counts, argmin
    ray codes, the argmin rays' triangles) and the two steps agree; excluded coordinates are
    counted, and so do the shadow march's (each pixel's minimising step, clamped samples and
    trilinear cells).  Perturbed states are recomputed in full by the oracle; of the argmin rays, those
    whose triangle touches the moved vertex are re-traced one by one, every other record must
    come back bit-identical."""
    import time
    t_start = time.time()
    sc = synth.scene_grad()
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    V32, T = sc.verts, sc.tris
    steps, bandw, x, key = sc.steps, sc.band, sc.rays, 0
    target = sc.extra["target"].astype(np.float64)
    timg = sc.extra["target_img"].astype(np.float64)
    s = orc.make_shadow(**sc.extra["shadow"])

    def state(Vf):
        seeds = orc.jfa(orc.voxelize(Vf, T, g), g, steps)
        band = orc.band(seeds, g, bandw)
        bvh = orc.BVH(Vf, T, orc.hit_pad(g))
        dmin, hits, argmin = orc.raysample(bvh, g, band, x, key, 0)
        return seeds, band, bvh, hits, argmin

    def argmin_tri(bvh, band, argmin, q):
        code = int(argmin[q]) & 0xFFFFFFFF
        w, _ = orc.direction(key, int(band[q]), code // x, code % x)
        ok, _, tri, _ = bvh.closest(orc.voxel_centre(g, band[q]), w)
        return tri if ok else -1

    seeds0, band0, bvh0, hits0, argmin0 = state(V32)
    coarse, _ = orc.combine(seeds0, np.full(len(seeds0), np.inf, np.float32), np.zeros(len(seeds0), np.uint32), g,
                            bandw, sc.h / 2, 0.0, 0)
    use = np.flatnonzero(hits0 > 0)
    tri0 = np.array([argmin_tri(bvh0, band0, argmin0, q) for q in use])
    assert (tri0 >= 0).all()
    codes0 = argmin0 & 0xFFFFFFFF
    O = np.array([orc.voxel_centre(g, band0[q]) for q in use], np.float64)
    W = np.array([orc.direction(key, int(band0[q]), int(codes0[q]) // x, int(codes0[q]) % x)[0] for q in use],
                 np.float64)
    sign = np.where((hits0[use] >> 16) > (hits0[use] & 0xFFFF), -1.0, 1.0)
    tv = T[tri0]

    def loss64(Vd):
        a, b, c = Vd[tv[:, 0]], Vd[tv[:, 1]], Vd[tv[:, 2]]
        n = np.cross(b - a, c - a)
        t = np.einsum("ij,ij->i", n, a - O) / np.einsum("ij,ij->i", n, W)
        fine = coarse.astype(np.float64).copy()
        fine[band0[use]] = sign * t
        img = orc.shadow_forward(fine, g, s)
        return ((fine - target) ** 2).sum() + ((img - timg) ** 2).sum(), fine, img

    L0, fine0, img0 = loss64(V32.astype(np.float64))
    path0 = orc.shadow_path(fine0, g, s)
    gfine = 2.0 * (fine0 - target) + orc.shadow_backward(fine0, g, s, 2.0 * (img0 - timg))
    gv = orc.sdf_backward(gfine, hits0, argmin0, band0, bvh0, V32, T, g, x, key)

    def unchanged(Vd32, vi):
        seeds, band, bvh, hits, argmin = state(Vd32)
        if not (np.array_equal(seeds, seeds0) and np.array_equal(band, band0) and np.array_equal(hits, hits0)
                and np.array_equal(argmin & 0xFFFFFFFF, codes0)):
            return False
        touched = np.isin(tri0, np.flatnonzero((T == vi).any(axis=1)))
        rest = use[~touched]
        if not np.array_equal(argmin[rest], argmin0[rest]):
            return False
        return all(argmin_tri(bvh, band, argmin, q) == t for q, t in zip(use[touched], tri0[touched]))

    rng = np.random.default_rng(4)
    coords = rng.permutation(np.flatnonzero(np.abs(gv).ravel() > 0))
    checked = excluded = 0
    for c in coords:
        if checked == 12 or checked + excluded == 80:
            break
        vi, ax = divmod(int(c), 3)
        fds, ok = [], True
        for hh in (1e-4, 5e-5):
            vals = []
            for sgn in (1, -1):
                Vd = V32.astype(np.float64)
                Vd[vi, ax] += sgn * hh
                if not unchanged(Vd.astype(np.float32), vi):
                    ok = False
                    break
                L, fine, _ = loss64(Vd)
                if not np.array_equal(orc.shadow_path(fine, g, s), path0):  # a march decision flipped
                    ok = False
                    break
                vals.append(L)
            if not ok:
                break
            fds.append((vals[0] - vals[1]) / (2 * hh))
        if not ok or abs(fds[0] - fds[1]) > 1e-4 * (1 + abs(fds[0])):
            excluded += 1
            continue
        rich = (4.0 * fds[1] - fds[0]) / 3.0  # Richardson: cancels the O(h^2) term
        assert abs(gv[vi, ax] - rich) <= 2e-6 * (1 + abs(rich)), (vi, ax, gv[vi, ax], fds)
        checked += 1
    print("masked points with hits", len(use), "checked", checked, "excluded", excluded,
          "seconds %.1f" % (time.time() - t_start))
    assert checked >= 6
