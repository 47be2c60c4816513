"""Pins of the oracle's clip map (the multi-resolution field around a camera that the
paper proposes for large scenes): level placement, level choice, sampling from the
concatenated levels, and the full shadow pass over a clip map with its adjoint.

  * placement: every level's box lies inside the next one's, the camera lies inside every
    level's box of grid-point centres, and a level stays put while the camera moves inside
    one of its voxels;
  * sampling: with a different affine field on every level (trilinear sampling reproduces
    affine fields exactly) the sampled value names the level read; the camera reads level
    0, a point just outside level 0's box of centres reads level 1, far points the coarsest;
  * one level equals the single-grid sampler and shadow pass bit for bit;
  * a constant field on every level gives the single-grid march bounded by the coarsest
    level's box;
  * the adjoint over a two-level clip map agrees with binary64 central differences.
"""
import numpy as np
import pytest

from paper_2210_06160_amd import synth


def centres(g):
    k, j, i = np.meshgrid(np.arange(g.nz), np.arange(g.ny), np.arange(g.nx), indexing="ij")
    return np.stack([g.org[0] + g.h * (i.ravel() + 0.5), g.org[1] + g.h * (j.ravel() + 0.5),
                     g.org[2] + g.h * (k.ravel() + 0.5)], 1)


def box(g):
    lo = np.array(g.org[:], np.float64)
    return lo, lo + np.float64(g.h) * np.array([g.nx, g.ny, g.nz])


def test_placement_nests_and_snaps(orc):
    rng = np.random.default_rng(0)
    for _ in range(50):
        cam = rng.uniform(-3, 3, 3).astype(np.float32)
        n = int(rng.choice([4, 8, 32, 64]))
        G = orc.clipmap_levels(cam, 0.01, n, 4)
        for l, g in enumerate(G):
            assert (g.nx, g.ny, g.nz) == (n, n, n)
            lo, hi = box(g)
            assert (lo + g.h / 2 <= cam).all() and (cam <= hi - g.h / 2).all()
            if l:
                plo, phi = box(G[l - 1])
                assert (lo <= plo).all() and (phi <= hi).all()
        # moving within the camera's level-2 voxel keeps level 2 (and coarser) in place
        h2 = float(G[2].h)
        base = (np.floor(cam / h2) + 0.5) * h2
        G2 = orc.clipmap_levels((base + rng.uniform(-0.45, 0.45, 3) * h2).astype(np.float32), 0.01, n, 4)
        for l in (2, 3):
            assert list(G2[l].org) == list(orc.clipmap_levels(base.astype(np.float32), 0.01, n, 4)[l].org)


def affine_levels(orc, G):
    coef = [(np.array([0.3 + l, -0.7, 0.2 * l]), 10.0 * l) for l in range(len(G))]
    return [centres(g) @ a + b for g, (a, b) in zip(G, coef)], coef


def test_sampling_names_the_level(orc):
    cam = np.array([1.0, 0.5, 1.0], np.float32)
    G = orc.clipmap_levels(cam, 1.0 / 64, 32, 3)
    F, coef = affine_levels(orc, G)
    lo0, hi0 = box(G[0])
    lo1, hi1 = box(G[1])
    pts = np.array([cam, [hi0[0] - G[0].h * 0.51, cam[1], cam[2]],      # inside level 0's centre box
                    [hi0[0] - G[0].h * 0.49, cam[1], cam[2]],             # just outside it, inside level 1's
                    [hi1[0] + 0.05, cam[1], cam[2]],                      # beyond level 1
                    [50.0, 50.0, 50.0]], np.float64)                      # beyond everything
    want = [0, 0, 1, 2, 2]
    val, lev = orc.clipmap_sample(G, F, pts)
    assert list(lev) == want
    for p, v, l in zip(pts[:4], val[:4], want[:4]):
        a, b = coef[l]
        assert v == pytest.approx(p @ a + b, rel=1e-12, abs=1e-12)
    # random points: the value is the affine function of the level reported
    rng = np.random.default_rng(1)
    X = rng.uniform(box(G[2])[0] + G[2].h, box(G[2])[1] - G[2].h, size=(400, 3))
    val, lev = orc.clipmap_sample(G, F, X)
    assert set(lev) == {0, 1, 2}
    for x, v, l in zip(X, val, lev):
        a, b = coef[l]
        assert v == pytest.approx(x @ a + b, rel=1e-12, abs=1e-9)


def test_one_level_is_the_single_grid(orc):
    g = orc.make_grid((20, 16, 24), (0.1, 0.0, -0.2), 0.05)
    rng = np.random.default_rng(2)
    f = rng.normal(size=20 * 16 * 24)
    X = rng.uniform(0, 1, size=(300, 3))
    v1, _ = orc.clipmap_sample([g], [f], X)
    v0, _ = orc.sample(f, g, X)
    assert np.array_equal(v0, v1)
    b = orc.make_shadow(**synth.shadow_setup(0.05, width=12, height=9, steps=80))
    s = orc.make_shadow_ex(b, [(0.3, 0.9, 0.3)], triangulate=True, jitter=0.02, key=3, bounded=True)
    assert np.array_equal(orc.shadow_forward_clip([g], [f], s), orc.shadow_forward_ex(f, g, s))


def test_constant_field_bounded_by_the_coarsest_box(orc):
    cam = np.array([0.5, 0.3, 0.5], np.float32)
    G = orc.clipmap_levels(cam, 1.0 / 32, 16, 3)
    c = 0.3
    b = orc.make_shadow(**synth.shadow_setup(1.0 / 32, width=10, height=8, steps=200, k=0.05))
    s = orc.make_shadow_ex(b, [(0.32, 0.92, 0.23)], bounded=True)
    img = orc.shadow_forward_clip(G, [np.full(16 ** 3, c)] * 3, s)
    assert np.array_equal(img, orc.shadow_forward_ex(np.full(16 ** 3, c), G[2], s))
    assert img.min() < 1.0


def test_adjoint_over_two_levels_matches_central_differences(orc):
    cam = np.array([0.5, 0.35, 0.5], np.float32)
    G = orc.clipmap_levels(cam, 1.0 / 48, 16, 2)     # the sphere straddles level 0's box
    C = np.array([0.52, 0.45, 0.5])
    F = [np.linalg.norm(centres(g) - C, axis=1) - 0.12 for g in G]
    b = orc.make_shadow(**synth.shadow_setup(1.0 / 48, width=64, height=64, steps=96))
    s = orc.make_shadow_ex(b, [(0.32, 0.92, 0.23)], triangulate=True, jitter=0.01, key=5, bounded=True)
    f = np.concatenate(F)
    n0 = len(F[0])
    split = lambda v: [v[:n0], v[n0:]]
    img = orc.shadow_forward_clip(G, F, s)
    rng = np.random.default_rng(4)
    d = rng.normal(size=f.size)

    def fd(eps):
        return (orc.shadow_forward_clip(G, split(f + eps * d), s) - orc.shadow_forward_clip(G, split(f - eps * d), s)) / (2 * eps)

    d1, d2 = fd(1e-6), fd(5e-7)
    pix = rng.choice(np.flatnonzero((img > 0) & (img < 1)), 100, replace=False)
    checked = 0
    for p in pix:
        if abs(d1[p] - d2[p]) > 1e-6 * (1 + abs(d1[p])):
            continue
        e = np.zeros(img.size)
        e[p] = 1.0
        adj = orc.shadow_backward_clip(G, F, s, e) @ d
        assert abs(adj - d1[p]) <= 1e-6 * (1 + abs(d1[p])), (p, adj, d1[p])
        checked += 1
    assert checked >= 70
    # both levels receive gradient
    g = orc.shadow_backward_clip(G, F, s, np.where((img > 0) & (img < 1), 1.0, 0.0))
    assert np.abs(g[:n0]).max() > 0 and np.abs(g[n0:]).max() > 0
