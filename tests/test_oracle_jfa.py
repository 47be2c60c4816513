"""Pins of the oracle's jump flooding (section 2.2).

Reading: each grid point keeps its stored seed and queries p + k*e, e in {-1,0,1}^3 \\ {0},
in the order ez, ey, ex ascending; an in-grid query replaces the stored seed only if its
seed is strictly closer.  Pins: single-seed exactness (closed form, any grid shape),
outputs are input seeds, seeds keep themselves, never closer than the exact EDT (scipy),
hand-worked tie cases, and an independent numpy implementation of the same definition.
"""
import numpy as np
import pytest
from scipy import ndimage

from geom import unpack
from paper_2210_06160_amd import synth

EMPTY = -1
ORDER = [(ex, ey, ez) for ez in (-1, 0, 1) for ey in (-1, 0, 1) for ex in (-1, 0, 1)
         if (ex, ey, ez) != (0, 0, 0)]


def np_jfa_pass(a, dims, k):
    """Independent vectorised implementation of one pass ([nz, ny, nx] array)."""
    nx, ny, nz = dims
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def d2(ids):
        c = unpack(ids.ravel()).reshape(ids.shape + (3,))
        return (c[..., 0] - x) ** 2 + (c[..., 1] - y) ** 2 + (c[..., 2] - z) ** 2

    best = a.copy()
    bestd = np.where(best == EMPTY, 0, d2(best))
    for ex, ey, ez in ORDER:
        sh = np.full_like(a, EMPTY)
        src = [slice(None)] * 3
        dst = [slice(None)] * 3
        for ax, off, n in ((2, ex * k, nx), (1, ey * k, ny), (0, ez * k, nz)):
            if abs(off) >= n:
                src = None
                break
            if off >= 0:
                dst[ax], src[ax] = slice(0, n - off), slice(off, n)
            else:
                dst[ax], src[ax] = slice(-off, n), slice(0, n + off)
        if src is None:
            continue
        sh[tuple(dst)] = a[tuple(src)]
        dd = d2(sh)
        take = (sh != EMPTY) & ((best == EMPTY) | (dd < bestd))
        best = np.where(take, sh, best)
        bestd = np.where(take, dd, bestd)
    return best


def np_jfa(seeds, dims, steps):
    a = seeds.reshape(dims[2], dims[1], dims[0]).copy()
    for k in steps:
        a = np_jfa_pass(a, dims, k)
    return a.ravel()


def random_seeds(rng, dims, n):
    nx, ny, nz = dims
    s = np.full(nx * ny * nz, EMPTY, np.int32)
    vid = rng.choice(nx * ny * nz, size=n, replace=False)
    i, j, k = vid % nx, (vid // nx) % ny, vid // (nx * ny)
    s[vid] = i | (j << 10) | (k << 20)
    return s


@pytest.mark.parametrize("dims", [(32, 32, 32), (37, 20, 51), (3, 50, 7), (1, 1, 9), (64, 2, 5)])
def test_single_seed_exact(orc, dims):
    rng = np.random.default_rng(sum(dims))
    g = orc.make_grid(dims, (0, 0, 0), 0.5)
    steps = orc.jfa_steps(dims)
    for _ in range(4):
        seeds = random_seeds(rng, dims, 1)
        sid = seeds[seeds != EMPTY][0]
        out = orc.jfa(seeds, g, steps)
        assert (out == sid).all()


def test_tie_rules(orc):
    # one pass, k = 2, on a hand-made 8x1x8 buffer around p = (4, 0, 4)
    dims = (8, 1, 8)
    g = orc.make_grid(dims, (0, 0, 0), 1.0)

    def vid(x, z):
        return x + 8 * z

    def sid(x, z):
        return x | (z << 20)

    buf = np.full(64, EMPTY, np.int32)
    buf[vid(4, 2)] = sid(6, 6)      # queried first (ez = -1): d2 = 8
    buf[vid(4, 6)] = sid(2, 2)      # queried later (ez = +1): d2 = 8, smaller id
    out = orc.jfa_pass(buf, g, 2)
    assert out[vid(4, 4)] == sid(6, 6)          # an equally close later query does not replace
    buf2 = buf.copy()
    buf2[vid(4, 4)] = sid(6, 6)
    buf2[vid(4, 2)] = sid(2, 2)
    out2 = orc.jfa_pass(buf2, g, 2)
    assert out2[vid(4, 4)] == sid(6, 6)         # the stored seed wins ties
    buf3 = buf.copy()
    buf3[vid(2, 4)] = sid(4, 5)                 # (ez=0, ex=-1): d2 = 1, strictly closer
    out3 = orc.jfa_pass(buf3, g, 2)
    assert out3[vid(4, 4)] == sid(4, 5)


@pytest.mark.parametrize("case", ["tiny", "rand24", "rand_odd", "sparse40"])
def test_matches_numpy_and_invariants(orc, case):
    rng = np.random.default_rng(7)
    if case == "tiny":
        sc = synth.scene_tiny()
        dims, steps = sc.dims, sc.steps
        g = orc.make_grid(dims, sc.org, sc.h)
        seeds = orc.voxelize(sc.verts, sc.tris, g)
    elif case == "rand24":
        dims, steps = (24, 24, 24), [8, 4, 2, 1, 1]
        seeds = random_seeds(rng, dims, 40)
    elif case == "rand_odd":
        dims, steps = (29, 13, 21), orc.jfa_steps((29, 13, 21), 1)
        seeds = random_seeds(rng, dims, 25)
    else:
        dims, steps = (40, 12, 40), orc.jfa_steps((40, 12, 40))
        seeds = random_seeds(rng, dims, 6)
    g = orc.make_grid(dims, (0, 0, 0), 1.0)
    out = orc.jfa(seeds, g, steps)
    assert np.array_equal(out, np_jfa(seeds, dims, steps))
    # every output is an input seed; seeds keep themselves
    sset = set(seeds[seeds != EMPTY].tolist())
    assert set(out[out != EMPTY].tolist()) <= sset
    isseed = seeds != EMPTY
    assert np.array_equal(out[isseed], seeds[isseed])
    assert (out != EMPTY).all()
    # never closer than the exact Euclidean distance transform
    mask = (seeds == EMPTY).reshape(dims[2], dims[1], dims[0])
    edt2 = np.rint(ndimage.distance_transform_edt(mask) ** 2).astype(np.int64).ravel()
    d2 = orc.seed_d2(out, g).astype(np.int64)
    assert (d2 >= edt2).all()
    # the approximation is close: report, and bound loosely
    assert (d2 == edt2).mean() > 0.9


def test_empty_stays_empty(orc):
    dims = (9, 10, 11)
    g = orc.make_grid(dims, (0, 0, 0), 1.0)
    out = orc.jfa(np.full(990, EMPTY, np.int32), g, [8, 4, 2, 1])
    assert (out == EMPTY).all()
