"""Pins of the oracle's voxelization (section 2.2) and seed ids, independent of the oracle.

Reading: a voxel is a seed iff its closed cell meets the closed triangle, after snapping
vertices to 1/256 voxel.  Pins: exact shell of a voxel-aligned box (closed form), vertex
voxels are seeds, voxels whose centre is within h/2 - snap of the mesh are seeds, no seed
lies farther than sqrt(3)/2 h + snap from the mesh (exact point-triangle distance).
"""
import numpy as np
import pytest

from geom import point_mesh_distance, voxel_centres, unpack
from paper_2210_06160_amd import synth


def test_pack_roundtrip(orc):
    rng = np.random.default_rng(0)
    coords = np.concatenate([rng.integers(0, 1024, size=(2000, 3)),
                             np.array([[0, 0, 0], [1023, 1023, 1023], [1023, 0, 0], [0, 1023, 0],
                                       [0, 0, 1023]])])
    for i, j, k in coords:
        s = orc.pack_id(int(i), int(j), int(k))
        assert s != orc.EMPTY and s >= 0
        assert tuple(unpack([s])[0]) == (i, j, k)


def test_aligned_box_shell(orc):
    # box [5h,15h] x [5h,12h] x [5h,20h]: faces lie on voxel faces, so the closed-cell
    # rule marks exactly the cells of [4,15]x[4,12]x[4,20] that touch a face plane.
    h = 1.0 / 32
    lo, hi = np.array([5, 5, 5]), np.array([15, 12, 20])
    v, t = synth.box((hi - lo) * h / 2, (hi + lo) * h / 2)
    g = orc.make_grid((32, 32, 32), (0, 0, 0), h)
    seeds = orc.voxelize(v, t, g)
    k, j, i = np.meshgrid(np.arange(32), np.arange(32), np.arange(32), indexing="ij")
    inblock = (i >= 4) & (i <= 15) & (j >= 4) & (j <= 12) & (k >= 4) & (k <= 20)
    touch = (np.isin(i, [4, 5, 14, 15]) | np.isin(j, [4, 5, 11, 12]) | np.isin(k, [4, 5, 19, 20]))
    expect = (inblock & touch).ravel()
    assert np.array_equal(seeds != orc.EMPTY, expect)
    ids = np.flatnonzero(seeds != orc.EMPTY)
    assert np.array_equal(seeds[ids], i.ravel()[ids] | (j.ravel()[ids] << 10) | (k.ravel()[ids] << 20))


def test_empty_mesh(orc):
    g = orc.make_grid((8, 9, 10), (0, 0, 0), 0.1)
    seeds = orc.voxelize(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), g)
    assert (seeds == orc.EMPTY).all()


@pytest.mark.parametrize("which", ["ico", "static"])
def test_distance_bounds(orc, which):
    if which == "ico":
        sc = synth.scene_tiny()
        verts, tris, dims, h = sc.verts, sc.tris, sc.dims, sc.h
    else:
        sc = synth.scene_static(dims=(40, 20, 40), nprims=12, seed=3)
        verts, tris, dims, h = sc.verts, sc.tris, sc.dims, sc.h
    g = orc.make_grid(dims, (0, 0, 0), h)
    seeds = orc.voxelize(verts, tris, g)
    snap = np.sqrt(3) * h / 512 + 1e-6 * h
    cen = voxel_centres(dims, (0, 0, 0), h)
    dist = point_mesh_distance(cen, verts, tris, chunk=64, max_dist=1.5 * h)
    is_seed = seeds != orc.EMPTY
    # V2: a ball of radius h/2 around the centre lies in the cell.
    assert is_seed[dist <= h / 2 - snap].all()
    # V3: a cell touching the mesh has its centre within half a cell diagonal.
    assert (dist[is_seed] <= np.sqrt(3) / 2 * h + snap).all()
    # V1: voxels holding a vertex (strictly inside, away from cell faces).
    q = np.asarray(verts, np.float64) / h
    ijk = np.floor(q).astype(np.int64)
    frac = q - ijk
    inside = ((frac > 1e-3) & (frac < 1 - 1e-3)).all(1) & (ijk >= 0).all(1) & (ijk < np.array(dims)).all(1)
    vid = ijk[inside, 0] + dims[0] * (ijk[inside, 1] + dims[1] * ijk[inside, 2])
    assert is_seed[vid].all()


def test_out_of_range_index(orc):
    g = orc.make_grid((4, 4, 4), (0, 0, 0), 0.25)
    with pytest.raises(ValueError):
        orc.voxelize(np.zeros((3, 3), np.float32), np.array([[0, 1, 3]], np.int32), g)
