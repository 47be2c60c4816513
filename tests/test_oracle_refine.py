"""Pins of the oracle's two-level field (section 2.3 mask of a finer traced field; section
2.5.1 coarse and fine resolutions): refinement must commute with the coarse field.

  * the fine mask equals the coarse mask with every point repeated `ratio` times per axis
    (numpy repeat of the coarse mask, not the oracle's index arithmetic);
  * with inputs that are constant over the children of each coarse point (dmin, hits,
    state), the refined combine equals the coarse combine of those inputs, repeated, in
    both the running-minimum and the decay mode;
  * ratio 1 reproduces the single-level calls.
"""
import numpy as np
import pytest

from paper_2210_06160_amd import synth


def repeat3(a, dims, r):
    nx, ny, nz = dims
    v = np.asarray(a).reshape(nz, ny, nx)
    return v.repeat(r, axis=0).repeat(r, axis=1).repeat(r, axis=2).ravel()


@pytest.fixture(scope="module")
def coarse(orc):
    sc = synth.scene_static(dims=(40, 20, 40), nprims=30, seed=4)
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    jfa = orc.jfa(orc.voxelize(sc.verts, sc.tris, g), g, sc.steps)
    return sc, g, jfa


@pytest.mark.parametrize("r", [1, 2, 3])
def test_refined_mask_is_repeated_coarse_mask(orc, coarse, r):
    sc, g, jfa = coarse
    cmask = np.zeros(len(jfa), bool)
    cmask[orc.band(jfa, g, 2)] = True
    fine = orc.band(jfa, g, 2, ratio=r)
    assert np.array_equal(fine, np.flatnonzero(repeat3(cmask, sc.dims, r)))
    if r == 1:
        assert np.array_equal(fine, orc.band(jfa, g, 2))


@pytest.mark.parametrize("r", [2, 3])
@pytest.mark.parametrize("mode", [0, 1])
def test_refined_combine_commutes_with_repetition(orc, coarse, r, mode):
    sc, g, jfa = coarse
    rng = np.random.default_rng(r + 10 * mode)
    N = len(jfa)
    dmin = rng.uniform(0.001, 0.03, N).astype(np.float32)
    front = rng.integers(0, 5, N)
    back = rng.integers(0, 5, N)
    hits = (front + (back << 16)).astype(np.uint32)
    state = rng.uniform(-0.05, 0.05, N).astype(np.float32)
    kw = dict(beta=sc.h / 2, bias=0.002, mode=mode, alpha=0.9, reset=False)
    cf, cs = orc.combine(jfa, dmin, hits, g, 3, state=state.copy(), **kw)
    ff, fs = orc.combine(jfa, repeat3(dmin, sc.dims, r), repeat3(hits, sc.dims, r), g, 3,
                         state=repeat3(state, sc.dims, r).copy(), ratio=r, **kw)
    assert np.array_equal(ff, repeat3(cf, sc.dims, r))
    if mode == 1:
        assert np.array_equal(fs, repeat3(cs, sc.dims, r))
