"""The allocation-free ray-sampling entry point (work cursors in the library's static
per-GPU scratch) against the entry point that takes a caller workspace.

Both run the same kernel over the same inputs; ray sampling's accumulators are order-free
(minimum, sum, minimum), so the bar is bit equality of dmin, hits and argmin.  Two calls in
a row, the second over a smaller mask, show that nothing the first call left in the shared
scratch changes the second; the first call's mask is large enough to spread its units over
every cursor range.
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


def prepared(R, sc):
    """A static scene flooded, masked and with its hierarchy built (no rays yet)."""
    S = R.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames)
    S.voxelize()
    S.jfa()
    S.mask()
    S.build_bvh()
    return S


def trace_both(R, S, frame, key=7):
    """dmin, hits, argmin from each entry point over the same mask."""
    import torch
    outs = []
    for noalloc in (False, True):
        dmin = torch.empty_like(S.dmin)
        hits = torch.empty_like(S.hits)
        argmin = torch.empty_like(S.argmin)
        R.rtsdf_reset_accum(dmin, hits, argmin)
        if noalloc:
            R.rtsdf_raysample_noalloc(S.bvh, S.gf, S.band_list, S.band_count, S.rays, key, frame, dmin, hits,
                                      argmin=argmin, band_capacity=S.band_n)
        else:
            R.rtsdf_raysample(S.bvh, S.gf, S.band_list, S.band_count, S.rays, key, frame, dmin, hits, S.ray_work,
                              argmin=argmin, band_capacity=S.band_n)
        torch.cuda.synchronize()
        outs.append((dmin.cpu().numpy().view(np.uint32), hits.cpu().numpy(), argmin.cpu().numpy()))
    return outs


def test_noalloc_matches_workspace_entry_point(R):
    big = synth.scene_grad(dims=(96, 96, 96), subdiv=4)
    small = synth.scene_tiny()
    for name, sc, frame in (("icosphere-96^3", big, 0), ("icosphere-32^3", small, 3)):
        log("case", name, sc.dims, "triangles", len(sc.tris))
        S = prepared(R, sc)
        n = int(S.band_count.item())
        assert n > 0
        (d0, h0, a0), (d1, h1, a1) = trace_both(R, S, frame)
        assert h0.any(), "no ray hit anything"
        assert np.array_equal(d0, d1), "dmin differs"
        assert np.array_equal(h0, h1), "hit counts differ"
        assert np.array_equal(a0, a1), "argmin records differ"
        log("  masked", n, "equal")


def test_noalloc_rejects_bad_arguments_without_launching(R):
    import torch
    sc = synth.scene_tiny()
    S = prepared(R, sc)
    with pytest.raises(R.RtsdfError):
        R.rtsdf_raysample_noalloc(S.bvh, S.gf, S.band_list, S.band_count, 0, 0, 0, S.dmin, S.hits)
    torch.cuda.synchronize()
