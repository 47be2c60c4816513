"""Deforming mesh (section 2.5.1, Eq. 1): GPU per-frame chain vs the CPU oracle, and the
HIP-graph replays of every frame vs the eager chain.

A reduced grid (100 x 50 x 100 over the same world box) is compared element by element over
a sequence of frames, including the Eq. 1 state carried from frame to frame.  At the full
400 x 200 x 400 size, the first and last frames are compared stage by stage (seed ids, mask
exact over every voxel; per-frame ray results on sampled masked voxels), and 60 frames
replayed (twice over) from one HIP graph recorded once (the frame index in device memory)
must equal the eager chain bit for bit.
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


def oracle_frames(orc, sc, frames, alpha):
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    N = g.nx * g.ny * g.nz
    state = np.zeros(N, np.float32)
    outs = []
    for f in range(frames):
        v = sc.extra["frames"][f]
        seeds = orc.jfa(orc.voxelize(v, sc.tris, g), g, sc.steps)
        band = orc.band(seeds, g, sc.band)
        bvh = orc.BVH(v, sc.tris, orc.hit_pad(g))
        dmin, hits, _ = orc.raysample(bvh, g, band, sc.rays, 0, f)
        D = np.full(N, np.inf, np.float32)
        H = np.zeros(N, np.uint32)
        D[band], H[band] = dmin, hits
        fine, state = orc.combine(seeds, D, H, g, sc.band, sc.h / 2, 0.0, 1, alpha, reset=(f == 0), state=state)
        outs.append(dict(seeds=seeds, band=band, dmin=dmin, hits=hits, fine=fine.copy(), state=state.copy()))
    return outs


def test_reduced_sequence_vs_oracle(R, orc):
    import torch
    sc = synth.scene_deform(dims=(100, 50, 100), frames=8)
    sc.band = 3
    alpha = sc.extra["alpha"]
    log("case: deforming knot 100x50x100, 8 frames")
    D = R.DeformSDF(sc.extra["frames"], sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, alpha)
    O = oracle_frames(orc, sc, 8, alpha)
    for f in range(8):
        # stage by stage through the public entry points for the per-frame ray results
        v = D.verts[f]
        if f == 0:
            R.rtsdf_reset_accum(D.dmin, D.hits)
        R.rtsdf_voxelize(v, D.tris, D.g, D.seeds, D.work)
        out = R.rtsdf_jfa(D.seeds, D.scratch, D.g, D.steps)
        R.rtsdf_band(out, D.g, D.band, D.band_list, D.band_count, D.work)
        R.rtsdf_build_bvh(v, D.tris, D.g, D.bvh, D.work)
        R.rtsdf_raysample(D.bvh, D.g, D.band_list, D.band_count, D.rays, 0, f, D.dmin, D.hits, D.ray_work)
        torch.cuda.synchronize()
        o = O[f]
        n = int(D.band_count.item())
        assert np.array_equal(out.cpu().numpy(), o["seeds"])
        assert np.array_equal(D.band_list[:n].cpu().numpy(), o["band"])
        hits = D.hits.cpu().numpy().view(np.uint32)[o["band"]]
        dmin = D.dmin.cpu().numpy()[o["band"]]
        assert np.array_equal(hits, o["hits"])
        fin = np.isfinite(o["dmin"])
        assert np.array_equal(np.isfinite(dmin), fin)
        np.testing.assert_allclose(dmin[fin], o["dmin"][fin], rtol=1e-5, atol=0)
        R.rtsdf_combine(out, D.dmin, D.hits, D.g, D.band, D.beta, D.bias, R.DECAY, D.fine, alpha=alpha,
                        first_frame=(f == 0), consume=True, state=D.state)
        torch.cuda.synchronize()
        np.testing.assert_allclose(D.fine.cpu().numpy(), o["fine"], rtol=1e-5, atol=0)
        np.testing.assert_allclose(D.state.cpu().numpy(), o["state"], rtol=1e-5, atol=0)
        # consume left the accumulators clear for the next frame
        assert (D.hits.cpu().numpy() == 0).all()


def test_full_size_frames_vs_oracle(R, orc):
    import torch
    sc = synth.scene_deform()
    log("case:", sc.name)
    D = R.DeformSDF(sc.extra["frames"], sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays,
                    sc.extra["alpha"])
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    rng = np.random.default_rng(5)
    for f in (0, sc.frames - 1):
        v = D.verts[f]
        R.rtsdf_reset_accum(D.dmin, D.hits)
        R.rtsdf_voxelize(v, D.tris, D.g, D.seeds, D.work)
        out = R.rtsdf_jfa(D.seeds, D.scratch, D.g, D.steps)
        R.rtsdf_band(out, D.g, D.band, D.band_list, D.band_count, D.work)
        R.rtsdf_build_bvh(v, D.tris, D.g, D.bvh, D.work)
        R.rtsdf_raysample(D.bvh, D.g, D.band_list, D.band_count, D.rays, 0, f, D.dmin, D.hits, D.ray_work)
        torch.cuda.synchronize()
        vn = sc.extra["frames"][f]
        seeds = orc.jfa(orc.voxelize(vn, sc.tris, g), g, sc.steps)
        band = orc.band(seeds, g, sc.band)
        n = int(D.band_count.item())
        assert np.array_equal(out.cpu().numpy(), seeds)
        assert np.array_equal(D.band_list[:n].cpu().numpy(), band)
        vids = np.sort(rng.choice(band, 3000, replace=False))
        dmin, hits, _ = orc.raysample(orc.BVH(vn, sc.tris, orc.hit_pad(g)), g, vids, sc.rays, 0, f)
        assert np.array_equal(D.hits.cpu().numpy().view(np.uint32)[vids], hits)
        fin = np.isfinite(dmin)
        np.testing.assert_allclose(D.dmin.cpu().numpy()[vids][fin], dmin[fin], rtol=1e-5, atol=0)
        log("  frame", f, "band", n, "ok")


def test_graph_replays_equal_eager(R):
    import torch
    sc = synth.scene_deform()
    D = R.DeformSDF(sc.extra["frames"], sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays,
                    sc.extra["alpha"])
    eager = []
    for f in range(sc.frames):
        D.frame(f)
        torch.cuda.synchronize()
        eager.append(D.fine.cpu().numpy().view(np.uint32).copy())
    D.capture()
    torch.cuda.synchronize()
    for rep in range(2):
        for f in range(sc.frames):
            D.replay(f)
            torch.cuda.synchronize()
            got = D.fine.cpu().numpy().view(np.uint32)
            assert np.array_equal(got, eager[f]), "replay %d frame %d differs" % (rep, f)
        log("  replay pass", rep, "ok")
        # eager work between the passes
        D.frame(0)
        torch.cuda.synchronize()
        assert np.array_equal(D.fine.cpu().numpy().view(np.uint32), eager[0])
