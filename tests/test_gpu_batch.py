"""Batched objects (one launch per stage over many grids) on the GPU.

Each object of a batch computes exactly what the single-object calls compute for it with
counter word obj = its index, so the bar against the single-object path is bit equality of
every output (seeds, mask, hits, argmin, dmin and fine); against the oracle it is the same
bar as the single-object parity tests (integers bit-exact, distances within 1e-5 relative).
The vertex adjoint sums binary32 atomics in a varying order, so it is compared within
|diff| <= 1e-3 |g| + 1e-4 max|g| (same as the single-object adjoint).
Cases: a mixed batch of small objects with odd and even JFA pass counts, grids that are not
multiples of any tile, a flat grid, a single-voxel grid and an empty mesh; the batched chain
captured into a HIP graph and replayed; and the full 64-object workload (about 1.9e8 grid
points, 2.2 M triangles), compared object by object with the single-object path.
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


def mixed_batch():
    objs = synth.scene_batch(nobj=7, seed=5, tri_range=(80, 3000), n_range=(12, 70))
    v, t = synth.icosphere(1, 0.3, (0.5, 0.5, 0.5))
    flat = synth.Scene(v, t, (20, 17, 1), (0.0, 0.0, 0.5), 1.0 / 20, synth.jfa_offsets((20, 17, 1), extra=2), 2, 8, 1)
    one = synth.Scene(v, t, (1, 1, 1), (0.4, 0.4, 0.4), 0.2, synth.jfa_offsets((1, 1, 1)), 1, 8, 1)
    empty = synth.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), (5, 7, 3), (0, 0, 0), 0.2,
                        synth.jfa_offsets((5, 7, 3)), 2, 8, 1)
    return objs[:3] + [flat, empty] + objs[3:] + [one]


def single(R, sc, o, rays, key, frames=1):
    S = R.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, rays, frames, rng_key=key, obj=o)
    S.run()
    return S


def compare_object(R, B, S, o):
    import torch
    off = B.offsets[o][0]
    n = S.g.n
    nb = int(B.band_count.item())
    lst = B.band_list[:nb]
    mine = lst[(lst >= off) & (lst < off + n)] - off
    ns = int(S.band_count.item())
    assert torch.equal(B.view(B.seeds, o), S.jfa_out), "object %d: seeds differ" % o
    assert torch.equal(mine, S.band_list[:ns]), "object %d: mask differs" % o
    assert torch.equal(B.view(B.hits, o), S.hits), "object %d: hits differ" % o
    assert torch.equal(B.view(B.argmin, o), S.argmin), "object %d: argmin differs" % o
    assert torch.equal(B.view(B.dmin, o).view(torch.int32), S.dmin.view(torch.int32)), "object %d: dmin differs" % o
    assert torch.equal(B.view(B.fine, o).view(torch.int32), S.fine.view(torch.int32)), "object %d: fine differs" % o


@pytest.mark.parametrize("frames,key,rays", [(1, 0, 8), (2, 9, 8), (1, 3, 3), (2, 4, 1)])
def test_batched_equals_single_calls(R, frames, key, rays):
    """Also with fewer than 8 rays per voxel, where ray sampling's pool fills span more voxels
    than they have LDS slots for (a separate kernel instance in both the batched and the
    single-object case)."""
    import torch
    objs = mixed_batch()
    log("case: mixed batch of %d objects, frames %d, key %d, rays %d" % (len(objs), frames, key, rays))
    B = R.BatchSDF(objs, rays=rays, frames=frames, rng_key=key)
    B.run()
    torch.cuda.synchronize()
    for o, sc in enumerate(objs):
        S = single(R, sc, o, rays, key, frames)
        torch.cuda.synchronize()
        compare_object(R, B, S, o)
    assert int(B.band_count.item()) > 0


def test_batched_vs_oracle(R, orc):
    objs = mixed_batch()
    log("case: mixed batch vs oracle")
    B = R.BatchSDF(objs, rays=8)
    B.run()
    for o, sc in enumerate(objs):
        g = orc.make_grid(sc.dims, sc.org, sc.h)
        seeds = orc.voxelize(sc.verts, sc.tris, g)
        jfa = orc.jfa(seeds, g, sc.steps)
        band = orc.band(jfa, g, sc.band)
        assert np.array_equal(B.view(B.seeds, o).cpu().numpy(), jfa), o
        if len(sc.tris) == 0:
            assert (B.view(B.hits, o) == 0).all()
            continue
        bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
        dmin, hits, argmin = orc.raysample(bvh, g, band, 8, 0, 0, obj=o)
        hb = B.view(B.hits, o).cpu().numpy().view(np.uint32)[band]
        ab = B.view(B.argmin, o).cpu().numpy().view(np.uint64)[band]
        db = B.view(B.dmin, o).cpu().numpy()[band]
        assert np.array_equal(hb, hits), o
        assert np.array_equal(ab, argmin), o
        fin = np.isfinite(dmin)
        np.testing.assert_allclose(db[fin], dmin[fin], rtol=1e-5)
        N = len(jfa)
        D = np.full(N, np.inf, np.float32)
        H = np.zeros(N, np.uint32)
        D[band], H[band] = dmin, hits
        fine, _ = orc.combine(jfa, D, H, g, sc.band, sc.h / 2, 0.0, 0)
        np.testing.assert_allclose(B.view(B.fine, o).cpu().numpy(), fine, rtol=1e-5)


def close(a, b, rtol=1e-3, arel=1e-4):
    b = np.asarray(b, np.float64)
    tol = rtol * np.abs(b) + arel * max(np.abs(b).max(), 1e-30)
    err = np.abs(np.asarray(a, np.float64) - b)
    assert (err <= tol).all(), "%d elements differ; worst %g" % ((err > tol).sum(), err.max())


def test_batched_backward(R, orc):
    import torch
    objs = mixed_batch()
    log("case: batched vertex adjoint")
    B = R.BatchSDF(objs, rays=8)
    B.run()
    w = torch.from_numpy(np.random.default_rng(8).normal(size=B.fine.numel()).astype(np.float32)).cuda()
    gb = B.backward(w).cpu().numpy()
    vo = np.cumsum([0] + [len(sc.verts) for sc in objs])
    for o, sc in enumerate(objs):
        if len(sc.tris) == 0:
            continue
        S = single(R, sc, o, 8, 0)
        gs = S.backward(B.view(w, o).contiguous()).cpu().numpy()
        close(gb[vo[o]:vo[o + 1]], gs)
    # one object against the oracle
    o = 1
    sc = objs[o]
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    jfa = orc.jfa(orc.voxelize(sc.verts, sc.tris, g), g, sc.steps)
    band = orc.band(jfa, g, sc.band)
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    dmin, hits, argmin = orc.raysample(bvh, g, band, 8, 0, 0, obj=o)
    go = orc.sdf_backward(B.view(w, o).cpu().numpy().astype(np.float64), hits, argmin, band, bvh, sc.verts, sc.tris,
                          g, 8, 0, obj=o)
    close(gb[vo[o]:vo[o + 1]], go)


def test_batched_full_workload(R):
    """The 64-object workload in the benchmark's configuration, object by object."""
    import torch
    objs = synth.scene_batch()
    log("case: 64-object batch, %d triangles, %d grid points" % (sum(len(s.tris) for s in objs),
                                                                 sum(int(np.prod(s.dims)) for s in objs)))
    B = R.BatchSDF(objs, rays=8)
    B.run()
    torch.cuda.synchronize()
    for o, sc in enumerate(objs):
        S = single(R, sc, o, 8, 0)
        torch.cuda.synchronize()
        compare_object(R, B, S, o)
        del S


def test_batched_graph_replays(R):
    """The whole batched chain captured once into a HIP graph: three replays, with eager work
    and synchronisations between them, each equal to the eager chain bit for bit."""
    import torch
    objs = mixed_batch()
    log("case: batched chain in a HIP graph, %d objects" % len(objs))
    E = R.BatchSDF(objs, rays=8, frames=2, rng_key=3)
    E.run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (E.seeds, E.hits, E.argmin, E.dmin, E.fine)]
    G = R.BatchSDF(objs, rays=8, frames=2, rng_key=3)
    G.run()  # warm-up outside capture
    torch.cuda.synchronize()
    G.capture()
    for rep in range(3):
        G.fine.fill_(123.0)
        G.hits.zero_()
        torch.cuda.synchronize()
        G.replay()
        torch.cuda.synchronize()
        got = (G.seeds, G.hits, G.argmin, G.dmin, G.fine)
        # every object's own grid points (the padding between objects is never written)
        for o in range(len(objs)):
            for name, a, b in zip(("seeds", "hits", "argmin", "dmin", "fine"), got, ref):
                a, b = G.view(a, o), G.view(b, o)
                assert torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else a,
                                   b.view(torch.int32) if b.dtype == torch.float32 else b), (rep, o, name)
        nb = int(G.band_count.item())
        assert torch.equal(G.band_list[:nb], E.band_list[:nb])
