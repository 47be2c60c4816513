"""Two-level field on the GPU (sections 2.3 and 2.5.1): jump flooding on a coarse grid,
mask, rays and combination on the grid refined by an integer ratio, against the oracle.

Bar as the single-level parity tests: coarse seed ids and the fine mask list bit-exact
(the mask over every fine point), hit counts and argmin records bit-exact, binary32
distances and field values within 1e-5 relative.
Cases: the icosphere at 16^3 refined by 2; a ragged 13 x 7 x 9 grid refined by 3 (no
axis a multiple of any tile); a 50 x 25 x 50 static scene refined by 2 compared
everywhere; the paper-shaped static scene flooded at 200 x 100 x 200 and traced at
400 x 200 x 400 (the benchmark's two-level configuration; rays on sampled fine points,
the field off the mask everywhere); a deforming sequence with the Eq. 1 decay on the
refined grid; and the refined chain with ratio 1 equal to the single-level chain.
"""
import sys

import numpy as np
import pytest

from paper_2210_06160_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-5


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


def gpu_chain(R, sc, ratio, key=0):
    import torch
    S = R.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames,
                    rng_key=key, ratio=ratio)
    S.run()
    torch.cuda.synchronize()
    n = int(S.band_count.item())
    return dict(jfa=S.jfa_out.cpu().numpy(), band=S.band_list[:n].cpu().numpy(), dmin=S.dmin.cpu().numpy(),
                hits=S.hits.cpu().numpy().view(np.uint32), argmin=S.argmin.cpu().numpy().view(np.uint64),
                fine=S.fine.cpu().numpy(), S=S)


def oracle_chain(orc, sc, ratio, key=0, sample=None, rng=None):
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    gf = orc.refine_grid(g, ratio)
    jfa = orc.jfa(orc.voxelize(sc.verts, sc.tris, g), g, sc.steps)
    band = orc.band(jfa, g, sc.band, ratio=ratio)
    vids = band if sample is None or sample >= len(band) else np.sort(rng.choice(band, sample, replace=False))
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(gf))
    acc = orc.new_accum(len(vids))
    for f in range(sc.frames):
        orc.raysample(bvh, gf, vids, sc.rays, key, f, acc=acc)
    dmin, hits, argmin = acc
    Nf = gf.nx * gf.ny * gf.nz
    D = np.full(Nf, np.inf, np.float32)
    H = np.zeros(Nf, np.uint32)
    D[vids], H[vids] = dmin, hits
    fine, _ = orc.combine(jfa, D, H, g, sc.band, sc.h / 2, 0.0, 0, ratio=ratio)
    return dict(jfa=jfa, band=band, vids=vids, dmin=dmin, hits=hits, argmin=argmin, fine=fine)


def compare(G, O, everywhere=True):
    v = O["vids"]
    assert np.array_equal(G["jfa"], O["jfa"])
    assert np.array_equal(G["band"], O["band"]), "fine mask differs"
    assert np.array_equal(G["hits"][v], O["hits"])
    assert np.array_equal(G["argmin"][v], O["argmin"])
    dg, do = G["dmin"][v], O["dmin"]
    fin = np.isfinite(do)
    assert np.array_equal(np.isfinite(dg), fin)
    np.testing.assert_allclose(dg[fin], do[fin], rtol=RTOL, atol=0)
    if everywhere:
        np.testing.assert_allclose(G["fine"], O["fine"], rtol=RTOL, atol=0)
    else:
        np.testing.assert_allclose(G["fine"][v], O["fine"][v], rtol=RTOL, atol=0)
        off = np.ones(len(G["fine"]), bool)
        off[O["band"]] = False
        np.testing.assert_allclose(G["fine"][off], O["fine"][off], rtol=RTOL, atol=0)


def ico_scene(dims, h, org=(0.0, 0.0, 0.0), band=2, rays=16, frames=1):
    v, t = synth.icosphere(1, 0.3, (0.5, 0.5, 0.5))
    return synth.Scene(v, t, dims, org, h, synth.jfa_offsets(dims), band, rays, frames)


@pytest.mark.parametrize("case", ["ico16x2", "ragged_x3", "static50x2"])
def test_two_level_vs_oracle(R, orc, case):
    if case == "ico16x2":
        sc, r = ico_scene((16, 16, 16), 1.0 / 16), 2
    elif case == "ragged_x3":
        sc, r = ico_scene((13, 7, 9), 0.077, org=(0.02, 0.25, 0.15), band=1, rays=5, frames=2), 3
    else:
        sc, r = synth.scene_static(dims=(50, 25, 50), nprims=40, seed=1), 2
        sc.band, sc.frames = 2, 3
    log("case: two-level %s, coarse %s, ratio %d, %d tris" % (case, sc.dims, r, len(sc.tris)))
    G = gpu_chain(R, sc, r, key=0x5EED)
    O = oracle_chain(orc, sc, r, key=0x5EED)
    assert len(O["band"]) > 0
    compare(G, O)


def test_two_level_paper_scale(R, orc):
    """Flooded at 200 x 100 x 200, traced at 400 x 200 x 400: 2-coarse-voxel mask, 8 rays x 16
    frames, the configuration the benchmark times."""
    sc = synth.scene_static(dims=(200, 100, 200))
    sc.band = 2
    log("case: two-level static, coarse %s ratio 2, %d tris" % (sc.dims, len(sc.tris)))
    G = gpu_chain(R, sc, 2)
    log("  gpu done, fine mask", len(G["band"]))
    O = oracle_chain(orc, sc, 2, sample=3000, rng=np.random.default_rng(77))
    log("  oracle done")
    compare(G, O, everywhere=False)


def test_ratio_one_is_single_level(R):
    import torch
    sc = synth.scene_static(dims=(60, 30, 60), nprims=20, seed=3)
    sc.frames = 2
    log("case: ratio 1 through the refined entries vs the single-level entries")
    a = gpu_chain(R, sc, 1)
    S = a["S"]
    fine = torch.empty_like(S.fine)
    lst = torch.empty_like(S.band_list)
    cnt = torch.zeros_like(S.band_count)
    R.rtsdf_band_refined(S.jfa_out, S.g, 1, S.band, lst, cnt, S.work)
    R.rtsdf_combine_refined(S.jfa_out, S.dmin, S.hits, S.g, 1, S.band, S.beta, S.bias, R.ACCUM, fine)
    torch.cuda.synchronize()
    n = int(cnt.item())
    assert n == len(a["band"]) and np.array_equal(lst[:n].cpu().numpy(), a["band"])
    assert torch.equal(fine.view(torch.int32), S.fine.view(torch.int32))


def test_two_level_decay_sequence(R, orc):
    """Deforming knot flooded at 50 x 25 x 50 and traced at 100 x 50 x 100, Eq. 1 decay over
    five frames (the state carried on the fine grid), element by element."""
    import torch
    sc = synth.scene_deform(dims=(50, 25, 50), frames=5)
    sc.band = 2
    alpha = sc.extra["alpha"]
    log("case: two-level deforming knot, coarse %s ratio 2, 5 frames" % (sc.dims,))
    D = R.DeformSDF(sc.extra["frames"], sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, alpha, ratio=2)
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    gf = orc.refine_grid(g, 2)
    Nf = gf.nx * gf.ny * gf.nz
    state = np.zeros(Nf, np.float32)
    for f in range(5):
        D.frame(f)
        torch.cuda.synchronize()
        v = sc.extra["frames"][f]
        seeds = orc.jfa(orc.voxelize(v, sc.tris, g), g, sc.steps)
        band = orc.band(seeds, g, sc.band, ratio=2)
        dmin, hits, _ = orc.raysample(orc.BVH(v, sc.tris, orc.hit_pad(gf)), gf, band, sc.rays, 0, f)
        Dm = np.full(Nf, np.inf, np.float32)
        H = np.zeros(Nf, np.uint32)
        Dm[band], H[band] = dmin, hits
        fine, state = orc.combine(seeds, Dm, H, g, sc.band, sc.h / 2, 0.0, 1, alpha, reset=(f == 0), state=state,
                                  ratio=2)
        n = int(D.band_count.item())
        assert np.array_equal(D.jfa_out.cpu().numpy(), seeds), f
        assert np.array_equal(D.band_list[:n].cpu().numpy(), band), f
        np.testing.assert_allclose(D.fine.cpu().numpy(), fine, rtol=RTOL, atol=0)
        np.testing.assert_allclose(D.state.cpu().numpy(), state, rtol=RTOL, atol=0)
        assert (D.hits.cpu().numpy() == 0).all()
        log("  frame", f, "mask", n, "ok")
