"""GPU (HIP, gfx950) versus CPU oracle, through the C ABI.

Bar: seed ids, mask lists, hit counts and argmin records bit-exact; FP32 distances and
fine values within 1e-5 relative (bit-exact is expected: both sides use the same binary32
operation order, correctly rounded '/' and sqrt, no contraction).
Sizes: the 32^3 icosphere; a 100x50x100 static scene compared element by element; and the
full 400x200x400 static scene in the launch configuration the benchmark times, compared
in full for the integer stages and on sampled voxels for the ray stages.  Edge cases: an
empty mesh, one triangle (a single-leaf hierarchy), two triangles on a voxel face, a grid
of 128 coplanar triangles (hierarchy nodes flat on one axis), grids with the largest
allowed side (1024) on each axis, and jump flooding with arbitrary offset lists on odd grids.
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


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def gpu_pipeline(R, sc, frames=None, key=0, beta=None, bias=0.0):
    import torch
    frames = sc.frames if frames is None else frames
    S = R.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, frames,
                    beta=beta, bias=bias, rng_key=key)
    S.voxelize()
    seeds0 = S.seeds.clone()
    S.jfa()
    S.mask()
    S.build_bvh()
    R.rtsdf_reset_accum(S.dmin, S.hits, S.argmin)
    for f in range(frames):
        S.trace(f)
    S.combine()
    torch.cuda.synchronize()
    n = int(S.band_count.item())
    return dict(seeds0=seeds0.cpu().numpy(), jfa=S.jfa_out.cpu().numpy(), band=S.band_list[:n].cpu().numpy(),
                dmin=S.dmin.cpu().numpy(), hits=u32(S.hits), argmin=u64(S.argmin), fine=S.fine.cpu().numpy(),
                S=S)


def oracle_pipeline(orc, sc, frames=None, key=0, beta=None, bias=0.0, sample=None, rng=None):
    frames = sc.frames if frames is None else frames
    beta = sc.h / 2 if beta is None else beta
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    seeds0 = orc.voxelize(sc.verts, sc.tris, g)
    jfa = orc.jfa(seeds0, g, sc.steps)
    band = orc.band(jfa, g, sc.band)
    vids = band if sample is None or sample >= len(band) else np.sort(rng.choice(band, sample, replace=False))
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    acc = orc.new_accum(len(vids))
    for f in range(frames):
        orc.raysample(bvh, g, vids, sc.rays, key, f, acc=acc)
    dmin, hits, argmin = acc
    # combine needs full-grid accumulators only at the sampled voxels
    N = len(seeds0)
    D = np.full(N, np.inf, np.float32)
    H = np.zeros(N, np.uint32)
    D[vids], H[vids] = dmin, hits
    fine_all, _ = orc.combine(jfa, D, H, g, sc.band, beta, bias, 0)
    return dict(seeds0=seeds0, jfa=jfa, band=band, vids=vids, dmin=dmin, hits=hits, argmin=argmin,
                fine=fine_all)


def compare_rays(G, O, vids):
    hits_g = G["hits"][vids]
    assert np.array_equal(hits_g, O["hits"]), "hit counts differ at %d voxels" % (hits_g != O["hits"]).sum()
    dg, do = G["dmin"][vids], O["dmin"]
    fin = np.isfinite(do)
    assert np.array_equal(np.isfinite(dg), fin)
    np.testing.assert_allclose(dg[fin], do[fin], rtol=RTOL)
    # same binary32 operations on both sides and exact culling: distances and argmin records
    # are bit-identical at every compared voxel
    nbits = int((dg[fin].view(np.uint32) != do[fin].view(np.uint32)).sum())
    ag = G["argmin"][vids]
    narg = int((ag != O["argmin"]).sum())
    log("  compared voxels", len(vids), "dmin bit differences", nbits, "argmin differences", narg)
    assert nbits == 0 and narg == 0


def test_tiny_full_parity(R, orc):
    sc = synth.scene_tiny()
    log("case: icosphere 80 tris, 32^3")
    G = gpu_pipeline(R, sc)
    O = oracle_pipeline(orc, sc)
    assert np.array_equal(G["seeds0"], O["seeds0"])
    assert np.array_equal(G["jfa"], O["jfa"])
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])
    np.testing.assert_allclose(G["fine"], O["fine"], rtol=RTOL, atol=0)


@pytest.mark.parametrize("case", ["static100", "static_odd"])
def test_static_reduced_full_parity(R, orc, case):
    if case == "static100":
        sc = synth.scene_static(dims=(100, 50, 100), nprims=40, seed=1)
        sc.frames = 3
    else:
        sc = synth.scene_static(dims=(77, 41, 93), nprims=15, seed=2)
        sc.frames, sc.rays, sc.band = 2, 5, 3
    log("case:", sc.name, "tris", len(sc.tris))
    G = gpu_pipeline(R, sc, key=0xDEADBEEF12345)
    O = oracle_pipeline(orc, sc, key=0xDEADBEEF12345)
    assert np.array_equal(G["seeds0"], O["seeds0"])
    assert np.array_equal(G["jfa"], O["jfa"])
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])
    np.testing.assert_allclose(G["fine"], O["fine"], rtol=RTOL, atol=0)


@pytest.mark.parametrize("case", ["x1", "x3", "x7", "x64", "x65", "x100", "x1_large", "x5_large", "x9_large"])
def test_rays_per_voxel_pool_boundaries(R, orc, case):
    """Ray counts that split a wave's pool of 64 rays unevenly: fills with more voxels than
    LDS slots (x < 8: those voxels' rays add to the global accumulators themselves), voxels
    continued from one fill to the next (x not dividing 64, on a mask large enough for
    chunks longer than one fill), a voxel filling a pool exactly (x = 64), and a voxel
    spanning several fills (x = 65, x = 100).  Small grids
    are compared at every masked voxel, the larger ones at 4000 sampled voxels."""
    x = int(case[1:].split("_")[0])
    if case.endswith("_large"):
        sc = synth.scene_static(dims=(160, 80, 160), nprims=60, seed=6)
        sc.frames, sc.rays, sc.band = 1, x, 4
        sample = 4000
    else:
        sc = synth.scene_static(dims=(60, 40, 60), nprims=12, seed=4)
        sc.frames, sc.rays, sc.band = (1 if x > 64 else 2), x, 3
        sample = None
    log("case:", case, "tris", len(sc.tris), "rays", x)
    G = gpu_pipeline(R, sc, key=77)
    O = oracle_pipeline(orc, sc, key=77, sample=sample, rng=np.random.default_rng(5))
    log("  masked voxels", len(G["band"]))
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])


def test_paper_scale_static(R, orc):
    """400x200x400, ~102k triangles, 10 passes, 4-voxel mask, 8 rays x 16 frames."""
    sc = synth.scene_static()
    log("case:", sc.name, "tris", len(sc.tris))
    G = gpu_pipeline(R, sc)
    log("  gpu done, band", len(G["band"]))
    O = oracle_pipeline(orc, sc, sample=3000, rng=np.random.default_rng(123))
    log("  oracle done")
    assert np.array_equal(G["seeds0"], O["seeds0"])
    assert np.array_equal(G["jfa"], O["jfa"])
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])
    v = O["vids"]
    np.testing.assert_allclose(G["fine"][v], O["fine"][v], rtol=RTOL, atol=0)
    # outside the mask the fine value is the coarse one: compare everywhere off-mask
    off = np.ones(len(G["fine"]), bool)
    off[O["band"]] = False
    np.testing.assert_allclose(G["fine"][off], O["fine"][off], rtol=RTOL, atol=0)


def test_edge_cases(R, orc):
    import torch
    # empty mesh: all EMPTY, empty mask, no hits, +inf everywhere
    sc = synth.scene_tiny()
    sc.verts, sc.tris = np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32)
    G = gpu_pipeline(R, sc)
    assert (G["seeds0"] == -1).all() and (G["jfa"] == -1).all() and len(G["band"]) == 0
    assert np.isinf(G["fine"]).all()
    # one triangle (the hierarchy is a single leaf), band 0, odd grid
    sc = synth.scene_tiny()
    sc.dims, sc.steps = (13, 7, 21), [16, 8, 4, 2, 1, 1]
    sc.verts = np.array([[0.1, 0.05, 0.2], [0.3, 0.15, 0.25], [0.12, 0.2, 0.5]], np.float32)
    sc.tris = np.array([[0, 1, 2]], np.int32)
    for band in (0, 1):
        sc.band = band
        G = gpu_pipeline(R, sc)
        O = oracle_pipeline(orc, sc)
        assert np.array_equal(G["seeds0"], O["seeds0"]) and np.array_equal(G["jfa"], O["jfa"])
        assert np.array_equal(G["band"], O["band"])
        compare_rays(G, O, O["vids"])
    # two triangles sharing an edge on a voxel face (closed-cell rule on both sides)
    sc.verts = np.array([[0.0, 0.25, 0.0], [0.0, 0.25, 0.5], [0.4, 0.25, 0.5], [0.4, 0.25, 0.0]], np.float32)
    sc.tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    sc.dims, sc.h = (16, 16, 16), 1.0 / 32
    sc.steps = [8, 4, 2, 1]
    G = gpu_pipeline(R, sc)
    O = oracle_pipeline(orc, sc)
    assert np.array_equal(G["seeds0"], O["seeds0"]) and np.array_equal(G["jfa"], O["jfa"])
    compare_rays(G, O, O["vids"])
    # 128 coplanar triangles on that face plus a tilted pair above it: hierarchy nodes flat on
    # y, whose quantised boxes use the smallest steps (the hit test's widening must still
    # cover them)
    xs = np.linspace(0.05, 0.45, 9, dtype=np.float32)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    v = np.stack([X.ravel(), np.full(X.size, 0.25, np.float32), Z.ravel()], 1)
    k = lambda i, j: i * 9 + j
    t = [[k(i, j), k(i, j + 1), k(i + 1, j + 1)] for i in range(8) for j in range(8)]
    t += [[k(i, j), k(i + 1, j + 1), k(i + 1, j)] for i in range(8) for j in range(8)]
    extra = np.array([[0.1, 0.3, 0.1], [0.35, 0.4, 0.15], [0.2, 0.33, 0.4], [0.3, 0.28, 0.3]], np.float32)
    sc.verts = np.concatenate([v, extra]).astype(np.float32)
    sc.tris = np.array(t + [[81, 82, 83], [81, 83, 84]], np.int32)
    log("case: flat grid of 128 triangles + 2, 16^3")
    G = gpu_pipeline(R, sc)
    O = oracle_pipeline(orc, sc)
    assert np.array_equal(G["seeds0"], O["seeds0"]) and np.array_equal(G["jfa"], O["jfa"])
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])


def test_deterministic(R):
    sc = synth.scene_static(dims=(100, 50, 100), nprims=30, seed=4)
    sc.frames = 2
    a = gpu_pipeline(R, sc)
    b = gpu_pipeline(R, sc)
    for k in ("jfa", "band", "hits", "argmin"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["fine"].view(np.uint32), b["fine"].view(np.uint32))


@pytest.mark.parametrize("dims,steps", [
    ((700, 97, 9), [256, 128, 64, 48, 33, 17, 12, 5, 2, 1]),   # rows walked in residue order for k = 12 ... 64
    ((430, 250, 7), [512, 300, 200, 129, 64, 31, 1]),           # k >= nx, k >= ny, odd row counts per residue
    ((37, 1001, 5), [600, 257, 64, 1]),                         # one-row-per-residue and tall planes
    ((1024, 6, 5), [512, 256, 3, 1]),                           # the largest side on each axis: ids with
    ((5, 1024, 6), [512, 100, 1]),                              # coordinates up to 1023
    ((6, 5, 1024), [1024, 512, 256, 128, 7, 1]),
])
def test_jfa_offsets_and_row_orders(R, orc, dims, steps):
    """Arbitrary offset lists on grids whose passes take every work layout (rows in residue
    order, neighbour rows or columns dropped, the sparse first passes): seed ids bit-exact
    against the oracle pass by pass, from ~0.2 % random seeds."""
    import torch
    rng = np.random.default_rng(sum(dims))
    nx, ny, nz = dims
    n = nx * ny * nz
    seeds = np.full(n, -1, np.int32)
    pick = rng.choice(n, size=max(1, n // 500), replace=False)
    x, y, z = pick % nx, (pick // nx) % ny, pick // (nx * ny)
    seeds[pick] = (x | (y << 10) | (z << 20)).astype(np.int32)
    g = R.make_grid(dims, (0.0, 0.0, 0.0), 1.0 / 512)
    go = orc.make_grid(dims, (0.0, 0.0, 0.0), 1.0 / 512)
    cur = torch.from_numpy(seeds).cuda()
    nxt = torch.empty_like(cur)
    ref = seeds
    for k in steps:
        log("case: jfa %s k=%d" % (dims, k))
        res = R.rtsdf_jfa(cur, nxt, g, [k])
        ref = orc.jfa_pass(ref, go, k)
        got = res.cpu().numpy()
        assert np.array_equal(got, ref), "k=%d: %d ids differ" % (k, (got != ref).sum())
        cur, nxt = res, cur


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_max_side_pipeline(R, orc, axis):
    """The whole chain on a grid whose side along `axis` is the largest allowed (1024 points,
    coordinates up to 1023) and a few points across: a slab through the icosphere, compared
    element by element (seeds, flood, mask, hits, distances, argmin records, fine values)."""
    sc = synth.scene_tiny()
    dims = [6, 5, 7]
    dims[axis] = 1024
    sc.h = 1.0 / 1024
    org = [0.5 - 3 * sc.h, 0.5 - 2.5 * sc.h, 0.5 - 3.5 * sc.h]
    org[axis] = 0.0
    sc.dims, sc.org = tuple(dims), tuple(org)
    sc.steps = orc.jfa_steps(sc.dims, 1)
    log("case: max side", sc.dims)
    G = gpu_pipeline(R, sc)
    O = oracle_pipeline(orc, sc)
    assert (O["seeds0"] != -1).sum() > 0 and len(O["band"]) > 0
    assert np.array_equal(G["seeds0"], O["seeds0"]) and np.array_equal(G["jfa"], O["jfa"])
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])
    np.testing.assert_allclose(G["fine"], O["fine"], rtol=RTOL, atol=0)
