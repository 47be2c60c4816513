"""The hierarchy builders on the GPU: every blob decoded and validated on the host (leaf
ranges partition the triangles, child boxes contain their triangles, records match the
mesh), ray sampling bit-identical whichever tree is built (culling is exact), and the
batched build equal byte for byte to the single-object build of every object.
Cases: 1, 2, 3, 4 and 5 triangles, triangles sharing one centroid, the 32^3 icosphere, a
grid of coplanar triangles (nodes flat on one axis, the smallest quantisation steps), an
icosphere a thousand units from the origin, a reduced static scene, a mixed batch, the
full static scene (PLOC), and a clustering tree deeper than the traversal stack holds
(rays then test every triangle, which gives the same closest hit)."""
import sys

import numpy as np
import pytest

from bvh_check import check
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


def build(R, verts, tris, dims, h, method):
    import torch
    g = R.make_grid(dims, (0, 0, 0), h)
    V = torch.from_numpy(np.ascontiguousarray(verts, np.float32)).cuda()
    T = torch.from_numpy(np.ascontiguousarray(tris, np.int32).reshape(-1, 3)).cuda()
    bvh = torch.empty(R.rtsdf_bvh_bytes(len(tris)), dtype=torch.uint8, device="cuda")
    work = R.workspace(R.rtsdf_bvh_work_bytes(len(tris)))
    R.rtsdf_build_bvh(V, T, g, bvh, work, method)
    torch.cuda.synchronize()
    return bvh.cpu().numpy()


def flat_grid(n, y):
    """2 n^2 triangles tiling a square of the plane at height y: nodes flat on y."""
    xs = np.linspace(0.1, 0.9, n + 1, dtype=np.float32)
    X, Z = np.meshgrid(xs, xs, indexing="ij")
    v = np.stack([X.ravel(), np.full(X.size, y, np.float32), Z.ravel()], 1).astype(np.float32)
    idx = lambda i, j: i * (n + 1) + j
    t = [[idx(i, j), idx(i, j + 1), idx(i + 1, j + 1)] for i in range(n) for j in range(n)]
    t += [[idx(i, j), idx(i + 1, j + 1), idx(i + 1, j)] for i in range(n) for j in range(n)]
    return v, np.array(t, np.int32)


def small_meshes():
    rng = np.random.default_rng(3)
    out = []
    for n in (1, 2, 3, 4, 5, 17):
        v = rng.uniform(0.2, 0.8, size=(3 * n, 3)).astype(np.float32)
        out.append(("random%d" % n, v, np.arange(3 * n, dtype=np.int32).reshape(n, 3)))
    # eight triangles rotated about one point: identical centroids (equal Morton codes)
    base = np.array([[0.1, 0, 0], [-0.05, 0.08, 0], [-0.05, -0.08, 0]], np.float32)
    tris_v = []
    for k in range(8):
        a = k * np.pi / 8
        rot = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]], np.float32)
        tris_v.append(base @ rot.T + 0.5)
    out.append(("same-centroid", np.concatenate(tris_v).astype(np.float32), np.arange(24, dtype=np.int32).reshape(8, 3)))
    v, t = synth.icosphere(1, 0.3, (0.5, 0.5, 0.5))
    out.append(("icosphere80", v, t))
    out.append(("flat-grid", *flat_grid(8, 0.25)))
    # small triangles a thousand units from the origin (quantised against a far node corner)
    v, t = synth.icosphere(1, 0.3, (0.5, 0.5, 0.5))
    out.append(("far-icosphere80", (v + np.float32(1000.0)).astype(np.float32), t))
    sc = synth.scene_static(dims=(100, 50, 100), nprims=40, seed=1)
    out.append(("static-reduced", sc.verts, sc.tris))
    return out


@pytest.mark.parametrize("method", [0, 1])
def test_blob_valid(R, method):
    for name, v, t in small_meshes():
        log("case: %s, %d triangles, method %d" % (name, len(t), method))
        blob = build(R, v, t, (32, 32, 32), 1.0 / 32, method)
        check(blob, v, t, np.float32(1.0 / 32) * np.float32(1.0 / 256))


def test_raysample_independent_of_tree(R):
    import torch
    sc = synth.scene_static(dims=(100, 50, 100), nprims=40, seed=1)
    sc.frames = 2
    log("case: static 100x50x100, LBVH vs PLOC")
    out = []
    for method in (0, 1):
        S = R.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames,
                        bvh_method=method)
        S.run()
        torch.cuda.synchronize()
        out.append((S.dmin.clone(), S.hits.clone(), S.argmin.clone(), S.fine.clone()))
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a.view(torch.int32) if a.dtype == torch.float32 else a,
                           b.view(torch.int32) if b.dtype == torch.float32 else b)


@pytest.mark.parametrize("method", [0, 1])
def test_batched_build_equals_single(R, method):
    import torch
    objs = synth.scene_batch(nobj=6, seed=5, tri_range=(80, 5000), n_range=(12, 70))
    v, t = synth.icosphere(1, 0.3, (0.5, 0.5, 0.5))
    empty = synth.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), (5, 7, 3), (0, 0, 0), 0.2,
                        synth.jfa_offsets((5, 7, 3)), 2, 8, 1)
    one = synth.Scene(v[:3], np.array([[0, 1, 2]], np.int32), (9, 9, 9), (0, 0, 0), 1 / 9, synth.jfa_offsets((9, 9, 9)),
                      2, 8, 1)
    objs = objs[:2] + [empty] + objs[2:4] + [one] + objs[4:]
    log("case: batched build of %d objects, method %d" % (len(objs), method))
    B = R.BatchSDF(objs, rays=8, bvh_method=method)
    B.build_bvh()
    torch.cuda.synchronize()
    blob = B.bvh.cpu().numpy()
    for o, sc in enumerate(objs):
        off = B.offsets[o][1]
        nbytes = R.rtsdf_bvh_bytes(len(sc.tris))
        single = build(R, sc.verts, sc.tris, sc.dims, sc.h, method)
        assert np.array_equal(blob[off:off + nbytes], single[:nbytes]), "object %d" % o
        check(single, sc.verts, sc.tris, np.float32(sc.h) * np.float32(1.0 / 256))


def test_full_static_ploc_blob(R):
    sc = synth.scene_static()
    log("case: static 400x200x400 scene, PLOC blob")
    blob = build(R, sc.verts, sc.tris, sc.dims, sc.h, 1)
    nodes = check(blob, sc.verts, sc.tris, np.float32(sc.h) * np.float32(1.0 / 256))
    depth = header_depth(blob)
    log("  reachable 4-wide nodes", nodes, "depth", depth)
    assert 3 * depth + 1 <= 176  # traversed as a tree, not triangle by triangle


def chain(n=300, r=1.031, leg=5e-5, corner=(0.3, 0.3, 0.5)):
    """n nested right triangles sharing one corner, legs growing geometrically: the merged
    box of any two is the larger one's, so the clustering builder can only merge the two
    smallest clusters at each step and its binary tree is a chain of depth n - 1 (a 4-wide
    depth near n / 3, beyond what the traversal stack holds)."""
    c = np.array(corner, np.float32)
    v = []
    for i in range(n):
        L = np.float32(leg * r ** i)
        v += [c, c + np.array([L, 0, 0], np.float32), c + np.array([0, L, 0], np.float32)]
    return np.array(v, np.float32), np.arange(3 * n, dtype=np.int32).reshape(n, 3)


def header_depth(blob):
    return int(np.asarray(blob[12:16], np.uint8).view(np.int32)[0])


def test_deep_hierarchy_traced_exactly(R, orc):
    """A clustering tree deeper than the stack bound is recorded as such, and ray sampling
    and the vertex adjoint through it test every triangle: results equal the oracle's."""
    import torch
    from test_gpu_parity import compare_rays, gpu_pipeline, oracle_pipeline
    v, t = chain()
    pad = np.float32(1.0 / 16) * np.float32(1.0 / 256)
    blob = build(R, v, t, (16, 16, 16), 1.0 / 16, 1)
    check(blob, v, t, pad)
    depth = header_depth(blob)
    log("case: chain of %d nested triangles, PLOC 4-wide depth %d" % (len(t), depth))
    assert 3 * depth + 1 > 176
    sc = synth.Scene(v, t, (16, 16, 16), (0, 0, 0), 1.0 / 16, synth.jfa_offsets((16, 16, 16)), 2, 8, 2)
    G = gpu_pipeline(R, sc)
    assert header_depth(G["S"].bvh.cpu().numpy()) == depth
    O = oracle_pipeline(orc, sc)
    assert np.array_equal(G["band"], O["band"])
    compare_rays(G, O, O["vids"])
    S = G["S"]
    w = np.random.default_rng(2).normal(size=S.g.n).astype(np.float32)
    gg = S.backward(torch.from_numpy(w).cuda()).cpu().numpy()
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    go = orc.sdf_backward(w.astype(np.float64), O["hits"], O["argmin"], O["band"], orc.BVH(v, t, orc.hit_pad(g)),
                          v, t, g, sc.rays, 0)
    tol = 1e-3 * np.abs(go) + 1e-4 * np.abs(go).max()
    assert np.abs(go).max() > 0 and (np.abs(gg - go) <= tol).all()


def test_depth_fallback_equals_tree(R):
    """Marking a hierarchy as too deep (its header's depth) switches ray sampling and the
    vertex adjoint to testing every triangle, with bit-identical hits, distances and argmin
    records; the regular static hierarchy stays within the stack bound."""
    import torch
    sc = synth.scene_static(dims=(50, 25, 50), nprims=20, seed=3)
    sc.frames = 2
    log("case: static 50x25x50, tree vs every triangle")
    out = []
    for deep in (False, True):
        S = R.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames)
        S.voxelize()
        S.jfa()
        S.mask()
        S.build_bvh()
        torch.cuda.synchronize()
        d = header_depth(S.bvh.cpu().numpy())
        assert 0 < d and 3 * d + 1 <= 176
        if deep:
            S.bvh[12:16] = torch.tensor([200], dtype=torch.int32).view(torch.uint8).cuda()
        R.rtsdf_reset_accum(S.dmin, S.hits, S.argmin)
        for f in range(sc.frames):
            S.trace(f)
        S.combine()
        w = torch.from_numpy(np.random.default_rng(4).normal(size=S.g.n).astype(np.float32)).cuda()
        gv = S.backward(w)
        torch.cuda.synchronize()
        out.append((S.dmin.view(torch.int32).clone(), S.hits.clone(), S.argmin.clone(), gv.cpu().numpy()))
    for a, b in zip(out[0][:3], out[1][:3]):
        assert torch.equal(a, b)
    ga, gb = out[0][3], out[1][3]
    assert np.abs(ga).max() > 0 and (np.abs(ga - gb) <= 1e-5 * np.abs(ga).max()).all()
