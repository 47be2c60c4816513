"""Host-side checks of a batch plan (no GPU): the layout the batched kernels index with.

The plan's bytes are decoded with numpy and every table is recomputed independently here:
voxel offsets (aligned, disjoint, covering each grid), hierarchy offsets, per-object JFA
offsets (equal to the single-object step list), the start-buffer parity, and for every JFA
pass the work-group prefix that the batched kernel searches, replayed to show that every
work-group decodes to an in-range tile of exactly one object.
"""
import numpy as np
import pytest

from paper_2210_06160_amd import synth

MAX_PASSES = 19
HEADER = np.dtype([("magic", "<u4"), ("nobj", "<i4"), ("max_passes", "<i4"), ("r0", "<i4"), ("total_vox", "<i8"),
                   ("total_verts", "<i8"), ("total_tris", "<i8"), ("bvh_bytes", "<u8"), ("plan_bytes", "<u8"),
                   ("device", "<u8"), ("pass_blocks", "<i4", (MAX_PASSES,)), ("total_tiles", "<i4"),
                   ("rest", "V%d" % (256 - 68 - 4 * MAX_PASSES))])
OBJECT = np.dtype([("n", "<i4", (3,)), ("org", "<f4", (3,)), ("h", "<f4"), ("band_vox", "<i4"), ("vox_off", "<i8"),
                   ("bvh_off", "<i8"), ("vert_off", "<i4"), ("tri_off", "<i4"), ("nv", "<i4"), ("nt", "<i4"),
                   ("nsteps", "<i4"), ("nhalf", "<i4"), ("k0", "<i4"), ("flip", "<i4"), ("beta", "<f4"),
                   ("bias", "<f4"), ("tile_off", "<i4"), ("r1", "<i4")])


@pytest.fixture(scope="module")
def R():
    import os
    from paper_2210_06160_amd import rtsdf
    if not os.path.exists(rtsdf.LIB_PATH):
        pytest.skip("librtsdf.so not built")
    return rtsdf


def decode(plan):
    raw = np.frombuffer(plan.host.raw, np.uint8)
    h = raw[:256].view(HEADER)[0]
    n = int(h["nobj"])
    p = 256
    objs = raw[p:p + OBJECT.itemsize * n].view(OBJECT)
    p += OBJECT.itemsize * n
    vox_prefix = raw[p:p + 8 * (n + 1)].view("<i8")
    p += 8 * (n + 1)
    tri_prefix = raw[p:p + 4 * (n + 1)].view("<i4")
    p += 4 * (n + 1)
    pass_prefix = raw[p:p + 4 * (n + 1) * MAX_PASSES].view("<i4").reshape(MAX_PASSES, n + 1)
    assert p + 4 * (n + 1) * MAX_PASSES == len(raw)
    return h, objs, vox_prefix, tri_prefix, pass_prefix


def find_object(prefix, n, i):
    """last o in [0, n) with prefix[o] <= i"""
    return int(np.searchsorted(prefix[:n], i, side="right") - 1)


def tuning():
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2210_06160_amd", "csrc",
                        "tuning.h")
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (RTSDF_\w+) (\d+)", open(path).read())}


WAVES, CHUNK = tuning()["RTSDF_JFA_WAVES"], tuning()["RTSDF_JFA_CHUNK"]


def z_tasks(nz, k):
    """z tasks of a pass: chunks of CHUNK lattice points of one residue class, or, when the
    classes are short, several whole classes per task -> (classes, chunks per class,
    classes per task, tasks)."""
    res = min(k, nz)
    mmax = -(-nz // k)
    per_res = -(-mmax // CHUNK)
    group = 1 if per_res > 1 else max(1, CHUNK // mmax)
    count = res * per_res if per_res > 1 else -(-res // group)
    return res, per_res, group, count


def chunk_len(nz, k):
    """Lattice points per chunk when classes are split: equal lengths, each <= CHUNK."""
    mmax = -(-nz // k)
    per_res = -(-mmax // CHUNK)
    return -(-mmax // per_res)


def jfa_blocks(n, k):
    nx, ny, nz = n
    return -(-(nx * ny) // (64 * WAVES)) * z_tasks(nz, k)[3]


def batch_scenes():
    v, t = synth.icosphere(1, 0.3, (0.5, 0.5, 0.5))
    objs = synth.scene_batch(nobj=5, seed=5, tri_range=(80, 3000), n_range=(12, 70))
    objs.append(synth.Scene(v, t, (20, 17, 1), (0, 0, 0.5), 0.05, synth.jfa_offsets((20, 17, 1), extra=2), 2, 8, 1))
    objs.append(synth.Scene(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), (5, 7, 3), (0, 0, 0), 0.2,
                            synth.jfa_offsets((5, 7, 3)), 2, 8, 1))
    objs.append(synth.Scene(v, t, (1, 1, 1), (0.4, 0.4, 0.4), 0.2, synth.jfa_offsets((1, 1, 1)), 1, 8, 1))
    return objs


def make_plan(R, scenes):
    recs = []
    for sc in scenes:
        extra = len(sc.steps) - len(synth.jfa_offsets(sc.dims))
        recs.append(R.make_object(sc.dims, sc.org, sc.h, len(sc.verts), len(sc.tris), sc.band, extra, sc.h / 2))
    return R.Plan(recs, upload=False)


@pytest.mark.parametrize("which", ["mixed", "full"])
def test_plan_tables(R, which):
    scenes = batch_scenes() if which == "mixed" else synth.scene_batch()
    plan = make_plan(R, scenes)
    h, objs, vox_prefix, tri_prefix, pass_prefix = decode(plan)
    n = len(scenes)
    assert h["magic"] == 0x52534442 and h["nobj"] == n
    # voxel layout: aligned, disjoint, each grid inside its range
    off = 0
    for o, sc in enumerate(scenes):
        N = int(np.prod(sc.dims))
        assert objs[o]["vox_off"] == off == vox_prefix[o] and off % 4096 == 0
        assert plan.offsets(o)[0] == off
        off += -(-N // 4096) * 4096
    assert vox_prefix[n] == off == h["total_vox"] == plan.sizes.voxels
    # vertices, triangles and hierarchies
    assert list(np.cumsum([0] + [len(s.tris) for s in scenes])) == list(tri_prefix)
    assert list(objs["vert_off"]) == list(np.cumsum([0] + [len(s.verts) for s in scenes])[:-1])
    b = 0
    for o, sc in enumerate(scenes):
        assert objs[o]["bvh_off"] == b and b % 256 == 0 and plan.offsets(o)[1] == b
        b += -(-R.rtsdf_bvh_bytes(len(sc.tris)) // 256) * 256
    assert b == h["bvh_bytes"] == plan.sizes.bvh_bytes
    tiles = np.cumsum([0] + [-(-len(s.tris) // 1024) for s in scenes])
    assert list(objs["tile_off"]) == list(tiles[:-1]) and h["total_tiles"] == tiles[-1]
    # JFA offsets and start-buffer parity
    for o, sc in enumerate(scenes):
        ob = objs[o]
        steps = [int(ob["k0"]) >> p if p < ob["nhalf"] else 1 for p in range(ob["nsteps"])]
        assert steps == list(sc.steps), (o, steps, sc.steps)
        assert ob["flip"] == ob["nsteps"] % 2
    assert h["max_passes"] == max(len(s.steps) for s in scenes) == plan.sizes.max_passes
    # per-pass work-group tables, replayed the way the batched kernel decodes them
    for p in range(h["max_passes"]):
        counts = [jfa_blocks(sc.dims, sc.steps[p]) if p < len(sc.steps) else 0 for sc in scenes]
        assert list(pass_prefix[p]) == list(np.cumsum([0] + counts))
        assert h["pass_blocks"][p] == sum(counts)
        seen = np.zeros(n, np.int64)
        rng = np.random.default_rng(p)
        total = int(h["pass_blocks"][p])
        sample = np.unique(np.concatenate([np.arange(min(total, 4096)), rng.integers(0, total, 4096),
                                           pass_prefix[p][1:-1], pass_prefix[p][1:-1] - 1]))
        for blk in sample[(sample >= 0) & (sample < total)]:
            o = find_object(pass_prefix[p], n, blk)
            sc = scenes[o]
            k = sc.steps[p]
            l = blk - pass_prefix[p][o]
            assert 0 <= l < counts[o]
            nx, ny, nz = sc.dims
            gc = -(-(nx * ny) // (64 * WAVES))
            bz = l // gc
            res, per_res, group, count = z_tasks(nz, k)
            assert bz < count
            assert (bz // per_res if per_res > 1 else bz * group) < res
            seen[o] += 1
        assert all(seen[o] > 0 for o in range(n) if counts[o] > 0)
    # mask / combine tiles: each lies in one object's range
    for t in range(0, int(h["total_vox"]), 4096 * 97):
        o = find_object(vox_prefix, n, t)
        assert vox_prefix[o] <= t < vox_prefix[o + 1]
    # workspace covers every stage
    need = max(R.rtsdf_voxelize_work_bytes(int(h["total_tris"])), max(R.rtsdf_bvh_work_bytes(len(s.tris)) for s in scenes))
    assert OBJECT.itemsize == 96
    assert plan.sizes.work_bytes >= need


def test_plan_validation(R):
    import ctypes
    lib = R.lib()
    g = R.make_grid((8, 8, 8), (0, 0, 0), 0.1)
    good = R.make_object((8, 8, 8), (0, 0, 0), 0.1, 3, 1, 2, 1, 0.05)
    nbytes = lib.rtsdf_batch_plan_bytes(1)
    host = ctypes.create_string_buffer(nbytes)
    sizes = R.BatchSizes()

    def plan(o, nb=nbytes, n=1):
        arr = (R.Object * 1)(o)
        return lib.rtsdf_batch_plan(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.cast(host, ctypes.c_void_p),
                                    ctypes.c_void_p(0x1000), nb, ctypes.byref(sizes))

    assert plan(good) == 0
    assert plan(good, nb=nbytes - 1) == -3
    assert plan(good, n=0) == -2
    bad = R.make_object((0, 8, 8), (0, 0, 0), 0.1, 3, 1, 2, 1, 0.05)
    assert plan(bad) == -2 and b"object 0" in lib.rtsdf_last_error()
    assert plan(R.make_object((8, 8, 8), (0, 0, 0), 0.1, 3, 1, 2, 9, 0.05)) == -2
    assert plan(R.make_object((8, 8, 8), (0, 0, 0), 0.1, 3, 1, 2, 1, float("nan"))) == -1
    assert plan(R.make_object((8, 8, 8), (0, 0, 0), 0.1, 0, 1, 2, 1, 0.05)) == -2
    assert lib.rtsdf_jfa_batched(None, ctypes.c_void_p(0x10), ctypes.c_void_p(0x20), None) == -1
    junk = ctypes.create_string_buffer(nbytes)
    assert lib.rtsdf_jfa_batched(ctypes.cast(junk, ctypes.c_void_p), ctypes.c_void_p(0x10),
                                 ctypes.c_void_p(0x20), None) == -1
    assert b"not a batch plan" in lib.rtsdf_last_error()


def test_jfa_tasks_cover_every_point_once():
    """The z tasks of a pass, decoded the way the pass kernel decodes them, visit every z of
    the grid exactly once (as lattice point m of residue class z mod k), for grids and
    offsets that give long classes split into chunks, short classes grouped, and offsets
    beyond the grid.  For the halving offsets of a grid whose classes are grouped, every
    task holds the same number of lattice points up to one class's (the XCDs run
    contiguous task ranges, so unequal tasks would leave some of them idle)."""
    for nz in (1, 2, 3, 7, 31, 32, 33, 64, 100, 200, 400, 1023):
        for k in sorted({1, 2, 3, 4, 8, 16, 31, 32, 64, 128, 256, 512, 1024, nz, max(1, nz // 2)}):
            res, per_res, group, count = z_tasks(nz, k)
            seen = np.zeros(nz, np.int64)
            for bz in range(count):
                if per_res > 1:
                    L = chunk_len(nz, k)
                    assert L <= CHUNK
                    r0 = bz // per_res
                    r1, mlo, mhi = r0 + 1, (bz - r0 * per_res) * L, (bz - r0 * per_res + 1) * L
                    rstep = 1
                else:
                    r0, r1, mlo, mhi, rstep = bz, res, 0, 1 << 31, count  # classes bz, bz + count, ...
                for r in range(r0, r1, rstep):
                    mcount = (nz - r + k - 1) // k
                    for m in range(mlo, min(mhi, mcount)):
                        seen[r + m * k] += 1
            assert (seen == 1).all(), (nz, k)
            if per_res == 1 and k & (k - 1) == 0 and 2 * k > nz // 2:
                work = [sum((nz - r + k - 1) // k for r in range(bz, res, count)) for bz in range(count)]
                assert max(work) - min(work) <= -(-nz // k), (nz, k, work)


NEAR_BLOCKS = 32  # rows k apart within this many work-groups keep the plain order


def pass_row(i, nx, ny, k):
    """Row of a plane at position i of a pass's row order: rows grouped by residue mod k
    (rho, rho + k, rho + 2k, ...) unless k = 1, k >= ny or rows k apart are near anyway."""
    if k * nx <= NEAR_BLOCKS * 64 * WAVES or k >= ny:
        return i
    c0, r = divmod(ny, k)
    split = r * (c0 + 1)
    if i < split:
        rho, j = divmod(i, c0 + 1)
    else:
        rho, j = divmod(i - split, c0)
        rho += r
    return rho + j * k


def test_jfa_row_order_is_a_permutation_grouping_residues():
    """The pass's row order visits every row of the plane once, and when it is not the plain
    order, rows of one residue class mod k follow each other in ascending order, so a row's
    y - k and y + k neighbour rows are the positions just before and after it."""
    for nx in (1, 7, 64, 100, 400, 1000):
        for ny in (1, 2, 5, 31, 64, 100, 200, 255, 401):
            for k in sorted({1, 2, 3, 8, 16, 32, 33, 64, 128, 256, max(1, ny // 2), ny, ny + 1}):
                rows = [pass_row(i, nx, ny, k) for i in range(ny)]
                assert sorted(rows) == list(range(ny)), (nx, ny, k)
                if rows == list(range(ny)):
                    continue
                for i, y in enumerate(rows):
                    if y + k < ny:
                        assert rows[i + 1] == y + k, (nx, ny, k, i)
                    if y - k >= 0:
                        assert rows[i - 1] == y - k, (nx, ny, k, i)
