"""The BVH blob validator used by the GPU tests, pinned on a hand-built blob: it accepts a
correct two-leaf hierarchy and rejects a shrunk box, a duplicated leaf, a wrong vertex and
an unused slot whose box is not the empty one."""
import numpy as np
import pytest

from bvh_check import NODE, TRI, check


def blob(verts, tris, pad, shrink=False, dup=False, bad_vertex=False, open_slot=False):
    nt = len(tris)
    nodes = np.zeros(max(nt - 1, 1), NODE)
    recs = np.zeros(nt, TRI)
    for p in range(nt):
        recs[p]["v"][:, :3] = verts[tris[p]]
        recs[p]["v"][0, 3] = np.int32(p).view(np.float32)
    if bad_vertex:
        recs[1]["v"][2, 0] += 0.5
    V = verts[tris]
    lo, hi = V.min(1) - 2 * pad, V.max(1) + 2 * pad
    ranges = [(0, 3), (3, 1)]
    if dup:
        ranges = [(0, 3), (2, 2)]
    nodes[0]["lo"][:] = np.inf
    nodes[0]["hi"][:] = -np.inf
    nodes[0]["child"][:] = -2 ** 31
    for q, (f, n) in enumerate(ranges):
        nodes[0]["lo"][:, q] = lo[f:f + n].min(0)
        nodes[0]["hi"][:, q] = hi[f:f + n].max(0)
        nodes[0]["child"][q] = ~(f | ((n - 1) << 26))
    if shrink:
        nodes[0]["hi"][0, 0] -= 0.1
    if open_slot:   # an unused slot whose box a ray could enter
        nodes[0]["lo"][:, 3] = 0.0
        nodes[0]["hi"][:, 3] = 1.0
    hdr = np.zeros(64, np.int32)
    hdr[0], hdr[1] = nt, 0
    hdr[2] = np.float32(pad).view(np.int32)
    return np.concatenate([hdr.view(np.uint8), nodes.view(np.uint8), recs.view(np.uint8)])


def mesh():
    rng = np.random.default_rng(0)
    v = rng.uniform(0, 1, size=(12, 3)).astype(np.float32)
    t = np.arange(12, dtype=np.int32).reshape(4, 3)
    return v, t


def test_accepts_valid_blob():
    v, t = mesh()
    assert check(blob(v, t, 0.01), v, t, 0.01) == 1


@pytest.mark.parametrize("bad", ["shrink", "dup", "bad_vertex", "open_slot"])
def test_rejects_corrupt_blob(bad):
    v, t = mesh()
    with pytest.raises(AssertionError):
        check(blob(v, t, 0.01, **{bad: True}), v, t, 0.01)
