"""The BVH blob validator used by the GPU tests, pinned on a hand-built blob: it accepts a
correct two-leaf hierarchy and rejects a shrunk box, a duplicated leaf, a wrong vertex and
an unused slot whose quantised box is not inverted."""
import numpy as np
import pytest

from bvh_check import NODE, TRI, check


def quantise(node, boxes):
    """Writes the quantised child boxes [(lo, hi) per slot, None for unused] into node."""
    used = [bx for bx in boxes if bx is not None]
    blo = np.min([bx[0] for bx in used], axis=0).astype(np.float32)
    bhi = np.max([bx[1] for bx in used], axis=0).astype(np.float32)
    node["o"] = blo
    exps, lo, hi = 0, [0, 0, 0], [0, 0, 0]
    for a in range(3):
        ext = float(bhi[a]) - float(blo[a])
        k = max(int(np.frexp(ext / 255.0)[1]), -126) if ext > 0 else -126
        exps |= (k + 127) << (8 * a)
        step = np.ldexp(1.0, k)
        for q, bx in enumerate(boxes):
            ql, qh = (255, 0) if bx is None else (
                int(np.clip(np.floor((float(bx[0][a]) - float(blo[a])) / step), 0, 255)),
                int(np.clip(np.ceil((float(bx[1][a]) - float(blo[a])) / step), 0, 255)))
            lo[a] |= ql << (8 * q)
            hi[a] |= qh << (8 * q)
    node["exps"], node["lo"], node["hi"] = exps, lo, hi


def blob(verts, tris, pad, shrink=False, dup=False, bad_vertex=False, open_slot=False, depth=1):
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
    boxes = [None] * 4
    nodes[0]["child"][:] = -2 ** 31
    for q, (f, n) in enumerate(ranges):
        boxes[q] = (lo[f:f + n].min(0), hi[f:f + n].max(0))
        nodes[0]["child"][q] = ~(f | ((n - 1) << 26))
    quantise(nodes[0], boxes)
    if shrink:   # child 0's high x plane one step lower than its triangles need
        w = int(nodes[0]["hi"][0])
        nodes[0]["hi"][0] = (w & ~0xFF) | max((w & 0xFF) - 1, 0)
    if open_slot:   # an unused slot whose quantised box is not inverted
        nodes[0]["lo"][0] = int(nodes[0]["lo"][0]) & ~(0xFF << 24)
    hdr = np.zeros(64, np.int32)
    hdr[0], hdr[1] = nt, 0
    hdr[2] = np.float32(pad).view(np.int32)
    hdr[3] = depth  # one node whose children are leaf ranges
    return np.concatenate([hdr.view(np.uint8), nodes.view(np.uint8), recs.view(np.uint8)])


def mesh():
    rng = np.random.default_rng(0)
    v = rng.uniform(0, 1, size=(12, 3)).astype(np.float32)
    t = np.arange(12, dtype=np.int32).reshape(4, 3)
    return v, t


def test_accepts_valid_blob():
    v, t = mesh()
    assert check(blob(v, t, 0.01), v, t, 0.01) == 1


@pytest.mark.parametrize("bad", ["shrink", "dup", "bad_vertex", "open_slot", "depth"])
def test_rejects_corrupt_blob(bad):
    v, t = mesh()
    with pytest.raises(AssertionError):
        check(blob(v, t, 0.01, **{bad: 2 if bad == "depth" else True}), v, t, 0.01)
