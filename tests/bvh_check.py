"""Host-side decoder and validator of a BVH blob (the layout in csrc/internal.h).

A blob is valid when: the header holds the triangle count and the hit padding; the leaf
ranges reachable from the root partition the positions [0, nt) exactly once; every child
box, decoded from its 8-bit planes (origin + byte * 2^(e - 127) per axis, exactly in
binary64), contains the boxes of all triangles under it (widened by twice the padding, see
traverse.h); every unused slot of a reachable node holds low bytes 255 and high bytes 0;
and the triangle records are a permutation of the input triangles with their vertices;
and the header's depth equals the number of 4-wide nodes on the longest root-to-leaf path
(0 when the root is a leaf range).  Returns the number of reachable 4-wide nodes.
"""
import numpy as np

NODE = np.dtype([("o", "<f4", (3,)), ("exps", "<u4"), ("child", "<i4", (4,)), ("lo", "<u4", (3,)), ("hi", "<u4", (3,)),
                 ("unused", "<u4", (2,))])


def child_box(node, q):
    """Binary64 low and high corners of child q's quantised box."""
    e = np.array([(int(node["exps"]) >> (8 * a)) & 0xFF for a in range(3)])
    step = np.ldexp(1.0, e - 127)
    o = node["o"].astype(np.float64)
    lq = np.array([(int(node["lo"][a]) >> (8 * q)) & 0xFF for a in range(3)], np.float64)
    hq = np.array([(int(node["hi"][a]) >> (8 * q)) & 0xFF for a in range(3)], np.float64)
    return o + lq * step, o + hq * step
TRI = np.dtype([("v", "<f4", (3, 4))])
EMPTY = -2 ** 31


def leaf_range(code):
    c = ~int(code)
    return c & 0x3FFFFFF, (c >> 26) + 1


def check(blob, verts, tris, pad):
    raw = np.asarray(blob, np.uint8)
    nt = len(tris)
    hdr = raw[:256].view(np.int32)
    assert hdr[0] == nt, (hdr[0], nt)
    root = int(hdr[1])
    assert raw[8:12].view(np.float32)[0] == np.float32(pad)
    nnodes = max(nt - 1, 1)
    nodes = raw[256:256 + NODE.itemsize * nnodes].view(NODE)
    trirec = raw[256 + NODE.itemsize * nnodes:256 + NODE.itemsize * nnodes + TRI.itemsize * nt].view(TRI)
    if nt == 0:
        assert root == EMPTY
        return 0
    ids = trirec["v"][:, 0, 3].view(np.int32)
    assert np.array_equal(np.sort(ids), np.arange(nt)), "triangle records are not a permutation"
    V = np.asarray(verts, np.float32)[np.asarray(tris)[ids]]       # [nt, 3 vertices, 3]
    assert np.array_equal(trirec["v"][:, :, :3], V), "triangle records differ from the mesh"
    lo_t = V.min(axis=1) - np.float32(2 * pad)
    hi_t = V.max(axis=1) + np.float32(2 * pad)
    # post-order walk: subtree ranges of every reachable node
    rng = {}
    order, stack = [], [root]
    while stack:
        c = stack.pop()
        if c < 0:
            continue
        assert 0 <= c < nnodes and c not in rng, "node %d out of range or reached twice" % c
        rng[c] = None
        order.append(c)
        for ch in nodes[c]["child"]:
            if ch != EMPTY:
                stack.append(int(ch))

    def span(code):
        return leaf_range(code) if code < 0 else rng[code]

    covered = np.zeros(nt, np.int32)
    depth = {}
    for c in reversed(order):
        depth[c] = 1 + max([depth[int(ch)] for ch in nodes[c]["child"] if ch >= 0] or [0])
        lo, hi = None, None
        for q in range(4):
            ch = int(nodes[c]["child"][q])
            if ch == EMPTY:
                assert all((int(nodes[c]["lo"][a]) >> (8 * q)) & 0xFF == 255 and
                           (int(nodes[c]["hi"][a]) >> (8 * q)) & 0xFF == 0 for a in range(3)), \
                    "unused slot %d of node %d is not the inverted box" % (q, c)
                continue
            f, n = span(ch)
            if ch < 0:
                covered[f:f + n] += 1
            blo, bhi = child_box(nodes[c], q)
            assert (lo_t[f:f + n].min(axis=0) >= blo).all() and (hi_t[f:f + n].max(axis=0) <= bhi).all(), \
                "child box of node %d misses a triangle" % c
            lo = f if lo is None else min(lo, f)
            hi = f + n if hi is None else max(hi, f + n)
        rng[c] = (lo, hi - lo)
    if root < 0:
        f, n = leaf_range(root)
        covered[f:f + n] += 1
    assert (covered == 1).all(), "leaf ranges do not partition the triangles"
    assert int(hdr[3]) == (depth[root] if root >= 0 else 0), ("header depth", int(hdr[3]), depth.get(root, 0))
    if root >= 0:
        assert rng[root] == (0, nt)
    return len(order)
