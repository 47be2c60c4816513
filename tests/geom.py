"""Exact (binary64) geometry used by the tests as ground truth for the oracle's pins.

Closest point on a triangle follows the Voronoi-region case analysis of Ericson,
"Real-Time Collision Detection" (2005), section 5.1.5, written here for numpy arrays.
"""
import numpy as np


def closest_point_on_triangles(p, a, b, c):
    """p: [P,3]; a, b, c: [T,3] -> closest points [P,T,3] (binary64)."""
    p = np.asarray(p, np.float64)[:, None, :]
    a, b, c = (np.asarray(x, np.float64)[None, :, :] for x in (a, b, c))
    ab, ac, ap = b - a, c - a, p - a
    d1 = (ab * ap).sum(-1)
    d2 = (ac * ap).sum(-1)
    bp = p - b
    d3 = (ab * bp).sum(-1)
    d4 = (ac * bp).sum(-1)
    cp = p - c
    d5 = (ab * cp).sum(-1)
    d6 = (ac * cp).sum(-1)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    with np.errstate(divide="ignore", invalid="ignore"):
        denom = va + vb + vc
        v = vb / denom
        w = vc / denom
        out = a + ab * v[..., None] + ac * w[..., None]
        # edge regions
        vbc = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        e_bc = b + (c - b) * vbc[..., None]
        w_ac = d2 / (d2 - d6)
        e_ac = a + ac * w_ac[..., None]
        v_ab = d1 / (d1 - d3)
        e_ab = a + ab * v_ab[..., None]
    bc_reg = (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0)
    out = np.where(bc_reg[..., None], e_bc, out)
    ac_reg = (vb <= 0) & (d2 >= 0) & (d6 <= 0)
    out = np.where(ac_reg[..., None], e_ac, out)
    ab_reg = (vc <= 0) & (d1 >= 0) & (d3 <= 0)
    out = np.where(ab_reg[..., None], e_ab, out)
    c_reg = (d6 >= 0) & (d5 <= d6)
    out = np.where(c_reg[..., None], np.broadcast_to(c, out.shape), out)
    b_reg = (d3 >= 0) & (d4 <= d3)
    out = np.where(b_reg[..., None], np.broadcast_to(b, out.shape), out)
    a_reg = (d1 <= 0) & (d2 <= 0)
    out = np.where(a_reg[..., None], np.broadcast_to(a, out.shape), out)
    return out


def point_mesh_distance(points, verts, tris, chunk=256, max_dist=None):
    """Exact unsigned distance from each point to the triangle mesh (binary64).

    With `max_dist`, distances beyond it are only guaranteed to be > max_dist (triangles
    whose box is farther than max_dist from a chunk's box are skipped; +inf if none is
    left)."""
    points = np.asarray(points, np.float64)
    v = np.asarray(verts, np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    tlo = np.minimum(np.minimum(a, b), c)
    thi = np.maximum(np.maximum(a, b), c)
    out = np.empty(len(points))
    for s in range(0, len(points), chunk):
        p = points[s:s + chunk]
        sel = slice(None)
        if max_dist is not None:
            plo, phi = p.min(0) - max_dist, p.max(0) + max_dist
            sel = np.flatnonzero(((thi >= plo) & (tlo <= phi)).all(1))
            if len(sel) == 0:
                out[s:s + chunk] = np.inf
                continue
        q = closest_point_on_triangles(p, a[sel], b[sel], c[sel])
        out[s:s + chunk] = np.sqrt(((q - p[:, None, :]) ** 2).sum(-1)).min(1)
    return out


def voxel_centres(dims, org, h, vids=None):
    nx, ny, nz = dims
    if vids is None:
        vids = np.arange(nx * ny * nz)
    vids = np.asarray(vids, np.int64)
    i, j, k = vids % nx, (vids // nx) % ny, vids // (nx * ny)
    return np.stack([org[0] + h * (i + 0.5), org[1] + h * (j + 0.5), org[2] + h * (k + 0.5)], 1)


def unpack(ids):
    ids = np.asarray(ids, np.int64)
    return np.stack([ids & 1023, (ids >> 10) & 1023, (ids >> 20) & 1023], 1)
