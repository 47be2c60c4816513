"""Seeded synthetic scenes (inputs only; none of the method's arithmetic lives here).

The paper measures on a living-room scene that is not available here (section 3); these
generators stand in for it with meshes of the shapes and sizes its 400 x 200 x 400 ray
texture implies (section 2.1).  Every mesh is a list of float32 vertices and int32
triangles wound counter-clockwise when seen from outside (geometric normal
(v1 - v0) x (v2 - v0) points out).  Both the GPU path and the CPU oracle consume these
arrays unchanged.
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Scene:
    verts: np.ndarray          # float32 [V, 3]
    tris: np.ndarray           # int32 [T, 3]
    dims: tuple                # (nx, ny, nz)
    org: tuple                 # grid origin (world units)
    h: float                   # voxel size (world units)
    steps: list                # jump-flooding offsets, in order
    band: int                  # ray-mask width in voxels
    rays: int                  # rays per masked voxel per frame
    frames: int                # frames accumulated
    name: str = ""
    extra: dict = field(default_factory=dict)


def merge(meshes):
    vs, ts, off = [], [], 0
    for v, t in meshes:
        vs.append(np.asarray(v, np.float32))
        ts.append(np.asarray(t, np.int64) + off)
        off += len(v)
    if not vs:
        return np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32)
    return np.concatenate(vs).astype(np.float32), np.concatenate(ts).astype(np.int32)


def signed_volume(verts, tris):
    """Enclosed volume of a closed mesh; positive when the winding is outward."""
    v = np.asarray(verts, np.float64)
    a, b, c = v[tris[:, 0]], v[tris[:, 1]], v[tris[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def icosphere(subdiv, radius=1.0, centre=(0.0, 0.0, 0.0)):
    """Subdivided icosahedron with vertices on the sphere (10 * 4^s + 2 vertices)."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p),
         (0, 1, -p), (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, np.float64) / np.linalg.norm(x) for x in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    V = np.array(verts) * radius + np.asarray(centre, np.float64)
    return V.astype(np.float32), np.array(faces, np.int32)


def uv_sphere(radius, centre, nseg=32, nring=16, rot=None):
    """Latitude/longitude sphere: 2 poles + (nring - 1) rings; 2*nseg*(nring-1) triangles."""
    pts = [(0.0, 0.0, 1.0)]
    for r in range(1, nring):
        th = np.pi * r / nring
        for s in range(nseg):
            ph = 2.0 * np.pi * s / nseg
            pts.append((np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)))
    pts.append((0.0, 0.0, -1.0))
    V = np.array(pts, np.float64)
    bottom = len(pts) - 1

    def ring(r, s):
        return 1 + (r - 1) * nseg + (s % nseg)

    T = []
    for s in range(nseg):
        T.append((0, ring(1, s), ring(1, s + 1)))
    for r in range(1, nring - 1):
        for s in range(nseg):
            a, b = ring(r, s), ring(r, s + 1)
            c, d = ring(r + 1, s), ring(r + 1, s + 1)
            T += [(a, c, d), (a, d, b)]
    for s in range(nseg):
        T.append((bottom, ring(nring - 1, s + 1), ring(nring - 1, s)))
    if rot is not None:
        V = V @ rot.T
    V = V * radius + np.asarray(centre, np.float64)
    return V.astype(np.float32), np.array(T, np.int32)


def torus(R, r, centre, nmaj=24, nmin=12, rot=None):
    """Ring torus around the z axis (before rotation): nmaj * nmin * 2 triangles."""
    pts = []
    for i in range(nmaj):
        u = 2.0 * np.pi * i / nmaj
        for j in range(nmin):
            v = 2.0 * np.pi * j / nmin
            pts.append(((R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)))
    V = np.array(pts, np.float64)

    def idx(i, j):
        return (i % nmaj) * nmin + (j % nmin)

    T = []
    for i in range(nmaj):
        for j in range(nmin):
            a, b, c, d = idx(i, j), idx(i + 1, j), idx(i + 1, j + 1), idx(i, j + 1)
            T += [(a, b, c), (a, c, d)]
    if rot is not None:
        V = V @ rot.T
    V = V + np.asarray(centre, np.float64)
    return V.astype(np.float32), np.array(T, np.int32)


def box(half, centre, rot=None):
    """Closed box with half extents `half`: 8 vertices, 12 triangles."""
    hx, hy, hz = half
    V = np.array([[sx * hx, sy * hy, sz * hz] for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)],
                 np.float64)
    # vertex index = (sx>0) + 2 (sy>0) + 4 (sz>0)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    T = []
    for a, b, c, d in quads:
        T += [(a, b, c), (a, c, d)]
    if rot is not None:
        V = V @ rot.T
    V = V + np.asarray(centre, np.float64)
    return V.astype(np.float32), np.array(T, np.int32)


def random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def jfa_offsets(dims, extra=0):
    n = max(dims)
    k = 1
    while k < n:
        k *= 2
    out = []
    k //= 2
    while k >= 1:
        out.append(k)
        k //= 2
    return (out or [1]) + [1] * extra


def scene_tiny():
    """One icosphere (subdivision 1, 80 triangles, radius 0.3) centred in the unit cube,
    32^3 grid, offsets 16..1, 2-voxel mask, 16 rays, one frame."""
    v, t = icosphere(1, 0.3, (0.5, 0.5, 0.5))
    return Scene(v, t, (32, 32, 32), (0.0, 0.0, 0.0), 1.0 / 32, [16, 8, 4, 2, 1], 2, 16, 1,
                 name="icosphere80-32^3")


def torus_knot_tube(p=2, q=3, R=0.6, a=0.25, tube=0.08, nseg=500, nring=50, centre=(1.0, 0.5, 1.0)):
    """Tube of radius `tube` around the (p, q) torus knot with radii R, a, lying in the
    x-z plane (so its height is +-(a + tube) around centre[1]); nseg x nring vertices,
    2 nseg nring triangles.  Returns (verts, tris, normals) in binary64 before rounding."""
    phi = 2.0 * np.pi * np.arange(nseg) / nseg

    def curve(f):
        r = R + a * np.cos(q * f)
        return np.stack([r * np.cos(p * f), -a * np.sin(q * f), r * np.sin(p * f)], -1)

    def d1(f):
        r = R + a * np.cos(q * f)
        dr = -a * q * np.sin(q * f)
        return np.stack([dr * np.cos(p * f) - r * p * np.sin(p * f), -a * q * np.cos(q * f),
                         dr * np.sin(p * f) + r * p * np.cos(p * f)], -1)

    eps = 1e-4
    c = curve(phi)
    T = d1(phi)
    T /= np.linalg.norm(T, axis=1, keepdims=True)
    Tn = d1(phi + eps)
    Tn /= np.linalg.norm(Tn, axis=1, keepdims=True)
    N = Tn - T                      # Frenet normal (the knot's curvature never vanishes)
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    B = np.cross(T, N)
    th = 2.0 * np.pi * np.arange(nring) / nring
    nrm = (np.cos(th)[None, :, None] * N[:, None, :] + np.sin(th)[None, :, None] * B[:, None, :])
    V = (c[:, None, :] + tube * nrm).reshape(-1, 3) + np.asarray(centre)
    nrm = nrm.reshape(-1, 3)
    T_ = []
    for i in range(nseg):
        for j in range(nring):
            a0 = i * nring + j
            a1 = i * nring + (j + 1) % nring
            b0 = ((i + 1) % nseg) * nring + j
            b1 = ((i + 1) % nseg) * nring + (j + 1) % nring
            T_ += [(a0, b0, b1), (a0, b1, a1)]
    tris = np.array(T_, np.int32)
    if signed_volume(V, tris) < 0:
        tris = tris[:, [0, 2, 1]].copy()
    return V, tris, nrm


def deform_frames(V, nrm, frames, amplitude=0.02, freqs=(2.0, 3.0, 5.0), periods=(60.0, 45.0, 30.0), seed=1):
    """Vertices of each frame: V + n * sum_i (amplitude/3) sin(2 pi (f_i (u_i . V) + t/P_i) + phi_i)
    along the undeformed normals n, with unit u_i and phases phi_i from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(3, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
    out = np.empty((frames, len(V), 3), np.float32)
    for t in range(frames):
        d = np.zeros(len(V))
        for i in range(3):
            d += (amplitude / 3.0) * np.sin(2.0 * np.pi * (freqs[i] * (V @ u[i]) + t / periods[i]) + ph[i])
        out[t] = (V + nrm * d[:, None]).astype(np.float32)
    return out


def scene_deform(dims=(400, 200, 400), frames=60):
    """Deforming mesh over the box [0,2] x [0,1] x [0,2]: a (2,3) torus-knot tube (R 0.6,
    a 0.25, tube radius 0.08, 500 x 50 segments: 25,000 vertices, 50,000 triangles) centred
    at (1, 0.5, 1), displaced every frame by three sinusoids along its normals (amplitude
    0.02).  Offsets n/2..1 plus one extra pass of 1, 4-voxel mask, 4 rays per masked voxel,
    Eq. 1 decay with alpha 0.95.  `extra["frames"]` holds the per-frame vertices."""
    V, tris, nrm = torus_knot_tube()
    fr = deform_frames(V, nrm, frames)
    h = 2.0 / dims[0]
    return Scene(fr[0], tris, tuple(dims), (0.0, 0.0, 0.0), h, jfa_offsets(dims, extra=1), 4, 4, frames,
                 name="torus-knot-50k-deforming-%dx%dx%d" % tuple(dims), extra={"frames": fr, "alpha": 0.95})


def ellipsoid_sdf(points, semi_axes, centre, iters=64):
    """Exact signed distance (negative inside) from points [n, 3] to an axis-aligned
    ellipsoid, by bisection on the monotone root of sum_i (e_i y_i / (t + e_i^2))^2 = 1
    (Eberly, "Distance from a point to an ellipse, an ellipsoid, or a hyperellipsoid",
    2013); binary64.  Points exactly on a symmetry plane of the smallest axis are not
    handled specially (a grid offset by half a voxel never produces them)."""
    e = np.asarray(semi_axes, np.float64)
    y = np.abs(np.asarray(points, np.float64) - np.asarray(centre, np.float64))
    e2 = e * e
    lo = np.full(len(y), -e2.min() + 1e-300)
    hi = np.maximum(np.linalg.norm(y, axis=1) * e.max(), 1e-12)

    def G(t):
        return (((e * y) / (t[:, None] + e2)) ** 2).sum(1)

    while True:
        bad = G(hi) > 1.0
        if not bad.any():
            break
        hi[bad] *= 2.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        g = G(mid)
        lo = np.where(g > 1.0, mid, lo)
        hi = np.where(g > 1.0, hi, mid)
    t = 0.5 * (lo + hi)
    x = e2 * y / (t[:, None] + e2)
    d = np.linalg.norm(x - y, axis=1)
    inside = ((y / e) ** 2).sum(1) < 1.0
    return np.where(inside, -d, d)


_GRID_SDF_CACHE = {}


def _grid_ellipsoid_sdf(dims, h, semi_axes, centre):
    """ellipsoid_sdf at every voxel centre (x fastest), float32.  The distance depends on
    |p - centre| per axis only, so it is evaluated once per distinct offset triple."""
    key = (dims, h, tuple(semi_axes), tuple(centre))
    if key not in _GRID_SDF_CACHE:
        axes = [np.abs((np.arange(n) + 0.5) * h - c) for n, c in zip(dims, centre)]
        uniq = [np.unique(a, return_inverse=True) for a in axes]
        ux, uy, uz = (u[0] for u in uniq)
        Z, Y, X = np.meshgrid(uz, uy, ux, indexing="ij")
        pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
        d = ellipsoid_sdf(pts, semi_axes, (0.0, 0.0, 0.0)).reshape(len(uz), len(uy), len(ux))
        ix, iy, iz = (u[1] for u in uniq)
        _GRID_SDF_CACHE[key] = d[iz[:, None, None], iy[None, :, None], ix[None, None, :]].astype(np.float32).ravel()
    return _GRID_SDF_CACHE[key]


def shadow_setup(h, width=512, height=512, plane_y=0.1, light=(0.35, 1.0, 0.25), k=8.0, steps=64,
                 smax=0.05):
    """Receiver plane y = plane_y over [0,1]^2 seen by a width x height image, a fixed
    directional light, penumbra k, a fixed number of sphere-tracing steps, steps clamped
    to [h/2, smax], start one voxel off the receiver (section 2.4, 2.5.2, 2.5.3)."""
    l = np.asarray(light, np.float64)
    l = l / np.linalg.norm(l)
    return dict(width=width, height=height, x0=0.0, z0=0.0, dx=1.0 / width, dz=1.0 / height, y=plane_y,
                light=tuple(float(a) for a in l), k=k, steps=steps, smin=h / 2.0, smax=smax, t0=h)


def scene_world(extent=8.0, nprims=800, seed=7):
    """A scene larger than one grid covers well, for the clip map: the static scene's
    primitives (boxes, UV spheres, tori, log-normal scales with median 0.1) over the box
    [0,extent] x [0,1] x [0,extent] on a ground quad at y = 0.05.  Returns (verts, tris)."""
    rng = np.random.default_rng(seed)
    meshes = [(np.array([[0.0, 0.05, 0.0], [0.0, 0.05, extent], [extent, 0.05, extent], [extent, 0.05, 0.0]],
                        np.float32), np.array([[0, 1, 2], [0, 2, 3]], np.int32))]
    for _ in range(nprims):
        kind = rng.integers(0, 3)
        c = (rng.uniform(0.0, extent), rng.uniform(0.05, 1.0), rng.uniform(0.0, extent))
        s = rng.lognormal(np.log(0.1), 0.5)
        rot = random_rotation(rng)
        if kind == 0:
            meshes.append(box(s * rng.uniform(0.5, 1.0, size=3), c, rot))
        elif kind == 1:
            meshes.append(uv_sphere(s, c, rot=rot))
        else:
            meshes.append(torus(s, 0.35 * s, c, rot=rot))
    return merge(meshes)


DL_LIGHTS = ((0.35, 1.0, 0.25), (-0.5, 1.0, 0.2), (0.15, 1.0, -0.45))


def dl_setup(h, width=512, height=512, steps=128, smax=0.05, frame=0, key=0x5EED5EED):
    """The full shadow pass (sections 2.5.2, 3.2): the receiver of shadow_setup, three
    fixed directional lights, 128 steps capped at 0.05, the two-sample triangulation, the
    start jittered by up to one maximal step, and the march ended where it leaves the field's
    box.  Returns (base parameters, unit light
    directions, the pass options)."""
    p = shadow_setup(h, width=width, height=height, steps=steps, smax=smax)
    lights = [tuple(float(a) for a in np.asarray(v) / np.linalg.norm(v)) for v in DL_LIGHTS]
    return p, lights, dict(triangulate=True, jitter=smax, frame=frame, key=key, bounded=True)


def scene_grad(dims=(128, 128, 128), subdiv=5, image=512):
    """Differentiation workload: icosphere (subdivision 5: 10,242 vertices, 20,480
    triangles, radius 0.3) centred in the unit cube on a 128^3 grid; offsets 64..1; 2-voxel
    mask; 16 rays; one frame; running minimum.  Targets: the exact signed distance of the
    ellipsoid with semi-axes (0.35, 0.3, 0.25) at the voxel centres, and a 512 x 512
    image uniform in [0, 1) from default_rng(3); the soft shadow of shadow_setup()."""
    v, t = icosphere(subdiv, 0.3, (0.5, 0.5, 0.5))
    h = 1.0 / dims[0]
    target = _grid_ellipsoid_sdf(tuple(dims), h, (0.35, 0.3, 0.25), (0.5, 0.5, 0.5))
    timg = np.random.default_rng(3).uniform(0.0, 1.0, size=image * image).astype(np.float32)
    return Scene(v, t, tuple(dims), (0.0, 0.0, 0.0), h, jfa_offsets(dims), 2, 16, 1,
                 name="icosphere-20480-%dx%dx%d" % tuple(dims),
                 extra={"target": target, "target_img": timg,
                        "shadow": shadow_setup(h, width=image, height=image)})


def scene_batch(nobj=64, seed=2, tri_range=(1e3, 2e5), n_range=(32, 256)):
    """Many uneven objects, each on its own unit-cube grid: triangle budget T_o log-uniform
    on tri_range, grid side n_o = round(log-uniform on n_range), h = 1/n_o; each object is the
    union of 4 UV spheres / tori (random type, rotation and position, inside [0.1, 0.9]^3)
    tessellated so that the four together have about T_o triangles.  Offsets
    2^(ceil(log2 n)-1)..1 plus one extra pass of 1, 4-voxel mask, 8 rays, one frame."""
    rng = np.random.default_rng(seed)
    out = []
    for o in range(nobj):
        T = float(np.exp(rng.uniform(np.log(tri_range[0]), np.log(tri_range[1]))))
        n = int(round(float(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))))
        meshes = []
        for _ in range(4):
            kind = int(rng.integers(0, 2))
            s = float(rng.uniform(0.08, 0.17))
            ext = s if kind == 0 else 1.35 * s
            c = rng.uniform(0.1 + ext, 0.9 - ext, size=3)
            rot = random_rotation(rng)
            m = max(3, int(round(np.sqrt(T / 4.0 / 4.0))))  # 4 m^2 triangles per primitive
            if kind == 0:
                meshes.append(uv_sphere(s, c, nseg=2 * m, nring=m + 1, rot=rot))
            else:
                meshes.append(torus(s, 0.35 * s, c, nmaj=2 * m, nmin=m, rot=rot))
        v, t = merge(meshes)
        dims = (n, n, n)
        out.append(Scene(v, t, dims, (0.0, 0.0, 0.0), 1.0 / n, jfa_offsets(dims, extra=1), 4, 8, 1,
                         name="object%02d-%d-tris-%d^3" % (o, len(t), n)))
    return out


def scene_static(dims=(400, 200, 400), nprims=200, seed=0):
    """Paper-shaped static scene over the box [0,2] x [0,1] x [0,2]: a ground quad at
    y = 0.05 (on a voxel face at the full resolution) plus `nprims` boxes, UV spheres and
    tori at uniform random positions with log-normal scales (median 0.1 = 0.05 of the box
    extent, sigma 0.5).  Offsets n/2..1 plus one extra pass of 1, 4-voxel mask, 8 rays per
    voxel per frame, 16 frames.  `dims` may be reduced (same world box) for fast tests."""
    rng = np.random.default_rng(seed)
    meshes = []
    g = np.array([[0.0, 0.05, 0.0], [0.0, 0.05, 2.0], [2.0, 0.05, 2.0], [2.0, 0.05, 0.0]], np.float32)
    meshes.append((g, np.array([[0, 1, 2], [0, 2, 3]], np.int32)))
    for _ in range(nprims):
        kind = rng.integers(0, 3)
        c = (rng.uniform(0.0, 2.0), rng.uniform(0.05, 1.0), rng.uniform(0.0, 2.0))
        s = rng.lognormal(np.log(0.1), 0.5)
        rot = random_rotation(rng)
        if kind == 0:
            meshes.append(box(s * rng.uniform(0.5, 1.0, size=3), c, rot))
        elif kind == 1:
            meshes.append(uv_sphere(s, c, rot=rot))
        else:
            meshes.append(torus(s, 0.35 * s, c, rot=rot))
    v, t = merge(meshes)
    h = 2.0 / dims[0]
    return Scene(v, t, tuple(dims), (0.0, 0.0, 0.0), h, jfa_offsets(dims, extra=1), 4, 8, 16,
                 name="ground+%d-prims-%dx%dx%d" % (nprims, *dims))
