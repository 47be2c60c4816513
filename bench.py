"""Benchmark: the RTSDF static hot path on a 400 x 200 x 400 grid (one MI355X).

One step = voxelize -> 10 jump-flooding passes -> ray mask -> LBVH build -> 16 frames of
ray sampling (8 rays per masked voxel) -> combine, on a synthetic scene shaped like the
paper's (ground plane + 200 boxes / spheres / tori, ~102k triangles) whose triangles are
already resident in HBM.  `value` is whole-field SDF voxels per second (32,000,000 grid
points per step); ray throughput, per-stage times, the roofline of the dominant kernel and
the CPU oracle baseline are reported beside it.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU ceiling from the unit counts: 256 CUs x 128 FP32 lanes per clock x 2.4 GHz =
# 78.6 T lane-ops/s, the published FP32 vector rate (157.3 TFLOP/s) counted one FMA per lane
# op.  The VALU probe (libvalupeak.so) shows which instructions issue at that rate (wave64
# in 2 clocks: v_fma_f32, v_add_u32, ...) and which at half of it (4 clocks: v_mad_u32_u24,
# v_min3_i32, v_dot2_i32_i16, ...); it is run live and reported beside the roofline.
ALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12  # T lane-ops/s
ALU_PEAK_SINGLE_RATE_TOPS = 256 * 64 * 2.4e9 / 1e12  # ... for the half-rate instructions
# Algorithmic lane-ops per ray of the method, independent of the hierarchy's width: about
# 1.05 Philox4x32-10 calls per direction (Marsaglia's rejection accepts pi/4 per pair, two
# pairs per call) x ~100 integer ops, 2 log2(T) ~ 34 box tests of a binary hierarchy over
# T ~ 1e5 triangles x ~20 flops, and ~8.6 triangle tests x ~30 flops.
OPS_PER_RAY = 1.05 * 100 + 34 * 20 + 8.6 * 30


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-deform", action="store_true", help="skip the deforming-mesh (graph) measurement")
    p.add_argument("--no-grad", action="store_true", help="skip the gradient-workload measurement")
    p.add_argument("--no-batch", action="store_true", help="skip the batched-objects measurement")
    p.add_argument("--no-two-level", action="store_true", help="skip the two-level (coarse/fine) measurement")
    p.add_argument("--no-dl", action="store_true", help="skip the full shadow pass measurement")
    p.add_argument("--no-clipmap", action="store_true", help="skip the clip-map measurement")
    p.add_argument("--no-tables", action="store_true", help="skip the Tables 3-4 re-run")
    p.add_argument("--no-valu", action="store_true", help="skip the VALU issue-rate probe")
    p.add_argument("--no-jfa-passes", action="store_true", help="skip the per-pass jump-flooding timings")
    p.add_argument("--only", choices=["static", "deform", "grad", "batch", "two_level", "tables", "dl", "clipmap",
                                      "valu", "jfa"],
                   help="run one workload alone and print its record (for profiling)")
    p.add_argument("--cpu-sample", type=int, default=4000000,
                   help="masked voxels ray-sampled by the oracle (about 6 s on 16 host cores)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy three times (to scale HBM counters)")
    return p.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "raysample_static_400x200x400_counters.md")
TRAFFIC_SOURCES = ["raysample.hip", "traverse.h", "sampling.h", "lbvh.hip", "layout.h", "tuning.h"]


def recorded_traffic():
    """HBM-side bytes per ray-sampling dispatch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (scaled by the plain-copy calibration), or None when the kernel
    sources have changed since those counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    csrc = os.path.join(ROOT, "paper_2210_06160_amd", "csrc")
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in TRAFFIC_SOURCES)).hexdigest()
    if fields.get("source_sha256") != sha or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


class StageTimer:
    """HIP events on the stream the kernels are launched on (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch
        self.events = []

    def mark(self, name):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.events.append((name, e))

    def durations(self):
        out = {}
        for (n0, e0), (n1, e1) in zip(self.events[:-1], self.events[1:]):
            out[n1] = out.get(n1, 0.0) + e0.elapsed_time(e1)
        return out


def gpu_step(S, rtsdf, timer):
    timer.mark("start")
    S.voxelize()
    timer.mark("voxelize")
    S.jfa()
    timer.mark("jfa")
    S.mask()
    timer.mark("mask")
    S.build_bvh()
    timer.mark("bvh")
    rtsdf.rtsdf_reset_accum(S.dmin, S.hits, S.argmin)
    timer.mark("reset")
    for f in range(S.frames):
        S.trace(f)
        timer.mark("raysample")
    S.combine()
    timer.mark("combine")


def deform_bench(torch, rtsdf, synth):
    """Deforming torus knot (50k triangles) on the same grid: 60 frames, each re-voxelized,
    re-flooded, re-masked, BVH rebuilt, 4 rays per masked voxel, Eq. 1 decay; the chain of
    frames >= 1 is one HIP graph recorded once and replayed per frame with the frame index
    in device memory (eager chain timed beside it)."""
    sc = synth.scene_deform()
    D = rtsdf.DeformSDF(sc.extra["frames"], sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays,
                        sc.extra["alpha"])
    for f in range(sc.frames):  # warm-up, eager
        D.frame(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(sc.frames):
        D.frame(f)
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) / sc.frames
    D.capture()
    for f in range(sc.frames):
        D.replay(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(sc.frames):
        D.replay(f)
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / sc.frames
    N = D.g.n
    return {"workload": sc.name, "frames": sc.frames, "triangles": int(len(sc.tris)),
            "ms_per_frame_graph": round(graph * 1e3, 3), "ms_per_frame_eager": round(eager * 1e3, 3),
            "sdf_voxels_per_s_graph": round(N / graph, 1), "masked_voxels_last_frame": int(D.band_count.item())}


def two_level_bench(torch, rtsdf, synth, steps=3):
    """Two-level field (sections 2.3, 2.5.1): the static scene flooded at 200 x 100 x 200 and
    traced at 400 x 200 x 400 (ratio 2, 2-coarse-voxel mask, 8 rays x 16 frames), and the
    deforming knot the same way (60 frames, Eq. 1 decay, every frame a replayed HIP graph).
    Voxel rates count points of the traced 400 x 200 x 400 field."""
    sc = synth.scene_static(dims=(200, 100, 200))
    sc.band = 2
    S = rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames, ratio=2)
    gpu_step(S, rtsdf, StageTimer(torch))
    torch.cuda.synchronize()
    timers = [StageTimer(torch) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        gpu_step(S, rtsdf, timers[k])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    stages = {}
    for tm in timers:
        for k, v in tm.durations().items():
            stages[k] = stages.get(k, 0.0) + v / steps
    band = int(S.band_count.item())
    Nf = S.gf.n
    out = {"static": {"workload": sc.name + "-ratio-2", "traced_grid": [S.gf.nx, S.gf.ny, S.gf.nz],
                      "ms_per_step": round(ms, 3), "sdf_voxels_per_s": round(Nf / (ms / 1e3), 1),
                      "masked_fine_voxels": band,
                      "rays_per_s": round(band * sc.rays * sc.frames / (stages["raysample"] / 1e3), 1),
                      "stages_ms": {k: round(v, 4) for k, v in stages.items()}}}
    del S
    sd = synth.scene_deform(dims=(200, 100, 200))
    sd.band = 2
    D = rtsdf.DeformSDF(sd.extra["frames"], sd.tris, sd.dims, sd.org, sd.h, sd.steps, sd.band, sd.rays,
                        sd.extra["alpha"], ratio=2)
    for f in range(sd.frames):
        D.frame(f)
    D.capture()
    for f in range(sd.frames):
        D.replay(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(sd.frames):
        D.replay(f)
    torch.cuda.synchronize()
    graph = (time.perf_counter() - t0) / sd.frames
    out["deform"] = {"workload": sd.name + "-ratio-2", "frames": sd.frames,
                     "ms_per_frame_graph": round(graph * 1e3, 3),
                     "sdf_voxels_per_s_graph": round(D.gf.n / graph, 1),
                     "masked_fine_voxels_last_frame": int(D.band_count.item())}
    return out


# GPU timings (ms) the paper reports on its own scene and GPU (RTX 2080 Ti): Table 3
# (V, JF, RT per size and rays per texel x, mask distance d = 0.1) and Table 4 (RT of size M
# per x and d).  Context beside the re-run, not a target.
PAPER_TABLE3 = {"S": {"V": 0.49, "JF": 0.28, "RT": {0: 0.14, 1: 0.16, 5: 0.71, 10: 1.41}},
                "M": {"V": 0.49, "JF": 2.37, "RT": {0: 0.55, 1: 1.41, 5: 4.51, 10: 8.36}},
                "L": {"V": 1.12, "JF": 21.89, "RT": {0: 3.98, 1: 9.12, 5: 26.56, 10: 48.32}}}
PAPER_TABLE4 = {1: {0.01: 0.8, 0.05: 1.28, 0.1: 1.63, 0.5: 3.12, "inf": 4.08},
                5: {0.01: 1.43, 0.05: 3.17, 0.1: 4.82, 0.5: 11.71, "inf": 16.15},
                10: {0.01: 2.18, 0.05: 5.41, 0.1: 8.36, 0.5: 22.25, "inf": 30.69},
                15: {0.01: 3.17, 0.05: 7.7, 0.1: 12.42, 0.5: 32.7, "inf": 46.0}}
TABLE_SIZES = {"S": 64, "M": 128, "L": 256}  # coarse side; the fine side is twice it


def mask_vox(d, h):
    """Mask width in whole coarse voxels for a world distance d (infinity: every point)."""
    return 2048 if d == "inf" else int(round(d / h))


def table_frame(D, rtsdf, timer, f, x, band):
    """One frame of the two-level dynamic chain of a static mesh (hierarchy built once):
    V = voxelize, JF = all jump-flooding passes, RT = mask + x rays per masked fine point +
    Eq. 1 combine (x = 0: mask and combine only)."""
    v = D.verts[0]
    timer.mark("start")
    rtsdf.rtsdf_voxelize(v, D.tris, D.g, D.seeds, D.work)
    timer.mark("V")
    out = rtsdf.rtsdf_jfa(D.seeds, D.scratch, D.g, D.steps)
    timer.mark("JF")
    rtsdf.rtsdf_band_refined(out, D.g, D.ratio, band, D.band_list, D.band_count, D.work)
    timer.mark("mask")
    if x > 0:
        rtsdf.rtsdf_raysample(D.bvh, D.gf, D.band_list, D.band_count, x, D.rng_key, f, D.dmin, D.hits, D.ray_work)
        timer.mark("rays")
    rtsdf.rtsdf_combine_refined(out, D.dmin, D.hits, D.g, D.ratio, band, D.beta, D.bias, rtsdf.DECAY, D.fine,
                                alpha=D.alpha, first_frame=(f == 0), consume=True, state=D.state)
    timer.mark("combine")


def tables_bench(torch, rtsdf, synth, reps=7):
    """Tables 3 and 4 re-run on this GPU with the static scene generator over the cube
    [0,2]^3 (ground plane + 200 primitives): sizes S/M/L flood 64^3/128^3/256^3 and trace
    twice the resolution; Table 3 at d = 0.1 for x in {0, 1, 5, 10}, Table 4 at size M for
    x in {1, 5, 10, 15} and d in {0.01, 0.05, 0.1, 0.5, inf}.  Medians over `reps` frames after
    one warm-up frame (sustained load can slow single frames for a while)."""
    def run(D, x, band):
        table_frame(D, rtsdf, StageTimer(torch), 0, x, band)
        timers = [StageTimer(torch) for _ in range(reps)]
        for k in range(reps):
            table_frame(D, rtsdf, timers[k], k + 1, x, band)
        torch.cuda.synchronize()
        per = {}
        for tm in timers:
            for k, v in tm.durations().items():
                per.setdefault(k, []).append(v)
        st = {k: statistics.median(v) for k, v in per.items()}
        rt = st["mask"] + st.get("rays", 0.0) + st["combine"]
        return {"V": round(st["V"], 4), "JF": round(st["JF"], 4), "RT": round(rt, 4),
                "mask_ms": round(st["mask"], 4), "rays_ms": round(st.get("rays", 0.0), 4),
                "combine_ms": round(st["combine"], 4), "masked_fine_points": int(D.band_count.item())}

    out = {"table3": {}, "table4": {}}
    for size, n in TABLE_SIZES.items():
        sc = synth.scene_static(dims=(n, n, n))
        band = mask_vox(0.1, sc.h)
        D = rtsdf.DeformSDF(sc.verts[None], sc.tris, sc.dims, sc.org, sc.h, sc.steps, band, 15, ratio=2,
                            bvh_method=rtsdf.BVH_PLOC)
        t0 = StageTimer(torch)
        t0.mark("start")
        rtsdf.rtsdf_build_bvh(D.verts[0], D.tris, D.gf, D.bvh, D.work, D.bvh_method)
        t0.mark("bvh")
        torch.cuda.synchronize()
        rows = {"coarse": n, "fine": 2 * n, "band_vox": band, "triangles": int(len(sc.tris)),
                "bvh_ms_once": round(t0.durations()["bvh"], 4), "x": {}}
        for x in (0, 1, 5, 10):
            rows["x"][x] = run(D, x, band)
            rows["x"][x]["paper_RT"] = PAPER_TABLE3[size]["RT"][x]
        rows["paper_V"], rows["paper_JF"] = PAPER_TABLE3[size]["V"], PAPER_TABLE3[size]["JF"]
        out["table3"][size] = rows
        if size == "M":
            for x in (1, 5, 10, 15):
                out["table4"][x] = {}
                for d in (0.01, 0.05, 0.1, 0.5, "inf"):
                    r = run(D, x, mask_vox(d, sc.h))
                    out["table4"][x][str(d)] = {"RT": r["RT"], "rays_ms": r["rays_ms"], "band_vox": mask_vox(d, sc.h),
                                                "masked_fine_points": r["masked_fine_points"],
                                                "paper_RT": PAPER_TABLE4[x][d]}
        del D
        torch.cuda.empty_cache()
    return out


def dl_bench(torch, rtsdf, synth, reps=20):
    """The full shadow pass (sections 2.5.2, 3.2) over the 128^3 ellipsoid field: three
    lights, 128 steps capped at 0.05, two-sample triangulation, jittered start; 512^2 forward
    and adjoint, and a 1920 x 1080 forward.  Medians of `reps` launches (HIP events)."""
    sc = synth.scene_grad()
    g = rtsdf.make_grid(sc.dims, sc.org, sc.h)
    fine = torch.from_numpy(sc.extra["target"].astype("float32")).cuda()
    out = {"field": "ellipsoid SDF on 128^3", "lights": 3, "steps": 128, "triangulate": True}

    def med(fn):
        ts = []
        for it in range(reps + 2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            if it >= 2:
                ts.append(a.elapsed_time(b))
        return statistics.median(ts)

    for w, hgt, bwd in ((512, 512, True), (1920, 1080, False)):
        p, lights, kw = synth.dl_setup(sc.h, width=w, height=hgt)
        s = rtsdf.make_shadow_ex(rtsdf.make_shadow(**p), lights, **kw)
        img = torch.empty(len(lights), hgt, w, device="cuda")
        fwd_ms = med(lambda: rtsdf.rtsdf_shadow_forward_ex(fine, g, s, img))
        # pixel-light marches per second (a bounded march may end before its 128 steps)
        rec = {"fwd_ms": round(fwd_ms, 4), "marches_per_s_fwd": round(len(lights) * w * hgt / (fwd_ms / 1e3), 1)}
        if bwd:
            gi = torch.ones_like(img)
            gf = torch.zeros_like(fine)
            rec["bwd_ms"] = round(med(lambda: rtsdf.rtsdf_shadow_backward_ex(fine, g, s, gi, gf)), 4)
        out["%dx%d" % (w, hgt)] = rec
    return out


def clipmap_bench(torch, rtsdf, synth, reps=5):
    """A clip map around a camera in a scene larger than one grid (an 8 x 1 x 8 box, 800
    primitives): 4 levels of 128^3 with voxels 1/64 .. 1/8 (level 3 spans 16 units), built
    by the batched chain (2-voxel masks, 8 rays, one frame), then the full shadow pass over
    it (1920 x 1080, three lights, 128 steps, a receiver patch of 4 x 4 units around the
    camera).  Beside it, the same chain on one grid covering the box at the finest voxel size
    (512 x 128 x 512).  Medians of `reps` (HIP events)."""
    import numpy as np
    v, t = synth.scene_world()
    cam = (4.0, 0.4, 4.0)
    C = rtsdf.ClipMapSDF(v, t, cam, 1.0 / 64, 128, 4, band=2, rays=8)

    def med(fn):
        ts = []
        for it in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            if it:
                ts.append(a.elapsed_time(b))
        return statistics.median(ts)

    build = med(C.run)
    p, lights, kw = synth.dl_setup(1.0 / 64, width=1920, height=1080)
    p.update(x0=2.0, z0=2.0, dx=4.0 / 1920, dz=4.0 / 1080)
    s = rtsdf.make_shadow_ex(rtsdf.make_shadow(**p), lights, **kw)
    img = torch.empty(3, 1080, 1920, device="cuda")
    dl = med(lambda: rtsdf.rtsdf_shadow_forward_clip(C.plan, C.fine, s, img))
    vox = sum(g.nx * g.ny * g.nz for g in C.grids)
    out = {"workload": "world 8x1x8, %d triangles, camera %s" % (len(t), list(cam)), "levels": 4, "n": 128,
           "h0": 1.0 / 64, "voxels": vox, "build_ms": round(build, 3), "dl_1920x1080x3_ms": round(dl, 3),
           "lit_fraction": round(float((img == 1).float().mean().item()), 4)}
    del C
    torch.cuda.empty_cache()
    S = rtsdf.StaticSDF(v, t, (512, 128, 512), (0.0, 0.0, 0.0), 1.0 / 64, synth.jfa_offsets((512, 128, 512), extra=1),
                        2, 8, 1)
    out["single_grid_512x128x512"] = {"voxels": 512 * 128 * 512, "build_ms": round(med(S.run), 3)}
    return out


def grad_bench(torch, rtsdf, synth, reps=20):
    """Gradient workload (icosphere of 20,480 triangles on 128^3, 16 rays, 512^2 soft shadow):
    forward = the SDF chain + shadow image + loss, backward = shadow adjoint + SDF term +
    vertex adjoint.  Medians over `reps` repetitions after 3 warm-ups, HIP events on the
    launch stream."""
    import statistics
    sc = synth.scene_grad()
    # an optimisation loop rebuilds the hierarchy every step: the fast-to-build tree
    S = rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames,
                        bvh_method=rtsdf.BVH_LBVH)
    sh = rtsdf.make_shadow(**sc.extra["shadow"])
    tgt = torch.from_numpy(sc.extra["target"].astype("float32")).cuda()
    timg = torch.from_numpy(sc.extra["target_img"]).cuda().reshape(sh.height, sh.width)
    img = torch.empty(sh.height, sh.width, dtype=torch.float32, device="cuda")
    gverts = torch.zeros_like(S.verts)
    rec = {k: [] for k in ("sdf_fwd", "shadow_fwd", "loss", "shadow_bwd", "vertex_bwd", "fwd", "bwd")}
    for it in range(reps + 3):
        T = StageTimer(torch)
        T.mark("start")
        fine = S.run()
        T.mark("sdf_fwd")
        rtsdf.rtsdf_shadow_forward(fine, S.gf, sh, img)
        T.mark("shadow_fwd")
        loss = ((fine - tgt) ** 2).sum() + ((img - timg) ** 2).sum()
        T.mark("loss")
        gfine = 2.0 * (fine - tgt)
        rtsdf.rtsdf_shadow_backward(fine, S.gf, sh, 2.0 * (img - timg), gfine)
        T.mark("shadow_bwd")
        gverts.zero_()
        S.backward(gfine, gverts)
        T.mark("vertex_bwd")
        torch.cuda.synchronize()
        if it >= 3:
            d = T.durations()
            for k in ("sdf_fwd", "shadow_fwd", "loss", "shadow_bwd", "vertex_bwd"):
                rec[k].append(d[k])
            rec["fwd"].append(d["sdf_fwd"] + d["shadow_fwd"] + d["loss"])
            rec["bwd"].append(d["shadow_bwd"] + d["vertex_bwd"])
    med = {k: statistics.median(v) for k, v in rec.items()}
    n = int(S.band_count.item())
    return {"workload": sc.name + "-shadow-%dx%d" % (sh.width, sh.height), "reps": reps,
            "ms": {k: round(v, 4) for k, v in med.items()}, "bwd_over_fwd": round(med["bwd"] / med["fwd"], 4),
            "masked_voxels": n, "loss": float(loss.item()),
            "shadow_samples_per_s_fwd": round(sh.width * sh.height * sh.steps / (med["shadow_fwd"] / 1e3), 1)}


def batch_bench(torch, rtsdf, synth, reps=20):
    """64 uneven objects (grids 32^3..256^3, 1k..200k triangles): the batched chain (one
    launch per stage and per JFA pass) against the plain loop of 64 single-object chains on
    the same stream; then the batched vertex adjoint against 64 looped adjoint calls.  Wall
    time around each whole chain (host launch cost included), medians over `reps`."""
    import statistics
    scenes = synth.scene_batch()
    B = rtsdf.BatchSDF(scenes, rays=8)
    singles = [rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, 8, 1, obj=o)
               for o, sc in enumerate(scenes)]
    grad = torch.randn(B.fine.numel(), device="cuda")
    grads = [B.view(grad, o).contiguous() for o in range(len(scenes))]
    gv = torch.zeros_like(B.verts)
    gvs = [torch.zeros_like(S.verts) for S in singles]

    def timed(fn):
        out = []
        for it in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if it:
                out.append(time.perf_counter() - t0)
        return statistics.median(out)

    def plain():
        for S in singles:
            S.run()

    def plain_bwd():
        for S, gs, gvo in zip(singles, grads, gvs):
            gvo.zero_()
            S.backward(gs, gvo)

    def batched_bwd():
        gv.zero_()
        B.backward(grad, gv)

    t_batch = timed(B.run)
    t_plain = timed(plain)
    tb_bwd = timed(batched_bwd)
    tp_bwd = timed(plain_bwd)
    T = StageTimer(torch)
    T.mark("start")
    B.voxelize()
    T.mark("voxelize")
    B.jfa()
    T.mark("jfa")
    B.mask()
    T.mark("mask")
    B.build_bvh()
    T.mark("bvh")
    rtsdf.rtsdf_reset_accum(B.dmin, B.hits, B.argmin)
    T.mark("reset")
    B.trace(0)
    T.mark("raysample")
    B.combine()
    T.mark("combine")
    torch.cuda.synchronize()
    masked = int(B.band_count.item())
    voxels = sum(int(S.g.n) for S in singles)
    return {"workload": "%d objects, %d triangles, %d grid points" % (len(scenes), int(B.tris.shape[0]), voxels),
            "ms_batched": round(t_batch * 1e3, 3), "ms_plain_loop": round(t_plain * 1e3, 3),
            "speedup": round(t_plain / t_batch, 3), "sdf_voxels_per_s_batched": round(voxels / t_batch, 1),
            "rays_per_s_batched": round(masked * 8 / (T.durations()["raysample"] / 1e3), 1),
            "stages_ms_batched": {k: round(v, 4) for k, v in T.durations().items()},
            "bwd_ms_batched": round(tb_bwd * 1e3, 3), "bwd_ms_plain_loop": round(tp_bwd * 1e3, 3),
            "bwd_speedup": round(tp_bwd / tb_bwd, 3), "masked_voxels": masked}


def valu_peak(torch, blocks=8192, iters=1024, reps=3):
    """Measured VALU issue rate: the probe library's kernels issue blocks x 256 threads x
    iters x 16 instructions of one kind per lane; lane-ops/s = that count / the launch's
    median duration (HIP events on the launch stream)."""
    import ctypes
    from paper_2210_06160_amd import build as hb
    L = ctypes.CDLL(hb.PROBE_LIB)
    L.valu_peak_launch.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                                   ctypes.c_void_p, ctypes.c_void_p]
    L.valu_peak_name.restype = ctypes.c_char_p
    L.valu_peak_shape.restype = ctypes.c_char_p
    per_trip = L.valu_peak_per_trip()
    sink = torch.zeros(256, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"blocks": blocks, "threads_per_block": 256, "iters": iters, "per_trip": per_trip, "T_lane_ops_per_s": {}}
    for op in range(L.valu_peak_ops()):
        name = "%s %s" % (L.valu_peak_name(op).decode(), L.valu_peak_shape(op).decode())
        ts = []
        for it in range(reps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            rc = L.valu_peak_launch(op, blocks, iters, 12345 + it, sink.data_ptr(), stream.cuda_stream)
            b.record()
            torch.cuda.synchronize()
            if rc != 0:
                raise RuntimeError("valu probe %d failed (%d)" % (op, rc))
            if it:
                ts.append(a.elapsed_time(b))
        ms = statistics.median(ts)
        lane_ops = blocks * 256.0 * iters * per_trip
        out["T_lane_ops_per_s"][name] = round(lane_ops / (ms / 1e3) / 1e12, 3)
    return out


def jfa_pass_bench(torch, rtsdf, synth, reps=20):
    """Each jump-flooding pass of the static 400 x 200 x 400 scene as it runs inside the full
    chain (between the first and the last pass the buffers hold the internal complemented
    ids): the chains of the first 1, 2, ..., 10 offsets are timed from the voxelized seeds
    (median of `reps` launches each, HIP events, the input restored before every launch) and
    pass i is the difference of the medians of chains i + 1 and i."""
    sc = synth.scene_static()
    g = rtsdf.make_grid(sc.dims, sc.org, sc.h)
    S = rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames)
    S.voxelize()
    seeds0 = S.seeds.clone()
    a_buf, b_buf = torch.empty_like(seeds0), torch.empty_like(seeds0)
    N = g.n
    chain_ms, empty_in = [0.0], []
    prev_out = seeds0
    for i in range(len(sc.steps)):
        empty_in.append(float((prev_out == rtsdf.EMPTY).float().mean().item()))
        ts = []
        for it in range(reps + 2):
            a_buf.copy_(seeds0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            res = rtsdf.rtsdf_jfa(a_buf, b_buf, g, sc.steps[:i + 1])
            e1.record()
            torch.cuda.synchronize()
            if it >= 2:
                ts.append(e0.elapsed_time(e1))
        chain_ms.append(statistics.median(ts))
        prev_out = res.clone()
    rows = []
    for i, k in enumerate(sc.steps):
        ms = max(chain_ms[i + 1] - chain_ms[i], 1e-6)
        rows.append({"pass": i, "k": int(k), "ms": round(ms, 4), "empty_input_frac": round(empty_in[i], 4),
                     "algorithmic_GBps": round(8.0 * N / (ms / 1e3) / 1e9, 1)})
    total = chain_ms[-1]
    return {"grid": list(sc.dims), "passes": rows, "ms_total": round(total, 4),
            "hbm_frac_mean": round(8.0 * N * len(rows) / (total / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_thread_rays(sc, band, sample):
    """Rays per second of the oracle's ray sampling on one host thread: a child process with
    OMP_NUM_THREADS=1 traces `sample` of the masked voxels for one frame."""
    import subprocess
    import tempfile
    import numpy as np
    rng = np.random.default_rng(1)
    vids = np.sort(rng.choice(band, min(sample, len(band)), replace=False)).astype(np.int32)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "vids.npy")
        np.save(path, vids)
        code = ("import sys, time, json; sys.path.insert(0, %r)\n"
                "import numpy as np, oracle as orc\n"
                "from paper_2210_06160_amd import synth\n"
                "sc = synth.scene_static(); g = orc.make_grid(sc.dims, sc.org, sc.h)\n"
                "bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g)); v = np.load(%r)\n"
                "t0 = time.perf_counter(); orc.raysample(bvh, g, v, sc.rays, 0, 0)\n"
                "print(json.dumps(len(v) * sc.rays / (time.perf_counter() - t0)))\n") % (ROOT, path)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
        if r.returncode != 0:
            raise RuntimeError("single-thread oracle leg failed:\n" + r.stderr)
        return float(r.stdout.strip().splitlines()[-1])


def cpu_baseline(sc, sample):
    """The oracle as it stands, on the host cores, on a bounded sample of the same step:
    voxelize, all jump-flooding passes, mask, hierarchy and combine over the full grid;
    ray sampling of `sample` masked voxels for one frame, scaled to all masked voxels and
    frames."""
    import numpy as np
    import oracle as orc
    g = orc.make_grid(sc.dims, sc.org, sc.h)
    t = {}
    t0 = time.perf_counter()
    seeds = orc.voxelize(sc.verts, sc.tris, g)
    t["voxelize"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    jfa = orc.jfa(seeds, g, sc.steps)
    t["jfa"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    band = orc.band(jfa, g, sc.band)
    t["mask"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    bvh = orc.BVH(sc.verts, sc.tris, orc.hit_pad(g))
    t["bvh"] = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    vids = np.sort(rng.choice(band, min(sample, len(band)), replace=False))
    t0 = time.perf_counter()
    acc = orc.raysample(bvh, g, vids, sc.rays, 0, 0)
    ts = time.perf_counter() - t0
    rays_s = len(vids) * sc.rays / ts
    t["raysample"] = len(band) * sc.rays * sc.frames / rays_s
    N = len(seeds)
    D = np.full(N, np.inf, np.float32)
    H = np.zeros(N, np.uint32)
    D[vids], H[vids] = acc[0], acc[1]
    t0 = time.perf_counter()
    orc.combine(jfa, D, H, g, sc.band, sc.h / 2, 0.0, 0)
    t["combine"] = time.perf_counter() - t0
    total = sum(t.values())
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    one = single_thread_rays(sc, band, sample // 20)
    return {"value": N / total, "unit": "SDF voxels/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "rays_per_s": rays_s, "rays_per_s_1_thread": one,
            "sample": "full-grid voxelize/JFA/mask/BVH/combine; ray sampling of %d of %d masked voxels x %d "
                      "rays for one frame, scaled to %d frames; the 1-thread ray rate from %d masked voxels" %
                      (len(vids), len(band), sc.rays, sc.frames, min(sample // 20, len(band))),
            "stage_s": {k: round(v, 3) for k, v in t.items()}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2210_06160_amd import rtsdf, synth

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device="cuda")
        b = torch.empty(n, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n, "copy_calibration_bytes_written": n, "dispatches": 3}))
        return
    if args.only == "valu":
        print(json.dumps({"valu": valu_peak(torch)}))
        return
    if args.only in ("deform", "grad", "batch", "two_level", "tables", "dl", "clipmap", "jfa"):
        fn = {"deform": deform_bench, "grad": grad_bench, "batch": batch_bench, "two_level": two_level_bench,
              "tables": tables_bench, "dl": dl_bench, "clipmap": clipmap_bench, "jfa": jfa_pass_bench}[args.only]
        print(json.dumps({args.only: fn(torch, rtsdf, synth)}))
        return
    if args.only == "static":
        args.no_deform = args.no_grad = args.no_batch = args.no_two_level = args.no_dl = args.no_clipmap = True
        args.no_tables = args.no_valu = args.no_jfa_passes = True
    sc = synth.scene_static()
    S = rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames)
    N = S.g.n
    for _ in range(args.warmup):
        gpu_step(S, rtsdf, StageTimer(torch))
    torch.cuda.synchronize()
    timers = [StageTimer(torch) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        gpu_step(S, rtsdf, timers[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    stages = {}
    per_step = []
    ray_launches = []
    for tm in timers:
        d = tm.durations()
        per_step.append(sum(d.values()))
        for k, v in d.items():
            stages[k] = stages.get(k, 0.0) + v / args.steps
        # each frame's ray-sampling launch, bracketed by its own events
        ev = tm.events
        ray_launches += [e0.elapsed_time(e1) for (n0, e0), (n1, e1) in zip(ev[:-1], ev[1:]) if n1 == "raysample"]
    ms_median = statistics.median(per_step)
    band = int(S.band_count.item())
    rays = band * sc.rays * sc.frames
    rays_per_s = rays / (stages["raysample"] / 1e3)
    dominant = max(stages, key=stages.get)
    launch_ms = statistics.median(ray_launches)
    # ray sampling: bound by plain ALU issue (no dense contraction, no streaming); achieved =
    # the method's algorithmic lane-ops per ray (OPS_PER_RAY) x rays per launch / the median
    # launch duration
    achieved = band * sc.rays * OPS_PER_RAY / (launch_ms / 1e3) / 1e12
    traffic = recorded_traffic()
    roof = {"kernel": "raysample", "bound": "alu", "achieved": round(achieved, 3), "peak": round(ALU_PEAK_TOPS, 2),
            "unit": "T lane-ops/s", "frac": round(achieved / ALU_PEAK_TOPS, 4), "traffic": traffic,
            "launch_ms": round(launch_ms, 4), "units_per_launch": band * sc.rays,
            "ops_per_unit": round(OPS_PER_RAY, 1),
            "frac_of_single_rate_peak": round(achieved / ALU_PEAK_SINGLE_RATE_TOPS, 4)}
    jfa_ms = stages["jfa"]
    passes = len(sc.steps)
    jfa_gbs = 8.0 * N * passes / (jfa_ms / 1e3) / 1e9
    out = {
        "metric": "SDF voxels/s & rays/s at 400x200x400; batched/bwd vs plain, same GPU",
        "value": round(N / (ms_median / 1e3), 1),
        "unit": "SDF voxels/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_per_step_median": round(ms_median, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+i32", "data": "synthetic",
        "config": {"workload": sc.name, "grid": list(sc.dims), "triangles": int(len(sc.tris)),
                   "jfa_passes": passes, "band_vox": sc.band, "rays_per_voxel": sc.rays, "frames": sc.frames,
                   "masked_voxels": band},
        "rays_per_s": round(rays_per_s, 1),
        "stages_ms": {k: round(v, 4) for k, v in stages.items()},
        "dominant_kernel": dominant,
        "roofline": roof,
        "jfa": {"ms_per_pass": round(jfa_ms / passes, 4), "voxel_passes_per_s": round(N * passes / (jfa_ms / 1e3), 1),
                "algorithmic_GBps": round(jfa_gbs, 1), "hbm_frac": round(jfa_gbs / HBM_PEAK_GBS, 4)},
    }
    if not args.no_deform:
        out["deform"] = deform_bench(torch, rtsdf, synth)
    if not args.no_grad:
        out["grad"] = grad_bench(torch, rtsdf, synth)
    if not args.no_batch:
        out["batch"] = batch_bench(torch, rtsdf, synth)
    if not args.no_two_level:
        out["two_level"] = two_level_bench(torch, rtsdf, synth)
    if not args.no_dl:
        out["dl"] = dl_bench(torch, rtsdf, synth)
    if not args.no_clipmap:
        out["clipmap"] = clipmap_bench(torch, rtsdf, synth)
    if not args.no_tables:
        out["tables"] = tables_bench(torch, rtsdf, synth)
    if not args.no_jfa_passes:
        out["jfa_passes"] = jfa_pass_bench(torch, rtsdf, synth)
    if not args.no_valu:
        v = valu_peak(torch)
        out["roofline"]["measured_valu_T_lane_ops_per_s"] = {
            k: v["T_lane_ops_per_s"][k] for k in ("v_fma_f32 I3", "v_add_u32 I2", "v_mad_u32_u24 I3", "v_min3_i32 I3")}
        out["valu_probe"] = v
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
