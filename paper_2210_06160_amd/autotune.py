"""Autotuner of the kernels' tile shapes and work-distribution constants (csrc/tuning.h).

    python -m paper_2210_06160_amd.autotune build           # host: one library per candidate
    python -m paper_2210_06160_amd.autotune run --json F    # GPU: time every candidate -> F
    python -m paper_2210_06160_amd.autotune apply F         # write the fastest into tuning.h

Each group below is a set of constants that one kernel's launch shape depends on, a list
of candidate values, and the workload that times it (the benchmark's own configuration).
Candidates differ only in speed: every one computes identical results (the tile shapes
change which work-group does which point, never what a point computes).  Every candidate
library is timed in a process of its own (a library's kernels are loaded once per process).
"""
import argparse
import itertools
import json
import os
import re
import statistics
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TUNE_DIR = os.path.join(HERE, "_build", "tune")
TUNING_H = os.path.join(HERE, "csrc", "tuning.h")

GROUPS = {
    "jfa": {"RTSDF_JFA_CHUNK": [16, 32, 64], "RTSDF_JFA_WAVES": [2, 4, 8]},
    "jfa_sparse": {"RTSDF_JFA_SPARSE": [0, 2, 4, 8]},
    "ray": {"RTSDF_RAY_START_BATCH": [6, 8, 12], "RTSDF_RAY_WAVES": [6, 7], "RTSDF_RAY_POP_TRIPS": [1, 2]},
    "tree": {"RTSDF_LEAF_MAX": [1, 2, 3], "RTSDF_PLOC_RADIUS": [16, 32]},
    "waves": {"RTSDF_RAY_WAVES": [6, 7]},
    "restart": {"RTSDF_RAY_START_BATCH": [4, 6, 8, 12], "RTSDF_RAY_POP_TRIPS": [1, 2, 3]},
    "visits": {"RTSDF_RAY_VISITS": [2, 4, 6, 8], "RTSDF_RAY_START_BATCH": [4, 8]},
    "slots": {"RTSDF_RAY_SLOTS": [8, 16, 32]},
    "dist": {"RTSDF_RAY_CHUNK": [16, 32, 64], "RTSDF_RAY_RANGES": [8, 16]},
    "shadow": {"RTSDF_SHADOW_TILE_X": [1, 2, 4, 8]},
    "ray_small": {"RTSDF_RAY_RANGES": [8, 32, 64], "RTSDF_RAY_CHUNK": [16, 32]},
}


def current():
    """The values tuning.h holds now."""
    vals = {}
    for m in re.finditer(r"#define (RTSDF_\w+) (\d+)", open(TUNING_H).read()):
        vals[m.group(1)] = int(m.group(2))
    return vals


def candidates(group):
    names = sorted(GROUPS[group])
    for combo in itertools.product(*[GROUPS[group][n] for n in names]):
        yield dict(zip(names, combo))


def tag(group, defines):
    return group + "-" + "-".join("%s%d" % (k.replace("RTSDF_", "").lower(), v) for k, v in sorted(defines.items()))


def lib_path(group, defines):
    return os.path.join(TUNE_DIR, tag(group, defines), "librtsdf.so")


def cmd_build(args):
    from paper_2210_06160_amd import build as B
    for group in (args.groups.split(",") if args.groups else GROUPS):
        for d in candidates(group):
            path = lib_path(group, d)
            B.build(defines=d, out=os.path.dirname(path), lib=path)
            for f in os.listdir(os.path.dirname(path)):
                if f.endswith(".o"):
                    os.remove(os.path.join(os.path.dirname(path), f))
            print("built", tag(group, d), flush=True)


def time_candidate(group, path, reps):
    """Runs in its own process: loads `path` and times the group's workload (ms, median)."""
    import torch
    from paper_2210_06160_amd import rtsdf, synth
    rtsdf.LIB_PATH = path
    rtsdf.lib()

    def events(fn):
        out = []
        for it in range(reps + 1):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            if it:
                out.append(a.elapsed_time(b))
        return statistics.median(out)

    if group in ("jfa", "jfa_sparse", "ray", "tree", "waves", "restart", "visits", "slots", "dist"):
        sc = synth.scene_static()
        S = rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, sc.band, sc.rays, sc.frames)
        S.voxelize()
        if group in ("jfa", "jfa_sparse"):
            return events(S.jfa)
        S.jfa()
        S.mask()
        S.build_bvh()
        rtsdf.rtsdf_reset_accum(S.dmin, S.hits, S.argmin)
        return events(lambda: S.trace(0))
    if group == "ray_small":
        return sum(events(fn) for fn in small_ray_launches(rtsdf, synth))
    sc = synth.scene_grad()
    g = rtsdf.make_grid(sc.dims, sc.org, sc.h)
    sh = rtsdf.make_shadow(**sc.extra["shadow"])
    fine = torch.from_numpy(sc.extra["target"].astype("float32")).cuda()
    img = torch.empty(sh.height, sh.width, device="cuda")
    gi = torch.ones(sh.height, sh.width, device="cuda")
    gf = torch.zeros_like(fine)
    return events(lambda: (rtsdf.rtsdf_shadow_forward(fine, g, sh, img),
                           rtsdf.rtsdf_shadow_backward(fine, g, sh, gi, gf)))


def small_ray_launches(rtsdf, synth):
    """Ray-sampling launches far from the static workload's shape, where the work
    distribution constants matter: the gradient workload (92 k masked points x 16 rays), the
    deforming knot's first frame (4 rays), every fine point of a 128^3 -> 256^3 two-level
    field with one ray, and a 64^3 -> 128^3 two-level field (mask d = 0.1) with 10 rays."""
    out = []
    sg = synth.scene_grad()
    G = rtsdf.StaticSDF(sg.verts, sg.tris, sg.dims, sg.org, sg.h, sg.steps, sg.band, sg.rays, 1,
                        bvh_method=rtsdf.BVH_LBVH)
    G.run()
    out.append(lambda: G.trace(0))
    sd = synth.scene_deform(frames=1)
    D = rtsdf.StaticSDF(sd.verts, sd.tris, sd.dims, sd.org, sd.h, sd.steps, sd.band, sd.rays, 1)
    D.run()
    out.append(lambda: D.trace(0))
    for n, band, x in ((128, 2048, 1), (64, None, 10)):
        sc = synth.scene_static(dims=(n, n, n))
        band = int(round(0.1 / sc.h)) if band is None else band
        T = rtsdf.StaticSDF(sc.verts, sc.tris, sc.dims, sc.org, sc.h, sc.steps, band, x, 1, ratio=2,
                            keep_argmin=False)
        T.run()
        out.append(lambda T=T: T.trace(0))
    return out


def cmd_run(args):
    results = {}
    for group in (args.groups.split(",") if args.groups else GROUPS):
        results[group] = []
        for d in candidates(group):
            path = lib_path(group, d)
            if not os.path.exists(path):
                raise SystemExit("missing %s: run the build step first" % path)
            t0 = time.time()
            r = subprocess.run([sys.executable, "-m", "paper_2210_06160_amd.autotune", "time", "--group", group,
                                "--lib", path, "--reps", str(args.reps)], capture_output=True, text=True,
                               timeout=300)
            if r.returncode != 0:
                raise SystemExit("timing %s failed:\n%s" % (tag(group, d), r.stderr[-2000:]))
            ms = float(r.stdout.strip().splitlines()[-1])
            results[group].append({"defines": d, "ms": ms})
            print("%-40s %9.4f ms  (%.0f s)" % (tag(group, d), ms, time.time() - t0), flush=True)
    with open(args.json, "w") as f:
        json.dump(results, f, indent=1)


def cmd_time(args):
    print("%.6f" % time_candidate(args.group, args.lib, args.reps), flush=True)


def cmd_apply(args):
    res = json.load(open(args.json))
    text = open(TUNING_H).read()
    for group, rows in res.items():
        best = min(rows, key=lambda r: r["ms"])
        for name, v in best["defines"].items():
            text = re.sub(r"#define %s \d+" % name, "#define %s %d" % (name, v), text)
        print(group, best)
    open(TUNING_H, "w").write(text)


def main():
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--groups", help="comma-separated groups (default: all)")
    r = sub.add_parser("run")
    r.add_argument("--json", required=True)
    r.add_argument("--reps", type=int, default=5)
    r.add_argument("--groups", help="comma-separated groups (default: all)")
    t = sub.add_parser("time")
    t.add_argument("--group", required=True)
    t.add_argument("--lib", required=True)
    t.add_argument("--reps", type=int, default=5)
    a = sub.add_parser("apply")
    a.add_argument("json")
    args = p.parse_args()
    {"build": cmd_build, "run": cmd_run, "time": cmd_time, "apply": cmd_apply}[args.cmd](args)


if __name__ == "__main__":
    main()
