// Tile shapes and work-distribution constants of the kernels.  The values below are the
// ones paper_2210_06160_amd/autotune.py measured fastest on MI355X (gfx950) for the
// benchmark workloads; every choice computes identical results, only speed differs.
// A -D definition on the compiler command line overrides a value (the autotuner builds
// its candidate libraries that way).
#pragma once

// jump flooding: lattice points per work-group along z, and waves per work-group (each wave
// takes 64 consecutive columns of a plane)
#ifndef RTSDF_JFA_CHUNK
#define RTSDF_JFA_CHUNK 32
#endif
#ifndef RTSDF_JFA_WAVES
#define RTSDF_JFA_WAVES 4
#endif
// ... a pass first tests a plane's loaded ids for all-EMPTY (a mostly EMPTY input: the large
// offsets of the halving schedule) when RTSDF_JFA_SPARSE x offset >= the longest grid side
// (0: never; a power of two)
#ifndef RTSDF_JFA_SPARSE
#define RTSDF_JFA_SPARSE 0
#endif
static_assert((RTSDF_JFA_SPARSE & (RTSDF_JFA_SPARSE - 1)) == 0, "RTSDF_JFA_SPARSE: 0 or a power of two");

// ray sampling: listed voxels a wave takes per cursor atomic (at most; fewer when the
// mask is small, so that every wave gets work), the number of voxel ranges (each with its
// own cursor; a multiple of the 8 XCDs), the voxel slots per wave (a power of two; a pool
// fill starts at most half of them), and idle lanes restarted together
#ifndef RTSDF_RAY_CHUNK
#define RTSDF_RAY_CHUNK 32
#endif
#ifndef RTSDF_RAY_RANGES
#define RTSDF_RAY_RANGES 8
#endif
#ifndef RTSDF_RAY_SLOTS
#define RTSDF_RAY_SLOTS 16
#endif
#ifndef RTSDF_RAY_START_BATCH
#define RTSDF_RAY_START_BATCH 8
#endif
// ... waves per SIMD the single-object and the batched kernel are built for (their register
// budgets, and the depth of their per-lane LDS stacks, which share the CU's 160 KB among that
// many waves)
#ifndef RTSDF_RAY_WAVES
#define RTSDF_RAY_WAVES 6
#endif
#ifndef RTSDF_RAY_WAVES_BATCH
#define RTSDF_RAY_WAVES_BATCH 5
#endif
// ... the node visits per loop iteration (a triangle test runs after every second one), and
// the most stack entries a lane pops after a node visit (0: until it finds work); a lane that
// needs more pops carries on at the next visit
#ifndef RTSDF_RAY_VISITS
#define RTSDF_RAY_VISITS 6
#endif
#ifndef RTSDF_RAY_POP_TRIPS
#define RTSDF_RAY_POP_TRIPS 1
#endif

// soft shadows: pixels per wave along x (the tile is RTSDF_SHADOW_TILE_X x 64/RTSDF_SHADOW_TILE_X)
#ifndef RTSDF_SHADOW_TILE_X
#define RTSDF_SHADOW_TILE_X 4
#endif

// PLOC iterations run across all clusters of all objects before one work-group per object
// finishes the rest (the same step either way, so the tree does not depend on it)
#ifndef RTSDF_PLOC_WIDE
#define RTSDF_PLOC_WIDE 24
#endif

// hierarchy shape: most triangles in a leaf of the 4-wide tree, and the PLOC neighbourhood
// radius (positions searched on each side for a cluster's nearest neighbour)
#ifndef RTSDF_LEAF_MAX
#define RTSDF_LEAF_MAX 1
#endif
#ifndef RTSDF_PLOC_RADIUS
#define RTSDF_PLOC_RADIUS 16
#endif
