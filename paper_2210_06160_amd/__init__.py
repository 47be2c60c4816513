"""RTSDF signed-distance hot path for AMD Instinct MI355X (gfx950).

Voxelize a triangle scene into seed voxels, jump-flood them into a coarse distance field,
ray-sample the band near surfaces against a software LBVH and combine the result with the
paper's running-minimum or decay rule (arXiv 2210.06160, sections 2.1-2.5).

`paper_2210_06160_amd.rtsdf` binds the C ABI of `librtsdf.so` (hand-written HIP); it is
imported lazily so that the input generators in `synth` work without a GPU.
"""

__all__ = ["rtsdf", "synth"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
