"""FastBlend hot path (arXiv 2311.09265) for AMD MI355X (gfx950).

PatchMatch nearest-neighbour-field search between guide frames, NNF remapping
of style frames and sliding-window blending / keyframe interpolation, as
hand-written HIP kernels behind the C ABI declared in ``include/fastblend.h``.
The Python layer (``api``) only marshals arguments: it hands device pointers
of PyTorch tensors and the current HIP stream to ``libfastblend.so``.
"""
__version__ = "0.1.0"
