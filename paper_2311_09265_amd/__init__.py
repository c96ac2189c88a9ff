"""FastBlend hot path (arXiv 2311.09265) for AMD MI355X (gfx950).

PatchMatch nearest-neighbour-field search between guide frames, NNF remapping
of style frames and sliding-window blending / keyframe interpolation, as
hand-written HIP kernels behind the C ABI declared in ``include/fastblend.h``.
The Python binding (``fastblend``) only marshals arguments: it hands device
pointers of PyTorch tensors and the current HIP stream to ``libfastblend.so``.
``synth`` generates the seeded synthetic workloads; ``proposal`` trains the
learned proposal network with the library's own kernels.
"""
__version__ = "0.1.0"
