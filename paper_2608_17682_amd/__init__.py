"""MI355X-native differentiable Voronoi ray tracing: the per-ray cell walk.

The compute lives in ``libvoro.so`` (hand-written HIP kernels for gfx950,
C ABI declared in ``include/voro.h``).  This package is its thin binding:
``voro`` (ctypes marshalling of the C entry points, same names) and
``autograd`` (a torch.autograd.Function over sites, densities and texels).
``synth`` draws seeded synthetic inputs.
"""
__version__ = "0.1.0"
