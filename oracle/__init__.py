"""FP64 CPU oracle for the per-ray Voronoi walk renderer.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package; the
product path (the HIP library and its Python binding) never does, and this
package imports nothing from the product.

Every function here is a plain, slow, direct evaluation of what the paper
defines, in float64, from the float32 inputs upcast exactly:

* ``walk``       - the Voronoi partition (Sec. 3.1, cell definition) and the
                   per-ray cell intervals, found by brute force over *all*
                   sites in two independent ways (interval method and
                   stepwise nearest-forward-crossing).  It never reads the
                   Delaunay adjacency; it only validates it.
* ``appearance`` - the octahedral map and bilinear texel lookup (Sec. 5.1).
* ``render``     - piecewise-constant opacity, front-to-back compositing and
                   early termination (Sec. 3.2).
* ``adjoint``    - the analytic FP64 gradient of ``render`` with respect to
                   site positions, densities and texels.
* ``cameras``    - ray generation for the camera models of Sec. 6.5 / App. D.
"""
from . import appearance, cameras, walk, render, adjoint  # noqa: F401
