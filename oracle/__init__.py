"""CPU oracle for the octree level-of-detail build and the point splat.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP path (``paper_0811_2055_amd``) and never imports it.

The oracle is deliberately plain: numpy integer arithmetic and float64,
one node at a time, written from the definitions of Szalay, Springel and
Lemson, "GPU-Based Interactive Visualization of Billion Point Cosmological
Simulations" (arXiv:0811.2055):

* the octree paragraph: a spatial octree in which every node or leaf is
  represented by at most n points (n = 16000 in the paper), extra points
  being thinned by density-weighted random subselection, and children
  holding the parent's data at eight times the detail;
* the quantisation paragraph: positions stored as 2 bytes per coordinate,
  spanning the containing block;
* the rendering paragraph: each point drawn as a smeared blob evaluated
  for every pixel it covers;
* the block-choice paragraph: near regions drawn from deep in the tree,
  far regions from shallow nodes, the choice made on the CPU.

Where the paper leaves the method undefined (the density estimate, the
sampling scheme, the random generator, ties, mass assignment, the blob
kernel), the oracle implements one fixed reading; each is listed in the
project's design notes and in the docstring of the function that uses it.

Modules: ``philox`` (counter-based generator), ``lod`` (the build),
``splat`` (render and its adjoint), ``cut`` (view-dependent node choice),
``refine`` (one step of the gradient refinement of a node), ``cubic`` (the
radial cubic blob and the attribute channel), ``interp`` (time interpolation
between snapshots and the motion codes of stored points), ``stream`` (block
store loading policy under a byte budget).
"""
from . import philox, lod, splat, cut, refine, cubic, interp, stream  # noqa: F401
