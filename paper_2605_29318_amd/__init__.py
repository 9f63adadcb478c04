"""MI355X (gfx950) subspace-construction path of FreeForm (arXiv 2605.29318).

RKPM shape functions on particles, the weight-space Hessian of Prop. 1 and
the RKPM mass matrix, and the smallest generalized eigenpairs (skinning
eigenmodes), behind the C ABI of include/freeform.h. ``freeform`` is the
Python binding; ``synth`` builds seeded synthetic particle clouds.
"""
