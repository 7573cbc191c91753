"""FP64 CPU oracle for the SVLF per-ray render path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  It
shares no code with the HIP library and imports nothing from it.

What it computes (SVLF, arxiv 2205.07058, section 4):

* ``octree``  -- the sparse octree over occupied leaves (section 4.1, "Scene
  volume"): Morton-ordered levels, per-node child masks, the vertex table
  (one feature embedding per octree vertex) and each leaf's 8 corner vertices.
* ``trace``   -- the ray / voxel intersection (section 4.2 ray-AABB test; the
  hierarchical sparse ray-octree intersection of section 4.3) evaluated with an
  exactly specified FP32 slab predicate, both level by level and by brute force.
* ``render``  -- trilinear interpolation psi (section 4.1), the decoder MLP
  (section 4.5 activations), optical thickness (section 4 footnote) and
  alpha compositing (Eq. 3), in FP64, with an optional BF16-rounding mode;
  the hand-derived backward of all of it; the loss and its gradient.
* ``optim``   -- Adam (section 4.5), dense and restricted to touched rows.
* ``lightfield`` -- the paper's two-decoder voxel light-field function
  (sections 4.1-4.3: bounding-sphere ray parameterisation, density decoder
  on the features at the entry and exit points giving tau and eta, colour
  decoder on the features at the surface point, Eq. 3) and its backward.

Every function states the passage it follows.  Parity status: every function
is pinned by the ``-m "not gpu"`` tests (brute force, exact rationals, closed
forms, invariants and finite differences); none is "parity unpinned".
"""

from . import octree, trace, render, optim, lightfield  # noqa: F401
