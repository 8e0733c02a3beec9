"""Batched driving-simulator step (kinematic bicycle dynamics, oriented-box
collision, ego-frame radius-filter observations, reward/done and auto-reset)
for AMD Instinct MI355X (gfx950).

Submodules are imported explicitly so that importing the package never loads
the HIP library as a side effect:

* ``paper_2408_01584_amd.scenes`` -- seeded synthetic scenes and actions
  (input generation only).
* ``paper_2408_01584_amd.gd``     -- ctypes binding of the C-ABI library
  ``libgd.so`` (same entry-point names as ``include/gd.h``).
* ``paper_2408_01584_amd.sim``    -- torch convenience layer: buffer
  allocation, ``Sim`` and the ``DiffRollout`` autograd function.
"""
