"""Mixed virtual element saddle-point solver for MI355X (gfx950).

Submodules:
  inputs  - seeded synthetic meshes, coefficient fields and analytic data
  vem     - Python binding of the C-ABI HIP library (imported on demand)
  build   - compiles the HIP library in-tree
"""
