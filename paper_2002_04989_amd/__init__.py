"""libeeid: squared eigenvector components of Hermitian matrices on one MI355X
through the eigenvector-eigenvalue identity (arXiv 2002.04989).

Submodules:
  eeid    -- ctypes binding of the C ABI (include/eeid.h); needs the built
             libeeid.so and a GPU, and raises otherwise.
  inputs  -- seeded synthetic inputs shaped like the paper's workloads.
  build   -- compiles libeeid.so for gfx950 with hipcc.
"""
