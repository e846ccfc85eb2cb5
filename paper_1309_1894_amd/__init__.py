"""MI355X-native autotuned CSR SpMV and vector kernels (HIP, gfx950).

The compute path lives in ``libspk.so`` (HIP kernels behind a C ABI).
Submodules, imported explicitly:

* ``paper_1309_1894_amd.spk``    -- thin ctypes binding to ``libspk.so``;
* ``paper_1309_1894_amd.inputs`` -- seeded synthetic matrices and vectors
  (numpy only, usable without a GPU).
"""
