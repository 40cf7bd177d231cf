"""MI355X-native non-collinear real-time TDDFT time step (HIP kernels behind a C ABI).

`paper_2506_21908_amd.nct` is the ctypes binding of libnct.so (hand-written
HIP for gfx950); `paper_2506_21908_amd.inputs` draws the seeded synthetic
systems.  Importing the package does not load the library.
"""
