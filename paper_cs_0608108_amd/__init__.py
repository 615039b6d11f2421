"""libsphidx: spherical-indexing neighbourhood queries (Brodu, arXiv cs/0608108)
as hand-written HIP for gfx950 behind a C ABI.

Submodules are imported on demand so that ``synth`` (input generation) can be
used without loading the GPU library:

* ``paper_cs_0608108_amd.sphidx`` -- ctypes binding of ``libsphidx.so``;
* ``paper_cs_0608108_amd.synth``  -- seeded synthetic workloads;
* ``paper_cs_0608108_amd.build``  -- compiles ``csrc/`` into ``libsphidx.so``.
"""
