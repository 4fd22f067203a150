"""MI355X-native DSMC micro-solver for force-driven parallel-plate flow.

``paper_2311_14140_amd.dsmc`` is the ctypes binding of the HIP library
``libdsmc.so`` (built by ``paper_2311_14140_amd.build``); importing it fails if
the library is missing.  ``stats`` holds the host-side batch-means statistics
and ``serve`` the continuous-batching request loop.
"""
