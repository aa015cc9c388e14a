"""MI355X-native unified geometric multigrid for hybridized (HDG) trace systems.

The compute path is the HIP library ``_lib/libhdg.so`` (built by
``paper_1811_09909_amd.build``); ``hdg`` holds the thin torch/ctypes binding
and ``inputs`` the seeded synthetic workloads.  Importing the package loads
nothing; the library is opened on first use and its absence is an error.
"""
__all__ = ["build", "hdg", "inputs"]
