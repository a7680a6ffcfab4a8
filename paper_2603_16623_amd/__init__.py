"""MI355X-native gridless quasistatic plasma-ring wake solver.

The compute path lives in ``libwake.so`` (HIP kernels for gfx950 behind a
C ABI declared in ``include/wake.h``); ``paper_2603_16623_amd.wake`` is the
thin ctypes binding.  Importing this package imports nothing else, so that
the input generators in ``workloads`` can be used without a GPU.
"""
