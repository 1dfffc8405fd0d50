"""Randomized LUPP skeleton selection (ID and CUR) on AMD MI355X.

The compute path is the HIP library ``librpid.so`` behind the C-ABI declared
in ``include/rpid.h``; ``paper_2104_05877_amd.rpid`` is its thin ctypes
binding.  ``paper_2104_05877_amd.inputs`` builds seeded synthetic inputs.
"""
