"""MI355X-native density-fitted JK / generalized-Fock library (HIP, gfx950).

The compute path is the C-ABI shared library ``libnof.so`` built from
``csrc/``; ``nof`` is its thin ctypes binding.  Importing this package does not
load the library; ``paper_2512_13550_amd.nof`` does, and raises if it is
missing.
"""
