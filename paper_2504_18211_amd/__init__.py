"""hbheap: a device-side heap allocator for MI355X (gfx950).

A heap preallocated in HBM is cut into fixed-size chunks, split into
power-of-two pages, with one lock-free queue per size class; threads of a
running HIP kernel allocate and free from it.  The hot path is HIP in
``csrc/`` behind a C ABI (``include/hbheap.h``); ``hbheap`` is its thin
ctypes binding.  Importing this package loads nothing; ``hbheap`` loads the
built library on first use and fails loudly if it is missing.
"""

__all__ = ["hbheap", "inputs"]
