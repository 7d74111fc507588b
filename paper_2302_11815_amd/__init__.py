"""Walk on Stars (Sawhney, Miller, Gkioulekas, Crane 2023) on AMD MI355X.

The solver lives in a C-ABI shared library (``include/wost.h``) built from
``csrc/`` with hipcc for gfx950; ``paper_2302_11815_amd.wost`` is its ctypes
binding and ``paper_2302_11815_amd.inputs`` holds the seeded scene and point
generators. Importing this package loads nothing.
"""
