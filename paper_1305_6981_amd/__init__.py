"""MI355X-native FCIQMC (Booth, Smart & Alavi, arXiv:1305.6981).

The iteration runs in hand-written HIP kernels inside ``libfciqmc.so`` behind
the C ABI of ``include/fciqmc.h``; :mod:`.fciqmc` is a thin ctypes binding with
the same names. :mod:`.systems` generates seeded synthetic inputs.
"""
