"""TC2 / TC2-CPSCF response density matrix on MI355X (gfx950).

``tc2`` is the ctypes binding of the C ABI (``include/tc2.h``) implemented by
the in-tree ``libtc2.so``; ``workloads`` draws the seeded synthetic inputs;
``build`` compiles the library with hipcc.
"""
__all__ = ["tc2", "workloads", "build"]
