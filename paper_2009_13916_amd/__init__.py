"""EDFA-preconditioned GMRES for MHFE-FV Darcy systems on MI355X (gfx950).

``edfa``   -- Python binding of the HIP library (libedfa.so, C ABI in include/edfa.h).
``inputs`` -- seeded synthetic problems in the library's array layout.
``build``  -- hipcc build of the library.
"""
