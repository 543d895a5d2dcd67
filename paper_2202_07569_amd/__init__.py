"""Constant-weight PIR server path on AMD MI355X (gfx950).

The library (libcwpir.so, C ABI in include/cwpir.h) computes, for an encrypted constant-weight
codeword query, the selection vector by the plain constant-weight equality operator and its inner
product with the database (Mahdavi and Kerschbaum, arXiv 2202.07569, Sections 3.1 and 3.3).
This package holds its HIP sources (csrc/), the build step and a ctypes binding.
"""
from .binding import Context, Database, Graph, Key, PirError, Server, lib, library_path  # noqa: F401
