"""MI355X (gfx950) NER + pseudonymize path of AnonShield (arXiv 2606.15650).

The compute lives in ``libanon.so`` (HIP kernels behind the C ABI of
``include/anon.h``); ``api`` is its ctypes binding and ``pipeline`` the torch
plumbing (device buffers, workspaces, streams).  Importing the package loads
the library and fails if it has not been built.
"""
from . import api

api.lib()

__all__ = ["api"]
