"""MI355X (gfx950) NER + pseudonymize path of AnonShield (arXiv 2606.15650).

The compute lives in ``libanon.so`` (HIP kernels behind the C ABI of
``include/anon.h``); ``api`` is its ctypes binding and ``pipeline`` the torch
plumbing (device buffers, workspaces, streams).  Importing the package loads
the library and fails if it has not been built.
"""
# torch provides the device memory and streams; its HIP runtime must be the
# one libanon.so binds to, so it is loaded first.
import torch  # noqa: F401

from . import api

api.lib()

__all__ = ["api"]
