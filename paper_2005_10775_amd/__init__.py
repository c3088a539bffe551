"""MI355X (gfx950) assembler for the P1 nonlocal stiffness matrix of
D'Elia, Gunzburger, Vollmann (arXiv:2005.10775): libnlasm.so behind a C ABI
(include/nlasm.h) and this thin ctypes binding."""
from .binding import Plan, Batch, Mlp, NlaError, lib, LIB_PATH

__all__ = ["Plan", "Batch", "Mlp", "NlaError", "lib", "LIB_PATH"]
