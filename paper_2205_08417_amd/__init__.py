"""MI355X-native discrete-ordinates (S_N) step library (KiT-RT, arXiv 2205.08417).

The hot path -- one explicit S_N step on an unstructured triangle mesh -- runs in
hand-written HIP kernels for gfx950 behind the C ABI declared in ``include/snrt.h``
(``libsnrt.so``).  ``paper_2205_08417_amd.snrt`` is the thin ctypes binding of that ABI
and ``paper_2205_08417_amd.solver`` the torch-facing layer (problem upload, rollouts,
autograd adjoint).  ``paper_2205_08417_amd.inputs`` holds the seeded synthetic inputs
and is importable without the native library.

Submodules are imported lazily so that importing the input generators never loads HIP.
"""
import importlib

__all__ = ["inputs", "snrt", "solver"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
