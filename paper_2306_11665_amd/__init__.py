"""MI355X-native sum-factorized Hadamard products (flux-differencing volume term).

The compute path is the HIP library ``libsfhad.so`` (C-ABI declared in
``include/sfhad.h``); ``paper_2306_11665_amd.sfhad`` is its thin ctypes
binding.  Importing this package loads nothing: the library is opened on the
first call into the binding.
"""
__all__ = ["sfhad", "workloads"]
