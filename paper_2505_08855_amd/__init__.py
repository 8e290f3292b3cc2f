"""MI355X-native radiative cooling source step (two-temperature GRMHD).

The compute path is the C-ABI library ``libradcool.so`` (hand-written HIP for
gfx950); ``radcool`` is its ctypes binding and ``autograd`` wraps the adjoint
in a ``torch.autograd.Function``.  ``workloads`` draws seeded synthetic inputs.
Importing the package loads nothing; the library is opened on first use and a
missing or unbuilt library is an error, never a fallback.
"""
