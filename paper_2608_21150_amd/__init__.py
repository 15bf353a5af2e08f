"""MI355X (gfx950) ICON-style non-hydrostatic dynamical-core step.

The compute path is libdycore.so (hand-written HIP + host C++ behind the C
ABI of include/dycore.h); ``paper_2608_21150_amd.dycore`` is its ctypes
binding.  Importing the binding fails when the library is not built.
"""
