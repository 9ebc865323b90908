"""MI355X-native hot path of the kernel-free boundary integral method for the bidomain equations.

``workloads`` describes problems (no method arithmetic); ``kfbi`` binds the HIP library
``libkfbi.so`` built from ``csrc/`` by ``build``.  Importing the package does not load
the library; the first call into ``kfbi`` does, and fails loudly if it is missing.
"""
__all__ = ["workloads", "kfbi", "build"]
