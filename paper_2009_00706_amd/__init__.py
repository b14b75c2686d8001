"""MI355X-native VMS assembly and in-out hot path (immersogeometric octree LES).

The compute path lives in the HIP library ``libvms`` (see ``csrc/``); the
Python module :mod:`paper_2009_00706_amd.vms` is a thin ctypes binding over its
C-ABI. Importing this package does not load the library.
"""
__all__ = ["inputs", "vms"]
