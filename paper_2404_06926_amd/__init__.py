"""MI355X-native mapping step of a 3D Gaussian map (Gaussian-LIC, arXiv 2404.06926).

The compute path is a C-ABI HIP library (``csrc/``, declared in ``include/gslic.h``);
``gslic`` is its ctypes binding. Importing this package loads nothing; the library is
loaded on first use and a missing build raises instead of falling back.
"""

__all__ = ["gslic", "scenes"]
