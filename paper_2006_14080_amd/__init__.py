"""MI355X-native ADMM-TV reconstruction of multi-coil radial MRI data.

The compute path lives in the HIP shared library ``libmriadmm.so`` built from
``csrc/``; :mod:`paper_2006_14080_amd.mri` is the thin ctypes binding over its
C ABI (declared in ``include/mri_admm.h``).  :mod:`paper_2006_14080_amd.synth`
holds the seeded synthetic-input generators.

Importing this package loads nothing: the binding loads the library on first
use and raises if it has not been built.
"""
__all__ = ["mri", "synth"]
