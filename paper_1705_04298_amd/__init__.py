"""MI355X-native Gerchberg slope extension and Fourier wave-front reconstruction.

The compute path is the HIP library ``libfwr.so`` (C ABI declared in
``include/fwr.h``); :mod:`paper_1705_04298_amd.fwr` is its thin ctypes
binding and :mod:`paper_1705_04298_amd.inputs` generates seeded synthetic
workloads.  Importing the package loads nothing; the library is opened on
first use and a missing library is an error, never a fallback.
"""
