"""MI355X cell-wise matrix-free Q_k finite elements: C-ABI library (libfe.so) and its binding.

``paper_2607_03413_amd.fe`` is the ctypes binding; the compute path is the
HIP library built by ``paper_2607_03413_amd/build_lib.py``.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfe.so")
HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fe.h")
