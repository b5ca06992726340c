"""MI355X-native FFT-accelerated Lippmann–Schwinger operator (arXiv:1509.05063).

The compute path lives in the C-ABI shared library built from csrc/ (HIP for
gfx950 plus host C++ set-up); `paper_1509_05063_amd.binding` marshals
arguments to it.  Importing this package does not load the library.
"""
