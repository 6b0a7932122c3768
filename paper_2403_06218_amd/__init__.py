"""MI355X-native block Gram-Schmidt QR (CGS-QR with CholeskyQR2 / CGS-CQR2) and solve.

The compute path is the HIP library ``libcqr.so`` (C ABI declared in
``include/cqr.h``); this package only marshals torch device tensors into it.
The native library is loaded on first use and its absence is an error.
"""
