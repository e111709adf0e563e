"""ffx: fermionic state-vector evolution at fixed (N_alpha, N_beta) on AMD MI355X (gfx950).

The compute path is the C-ABI library libffx.so (hand-written HIP kernels plus a
C++ host layer); ``paper_2605_03123_amd.ffx`` is the thin Python binding over it.
Importing this package does not load the library; ``ffx`` does, and raises if
it is missing.
"""
