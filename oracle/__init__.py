"""Reference ("oracle") for polynomial-kernel Gaussian splatting.

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything in this package. The
GPU product (``paper_2603_18707_amd``) never imports it, and this package never
imports the product: the two share no code, header, table or constant
generator. Both sides receive the same seeded inputs from the generator module
``paper_2603_18707_amd.scenes``, which holds none of the method's arithmetic.

Contents
--------
``core``     ctypes binding of ``oracle.c``: FP64 projection and brute-force
             per-pixel compositing (every pixel against every depth-ordered
             splat, no tile lists).
``coeffs``   the paper's first-order coefficients and an independent L1 fit of
             orders 1-3 (Sec. 3.1), roots by bisection (Sec. 3.3, App. B).
``binning``  integer reference for tile duplication, stable sort and tile
             ranges (what a tile-based rasterizer must build, Sec. 2.1).
``grad``     FP64 PyTorch-CPU re-implementation of the forward used only for
             exact reverse-mode gradients (the paper's optimisation ablation,
             Sec. 4.3, needs the derivative of the ReLU-polynomial kernel).

Parity status of every function is listed in the module headers; functions
without an independent pin say "parity unpinned".
"""
