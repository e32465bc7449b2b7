"""MI355X-native Douglas-ADI solver for the single-factor HJM model with
stochastic volatility.

The solver itself is the C-ABI library ``libhjm.so`` (hand-written HIP kernels
for gfx950 plus a small C++ host layer, declared in ``include/hjm.h``).
``paper_1108_1688_amd.hjm`` is the thin ctypes binding; it loads the library
on first use and raises if it is missing -- there is no CPU fallback.
``paper_1108_1688_amd.workloads`` holds the seeded synthetic inputs.
"""
__all__ = ["hjm", "workloads"]
