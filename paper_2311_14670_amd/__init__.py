"""s2mi: spin spherical-harmonic and Wigner transforms on AMD MI355X (gfx950).

The transforms of Price & McEwen (arXiv 2311.14670) -- the O(L^3) Wigner-d
stage (descending-m recursion with running renormalisation, evaluated on the
fly per (theta ring, m) and fused with the l-contraction) and the per-ring
phi-DFT -- run in hand-written HIP kernels behind a C ABI (``include/s2mi.h``).
``paper_2311_14670_amd.binding`` is the thin Python binding over that ABI; the
native library is loaded on first use and every transform raises if it is
missing.
"""
