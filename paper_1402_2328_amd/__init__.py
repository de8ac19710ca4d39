"""Replica-exchange Wang-Landau sampling on AMD Instinct MI355X (gfx950).

The method is that of Li, Vogel, Wuest and Landau (arXiv:1402.2328); the
work runs in hand-written HIP kernels behind the C-ABI in include/rewl.h
(librewl.so), with a thin ctypes binding in ``rewl``.
"""
