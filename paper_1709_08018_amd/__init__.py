"""Indexed Kleinian-attractor renderer for AMD Instinct MI355X (gfx950).

Words over {a, b, A, B} are decoded from integer indices with no stored
words array, their Moebius maps are applied right to left to a seed point,
and the values are binned into a density image (Rosa, arXiv:1709.08018).
The compute path is the HIP library ``libkl.so`` behind the C ABI declared
in ``include/kl.h``; ``paper_1709_08018_amd.kl`` is its Python binding.
Submodules are imported on demand so that importing the package does not
load the GPU library.
"""
__all__ = ["kl", "workloads"]
