"""FT-CCSD imaginary-time hot path on AMD Instinct MI355X (gfx950).

The native library libftcc.so (C ABI in include/ftcc.h) holds every kernel;
`paper_2004_01729_amd.ftcc` is its Python binding and
`paper_2004_01729_amd.autograd` wraps it as a torch.autograd.Function.
Importing this package loads nothing; the library is loaded on first use.
"""
__all__ = ["ftcc", "build", "autograd"]
