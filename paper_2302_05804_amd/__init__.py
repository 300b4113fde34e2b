"""MI355X-native hot path of the multi-frame EM deconvolution / super-resolution
method of Sukurdeep, Navarro & Budavari (arXiv:2302.05804, Sec. 2, Eqs. (1)-(3)).

The compute lives in a C-ABI shared library (``libem.so``, HIP for gfx950);
``paper_2302_05804_amd.em`` is the thin ctypes binding.  Importing this package
does not load the library; ``paper_2302_05804_amd.em`` does, and fails loudly
when it has not been built.
"""
__all__ = ["synth", "em"]
