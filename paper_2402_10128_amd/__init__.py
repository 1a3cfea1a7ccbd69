"""MI355X (gfx950) rasterizer for Generalized Exponential Splatting (arXiv 2402.10128).

Layout:
  csrc/       HIP kernels and the C ABI (include/ges.h) compiled into libges.so
  build.py    in-tree hipcc build of libges.so
  ges.py      ctypes binding with the C entry-point names (argument marshalling only)
  autograd.py torch.autograd.Function over the forward and backward passes
  serve.py    Python front end of the continuous-batching render server
  synth.py    seeded synthetic scenes and cameras (inputs only)

Importing the package does not load libges.so; ``ges.lib()`` does, and raises when
the library has not been built.
"""
