"""CPU oracle for the GES tile rasterizer -- TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may import
this package.  The product path (the HIP library and its binding) never does.

Modules:
  oracle.py         ctypes wrapper over the C++ oracle (preprocess, keys, sort,
                    ranges, per-pixel compositing and its reverse pass)
  preprocess_f64.py differentiable binary64 preprocess in plain PyTorch (CPU)
  loss.py           L1 + frequency-masked L1 and the DoG mask (Sec. 4.3)
  gef1d.py          1-D GEF, Theorem-1 quadrature and mixtures (Sec. 3, App. A)
"""
