"""MI355X-native differentiable Gaussian pointmap rasterizer.

The compute path is the HIP library ``libgspm.so`` (built from ``csrc/``) behind a C ABI
declared in ``include/gspm.h``; ``binding`` marshals arguments to it, ``render`` adds the
autograd function and the batched keyframe window.  Importing this package loads nothing;
the library is opened on first use.
"""
