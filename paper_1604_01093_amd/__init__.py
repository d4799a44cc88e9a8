"""MI355X global pose alignment (BundleFusion Sec. 4.3-4.4) as HIP kernels behind a C ABI.

The compute path lives in ``libbf.so`` (``csrc/``, built by ``build.py``);
``bf`` is its ctypes binding.  Importing this package does not load the
library; ``bf.load()`` (called by every binding function) does, and raises if
it has not been built.
"""
