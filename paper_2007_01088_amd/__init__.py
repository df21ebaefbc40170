"""MI355X-native CC3 ground-state triples residual (arXiv 2007.01088, Algorithm 1).

The compute path is the HIP library libcc3.so (C ABI declared in include/cc3.h);
``paper_2007_01088_amd.cc3`` is its thin Python binding.  Importing this package
does not load the library; ``from paper_2007_01088_amd import cc3`` does.
"""
