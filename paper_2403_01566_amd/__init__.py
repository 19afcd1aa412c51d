"""MI355X-native adaptive H2-matrix multiplication with block-relative error control.

The compute path lives in the HIP shared library built from ``csrc/``; the
Python binding in ``h2`` only marshals arguments.  Importing this package does
not load the library: ``from paper_2403_01566_amd import h2`` does.
"""
