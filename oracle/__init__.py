"""Plain FP64 CPU oracle for the adaptive H2-matrix product.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything here.  The
oracle shares no code with the HIP path (``paper_2403_01566_amd``); both take
their inputs from ``paper_2403_01566_amd.workloads``, which holds no arithmetic
of the method.
"""
from .tree import ClusterTree, BlockTree, admissible
from .h2 import (H2Matrix, ClusterBasis, Interp, build_interpolated, identity_h2,
                 kernel_matrix, KERNEL_NEG_LOG, KERNEL_SLP, KERNEL_DLP, DIAG_ZERO, DIAG_ROW_MEAN)
from .mul import mul, recompress, block_errors, basis_products, MulInfo
from .error import power_norm, product_error
from .coarsen import agglomerate_sequential
