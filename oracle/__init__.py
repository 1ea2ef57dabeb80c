"""CPU FP64 oracle for randomized T-HOSVD / ST-HOSVD with the power scheme and
approximate matrix multiplication (Che, Wei, Yan).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It is an independent restatement of the paper in numpy and shares
no code with the HIP library.

Pinning status of each function (what fixes it other than itself) is recorded
in the oracle test files; every function here is pinned (none is "parity
unpinned") except the paper's plotted numbers, which the paper never prints.
"""
from .philox import philox4x64  # noqa: F401
from .tucker import (  # noqa: F401
    PROB_NEARLY_OPTIMAL, PROB_NONE, PROB_UNIFORM, TAG_GAUSS, TAG_SAMPLE,
    canonical_signs, ceil_log2, choose_rank, column_sq_norms, draw_columns, fold, frobenius,
    gaussian_matrix, leading_left_singular_vectors, mode_product, power_sketch,
    power_sketch_stabilised, rand_sthosvd, rand_thosvd, rand_tucker_adaptive, randsample,
    range_finder, reconstruct, related_factor, relative_error, sampling_weights, unfold,
)
