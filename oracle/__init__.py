"""FP64 CPU oracle for dense 3-way MTTKRP and CP-ALS -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding)
never calls it, and this package imports nothing from the product: the two
share no code.  Both consume inputs drawn by the seeded generators, which
hold none of the arithmetic checked here.

Source of the definitions.  The paper this work accompanies (Gameiro et al.,
"Towards Real Time Compton Imaging in Demanding Conditions", arXiv
2411.04785) describes Compton-camera event clustering (its Section 2) and 3D
back projection (its Section 3); it contains no passage on MTTKRP, CP-ALS,
Gram matrices or the FP8/bf16 formats.  Every operation here is therefore
the standard mathematical definition, written out directly in FP64:

* MTTKRP (mode n): the unfolded tensor times the Khatri-Rao product of the
  other two factors, ``M_1 = X_(1) (B kr C)``; entrywise
  ``M_1(i,r) = sum_{j,k} X(i,j,k) B(j,r) C(k,r)`` (likewise for modes 2, 3),
  and for an N-way tensor the same with the product of the N-1 other
  factors (``mttkrp_nway``); for a sparse tensor in coordinates, the same sum
  over the stored entries (``mttkrp_coo``).
* CP-ALS: block coordinate descent on ``||X - [[lambda; A, B, C]]||_F``,
  each factor solved from its normal equations ``A_n V = M_n`` with
  ``V = *_{m != n} A_m^T A_m`` (Hadamard product of Grams).
* bf16 / OCP e4m3 rounding: round-to-nearest, ties to the even code.

None of it is pinned by a value printed in the paper (the paper prints
none for these operations).  It is pinned by mathematics instead -- brute
force loops on tiny inputs, closed forms on exact CP tensors, special cases
that reduce to library routines, invariants and library casts -- in
``tests/test_oracle.py``.
"""

from .mttkrp import khatri_rao, unfold, mttkrp, mttkrp_rows, mttkrp_brute  # noqa: F401
from .mttkrp import khatri_rao_many, unfold_nway, mttkrp_nway, mttkrp_nway_brute, mttkrp_coo  # noqa: F401
from .cpals import (gram_hadamard, gram_solve, normalize_columns, cp_als, cp_als_extrapolated,  # noqa: F401
                     gram_hadamard_nway, fit_nway, cp_als_nway,
                     reconstruct_slices, fit)
from .formats import (bf16_round, bf16x2_split, e4m3_values, e4m3_encode,  # noqa: F401
                      e4m3_decode, slice_scale_exponent, quantize_slices_e4m3,
                      dequantize_slices_e4m3)
