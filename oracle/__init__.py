"""FP64 CPU oracle for the Grangeat / epipolar-consistency hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately
unoptimised restatement of the method (arxiv 1806.02637): the Radon-derivative
sinogram of Eq. 1, the pseudo-inverse-free epipolar lines of Eqs. 4, 5, 13
and 14, and the cost of Eqs. 15-17, plus an exact dual-number gradient.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the HIP engine shares no code with it and never calls it.

Modules: ``geometry`` (projective steps), ``sinogram`` (Eq. 1 on a flat
detector; its inner line integral is plain C in ``sino.c``), ``ecc`` (cost),
``grad`` (gradient), ``dual`` (forward-mode dual numbers), ``spline`` (the
Akima motion model), ``fdk`` (the reconstruction a compensated scan is
checked with).
"""
from .dual import Dual, ops  # noqa: F401
from .ecc import EccParams, ecc_cost, ecc_pair, pair_index, pair_list  # noqa: F401
from .grad import ecc_grad  # noqa: F401
from .sinogram import FullSinograms, LazySinograms, SinoGrid  # noqa: F401
