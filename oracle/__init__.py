"""FP64 CPU oracle of restarted reflected Halpern PDHG for LP.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP library; the only module both
sides use is ``lpgen`` (seeded inputs, none of the method's arithmetic).

Every function is a plain, slow, step-by-step rendering of the method as the
paper states it (Lu, Peng, Yang, "cuPDLPx", arXiv 2507.14051):

  pdhg      -- validation, diagonal rescaling, power iteration, the PDHG step
               (Sec. 2.2, eq. pdhg), Halpern anchoring and reflection (Sec. 3),
               the fixed-point residual and restart tests (Sec. 3, adaptive
               restart), the PID primal weight (Sec. 3, primal weight update)
               and the relative KKT termination test (Sec. 4, optimality
               termination criteria).
  kkt       -- the relative KKT error on the original LP (Sec. 4).
  brute     -- vertex enumeration for tiny LPs (an independent ground truth).
  mixed     -- iterative refinement in shifted coordinates with an FP32 inner
               solve (an extension of the method, not in the paper).
  adjoint   -- reverse mode of K unrolled iterations with the controller frozen
               (an extension of the method, not in the paper).

Pins: every function above is checked in ``tests/test_oracle_*.py`` against
something other than itself (vertex enumeration, HiGHS via scipy, closed forms,
fixed-point and firm-nonexpansiveness invariants, torch autograd on CPU,
finite differences).  Functions without such a check say "parity unpinned".
"""
from .kkt import kkt, proj_R, dual_objective  # noqa: F401
from .pdhg import Params, Result, validate, rescale, power_norm, solve, pdhg_operator  # noqa: F401
