"""FP64 CPU oracle for the LADMM mapping iteration.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, double-precision
restatement of the paper's Algorithm 2 (Sec. III-E) and of the objective it
minimises (Eqs. spat and l2, Sec. II-C). Only the test suite, the package
smoke check and the benchmark's CPU-baseline leg may import it. The GPU
library never does, and this package imports nothing from the library: the
two share no code. Inputs for both come from the seeded generator module,
which holds none of the method's arithmetic.
"""
from .algorithm2 import (dtd_apply, dtd_norm, f_step, ladmm, objective, rank_rule,
                    reg_value, thin_svd, xi_rule, z_step, d_step)

__all__ = ["dtd_apply", "dtd_norm", "f_step", "ladmm", "objective", "rank_rule",
           "reg_value", "thin_svd", "xi_rule", "z_step", "d_step"]
