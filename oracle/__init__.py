"""FP64 CPU oracle for the LADMM mapping iteration.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, double-precision
restatement of the paper's Algorithm 2 (Sec. III-E) and of the objective it
minimises (Eqs. spat and l2, Sec. II-C). Only the test suite, the package
smoke check and the benchmark's CPU-baseline leg may import it. The GPU
library never does, and this package imports nothing from the library: the
two share no code. Inputs for both come from the seeded generator module,
which holds none of the method's arithmetic.
"""
from .algorithm2 import (beta_heuristic, centre_patch, d_step, dtd_apply, dtd_apply_graph,
                         dtd_norm, dtd_norm_graph, f_step, graph_edges, ladmm, objective,
                         objective_masked, patch_data, rank_rule, reg_value, thin_svd, xi_rule,
                         z_step)
from .admm_previous import admm_previous, z_solve_dct

__all__ = ["beta_heuristic", "centre_patch", "d_step", "dtd_apply", "dtd_apply_graph",
           "dtd_norm", "dtd_norm_graph", "f_step", "graph_edges", "ladmm", "objective",
           "objective_masked", "patch_data", "rank_rule", "reg_value", "thin_svd", "xi_rule",
           "z_step", "admm_previous", "z_solve_dct"]
