"""MI355X (gfx950) implementation of the localized stochastic FBSDE / local-linear-regression scheme
for very high-dimensional semilinear parabolic PDEs: HIP kernels behind a C ABI (include/fbsde.h),
with a thin Python front end over PyTorch device memory and streams."""
from . import _native
from .api import (TIMED_CG_LOOP, TIMED_CG_PRODUCT, TIMED_LITERAL_ANCHORS, TIMED_LITERAL_GRAM, workspace_cg_rows, solve_noalloc, batched_cg_bytes, NOALLOC_SCRATCH_BYTES, CapturedBatch, CapturedSolve, FBSDEFunction, Problem, autotune, autotune_reset, batched_workspace, box_muller,
                  cholesky_solve, gemm, launch_timer, launch_timer_kinds, launch_timer_read, literal_coef_workspace_size, literal_workspace_size, coef_workspace_size, solve_coef, solve_coef_backward, solve_coef_autograd, sigma_workspace_size, solve_sigma, solve_sigma_backward, normals, solve, solve_autograd, solve_backward, solve_batched, solve_batched_backward, solve_literal, solve_literal_geometric, solve_step, state_ld, terminal, time_kernel,
                  workspace, workspace_size)
from ._native import (F32C, F64, F_ALLEN_CAHN, F_BURGERS, F_HJB, F_HJ_SINK, F_LOG_POT, F_ZERO, G_AC, G_AFFINE, G_CASE2,
                      G_HJ_GAUSS,
                      G_HJB_LOG, G_LOGISTIC, G_QUAD, SOLVER_AUTO, SOLVER_CG, ST_CG_MAXIT,
                      ST_NEWTON_FLAT, ST_NONFINITE, FbsdeError)

__all__ = ["TIMED_CG_LOOP", "workspace_cg_rows", "batched_cg_bytes", "solve_noalloc", "NOALLOC_SCRATCH_BYTES", "TIMED_CG_PRODUCT", "TIMED_LITERAL_GRAM", "TIMED_LITERAL_ANCHORS", "Problem", "CapturedSolve", "CapturedBatch", "autotune", "autotune_reset", "FBSDEFunction", "solve_autograd", "solve",
           "solve_step", "solve_backward", "solve_batched", "solve_batched_backward", "batched_workspace", "terminal", "normals", "box_muller", "state_ld", "workspace",
           "workspace_size", "gemm", "cholesky_solve", "time_kernel", "launch_timer", "launch_timer_kinds", "launch_timer_read", "solve_literal", "solve_literal_geometric", "literal_workspace_size", "literal_coef_workspace_size", "coef_workspace_size", "solve_coef", "solve_coef_backward", "solve_coef_autograd", "sigma_workspace_size", "solve_sigma", "solve_sigma_backward", "F64", "F32C", "F_ZERO", "F_ALLEN_CAHN",
           "F_HJB", "F_BURGERS", "F_HJ_SINK", "F_LOG_POT", "G_QUAD", "G_AC", "G_HJB_LOG", "G_AFFINE", "G_LOGISTIC", "G_HJ_GAUSS", "G_CASE2",
           "SOLVER_AUTO", "SOLVER_CG", "ST_CG_MAXIT", "ST_NEWTON_FLAT", "ST_NONFINITE",
           "FbsdeError"]
