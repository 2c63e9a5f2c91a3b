"""MI355X (gfx950) fast-diagonalisation preconditioned CG for isogeometric
Poisson problems (Sangalli & Tani, arXiv 1602.01636).

The solver lives in the HIP library libigafd.so (C ABI in include/igafd.h);
`binding` marshals arguments to it.  Importing this package does not load the
library; the first igafd_* call does, and fails loudly when it is not built.
"""
from .binding import (IgafdError, Context, Mlp, igafd_apply_A, igafd_apply_precond, igafd_autotune,
                      igafd_destroy, igafd_diagonals, igafd_features, igafd_features_noalloc, igafd_get_adi, igafd_get_eigen,
                      igafd_get_shape, igafd_last_error, igafd_load_vector, igafd_lshape_corner,
                      igafd_lshape_setup, igafd_mlp_create, igafd_mlp_destroy, igafd_mlp_fit_normalization,
                      igafd_mlp_forward, igafd_mlp_get_params, igafd_mlp_gradient, igafd_mlp_num_params,
                      igafd_mlp_set_params, igafd_mlp_train_step, igafd_scaling_gate, igafd_scaling_targets,
                      igafd_set_adi, igafd_set_adi_greedy, igafd_set_scaling, igafd_set_scaling_diag_ratio,
                      igafd_setup, igafd_setup_precond, igafd_sizes, igafd_solve, igafd_solve_batched,
                      igafd_spectral_bounds, igafd_univariate, lib)

__all__ = ["IgafdError", "Context", "Mlp", "igafd_apply_A", "igafd_apply_precond", "igafd_autotune",
           "igafd_destroy", "igafd_diagonals", "igafd_features", "igafd_features_noalloc", "igafd_get_adi", "igafd_get_eigen",
           "igafd_get_shape", "igafd_last_error", "igafd_load_vector", "igafd_lshape_corner",
           "igafd_lshape_setup", "igafd_mlp_create", "igafd_mlp_destroy", "igafd_mlp_fit_normalization",
           "igafd_mlp_forward", "igafd_mlp_get_params", "igafd_mlp_gradient", "igafd_mlp_num_params",
           "igafd_mlp_set_params", "igafd_mlp_train_step", "igafd_scaling_gate", "igafd_scaling_targets",
           "igafd_set_adi", "igafd_set_adi_greedy", "igafd_set_scaling", "igafd_set_scaling_diag_ratio",
           "igafd_setup", "igafd_setup_precond", "igafd_sizes", "igafd_solve", "igafd_solve_batched",
           "igafd_spectral_bounds", "igafd_univariate", "lib"]
