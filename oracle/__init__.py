"""CPU oracle (test infrastructure only).

Plain float64 direct-sum implementation of the RIME and its chi-squared, used
by the tests, the smoke check and the benchmark's CPU-baseline leg to judge
the HIP library.  Nothing in the product package imports it.
"""
from .rime_oracle import (  # noqa: F401
    C_LIGHT, GAUSS_K, apply_die, brightness, beam_e, brute_force_vis, chi2, chi2_and_grad,
    chi2_and_grad_ext, chi2_from_vis, disk_shape, gauss_shape, loglike_const, model_vis,
    n_minus_one, phase_K, phase_turns, spectral, total_flux,
)
