"""Test infrastructure: plain CPU FP64 oracle of ChASE (Algorithm 1).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the GPU library never imports, links or calls it.
"""
from .chase import (Options, Stats, chebyshev_filter, cheb_poly_value, degrees,
                    dos_mu, eigvec_adjoint, filter_coefficients, jacobi_eigh, lanczos_norm,
                    lanczos_runs,
                    qr_locked, rayleigh_ritz, residual_norms, solve,
                    spectral_bounds, tridiag_eig)

__all__ = ["Options", "Stats", "chebyshev_filter", "cheb_poly_value", "degrees",
           "dos_mu", "eigvec_adjoint", "filter_coefficients", "jacobi_eigh", "lanczos_norm", "lanczos_runs",
           "qr_locked", "rayleigh_ritz", "residual_norms", "solve",
           "spectral_bounds", "tridiag_eig"]
