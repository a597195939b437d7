"""The bound behind the cutoff far field's radius (host logic, CPU).

The radius z_c solves kappa/(2 pi) sqrt(pi/(2z)) e^-z (1 + 3/(8z)) L = eps: the
first two terms of the large-argument expansion of K1 (DLMF 10.40.2), which
bound K1 from above for every z > 0 because the remainder after a positive
term is negative and smaller in magnitude (DLMF 10.40.10).  The gradient's
kernel is bounded by kappa^2/(2 pi) (K0 + 3 K1 / z) <= kappa^2/(2 pi) K1 (1 + 3/z).
"""
import numpy as np
from scipy import special


def test_k1_two_term_bound_holds_and_is_tight():
    z = np.concatenate([np.geomspace(1e-3, 1.0, 200), np.linspace(1.0, 700.0, 5000)])
    bound = np.sqrt(np.pi / (2 * z)) * (1 + 3 / (8 * z))
    k1e = special.k1e(z)      # K1(z) e^z, free of underflow
    assert np.all(k1e <= bound * (1 + 1e-15))
    big = z > 50
    assert np.all(bound[big] / k1e[big] < 1 + 1e-3)   # tight where the cutoff lives


def test_gradient_kernel_bound():
    z = np.geomspace(1e-2, 600.0, 4000)
    k0e, k1e = special.k0e(z), special.k1e(z)
    assert np.all(k0e <= k1e)
    assert np.all(k0e + 3 * k1e / z <= k1e * (1 + 3 / z) * (1 + 1e-15))
