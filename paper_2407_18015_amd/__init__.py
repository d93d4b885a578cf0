"""Critical-point probabilities of uncertain 2-D fields on MI355X.

Implements the method of Athawale et al., "Uncertainty Visualization of
Critical Points of 2D Scalar Fields for Parametric and Nonparametric
Probabilistic Models" (arXiv 2407.18015): per-vertex probability of being a
local minimum / maximum (and saddle / regular point) on the 4-neighbour
stencil for uniform, Epanechnikov and histogram models (closed form), and a correlated Gaussian over the
stencil (Monte Carlo), with fitting from ensemble members, adjoints and a
batched persistent launch.  All computation runs in the HIP library
``libcpcrit.so`` behind the C ABI of ``include/cpcrit.h``.
"""
from . import _lib
from .ops import (CPProb, Field, backward, batched, batched_describe, batched_pin,
                  classify, critical_point_probability, field_of, fit, fit_error_bound, fit_forward,
                  forward, n_params, philox, semianalytical)

__all__ = ["CPProb", "Field", "backward", "batched", "batched_describe", "batched_pin",
           "classify", "critical_point_probability", "field_of", "fit", "fit_error_bound", "fit_forward", "forward",
           "n_params", "philox", "semianalytical", "_lib"]
