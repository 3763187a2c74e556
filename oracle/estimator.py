"""Exact moments of the one-sample light-sampling estimator.

Test infrastructure (see the package docstring).

Sec. 1: direct illumination is estimated by Monte Carlo, picking light i with
probability p_i and returning f_i V_i / p_i; it is unbiased when p_i > 0
wherever f_i V_i > 0, and its noise shrinks as p approaches f V.  Sec. 3.1
keeps every probability positive by clamping the predicted visibility.  For a
discrete pick these moments have closed forms, so no Monte Carlo noise enters
a comparison between sampling distributions:

    mu    = sum_i f_i V_i                      (the exact direct illumination)
    E     = sum_{p_i > 0} f_i V_i              (= mu iff unbiased)
    Var   = sum_{p_i > 0} (f_i V_i)^2 / p_i - E^2
    waste = sum_{V_i = 0} p_i                  (probability of picking an occluded light)
"""
from __future__ import annotations

import numpy as np


def moments(f, V, p):
    """Per-point (mu, E, Var, waste) for contributions f, true visibility V and pick pmf p, all [n,M]."""
    f = np.asarray(f, np.float64)
    V = np.asarray(V, np.float64)
    p = np.asarray(p, np.float64)
    c = f * V
    mu = c.sum(axis=1)
    pos = p > 0
    E = np.where(pos, c, 0.0).sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        second = np.where(pos, c * c / np.where(pos, p, 1.0), 0.0).sum(axis=1)
    var = second - E * E
    waste = np.where(V == 0, p, 0.0).sum(axis=1)
    return mu, E, var, waste
