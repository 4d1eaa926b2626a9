"""Marginal-CDF modelling of the inputs (Section IV.D, Fig. 4) -- TEST INFRASTRUCTURE ONLY.

Imported only by tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py.

Section IV.D replaces the affine moment analysis behind eq. (18) with a fitted marginal CDF
of the input samples: the square root of the fitted distribution's second moment is the
sigma_s (or sigma_k) that goes into eq. (18).  The paper fits a two-parameter Weibull to the
music-matching features and a zero-mean Laplacian to audio (Fig. 4), by expectation
maximization; for one component EM is maximum likelihood, which is what is computed here.

Readings (also listed in the design notes):
  R19 "bivariate Weibull" is the two-parameter Weibull (scale lambda, shape kappa, the two
      values Fig. 4(a) prints), fitted to the positive samples (the features are magnitudes;
      zero samples carry no likelihood and are left out).
  R20 the fitted sigma_s, sigma_k are per source (one value per signal and per kernel), not per
      block; the block maximum still sets the rounding noise sigma_v of eq. (18) per block.
  R21 the 16-sample sets of Fig. 4 do not change a marginal fit: all samples are pooled.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .core import BlockParams, FULL, SYM, ASYM2, kernel_stats, max_q, partition, snr_model_db, block_stats

LAPLACE, WEIBULL = "laplace", "weibull"


@dataclass
class MarginalFit:
    model: str
    scale: float   # Laplacian b, or Weibull lambda
    shape: float   # Weibull kappa (1.0 for the Laplacian)
    sigma: float   # square root of the fitted second moment
    n: int         # samples the fit used


def fit_laplace(x) -> MarginalFit:
    """Zero-mean Laplacian (Fig. 4(b)): the likelihood maximizer of the scale is mean |x|, and
    E[x^2] = 2 b^2."""
    x = np.asarray(x, dtype=np.float64).ravel()
    b = float(np.mean(np.abs(x))) if x.size else 0.0
    return MarginalFit(LAPLACE, b, 1.0, math.sqrt(2.0) * b, int(x.size))


def fit_weibull(x, tol: float = 1e-13, max_iter: int = 200) -> MarginalFit:
    """Two-parameter Weibull on the positive samples (reading R19), maximum likelihood.

    The shape kappa solves  sum(y^k ln y) / sum(y^k) - 1/k - mean(ln y) = 0  (the score equation
    once lambda is profiled out); Newton's method on it, with y = x / max(x) so that the powers
    stay in range.  Then lambda = (mean x^kappa)^(1/kappa) and E[x^2] = lambda^2 Gamma(1 + 2/kappa).
    """
    x = np.asarray(x, dtype=np.float64).ravel()
    x = x[x > 0.0]
    if x.size < 2:
        return MarginalFit(WEIBULL, 0.0, 1.0, 0.0, int(x.size))
    xm = float(np.max(x))
    ly = np.log(x / xm)
    mly = float(np.mean(ly))
    sd = float(np.std(ly))
    k = math.pi / (math.sqrt(6.0) * sd) if sd > 0.0 else 1.0  # moment start for the shape
    for _ in range(max_iter):
        yk = np.exp(k * ly)
        a0 = float(np.sum(yk))
        a1 = float(np.sum(yk * ly))
        a2 = float(np.sum(yk * ly * ly))
        g = a1 / a0 - 1.0 / k - mly
        dg = (a2 * a0 - a1 * a1) / (a0 * a0) + 1.0 / (k * k)
        step = g / dg
        k_new = k - step
        if k_new <= 0.0:
            k_new = 0.5 * k
        done = abs(k_new - k) <= tol * k
        k = k_new
        if done:
            break
    lam = xm * float(np.mean(np.exp(k * ly))) ** (1.0 / k)
    sigma = lam * math.sqrt(math.gamma(1.0 + 2.0 / k))
    return MarginalFit(WEIBULL, lam, k, sigma, int(x.size))


def fit(x, model: str) -> MarginalFit:
    return fit_laplace(x) if model == LAPLACE else fit_weibull(x)


def auto_params_sigma(s, k, W_block: int, target_db: float, sigma_s: float, sigma_k: float,
                      calib_db: float = 0.0, candidates=(SYM, ASYM2)):
    """Section IV.D selection with source-level sigmas (reading R20): as core.auto_params, with
    sigma_s and sigma_k in eq. (18) in place of each block's and the kernel's root second
    moment; the maxima stay per block and per kernel."""
    part = partition(np.asarray(s).size, np.asarray(k).size, W_block)
    kmax, _ = kernel_stats(k)
    ps = []
    for w in range(part.P):
        smax, rms = block_stats(part.window(s, w))
        chosen = BlockParams(FULL, 0, 0, 0.0, smax, rms, math.inf)
        for mode in candidates:
            q = max_q(mode, part.N_odd)
            if q < 1:
                continue
            if smax == 0.0 or kmax == 0.0:  # an all-zero operand is reproduced exactly
                chosen = BlockParams(mode, q, q, 0.0, smax, rms, math.inf)
                break
            snr = snr_model_db(sigma_s, smax, sigma_k, kmax, q, q) + calib_db
            if snr >= target_db:
                chosen = BlockParams(mode, q, q, 0.0, smax, rms, snr)
                break
        ps.append(chosen)
    return ps
