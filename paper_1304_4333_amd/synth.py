"""Seeded synthetic inputs for the multinomial-logit SPS hot path.

This module only draws numbers: covariate matrices, outcome vectors, particle
sets, normal and uniform variates, log-weights and integer weights.  It holds
none of the simulator's arithmetic (no log-likelihood, no log-sum-exp, no
weights, no resampling), so both the FP64 CPU oracle and the HIP path may take
their inputs from here without sharing any of the method.

Outcomes are drawn from the random-utility form of the logit model: with
utilities u_c = x' beta_c + e_c, e_c iid standard Gumbel and beta_0 = 0, the
outcome argmax_c u_c has exactly the multinomial-logit law of the paper's
eq. (plogit) (Section 2.1) with outcome 0 as the normalised base.  Drawing
through the argmax avoids evaluating the model's probabilities here.

Workloads (the paper's data sets are not available; these synthetic designs
stand in for them, scaled up from the sizes of Table 1):

  name        C   T(=n)    k    d    J x N       prior sd   precision
  small       2     500    5    5    4 x 256     5          fp64
  binary30    2  10 000   30   30   16 x 1024    5          fp32
  multi4      4  20 000   20   60   16 x 2048    5          bf16x3
  ar100       2  50 000  100  100   32 x 1024    1          bf16x3
  multi6      6 200 000   50  250   64 x 1024    1          bf16x3
  cars3       3     263    4    8   10 x 1000    g-prior    fp64

cars3 has the shape of the paper's smallest multinomial data set (Table 1:
T = 263, k = 4, C = 3; an intercept, one continuous covariate and two
indicators); the reliability and prior-tightness studies (Tables 2 and 3) run
on it with the g-prior of eq. (g-prior_def), J x N = 10 x 1000 and 40 x 2500.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "make_data", "make_particles",
    "make_normals", "make_uniforms", "make_u53", "make_log_weights",
    "make_int_weights", "rng",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape and recipe of one synthetic logit problem.

    C: number of outcomes (outcome 0 is the base, its coefficients are 0).
    T: number of observations.  k: covariates per outcome.
    J, N: particle groups and particles per group (Section 2.2).
    prior_sd: sd of the iid N(0, prior_sd^2) prior on each free parameter.
    design: covariate recipe ("gauss", "gauss_dummy", "gauss_cat", "ar1").
    beta_sd: sd of the data-generating coefficients (0 -> sparse design).
    precision / kernel: the likelihood precision and M-phase proposal the
    workload is exercised with.
    """
    name: str
    C: int
    T: int
    k: int
    J: int
    N: int
    prior_sd: float
    design: str
    beta_sd: float
    n_dummy: int = 0
    dummy_p: float = 0.0
    n_sparse: int = 0
    precision: str = "fp64"
    kernel: str = "rw"
    data_seed: int = 0

    @property
    def d(self) -> int:
        return self.k * (self.C - 1)

    @property
    def P(self) -> int:
        return self.J * self.N


WORKLOADS: Dict[str, Workload] = {
    "small": Workload("small", C=2, T=500, k=5, J=4, N=256, prior_sd=5.0,
                      design="gauss", beta_sd=1.0, precision="fp64",
                      kernel="rw", data_seed=1001),
    "binary30": Workload("binary30", C=2, T=10_000, k=30, J=16, N=1024,
                         prior_sd=5.0, design="gauss_dummy", beta_sd=0.5,
                         n_dummy=10, dummy_p=0.3, precision="fp32",
                         kernel="rw", data_seed=1002),
    "multi4": Workload("multi4", C=4, T=20_000, k=20, J=16, N=2048,
                       prior_sd=5.0, design="gauss_cat", beta_sd=0.5,
                       n_dummy=5, precision="bf16x3", kernel="rw",
                       data_seed=1003),
    "ar100": Workload("ar100", C=2, T=50_000, k=100, J=32, N=1024,
                      prior_sd=1.0, design="ar1", beta_sd=0.0, n_sparse=10,
                      precision="bf16x3", kernel="mala", data_seed=1004),
    "multi6": Workload("multi6", C=6, T=200_000, k=50, J=64, N=1024,
                       prior_sd=1.0, design="gauss_dummy", beta_sd=0.5,
                       n_dummy=10, dummy_p=0.2, precision="bf16x3",
                       kernel="mala", data_seed=1005),
    "cars3": Workload("cars3", C=3, T=263, k=4, J=10, N=1000, prior_sd=1.0,
                      design="gauss_dummy", beta_sd=0.7, n_dummy=2, dummy_p=0.4,
                      precision="fp64", kernel="rw", data_seed=1006),
}


def workload(name: str, **overrides) -> Workload:
    """Return a named workload, optionally with fields replaced (e.g. T)."""
    w = WORKLOADS[name]
    return dataclasses.replace(w, **overrides) if overrides else w


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _design(w: Workload, g: np.random.Generator) -> np.ndarray:
    T, k = w.T, w.k
    if w.design == "gauss":
        # intercept + (k-1) iid N(0,1)
        return np.concatenate([np.ones((T, 1)), g.standard_normal((T, k - 1))], axis=1)
    if w.design == "gauss_dummy":
        # intercept + Gaussian columns + Bernoulli(dummy_p) indicator columns
        ng = k - 1 - w.n_dummy
        Z = g.standard_normal((T, ng))
        D = (g.random((T, w.n_dummy)) < w.dummy_p).astype(np.float64)
        return np.concatenate([np.ones((T, 1)), Z, D], axis=1)
    if w.design == "gauss_cat":
        # intercept + Gaussian columns + one-hot of a uniform (n_dummy+1)-level
        # categorical, reference level dropped
        ng = k - 1 - w.n_dummy
        Z = g.standard_normal((T, ng))
        lev = g.integers(0, w.n_dummy + 1, size=T)
        D = np.zeros((T, w.n_dummy))
        rows = np.nonzero(lev > 0)[0]
        D[rows, lev[rows] - 1] = 1.0
        return np.concatenate([np.ones((T, 1)), Z, D], axis=1)
    if w.design == "ar1":
        # k columns with corr 0.5^|i-j| (AR(1) across columns), no intercept
        E = g.standard_normal((T, k))
        X = np.empty((T, k))
        X[:, 0] = E[:, 0]
        s = np.sqrt(0.75)
        for i in range(1, k):
            X[:, i] = 0.5 * X[:, i - 1] + s * E[:, i]
        return X
    raise ValueError(f"unknown design {w.design!r}")


def _beta(w: Workload, g: np.random.Generator) -> np.ndarray:
    """Data-generating coefficients, shape (C-1, k) for outcomes 1..C-1."""
    if w.n_sparse:
        B = np.zeros((w.C - 1, w.k))
        for c in range(w.C - 1):
            idx = g.choice(w.k, size=w.n_sparse, replace=False)
            B[c, idx] = g.standard_normal(w.n_sparse)
        return B
    return w.beta_sd * g.standard_normal((w.C - 1, w.k))


def make_data(w: Workload, seed: Optional[int] = None):
    """Draw (X, y, beta_true) for workload w.

    X: float64 (T, k) row-major; y: int32 (T,) in [0, C); beta_true (C-1, k).
    y_t = argmax_c (x_t' beta_c + Gumbel noise), beta_0 = 0.
    """
    g = rng(w.data_seed if seed is None else seed)
    X = _design(w, g)
    B = _beta(w, g)
    util = np.zeros((w.T, w.C))
    util[:, 1:] = X @ B.T
    util += g.gumbel(size=(w.T, w.C))
    y = np.argmax(util, axis=1).astype(np.int32)
    return np.ascontiguousarray(X), y, B


def make_particles(P: int, d: int, scale: float = 1.0, seed: int = 0,
                   center: Optional[np.ndarray] = None) -> np.ndarray:
    """P x d particle matrix (row p = particle p), N(center, scale^2) entries."""
    th = scale * rng(seed).standard_normal((P, d))
    if center is not None:
        th += np.asarray(center, dtype=np.float64).reshape(1, -1)
    return np.ascontiguousarray(th)


def make_normals(P: int, d: int, seed: int) -> np.ndarray:
    return np.ascontiguousarray(rng(seed).standard_normal((P, d)))


def make_uniforms(P: int, seed: int) -> np.ndarray:
    """Uniforms strictly inside (0, 1): (U + 1/2) 2^-53 with U a 53-bit integer."""
    U = make_u53(P, seed)
    return (U.astype(np.float64) + 0.5) * 2.0 ** -53


def make_u53(count: int, seed: int) -> np.ndarray:
    """Integers uniform on [0, 2^53) as uint64."""
    return rng(seed).integers(0, 1 << 53, size=count, dtype=np.uint64)


def make_log_weights(P: int, seed: int, spread: float = 3.0,
                     n_neg_inf: int = 0) -> np.ndarray:
    """Log-weights with a given spread; optionally some entries set to -inf."""
    g = rng(seed)
    lw = spread * g.standard_normal(P) - 50.0
    if n_neg_inf:
        lw[g.choice(P, size=n_neg_inf, replace=False)] = -np.inf
    return lw


def make_int_weights(J: int, N: int, seed: int, bits: int = 40) -> np.ndarray:
    """Integer weights in [0, 2^bits] with the group maximum equal to 2^bits."""
    g = rng(seed)
    W = g.integers(0, 1 << bits, size=(J, N), dtype=np.uint64)
    zero = g.random((J, N)) < 0.2
    W[zero] = 0
    W[np.arange(J), g.integers(0, N, size=J)] = np.uint64(1 << bits)
    return W.reshape(-1)
