"""Finite-difference references for the reverse-mode tests (oracle only).

A checkpoint segment of the differentiation workload (50k agents at area
fraction 3.9, a 256^2 grid on which one agent deposits 0.65 per step into
its four nodes) is a rough map: the interpolated gradient of such a spiky
field changes slope at every cell face, so two trajectories a float32
rounding apart can see derivatives that differ by percents.  The reference
for a float32 implementation is therefore an ensemble:

* fd_0: the FP64 oracle's central difference at the checkpoint;
* fd_m, m = 1..M: the same with a fixed perturbation of half a float32 ulp
  (random sign, per coordinate and per node) added to the state after every
  step, common to the +h and -h runs, so that the difference still sees only
  theta.  These are derivatives along trajectories a float32 state could
  equally have taken.

Their RMS deviation from fd_0 measures how well the derivative is defined
at float32 resolution.
"""
from __future__ import annotations

import numpy as np

import oracle


def _half_ulp_noise(a: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    sp = np.spacing(np.abs(a).astype(np.float32)).astype(np.float64)
    return 0.5 * sp * rng.choice([-1.0, 1.0], size=a.shape)


def run_perturbed(w, x0, sp, c0, step0: int, K: int, theta, noise_seed: int | None):
    """K oracle steps of one instance from (x0, c0) at theta; with a seed,
    half-ulp perturbations are added to positions and field after each step
    (the same ones for a given seed whatever theta is)."""
    wt = oracle.workload_at(w, theta)
    p = oracle.params(wt, 0)
    X = np.asarray(x0, np.float64).copy()
    c = np.asarray(c0, np.float64).copy()
    rng = np.random.default_rng(noise_seed) if noise_seed is not None else None
    st = step0
    for _ in range(K):
        X, c, st = oracle.step(p, X, sp, c, st)
        if rng is not None:
            X = X + _half_ulp_noise(X, rng)
            c = c + _half_ulp_noise(c, rng)
            if w.periodic:
                X = np.mod(X, w.L)
                X[X >= w.L] = 0.0
            else:
                np.clip(X, 0.0, w.L, out=X)
    return X, c


def segment_fd_ensemble(w, x0, sp, c0, step0: int, K: int, theta, funcs, M: int = 4,
                        rel: float = 1e-7, seed: int = 0):
    """Central differences in each theta_j, as derivatives with respect to the
    scale of theta_j (theta_j d/dtheta_j), of the functionals funcs(X, c) ->
    array after K steps: returns (fd0, members), arrays of shape
    (3, n_funcs) and (M, 3, n_funcs)."""
    theta = np.asarray(theta, np.float64)

    def F(th, ns):
        X, c = run_perturbed(w, x0, sp, c0, step0, K, th, ns)
        return np.asarray(funcs(X, c), np.float64)

    out = []
    for ns in [None] + [seed * 1000 + m for m in range(1, M + 1)]:
        rows = []
        for j in range(3):
            h = rel * theta[j]
            tp, tm = theta.copy(), theta.copy()
            tp[j] += h
            tm[j] -= h
            rows.append((F(tp, ns) - F(tm, ns)) / (2 * h) * theta[j])
        out.append(np.array(rows))
    return out[0], np.array(out[1:])
