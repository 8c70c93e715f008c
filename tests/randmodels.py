"""Seeded random reaction-diffusion models for parity tests (inputs only)."""
import numpy as np


def random_model(rng: np.random.Generator, S: int, R: int, n_regions: int = 1,
                 immobile_frac: float = 0.2) -> dict:
    """Random mass-action model: orders 0-2 (homodimers included), rate
    constants log-uniform, some immobile species, per-region rate tables."""
    D = 10.0 ** rng.uniform(-13, -11, S)
    D[rng.uniform(size=S) < immobile_frac] = 0.0
    if not (D > 0).any():
        D[0] = 1e-12
    lhs = np.zeros((R, S), np.int32)
    rhs = np.zeros((R, S), np.int32)
    k = np.zeros((n_regions, R))
    for r in range(R):
        kind = rng.integers(0, 5)
        if kind == 0:        # 0 -> X
            order = 0
        elif kind in (1, 2):  # X -> ...
            order = 1
        else:
            order = 2
        reac = list(rng.choice(S, size=order, replace=True)) if order else []
        for s in reac:
            lhs[r, s] += 1
        n_prod = int(rng.integers(0 if order else 1, 3))
        for s in rng.choice(S, size=n_prod, replace=True):
            rhs[r, s] += 1
        if order == 0:
            base = 10.0 ** rng.uniform(-4, -1)      # M/s
        elif order == 1:
            base = 10.0 ** rng.uniform(-1, 2)       # 1/s
        else:
            base = 10.0 ** rng.uniform(5, 8)        # 1/(M s)
        k[:, r] = base * rng.uniform(0.5, 1.5, n_regions)
        if n_regions > 1 and rng.uniform() < 0.3:
            k[int(rng.integers(0, n_regions)), r] = 0.0
    return dict(D=D, lhs=lhs, rhs=rhs, kcst=k)


def random_counts(rng: np.random.Generator, S: int, T: int, mean: float) -> np.ndarray:
    lam = rng.uniform(0, 2 * mean, S)[:, None] * np.ones((1, T))
    c = rng.poisson(lam).astype(np.int32)
    c[:, rng.uniform(size=T) < 0.3] = 0  # empty tets
    return c
