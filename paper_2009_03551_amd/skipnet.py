"""Training of the block-skip network from the solver's own runs.

1. ``collect`` runs solves with the exact screen and feature logging: every
   candidate output block that the norm bound cannot rule out contributes its
   features and whether the drop removed it.
2. ``train`` fits the network on the device with the library's own forward,
   gradient and Adam kernels (``tc2_mlp_train``).
3. Solves with ``skip="mlp"`` then skip the candidates whose predicted drop
   probability exceeds the threshold; the error this introduces is measured
   against the exact-screen run of the same input.
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Tuple

import numpy as np

from . import tc2 as T
from .workloads import System


def collect(systems: Iterable[System], precision: str = "fp64", cap: int = 4_000_000,
            **solver_kw) -> Tuple[np.ndarray, np.ndarray]:
    """Features and labels (1 = dropped) logged from solves of `systems`."""
    xs: List[np.ndarray] = []
    ys: List[np.ndarray] = []
    for s in systems:
        sv = T.Solver(s, precision=precision, export=False, skip="bound", log_capacity=cap,
                      **solver_kw)
        sv.run()
        x, y = sv.log()
        sv.close()
        xs.append(x)
        ys.append(y)
    return np.concatenate(xs), np.concatenate(ys)


def init_params(seed: int) -> np.ndarray:
    """He-style random initial parameters (drawn here, passed to the library)."""
    rng = np.random.default_rng(seed)
    nf, nh = T.MLP_IN, 64
    w1 = rng.normal(0.0, np.sqrt(2.0 / nf), (nh, nf))
    w2 = rng.normal(0.0, np.sqrt(2.0 / nh), (nh, nh))
    w3 = rng.normal(0.0, np.sqrt(1.0 / nh), nh)
    return np.concatenate([w1.ravel(), np.zeros(nh), w2.ravel(), np.zeros(nh), w3,
                           np.zeros(1)]).astype(np.float32)


def train(x: np.ndarray, y: np.ndarray, seed: int = 7, epochs: int = 20, batch: int = 2048,
          lr: float = 2e-3, shuffle_seed: Optional[int] = 11):
    """Trained parameters and loss per epoch (data shuffled once, seeded)."""
    if shuffle_seed is not None:
        perm = np.random.default_rng(shuffle_seed).permutation(len(y))
        x, y = x[perm], y[perm]
    return T.mlp_train(x, y, init_params(seed), epochs=epochs, batch=batch, lr=lr)


def confusion(theta, x, y, threshold: float) -> dict:
    """Rates of the skip decision (predicted drop probability > threshold)."""
    z = T.mlp_forward(theta, x)
    skip = z > np.log(threshold / (1 - threshold))
    drop = y > 0.5
    return dict(n=int(len(y)), dropped=float(drop.mean()), skipped=float(skip.mean()),
                skipped_but_kept=int(np.sum(skip & ~drop)),
                recall_of_dropped=float(np.sum(skip & drop) / max(1, drop.sum())))
