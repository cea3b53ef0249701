"""FP64 references of the training-loop steps of the paper's protocol (Sec. 4.4).

TEST INFRASTRUCTURE ONLY (see model.py for the import rule).

  adam_step  the Adam update (Kingma and Ba): m = b1 m + (1 - b1) g,
             v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) /
             (sqrt(v / (1 - b2^t)) + eps). The paper gives the learning rates
             (Gaussians 1e-2, MLP 8e-3, hyperparameter table), not the decays
             or epsilon; the usual 0.9, 0.999, 1e-8 are the reading.
  anneal_tx  anneal smoothing (Sec. 4.4, anneal-smoothing equations): the
             position gets gamma * n * (2 / cbrt(N_s)) * (1 - i / tau) in the
             unit cube the positions are normalised to (so each axis is scaled
             by the room's extent), n a standard 3D normal draw passed in; the
             decay is clamped at 0 past tau (the printed linear factor would go
             negative there).

Pins: tests/test_oracle_train.py (Adam's first step from zero moments moves
each parameter by lr g / (|g| + eps); a constant gradient keeps doing so; the
anneal noise vanishes from tau on and has the stated scale at i = 0).
"""
from __future__ import annotations

import numpy as np

BETA1, BETA2, EPS = 0.9, 0.999, 1e-8
LR_GAUSSIANS, LR_MLP = 1e-2, 8e-3
GAMMA, TAU = 1.0, 10_000


def adam_step(p, g, m, v, lr, t, b1=BETA1, b2=BETA2, eps=EPS):
    """One Adam step at step number t >= 1; returns (p, m, v) as new FP64 arrays."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def anneal_tx(tx, noise, i, gamma=GAMMA, tau=TAU, n_positions=1, room=((0, 0, 0), (6, 6, 3))):
    """Anneal-smoothed positions (B, 3) in metres."""
    lo, hi = np.asarray(room[0], np.float64), np.asarray(room[1], np.float64)
    f = gamma * 2.0 / np.cbrt(float(n_positions)) * max(0.0, 1.0 - i / tau)
    return np.asarray(tx, np.float64) + f * (hi - lo) * np.asarray(noise, np.float64)
