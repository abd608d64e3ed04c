"""Adam / AdamW update of the learned weight (the paper trains M with AdamW,
Sec. 3.1), float64.  Test infrastructure only.

One step at count t >= 1 (Kingma & Ba 2015; decoupled weight decay as in
Loshchilov & Hutter 2019):
    M <- M (1 - lr wd)
    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    M <- M - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
Pinned against torch.optim.Adam and AdamW on the CPU.
"""
from __future__ import annotations

import numpy as np


def adam_step(M, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, weight_decay=0.0):
    """Returns the updated (M, m, v); inputs are not modified."""
    M = np.asarray(M, np.float64) * (1.0 - lr * weight_decay)
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return M - lr * mhat / (np.sqrt(vhat) + eps), m, v
