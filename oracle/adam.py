"""Adam (Kingma & Ba 2015), float64, in torch.optim.Adam's update order.

TEST INFRASTRUCTURE ONLY (see the package docstring).

m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""

import numpy as np


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step (step counts from 1).  Returns new (theta, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    denom = np.sqrt(v / (1.0 - beta2 ** step)) + eps
    return np.asarray(theta, dtype=np.float64) - lr * mhat / denom, m, v
