"""Adam update of the training loop, FP64.

Paper, example parameter file: opt = "Adam", base_lr = 0.001, applied once per
iteration to the gradient of the loss.  The other hyperparameters are not
given; the reading is the standard bias-corrected Adam (Kingma & Ba, 2015) with
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and optimizer state kept across steps.

    m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
    p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

Pinned by: the first step from zero state moves every parameter by
-lr g/(|g| + eps), a constant gradient keeps the step at lr, and the second and
third steps with varying gradients match the closed forms of the bias-corrected
moments as weighted means of the gradients (which fix beta1 and beta2).
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
