"""Online training of the learned Poisson warm start from PIC runs.

Each step's field solve, with the context's warm start set to "record" (or
"unet"), records its pair: the input (r0 / sigma, phi_prev / V_ref), where
r0 = b - A phi_prev is the residual of the previous potential over the
unknowns and sigma its RMS, and the target (phi - phi_prev) / sigma of the
converged potential.  The exact correction A^-1 r0 is linear in r0, so the
normalised pair does not depend on the charge's magnitude.  The network
trains on these pairs with Adam (MSE loss, cosine learning-rate decay) in
the library's own BF16 forward and backward kernels; whatever it predicts,
the multigrid V-cycles finish every solve to the same residual.
"""
import math

import numpy as np


def collect_pairs(pic, dt, steps):
    """Run `steps` PIC steps recording the solve's pair after each one;
    returns [(input, target)] device tensors and the step diagnostics."""
    pairs, diags = [], []
    pic.set_warm_start("record")
    for _ in range(steps):
        _, d = pic.step(dt)
        pairs.append(pic.warm_pair())
        diags.append(d)
    pic.set_warm_start("prev")
    return pairs, diags


def cosine_lr(k, total, lr_max, lr_min):
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * k / total))


def train(net, pairs, epochs, lr_max=1e-3, lr_min=1e-5, seed=0, loss="mse",
          k0=1):
    """Adam over `epochs` shuffled passes of `pairs`; returns the mean loss
    of each epoch.  loss "mse" fits the normalised correction; "residual"
    minimises the residual of the start it produces (k0: first unknown
    plane of the grid)."""
    net.set_loss(loss, k0)
    rng = np.random.default_rng(seed)
    total = epochs * len(pairs)
    k = 0
    means = []
    for _ in range(epochs):
        losses = []
        for i in rng.permutation(len(pairs)):
            x, t = pairs[i]
            losses.append(net.train_step(x, t, lr=cosine_lr(k, total, lr_max, lr_min)))
            k += 1
        means.append(float(np.mean(losses)))
    return means
