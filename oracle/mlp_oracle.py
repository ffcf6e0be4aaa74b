"""FP64 NumPy reference of the learned C6 surrogate network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The surrogate is not part of the paper: it approximates the CN-dependent
C6 of Eq. 3 (and its two CN derivatives) for one element pair with a small
multilayer perceptron, trained on samples that Eq. 3 itself labels.  This
module holds the plain definition of that network, its mean-squared-error
loss, the loss gradient by backpropagation, one Adam step and the cosine
step-size schedule, so that the GPU training kernels can be checked
against it.

Network (row-vector convention, inputs already scaled to [-1, 1]):
    z1 = x W1 + b1      (2 -> 32),  h1 = silu(z1)
    z2 = h1 W2 + b2     (32 -> 32), h2 = silu(z2)
    y  = h2 W3 + b3     (32 -> 3)
with silu(z) = z / (1 + exp(-z)).  Parameter vector (1251 values):
W1[2][32], b1[32], W2[32][32], b2[32], W3[32][3], b3[3].
Loss of one element pair: mean over its samples and the 3 outputs of
(y - t)^2.

Parity: pinned (finite differences of the loss, closed-form networks).
"""

import numpy as np

HIDDEN = 32
N_PARAMS = 2 * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN * 3 + 3


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    o = 0
    out = {}
    for name, shape in (("W1", (2, HIDDEN)), ("b1", (HIDDEN,)),
                        ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
                        ("W3", (HIDDEN, 3)), ("b3", (3,))):
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def pack(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"],
                           p["W3"].ravel(), p["b3"]])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x):
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"] + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["W3"] + p["b3"]
    return y, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss_and_grad(theta, x, t):
    """Mean squared error over samples and outputs, and its gradient."""
    p = unpack(theta)
    y, c = forward(theta, x)
    t = np.asarray(t, dtype=np.float64)
    m = y.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / (3.0 * m)
    g = {"W3": c["h2"].T @ dy, "b3": dy.sum(0)}
    dz2 = (dy @ p["W3"].T) * silu_grad(c["z2"])
    g["W2"] = c["h1"].T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * silu_grad(c["z1"])
    g["W1"] = c["x"].T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def cosine_step_size(step, total, lr0, lr1):
    """Step size of training step ``step`` (0-based) of ``total`` under a
    cosine decay from lr0 (step 0) to lr1 (step total)."""
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + np.cos(np.pi * step / total))


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new theta, m, v."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
