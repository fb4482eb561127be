"""Double-precision reference of the warm-start network and its training (test infrastructure only).

The network maps the 12 per-contact features to 3 normalised impulses:
12 -> 64 (ReLU) -> 64 (ReLU) -> 3 (linear).  The flat parameter vector is
W1[12][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3] (row-major,
input index first).  The loss is the mean squared error over the batch and
the three outputs; the optimiser is Adam (Kingma & Ba 2015) with bias
correction.  Only the tests and the benchmark's baseline leg use this file.
"""
import numpy as np

N_IN, N_HID, N_OUT = 12, 64, 3
SIZES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unflatten(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def flatten(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    P = unflatten(p)
    X = np.asarray(X, np.float64)
    z1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"] + P["b3"]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(p, X, T):
    """Mean squared error over all outputs and its gradient with respect to the flat parameters."""
    P = unflatten(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    T = np.asarray(T, np.float64)
    n = X.shape[0]
    d = y - T
    loss = float((d * d).sum() / (n * N_OUT))
    dy = 2.0 * d / (n * N_OUT)
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dh2 = (dy @ P["W3"].T) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ P["W2"].T) * (z1 > 0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(0)
    return loss, flatten(g)


class Adam:
    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, p, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)
