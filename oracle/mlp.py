"""FP64 oracle of the (q, p) selector network (TEST INFRASTRUCTURE ONLY).

A three-layer perceptron maps the 131 sketch features to scores for the 15
(q, p) pairs: 131 -> 64 (ReLU) -> 64 (ReLU) -> 15, softmax, mean
cross-entropy over the batch.  Training uses Adam (Kingma & Ba, "Adam: A
Method for Stochastic Optimization", ICLR 2015, Algorithm 1).

Parameters are one flat vector, in this order (row-major matrices, inputs
along the rows):  W1 (131 x 64), b1 (64), W2 (64 x 64), b2 (64),
W3 (64 x 15), b3 (15)  --  13583 values.
"""
import numpy as np

N_IN, N_HID, N_OUT = 131, 64, 15
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Views of the flat parameter vector as the six named arrays."""
    out, off = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[off:off + size].reshape(shape)
        off += size
    return out


def forward(theta, X):
    """Layer values for a batch X (B x 131): dict with h1, h2, z (logits), prob."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ P["W3"] + P["b3"]
    zs = z - z.max(axis=1, keepdims=True)
    e = np.exp(zs)
    prob = e / e.sum(axis=1, keepdims=True)
    return dict(a1=a1, h1=h1, a2=a2, h2=h2, z=z, prob=prob)


def loss(theta, X, y):
    """Mean cross-entropy -log prob[b, y_b] over the batch."""
    f = forward(theta, X)
    z = f["z"]
    zmax = z.max(axis=1)
    lse = zmax + np.log(np.exp(z - zmax[:, None]).sum(axis=1))
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def loss_and_grad(theta, X, y):
    """Loss and its gradient by back-propagation (chain rule through the
    softmax cross-entropy, the affine maps and the ReLUs; ReLU'(0) = 0)."""
    theta = np.asarray(theta, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y)
    B = X.shape[0]
    P = unpack(theta)
    f = forward(theta, X)
    d3 = f["prob"].copy()
    d3[np.arange(B), y] -= 1.0
    d3 /= B                                   # d loss / d z
    d2 = (d3 @ P["W3"].T) * (f["a2"] > 0)     # d loss / d a2
    d1 = (d2 @ P["W2"].T) * (f["a1"] > 0)     # d loss / d a1
    g = dict(W3=f["h2"].T @ d3, b3=d3.sum(axis=0),
             W2=f["h1"].T @ d2, b2=d2.sum(axis=0),
             W1=X.T @ d1, b1=d1.sum(axis=0))
    grad = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return loss(theta, X, y), grad


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict(theta, X):
    """Class of the largest score (lowest index on ties)."""
    return np.argmax(forward(theta, X)["z"], axis=1)
