"""FP64 reference of the surrogate MLP: forward, backward and Adam (test infrastructure).

Network: 10 -> 128 -> 128 -> 128 -> 3, SiLU on the hidden layers, linear output;
loss = mean over samples and outputs of (y_hat - y)^2 on standardised targets.
Training keeps FP32 master weights and Adam moments; the products run on BF16 copies
of the weights, of the layer inputs and (backward) of the error signal, with wide
accumulation.  The reference takes those BF16 quantisation points as part of its
definition -- ``bf16()`` rounds to the nearest BF16 value (ties to even) before every
product -- and accumulates exactly in FP64, so the only differences left to the GPU are its FP32 accumulation order and,
rarely, a BF16 rounding that flips because an FP32 sum sits on a rounding boundary.

Parameter layout (flat FP32 vector, 34,819 values):
W1 [128 x 10], b1 [128], W2 [128 x 128], b2 [128], W3 [128 x 128], b3 [128],
W4 [3 x 128], b4 [3]; W is [out x in], row-major.
"""
import numpy as np

SIZES = (10, 128, 128, 128, 3)


def layer_shapes():
    return [(SIZES[k + 1], SIZES[k]) for k in range(len(SIZES) - 1)]


def n_params():
    return sum(o * i + o for o, i in layer_shapes())


def unflatten(theta):
    out, off = [], 0
    for o, i in layer_shapes():
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    return out


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(seed):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases, from a seeded generator."""
    rng = np.random.default_rng(seed)
    ps = []
    for o, i in layer_shapes():
        lim = np.sqrt(6.0 / i)
        ps.append((rng.uniform(-lim, lim, (o, i)), np.zeros(o)))
    return flatten(ps).astype(np.float32)


def forward(theta, X, quant=True):
    """X [B, 10] -> (Y [B, 3], cache of pre-activations and BF16 layer inputs).

    quant=False drops the BF16 rounding (a plain FP64 network, used to check the
    backward pass against finite differences)."""
    q = bf16 if quant else (lambda a: np.asarray(a, dtype=np.float64))
    params = unflatten(np.asarray(theta, dtype=np.float64))
    h = q(X)
    cache = []
    for k, (W, b) in enumerate(params):
        z = h @ q(W).T + b
        cache.append((h, z))
        if k < len(params) - 1:
            h = q(silu(z))
        else:
            h = z
    return h, cache


def loss_and_grad(theta, X, Y, quant=True):
    """MSE loss and its gradient with respect to the flat parameters (same layout).

    The BF16 roundings are passed through unchanged in the backward pass (the
    gradient of a rounding is taken as the identity)."""
    q = bf16 if quant else (lambda a: np.asarray(a, dtype=np.float64))
    params = unflatten(np.asarray(theta, dtype=np.float64))
    Yh, cache = forward(theta, X, quant)
    B = X.shape[0]
    L = np.mean((Yh - Y) ** 2)
    d = 2.0 * (Yh - Y) / (B * Y.shape[1])           # dL/dz of the output layer
    grads = [None] * len(params)
    for k in range(len(params) - 1, -1, -1):
        W, b = params[k]
        h, z = cache[k]
        if k < len(params) - 1:
            d = d * dsilu(z)
        # the error signal is a BF16 operand of both products; the bias gradient sums it unrounded
        grads[k] = (q(d).T @ h, d.sum(axis=0))
        if k > 0:
            d = q(d) @ q(W)
    return L, flatten(grads)


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
