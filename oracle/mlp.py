"""FP64 oracle of the learned shock sensor's network (10 -> 32 -> 32 -> 1,
ReLU, ReLU, sigmoid) and of its training step.

TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline).  Plain numpy,
written from the definitions: forward pass, class-weighted binary
cross-entropy, backpropagation, Adam.  Weights are evaluated as the GPU
stores them: rounded to bfloat16 (round to nearest even).

Flat parameter order (1441 values): W1[10][32] (input-major), b1[32],
W2[32][32] (input-major), b2[32], w3[32], b3.
"""
import numpy as np

NIN, NH = 10, 32
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """bfloat16 bit patterns (uint16) of x (round to nearest even)."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return b.astype(np.uint16)


def init(seed=0):
    """Glorot-uniform initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.uniform(-1, 1, (NIN, NH)) * np.sqrt(6.0 / (NIN + NH)),
         "b1": np.zeros(NH),
         "W2": rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / (2 * NH)),
         "b2": np.zeros(NH),
         "w3": rng.uniform(-1, 1, NH) * np.sqrt(6.0 / (NH + 1)),
         "b3": np.zeros(1)}
    return pack(p)


def forward(theta, X, round_activations=False):
    """Logits z of samples X (n, 10).  round_activations: the inference form,
    where the inputs of every layer are bfloat16."""
    p = unpack(bf16_round(theta))
    X = np.asarray(X, dtype=np.float64)
    if round_activations:
        X = bf16_round(X)
    a1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(a1, 0.0)
    if round_activations:
        h1 = bf16_round(h1)
    a2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(a2, 0.0)
    if round_activations:
        h2 = bf16_round(h2)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, (X, a1, h1, a2, h2, p)


def sample_weights(y, w_neg):
    return np.where(np.asarray(y) > 0, 1.0, float(w_neg))


def loss(theta, X, y, w_neg=10.0):
    """Mean class-weighted binary cross-entropy of sigmoid(z) against y;
    label-0 (not smooth) samples weigh w_neg (a false "smooth" costs more)."""
    z, _ = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    w = sample_weights(y, w_neg)
    # log(1 + e^z) - y z, evaluated stably
    sp = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    return float(np.mean(w * (sp - y * z)))


def grad(theta, X, y, w_neg=10.0):
    """Analytic gradient of `loss` with respect to the (bfloat16-rounded)
    weights, by backpropagation."""
    z, (Xr, a1, h1, a2, h2, p) = forward(theta, X)
    y = np.asarray(y, dtype=np.float64)
    n = len(y)
    w = sample_weights(y, w_neg)
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = w * (sig - y) / n                       # d loss / d z
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"]) * (a2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"].T) * (a1 > 0)
    g["W1"] = Xr.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def adam(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1) on the FP64 master weights."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
