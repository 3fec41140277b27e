"""FP64 reference of the transport surrogate's network. TEST INFRASTRUCTURE ONLY.

Network 5 -> 64 -> 64 -> 4 with ReLU hidden units and a linear output. Inputs are
mapped from the domain box to [-1, 1]; outputs are standardised with (mean, std).
Parameters are one flat vector: W1 [5, 64], b1 [64], W2 [64, 64], b2 [64],
W3 [64, 4], b3 [4] (4804 values; W[in, out]).

With quantize=True the forward pass rounds what the GPU kernels feed to its bf16
matrix cores (scaled inputs, weights, hidden activations) to bf16 and computes
everything else in FP64: the same network the kernels evaluate, without their
FP32 summation order. The backward pass then also rounds the operands the
training kernel feeds to its matrix cores: the output error dL/dy and the
back-propagated errors of both hidden layers (bias gradients are the sums of
those rounded errors).
"""
import numpy as np

SIZES = [("W1", (5, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 4)), ("b3", (4,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def scale_inputs(X, lo, hi):
    X = np.asarray(X, dtype=np.float64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (X - lo) / (hi - lo) - 1.0


def forward(theta, X, lo, hi, mean, std, quantize=True, return_all=False):
    P = unpack(theta)
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    xh = q(scale_inputs(X, lo, hi))
    z1 = xh @ q(P["W1"]) + P["b1"]
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ q(P["W2"]) + P["b2"]
    h2 = q(np.maximum(z2, 0.0))
    yh = h2 @ q(P["W3"]) + P["b3"]
    y = yh * np.asarray(std) + np.asarray(mean)
    if return_all:
        return dict(xh=xh, z1=z1, h1=h1, z2=z2, h2=h2, yh=yh, y=y, P=P)
    return y


def loss_and_grad(theta, X, Y, lo, hi, mean, std, quantize=True):
    """Mean over samples and outputs of the squared error of standardised outputs,
    and its gradient with respect to theta (FP64 back-propagation)."""
    f = forward(theta, X, lo, hi, mean, std, quantize=quantize, return_all=True)
    P = f["P"]
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    t = (np.asarray(Y, dtype=np.float64) - np.asarray(mean)) / np.asarray(std)
    n = X.shape[0]
    r = f["yh"] - t
    loss = float(np.mean(r * r))
    dy = q(2.0 * r / (n * 4))
    g = {}
    g["W3"] = f["h2"].T @ dy
    g["b3"] = dy.sum(0)
    dz2 = q((dy @ q(P["W3"]).T) * (f["z2"] > 0))
    g["W2"] = f["h1"].T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = q((dz2 @ q(P["W2"]).T) * (f["z1"] > 0))
    g["W1"] = f["xh"].T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, pack(g)


def init(seed):
    """He-uniform initial weights, zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            lim = np.sqrt(6.0 / shape[0])
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    return pack(d)
