"""Oracle for the learned iterate corrector (TEST INFRASTRUCTURE ONLY).

The paper has no corrector; this is the plain definition of the small network
that the library trains on OCI iterate histories to damp slow convergence in
optically thin cells (the weakness the paper states in its introduction and
conclusions).  Everything here follows textbook definitions, in FP64:

* a 1-D convolution over cells (cross-correlation, kernel width 5, zero
  padding of two cells at each mesh end, so the output has the input's cell
  count): y[b, o, j] = sum_i sum_t W[o, i, t] x[b, i, j + t - 2];
* four such layers, 32 channels between them, no biases, ReLU after each of
  the first three (so the network is positively homogeneous: f(a x) = a f(x)
  for a > 0, and a correction scales with the iterate difference it is fed);
* the mean squared error over all outputs and its gradient by the chain rule;
* Adam (Kingma and Ba, 2015) with bias-corrected first and second moments.

Layout: x [B][C_in][J], y [B][C_out][J]; the weights of layer l are
[C_o][C_i][5], all layers concatenated in order into one flat vector.

Parity pinned: against finite differences of the loss (every gradient),
against numpy's correlate (one channel), against exact shifts (off-centre
delta kernels), positive homogeneity, and Adam's closed-form first step.
"""
import numpy as np

KW = 5        # kernel width
HIDDEN = 32   # channels between layers
LAYERS = 4


def layer_shapes(c_in, c_out):
    chans = [c_in] + [HIDDEN] * (LAYERS - 1) + [c_out]
    return [(chans[l + 1], chans[l], KW) for l in range(LAYERS)]


def num_weights(c_in, c_out):
    return sum(int(np.prod(s)) for s in layer_shapes(c_in, c_out))


def unflatten(w, c_in, c_out):
    out, k = [], 0
    for s in layer_shapes(c_in, c_out):
        n = int(np.prod(s))
        out.append(np.asarray(w[k:k + n], dtype=np.float64).reshape(s))
        k += n
    return out


def conv1d(x, W):
    """y[b, o, j] = sum_i sum_t W[o, i, t] x[b, i, j + t - 2], zero outside [0, J)."""
    B, Ci, J = x.shape
    Co = W.shape[0]
    xp = np.zeros((B, Ci, J + KW - 1))
    xp[:, :, 2:2 + J] = x
    y = np.zeros((B, Co, J))
    for t in range(KW):
        # (Co, Ci) x (B, Ci, J) -> (B, Co, J): the tap t contribution
        y += np.einsum("oi,bij->boj", W[:, :, t], xp[:, :, t:t + J])
    return y


def forward(w, x, c_in, c_out):
    """Network output and the activations of every layer (inputs of layers 1..4)."""
    Ws = unflatten(w, c_in, c_out)
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for l, W in enumerate(Ws):
        h = conv1d(h, W)
        if l < LAYERS - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def loss(w, x, target, c_in, c_out):
    y, _ = forward(w, x, c_in, c_out)
    return float(np.mean((y - target) ** 2))


def grad(w, x, target, c_in, c_out):
    """Mean squared error and its gradient wrt the flat weights (chain rule)."""
    Ws = unflatten(w, c_in, c_out)
    y, acts = forward(w, x, c_in, c_out)
    n = y.size
    g = 2.0 * (y - target) / n            # dL/dy
    grads = [None] * LAYERS
    for l in range(LAYERS - 1, -1, -1):
        if l < LAYERS - 1:
            g = g * (acts[l + 1] > 0.0)   # through the ReLU of layer l
        xin = acts[l]
        B, Ci, J = xin.shape
        xp = np.zeros((B, Ci, J + KW - 1))
        xp[:, :, 2:2 + J] = xin
        dW = np.zeros_like(Ws[l])
        for t in range(KW):
            dW[:, :, t] = np.einsum("boj,bij->oi", g, xp[:, :, t:t + J])
        grads[l] = dW
        if l > 0:
            # dL/dx[b, i, j] = sum_o sum_t W[o, i, t] g[b, o, j - t + 2]
            gp = np.zeros((B, g.shape[1], J + KW - 1))
            gp[:, :, 2:2 + J] = g
            gx = np.zeros_like(xin)
            for t in range(KW):
                gx += np.einsum("oi,boj->bij", Ws[l][:, :, t], gp[:, :, KW - 1 - t:KW - 1 - t + J])
            g = gx
    return float(np.mean((y - target) ** 2)), np.concatenate([d.ravel() for d in grads])


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1, 2, ...): returns the new weights and moments."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
