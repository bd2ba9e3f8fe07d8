"""FP64 reference of the small convolutional coarse-grid correction network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper implements its solver as fixed-weight convolutional layers and points to trainable
multigrid as related work, but specifies no trained network; the network here is this project's
own: four 3 x 3 convolutions, channels 3 -> 32 -> 32 -> 32 -> 1, zero padding ("same" size),
ReLU after the first three, mean-squared-error loss, Adam.  Parameters are one flat float vector
in the order W1, b1, W2, b2, W3, b3, W4, b4 with W[c_out][c_in][ky][kx].  Activations are
[batch][channel][y][x].

Convolution semantics (cross-correlation, as the paper's convolutional filters):
out[b, co, y, x] = bias[co] + sum_{ci, v, u} W[co, ci, v+1, u+1] in[b, ci, y+v, x+u], zero outside.
"""
import numpy as np

CHANNELS = (3, 32, 32, 32, 1)


def layer_shapes(channels=CHANNELS):
    return [((co, ci, 3, 3), (co,)) for ci, co in zip(channels[:-1], channels[1:])]


def n_params(channels=CHANNELS):
    return sum(int(np.prod(w)) + b[0] for w, b in layer_shapes(channels))


def unpack(theta, channels=CHANNELS):
    out, off = [], 0
    for ws, bs in layer_shapes(channels):
        nw = int(np.prod(ws))
        W = theta[off:off + nw].reshape(ws)
        off += nw
        b = theta[off:off + bs[0]]
        off += bs[0]
        out.append((W, b))
    return out


def init_params(seed, channels=CHANNELS, scale=1.0):
    """He-style uniform initialisation (seeded), biases zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for (co, ci, kh, kw), (nb,) in layer_shapes(channels):
        bound = scale * np.sqrt(6.0 / (ci * kh * kw))
        parts.append(rng.uniform(-bound, bound, size=co * ci * kh * kw))
        parts.append(np.zeros(nb))
    return np.concatenate(parts)


def conv2d(x, W, b):
    """x[B, Ci, H, Wd] -> [B, Co, H, Wd], 3 x 3 cross-correlation with zero padding."""
    B, Ci, H, Wd = x.shape
    xp = np.zeros((B, Ci, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((B, W.shape[0], H, Wd)) + b[None, :, None, None]
    for v in range(3):
        for u in range(3):
            out += np.einsum("oc,bchw->bohw", W[:, :, v, u], xp[:, :, v:v + H, u:u + Wd])
    return out


def forward(theta, x, channels=CHANNELS):
    """Returns the output and the list of layer inputs / pre-activations for the backward pass."""
    layers = unpack(theta, channels)
    acts, pres = [x], []
    h = x
    for i, (W, b) in enumerate(layers):
        z = conv2d(h, W, b)
        pres.append(z)
        h = np.maximum(z, 0.0) if i < len(layers) - 1 else z
        acts.append(h)
    return h, acts, pres


def mse(out, target):
    return float(np.mean((out - target) ** 2))


def loss_and_grad(theta, x, target, channels=CHANNELS):
    """MSE loss and its gradient with respect to the flat parameter vector (reverse mode)."""
    layers = unpack(theta, channels)
    out, acts, pres = forward(theta, x, channels)
    loss = mse(out, target)
    d = 2.0 * (out - target) / out.size
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, b = layers[i]
        if i < len(layers) - 1:
            d = d * (pres[i] > 0)
        h = acts[i]
        B, Ci, H, Wd = h.shape
        hp = np.zeros((B, Ci, H + 2, Wd + 2))
        hp[:, :, 1:-1, 1:-1] = h
        gW = np.zeros_like(W)
        for v in range(3):
            for u in range(3):
                gW[:, :, v, u] = np.einsum("bohw,bchw->oc", d, hp[:, :, v:v + H, u:u + Wd])
        gb = d.sum(axis=(0, 2, 3))
        grads.append((gW, gb))
        # gradient with respect to the layer input: correlation with the flipped kernel
        dp = np.zeros((B, W.shape[0], H + 2, Wd + 2))
        dp[:, :, 1:-1, 1:-1] = d
        dh = np.zeros_like(h)
        for v in range(3):
            for u in range(3):
                dh += np.einsum("oc,bohw->bchw", W[:, :, v, u], dp[:, :, 2 - v:2 - v + H, 2 - u:2 - u + Wd])
        d = dh
    flat = []
    for gW, gb in reversed(grads):
        flat.append(gW.ravel())
        flat.append(gb)
    return loss, np.concatenate(flat)


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) at step t >= 1; returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
