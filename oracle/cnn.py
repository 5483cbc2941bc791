"""FP64 reference of the learned warm-start network (test infrastructure).

Only the tests (and the smoke check) use this module.  Plain numpy, FP64, no
fusion: every layer is written as its definition.

Network (3D, periodic, C = 16 channels, `levels` resolutions n, n/2, ...):
  encoder level l: conv + ReLU, conv + ReLU   -> e_l   (level 0 input: 1 channel)
  between levels:  2x2x2 average (the multigrid restriction filter)
  decoder level l (from levels-2 down to 0): u_l = up(d_{l+1}) + e_l,
                   conv + ReLU, conv + ReLU   -> d_l   (d_{levels-1} = e_{levels-1})
  output:          conv (16 -> 1), no activation
`up` is the cell-centred trilinear prolongation with periodic wrap (weights
3/4 and 1/4 per axis).  A convolution is the cross-correlation of the paper's
filter definition (Section 2.1): out[o, z, y, x] = b[o] + sum over taps t =
(dz, dy, dx) in {-1, 0, 1}^3 and input channels c of W[t, o, c] * in[c, z+dz,
y+dy, x+dx], indices wrapped.  Tap index t = (dz+1)*9 + (dy+1)*3 + (dx+1).

Parameters: one (W[27, 16, 16], b[16]) pair per convolution in network order
(2*levels encoder convs, 2*(levels-1) decoder convs, 1 output conv).  The
first conv uses input channel 0 only and the output conv output channel 0
only; the other entries stay zero.  Activations are arrays (C, n, n, n).
"""
import numpy as np

C = 16
OFFS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def n_convs(levels):
    return 2 * levels + 2 * (levels - 1) + 1


def conv(X, W, b):
    """Periodic 3x3x3 cross-correlation, channels (C_in, n, n, n) -> (C_out, ...)."""
    Y = np.zeros((W.shape[1],) + X.shape[1:])
    for t, (dz, dy, dx) in enumerate(OFFS):
        Xs = np.roll(X, shift=(-dz, -dy, -dx), axis=(1, 2, 3))  # Xs[c, z] = X[c, z + dz]
        Y += np.einsum("oc,czyx->ozyx", W[t], Xs)
    return Y + b[:, None, None, None]


def conv_backward(X, W, dY):
    """Gradients of conv for upstream dY: returns dX, dW, db."""
    dW = np.zeros_like(W)
    dX = np.zeros_like(X)
    for t, (dz, dy, dx) in enumerate(OFFS):
        Xs = np.roll(X, shift=(-dz, -dy, -dx), axis=(1, 2, 3))
        dW[t] = np.einsum("ozyx,czyx->oc", dY, Xs)
        # d/dX[c, z+dz] of W[t,o,c] X[c, z+dz] dY[o, z]: shift dY forward by the tap
        dX += np.roll(np.einsum("oc,ozyx->czyx", W[t], dY), shift=(dz, dy, dx), axis=(1, 2, 3))
    db = dY.sum(axis=(1, 2, 3))
    return dX, dW, db


def pool(X):
    c, n = X.shape[0], X.shape[1]
    return X.reshape(c, n // 2, 2, n // 2, 2, n // 2, 2).mean(axis=(2, 4, 6))


def pool_backward(dY):
    return np.repeat(np.repeat(np.repeat(dY, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def _up_matrix(nc):
    """1D periodic cell-centred linear interpolation matrix (2nc x nc)."""
    P = np.zeros((2 * nc, nc))
    for i in range(2 * nc):
        I = i // 2
        nb = (I - 1) % nc if i % 2 == 0 else (I + 1) % nc
        P[i, I] += 0.75
        P[i, nb] += 0.25
    return P


def up(X):
    P = _up_matrix(X.shape[1])
    Y = np.einsum("Zz,czyx->cZyx", P, X)
    Y = np.einsum("Yy,cZyx->cZYx", P, Y)
    return np.einsum("Xx,cZYx->cZYX", P, Y)


def up_backward(dY):
    P = _up_matrix(dY.shape[1] // 2)
    d = np.einsum("Zz,cZYX->czYX", P, dY)
    d = np.einsum("Yy,czYX->czyX", P, d)
    return np.einsum("Xx,czyX->czyx", P, d)


def relu(X):
    return np.maximum(X, 0.0)


def forward(params, f, levels, keep=False):
    """params: list of (W, b); f: (n, n, n) input.  Returns the prediction (n, n, n)
    and (when keep) the tape of activations for backward."""
    x = np.zeros((C,) + f.shape)
    x[0] = f
    tape = {"x": x}
    it = iter(range(n_convs(levels)))
    h = x
    enc = []
    for l in range(levels):
        if l > 0:
            h = pool(h)
            tape["p%d" % l] = h
        k = next(it)
        a = relu(conv(h, *params[k]))
        tape["a%d" % l] = (h, a, k)
        k = next(it)
        e = relu(conv(a, *params[k]))
        tape["e%d" % l] = (a, e, k)
        enc.append(e)
        h = e
    d = enc[-1]
    for l in range(levels - 2, -1, -1):
        u = up(d) + enc[l]
        k = next(it)
        c1 = relu(conv(u, *params[k]))
        tape["c%d" % l] = (u, c1, k)
        k = next(it)
        d = relu(conv(c1, *params[k]))
        tape["d%d" % l] = (c1, d, k)
    k = next(it)
    out = conv(d, *params[k])
    tape["out"] = (d, out, k)
    return (out[0], tape) if keep else out[0]


def loss_and_grads(params, f, target, levels):
    """MSE loss mean((N(f) - target)^2) and its gradient for every parameter."""
    y, tape = forward(params, f, levels, keep=True)
    V = y.size
    loss = float(np.mean((y - target) ** 2))
    grads = [None] * len(params)
    d_out = np.zeros((C,) + y.shape)
    d_out[0] = 2.0 * (y - target) / V

    def back(inp, k, dY):
        dX, dW, db = conv_backward(inp, params[k][0], dY)
        grads[k] = (dW, db)
        return dX

    d, _, k = tape["out"]
    g = back(d, k, d_out)
    g_enc = [np.zeros(0)] * levels
    for l in range(0, levels - 1):
        c1, dd, k2 = tape["d%d" % l]
        u, c1o, k1 = tape["c%d" % l]
        g = g * (dd > 0)
        g = back(c1, k2, g)
        g = g * (c1o > 0)
        g_u = back(u, k1, g)
        g_enc[l] = g_u                   # skip connection
        g = up_backward(g_u)             # to d_{l+1}
    # g is now the gradient with respect to e_{levels-1}
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            g = g + g_enc[l]
        a, e, k2 = tape["e%d" % l]
        h, ao, k1 = tape["a%d" % l]
        g = g * (e > 0)
        g = back(a, k2, g)
        g = g * (ao > 0)
        g = back(h, k1, g)
        if l > 0:
            g = pool_backward(g)
    return loss, grads


def init_params(levels, seed=0):
    """He-normal initialisation (seeded); first conv reads channel 0 only, output
    conv writes channel 0 only, biases zero."""
    rng = np.random.default_rng(seed)
    ps = []
    nc = n_convs(levels)
    for k in range(nc):
        cin = 1 if k == 0 else C
        W = np.zeros((27, C, C))
        std = np.sqrt(2.0 / (27 * cin))
        if k == 0:
            W[:, :, 0] = rng.standard_normal((27, C)) * std
        elif k == nc - 1:
            W[:, 0, :] = rng.standard_normal((27, C)) * np.sqrt(1.0 / (27 * C))
        else:
            W[:] = rng.standard_normal((27, C, C)) * std
        ps.append((W, np.zeros(C)))
    return ps


def flatten(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in params])


def unflatten(vec, levels):
    ps = []
    o = 0
    for _ in range(n_convs(levels)):
        W = vec[o:o + 27 * C * C].reshape(27, C, C)
        o += 27 * C * C
        b = vec[o:o + C]
        o += C
        ps.append((W.copy(), b.copy()))
    return ps


def bf16_round(a):
    """Round FP64 values to BF16 (through FP32, round to nearest even)."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
