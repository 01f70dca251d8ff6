"""CPU FP64 oracle of the learned-correction form (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; it imports nothing from the GPU library.

The learned-correction form is not part of the paper: the paper's fluid
example (Section 3) is the plain RK2 step.  The form corrects a 2x coarser
solve toward the fine solve restricted to the coarse mesh:
  - restriction: a coarse cell is the mean of the 2 x 2 x 2 fine cells it
    covers (conservative: totals over the mesh scale by exactly 1/8 per cell
    volume ratio);
  - a network of three 3 x 3 x 3 convolutions, 5 -> 32 -> 32 -> 5 channels,
    ReLU after the first two; ghost cells of each convolution follow the
    mesh's boundary kind (periodic wrap, or outflow: repeat the edge cell);
  - the mean-squared-error loss and its gradient, and the Adam update of the
    parameters.

Everything here is written from the definitions, in FP64, without blocking
or reordering: a convolution is the sum over the 27 shifts of a per-shift
channel contraction.  Arrays: activations (C, nz, ny, nx); weights
(Cout, Cin, 3, 3, 3) indexed [o, i, dz+1, dy+1, dx+1]; biases (Cout,).
"""
import numpy as np

OUTFLOW = 0
PERIODIC = 1

SHIFTS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _index(n, d, bc):
    """Cell index of the neighbour at offset d (-1, 0, 1) of every cell of
    an axis of n cells: wrapped (periodic) or clamped to the edge (outflow)."""
    i = np.arange(n) + d
    if bc == PERIODIC:
        return i % n
    return np.clip(i, 0, n - 1)


def shifted(x, shift, bc):
    """x[:, z + dz, y + dy, x + dx] with the boundary map, for all cells."""
    dz, dy, dx = shift
    nz, ny, nx = x.shape[1:]
    return x[:, _index(nz, dz, bc)][:, :, _index(ny, dy, bc)][:, :, :, _index(nx, dx, bc)]


def conv3(x, w, b, bc):
    """y[o, p] = b[o] + sum over shifts t and input channels i of
    w[o, i, t] x[i, p + t]."""
    cout = w.shape[0]
    y = np.empty((cout,) + x.shape[1:])
    y[:] = b[:, None, None, None]
    for (dz, dy, dx) in SHIFTS:
        xs = shifted(x, (dz, dy, dx), bc)
        wt = w[:, :, dz + 1, dy + 1, dx + 1]          # (cout, cin)
        y += np.tensordot(wt, xs, axes=([1], [0]))
    return y


def relu(x):
    return np.maximum(x, 0.0)


def forward(x, params, bc):
    """The network: returns (y, (a1, h1, a2, h2)) with a = pre-activation,
    h = ReLU(a)."""
    (w1, b1), (w2, b2), (w3, b3) = params
    a1 = conv3(x, w1, b1, bc)
    h1 = relu(a1)
    a2 = conv3(h1, w2, b2, bc)
    h2 = relu(a2)
    y = conv3(h2, w3, b3, bc)
    return y, (a1, h1, a2, h2)


def conv3_backward(x, w, dy, bc):
    """Gradients of sum(dy * conv3(x, w, b)) with respect to w, b and x.

    dw[o, i, t] = sum over cells p of dy[o, p] x[i, p + t]
    db[o]       = sum over p of dy[o, p]
    dx[i, q]    = sum over t, o, and the cells p with p + t mapping to q, of
                  w[o, i, t] dy[o, p]
    The last one scatters through the same boundary map the forward
    gathered through, so it is exact for both boundary kinds."""
    dw = np.zeros_like(w)
    db = dy.reshape(dy.shape[0], -1).sum(axis=1)
    dx = np.zeros_like(x)
    nz, ny, nx = x.shape[1:]
    for (dz, dy_, dx_) in SHIFTS:
        xs = shifted(x, (dz, dy_, dx_), bc)
        dw[:, :, dz + 1, dy_ + 1, dx_ + 1] = np.tensordot(dy, xs, axes=([1, 2, 3], [1, 2, 3]))
        contrib = np.tensordot(w[:, :, dz + 1, dy_ + 1, dx_ + 1], dy, axes=([0], [0]))  # (cin, ...)
        iz, iy, ix = _index(nz, dz, bc), _index(ny, dy_, bc), _index(nx, dx_, bc)
        Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
        for i in range(x.shape[0]):
            np.add.at(dx[i], (Z, Y, X), contrib[i])
    return dw, db, dx


def mse_loss(y, t):
    """Mean over all entries of (y - t)^2, and its gradient with respect to y."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(x, params, cache, dy, bc):
    """Parameter gradients of the network for the output gradient dy, by the
    chain rule through the three convolutions and the two ReLUs (derivative
    1 where the pre-activation is > 0, else 0)."""
    (w1, b1), (w2, b2), (w3, b3) = params
    a1, h1, a2, h2 = cache
    dw3, db3, dh2 = conv3_backward(h2, w3, dy, bc)
    da2 = dh2 * (a2 > 0.0)
    dw2, db2, dh1 = conv3_backward(h1, w2, da2, bc)
    da1 = dh1 * (a1 > 0.0)
    dw1, db1, _ = conv3_backward(x, w1, da1, bc)
    return [(dw1, db1), (dw2, db2), (dw3, db3)]


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) of parameter array p with
    gradient g and moment estimates m, v, at 1-based step number `step`.
    Returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def restrict2(U):
    """Coarse mesh from a fine one with even sizes: each coarse cell is the
    mean of the 2 x 2 x 2 fine cells it covers."""
    c, nz, ny, nx = U.shape
    return U.reshape(c, nz // 2, 2, ny // 2, 2, nx // 2, 2).mean(axis=(2, 4, 6))


def bf16_round(x):
    """Round FP64 values to the nearest bfloat16 (8 significand bits, ties to
    even) and return them as FP64.  Used to hand the oracle exactly the
    operands a BF16 kernel sees."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(U, gamma):
    """Scale-aware network inputs of a conserved state U (5, ...): log rho,
    the velocity components and log p (the Euler equations are invariant
    under rho, p -> lambda rho, lambda p, and log turns that into a shift)."""
    rho = U[0]
    v = U[1:4] / rho
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * np.sum(v * v, axis=0))
    return np.stack([np.log(rho), v[0], v[1], v[2], np.log(p)])


def scales(U, gamma):
    """Local scales of the corrections of each conserved field: rho for the
    density, rho c for the three momenta (c the sound speed), E for the
    energy."""
    rho = U[0]
    v = U[1:4] / rho
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * np.sum(v * v, axis=0))
    rc = rho * np.sqrt(gamma * p / rho)
    return np.stack([rho, rc, rc, rc, U[4]])
