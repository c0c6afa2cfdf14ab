"""FP64 oracle of the learned warm start: node features, the per-node network,
its gradient and one Adam step.  Test infrastructure only: nothing on the
product path imports this module.

The paper has no learned component; this module fixes, in plain code, the
definitions the GPU kernels implement:

Features of node i (the receptive field is the support of psi_i, the four cells
sharing the node: a = (ix, iy), b = (ix-1, iy), c = (ix-1, iy-1), d = (ix, iy-1),
periodic).  The particles of these cells are taken cell by cell in that order,
each cell in binned (ascending original index) order; the first K_MAX are kept
and n counts all of them.  For a kept particle in cell role r with in-cell
offsets (xi, eta) (the FP64 locate of the assembly): dx = xi - [r in (b, c)],
dy = eta - [r in (c, d)], so (dx, dy) is the offset from the node in cell units.
With the FLIP value base = b_i / w_i (0 for an orphan) and
s = sqrt(mean over kept particles of (A - base)^2), the value feature is
(A - base) / s.  The input row is [dx_1, dy_1, a_1, ..., dx_48, dy_48, a_48, n/48]
followed by 15 zeros (160 entries); rows of absent particles are 0.  A node is
usable when 1 <= n <= K_MAX, w_i > 0 and s > S_FLOOR * max |A| over the kept
particles (a spread that is not rounding noise); other nodes keep the FLIP value.

Network (3 hidden layers of 64, ReLU): z1 = W1 x + b1, h1 = relu(z1),
z2 = W2 h1 + b2, h2 = relu(z2), z3 = W3 h2 + b3, h3 = relu(z3), y = W4 . h3 + b4.
The start value is x0_i = base + s * y; the training target for y is
(exact_i - base) / s.  On the GPU W1..W3, x, h1 and h2 are BF16 (products
accumulated in FP32), W4, b and h3 are FP32; bf16() below is the same rounding
(round to nearest, ties to even) so that the oracle can mirror it.

Parameter vector (FP32, N_PARAM entries): W1 [64][160] (columns 145..159 stay
0), b1 [64], W2 [64][64], b2 [64], W3 [64][64], b3 [64], W4 [64], b4 [1].
"""
import numpy as np

K_MAX = 48
N_FEAT = 3 * K_MAX + 1        # 145
N_IN = 160                    # padded to whole MFMA K-steps
H = 64
S_FLOOR = 2.0 ** -20
OFFS = {}
_o = 0
for _name, _size in (("W1", H * N_IN), ("b1", H), ("W2", H * H), ("b2", H), ("W3", H * H),
                     ("b3", H), ("W4", H), ("b4", 1)):
    OFFS[_name] = (_o, _size)
    _o += _size
N_PARAM = _o                  # 18689


def unpack(theta):
    """Views of the parameter vector: W1 [64, 160], b1, W2 [64, 64], b2, W3, b3, W4 [64], b4 [1]."""
    theta = np.asarray(theta)
    out = {}
    for name, (o, n) in OFFS.items():
        v = theta[o:o + n]
        if name == "W1":
            v = v.reshape(H, N_IN)
        elif name in ("W2", "W3"):
            v = v.reshape(H, H)
        out[name] = v
    return out


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.  Works on the
    FP32 bit pattern: BF16 keeps the top 16 bits of an FP32 number."""
    f0 = np.asarray(a, dtype=np.float32)
    f = np.atleast_1d(f0)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)
    out[np.isnan(f)] = np.nan
    return out.reshape(f0.shape)


# ----------------------------------------------------------------------------
# features
# ----------------------------------------------------------------------------
def flip_base(b, w):
    """FLIP values b / w per field, 0 at orphan nodes (w == 0)."""
    b = np.atleast_2d(np.asarray(b, dtype=np.float64))
    w = np.asarray(w, dtype=np.float64)
    return np.where(w > 0, b / np.where(w > 0, w, 1.0), 0.0)


def node_features(prob, values, base, w, nodes, loc, perm, cell_start):
    """Feature rows of the listed nodes for every field.

    prob: 2D problem; values [F, N_p]; base [F, N_n] (flip_base); w [N_n];
    loc: p1.locate(prob); perm / cell_start: p1.bin_particles output.
    Returns X [len(nodes), F, 160] (FP64, not rounded), scale [len(nodes), F] (s, or
    0 when the node is not usable) and count [len(nodes)] (n, all particles of the
    four cells).
    """
    values = np.atleast_2d(np.asarray(values, dtype=np.float64))
    F = values.shape[0]
    nx, ny = prob["nx"], prob["ny"]
    xi = loc["xi"]
    eta = loc["eta"]
    X = np.zeros((len(nodes), F, N_IN))
    scale = np.zeros((len(nodes), F))
    count = np.zeros(len(nodes), dtype=np.int64)
    for r, node in enumerate(nodes):
        ix, iy = node % nx, node // nx
        cells = [(ix, iy, 0, 0), ((ix - 1) % nx, iy, 1, 0), ((ix - 1) % nx, (iy - 1) % ny, 1, 1),
                 (ix, (iy - 1) % ny, 0, 1)]
        plist = []
        for cx, cy, sx, sy in cells:
            c = cx + nx * cy
            for k in range(cell_start[c], cell_start[c + 1]):
                plist.append((perm[k], sx, sy))
        n = len(plist)
        count[r] = n
        kept = plist[:K_MAX]
        if not kept:
            continue
        for f in range(F):
            a = np.array([values[f, mu] for mu, _, _ in kept]) - base[f, node]
            s = np.sqrt(np.mean(a * a))
            for m, (mu, sx, sy) in enumerate(kept):
                X[r, f, 3 * m + 0] = xi[mu] - sx
                X[r, f, 3 * m + 1] = eta[mu] - sy
                X[r, f, 3 * m + 2] = a[m] / s if s > 0.0 else 0.0
            X[r, f, 3 * K_MAX] = min(n, K_MAX) / K_MAX
            amax = max(abs(values[f, mu]) for mu, _, _ in kept)
            usable = n <= K_MAX and s > S_FLOOR * amax and w[node] > 0.0
            scale[r, f] = s if usable else 0.0
    return X, scale, count


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------
def forward(theta, X, mirror_gpu=True):
    """Network outputs for rows X [B, 160].  With mirror_gpu the BF16 roundings of the
    GPU (weights W1..W3, inputs, h1, h2) are applied; all arithmetic is FP64.
    Returns (y [B], cache)."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    rnd = bf16 if mirror_gpu else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = rnd(p["W1"]), rnd(p["W2"]), rnd(p["W3"])
    x = rnd(X)
    z1 = x @ W1.T + p["b1"]
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + p["b2"]
    h2 = rnd(np.maximum(z2, 0.0))
    z3 = h2 @ W3.T + p["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ p["W4"] + p["b4"][0]
    return y, dict(x=x, W1=W1, W2=W2, W3=W3, W4=p["W4"], z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, h3=h3)


def loss_and_grad(theta, X, target, mirror_gpu=True):
    """Mean squared error (1/B) sum (y - t)^2 and its gradient (FP64 backward through
    the forward above; each rounding is passed through as the identity)."""
    y, c = forward(theta, X, mirror_gpu)
    B = X.shape[0]
    err = y - target
    loss = float(np.mean(err * err))
    dy = 2.0 * err / B
    g = {}
    g["W4"] = c["h3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, c["W4"]) * (c["z3"] > 0)
    g["W3"] = dz3.T @ c["h2"]
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ c["W3"]) * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ c["W2"]) * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(0)
    grad = np.zeros(N_PARAM)
    for name, (o, n) in OFFS.items():
        grad[o:o + n] = np.asarray(g[name]).reshape(-1)
    return loss, grad, y


def adam_step(theta, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1) with bias correction; step >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed):
    """He-normal hidden layers, a small output layer, zero biases, zero padding columns."""
    g = np.random.Generator(np.random.PCG64(seed))
    theta = np.zeros(N_PARAM)
    p = unpack(theta)
    p["W1"][:, :N_FEAT] = g.normal(0.0, np.sqrt(2.0 / N_FEAT), (H, N_FEAT))
    p["W2"][:] = g.normal(0.0, np.sqrt(2.0 / H), (H, H))
    p["W3"][:] = g.normal(0.0, np.sqrt(2.0 / H), (H, H))
    p["W4"][:] = g.normal(0.0, 0.01, H)
    return theta.astype(np.float32)
