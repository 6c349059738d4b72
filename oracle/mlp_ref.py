"""FP64 reference of the false-alarm surrogate network -- TEST INFRASTRUCTURE ONLY.

Plain numpy, written from the network's definition (not from the GPU code):
  features (68) -> standardize -> Linear 256 -> GELU -> Linear 256 -> GELU
  -> Linear 256 -> GELU -> Linear 9 -> monotone head
  q_0 = mu + sigma r_0, q_i = q_{i-1} + sigma softplus(r_i).
GELU is the tanh form 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).
With bf=True the values that the GPU feeds to its BF16 matrix products
(standardized inputs, weights, activations, back-propagated gradients) are
rounded to BF16 (round to nearest even) at the same points; everything else
is FP64.  Loss: the pinball loss averaged over patterns, quantile levels and
Monte-Carlo samples.  Optimizer: Adam as in Kingma & Ba's Algorithm 1.
"""
import numpy as np

TAU = np.array([0.5, 0.75, 0.9, 0.95, 0.975, 0.99, 0.995, 0.998, 0.999])
SHAPES = [(256, 68), (256, 256), (256, 256), (9, 256)]
N_PARAMS = sum(o * i + o for o, i in SHAPES)
C_GELU = np.sqrt(2.0 / np.pi)


def bf16(x):
    """Round to the nearest BF16 (ties to even), via FP32; returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unflatten(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = [], 0
    for (n_out, n_in) in SHAPES:
        W = p[o:o + n_out * n_in].reshape(n_out, n_in)
        o += n_out * n_in
        b = p[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == p.size
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_grad(z):
    th = np.tanh(C_GELU * (z + 0.044715 * z ** 3))
    return 0.5 * (1.0 + th) + 0.5 * z * (1.0 - th ** 2) * C_GELU * (1.0 + 3 * 0.044715 * z ** 2)


def softplus(r):
    return np.where(r > 20, r, np.log1p(np.exp(np.minimum(r, 20))))


def head(raw, mu, sigma):
    q = np.empty((raw.shape[0], 9))
    q[:, 0] = mu + sigma * raw[:, 0]
    for i in range(1, 9):
        q[:, i] = q[:, i - 1] + sigma * softplus(raw[:, i])
    return q


def forward(p, feat, mean, std, mu, sigma, bf=True):
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unflatten(p)
    X = rnd((np.asarray(feat, dtype=np.float64) - mean) / std)
    acts = [X]
    Zs = []
    h = X
    for li, (W, b) in enumerate(layers):
        z = h @ rnd(W).T + b
        if li < 3:
            Zs.append(z)
            h = rnd(gelu(z))
            acts.append(h)
        else:
            raw = z
    return {"X": X, "acts": acts, "Z": Zs, "raw": raw, "q": head(raw, mu, sigma)}


def pinball(q, y):
    """L = 1/(9B) sum_b sum_i mean_r rho_tau_i(y_br - q_bi) and dL/dq."""
    B = q.shape[0]
    u = y[:, None, :] - q[:, :, None]                      # [B, 9, R]
    rho = u * (TAU[None, :, None] - (u < 0))
    L = rho.mean(axis=2).sum() / (9 * B)
    dq = ((u < 0).mean(axis=2) - TAU[None, :]) / (9 * B)
    return L, dq


def loss_and_grad(p, feat, y, mean, std, mu, sigma, bf=True):
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    f = forward(p, feat, mean, std, mu, sigma, bf)
    raw, q = f["raw"], f["q"]
    L, dq = pinball(q, np.asarray(y, dtype=np.float64))
    # back through the head
    dr = np.zeros_like(raw)
    tail = np.zeros(raw.shape[0])
    for i in range(8, 0, -1):
        tail += dq[:, i]
        dr[:, i] = tail * sigma / (1.0 + np.exp(-raw[:, i]))
    dr[:, 0] = (tail + dq[:, 0]) * sigma
    layers = unflatten(p)
    grads = [None] * 4
    dz = dr
    for li in range(3, -1, -1):
        W, _ = layers[li]
        a_in = f["acts"][li]
        grads[li] = (rnd(dz).T @ a_in, dz.sum(axis=0))
        if li > 0:
            dh = rnd(dz) @ rnd(W)
            dz = dh * gelu_grad(f["Z"][li - 1])
    return L, flatten(grads), f


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def fap_from_quantiles(q, p):
    """P(max >= p) from one set of nine quantiles: linear in y = -ln(-ln tau)
    between neighbouring quantiles, extended along the end segments."""
    y = -np.log(-np.log(TAU))
    q = np.asarray(q, dtype=np.float64)
    i = 0
    while i < 7 and p > q[i + 1]:
        i += 1
    yy = y[i] + (p - q[i]) * (y[i + 1] - y[i]) / max(q[i + 1] - q[i], 1e-12)
    return -np.expm1(-np.exp(-yy))
