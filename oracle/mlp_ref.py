"""FP64 reference of the false-alarm surrogate network -- TEST INFRASTRUCTURE ONLY.

Plain numpy, written from the network's definition (not from the GPU code):
  features (68) -> standardize -> Linear 256 -> GELU -> Linear 256 -> GELU
  -> Linear 256 -> GELU -> Linear 2 -> (m, beta).
GELU is the tanh form 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))).

The two outputs set the law of the maximum power of white noise over the
pattern's grid.  A single frequency's power z exceeds a level with the
probability of the beta law of Section 3, (1 - 2z/Nt)^((Nt-3)/2) = exp(-w(z)),
w(z) = -((Nt-3)/2) ln(1 - 2z/Nt); the maximum is modelled as Gumbel in w,
  P(max <= z) = exp(-exp(-u)),  u = (w(z) - ln Nf - m) / beta,
  m = mu + sigma r_0,  beta = softplus(r_1 + ln(e - 1))   (beta = 1 at r_1 = 0),
which is Eq. (3) with Nf independent frequencies when m = 0, beta = 1 (up to
the Poisson limit of the binomial power).  Quantiles at tau:
w = ln Nf + m + beta (-ln(-ln tau)), z = (Nt/2)(1 - exp(-2w/(Nt-3))).
Nt and Nf come from the raw features (feat[64] = log10 Nt, feat[67] = log10 Nf).

With bf=True the values that the GPU feeds to its BF16 matrix products
(standardized inputs, weights, activations, back-propagated gradients) are
rounded to BF16 (round to nearest even) at the same points; everything else
is FP64.  Loss: the negative log-likelihood of the R Monte-Carlo maxima per
pattern under that law (in w, whose Jacobian does not depend on the
parameters), averaged over samples and patterns.  Optimizer: Adam as in
Kingma & Ba's Algorithm 1.
"""
import numpy as np

TAU = np.array([0.5, 0.75, 0.9, 0.95, 0.975, 0.99, 0.995, 0.998, 0.999])
SHAPES = [(256, 68), (256, 256), (256, 256), (2, 256)]
N_PARAMS = sum(o * i + o for o, i in SHAPES)
C_GELU = np.sqrt(2.0 / np.pi)
BETA_SHIFT = np.log(np.e - 1.0)
G_TAU = -np.log(-np.log(TAU))


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


def nt_nf(feat):
    """Nt and Nf of each pattern from its raw features."""
    feat = np.asarray(feat, dtype=np.float64)
    return np.rint(10.0 ** feat[:, 64]), np.rint(10.0 ** feat[:, 67])


def w_of(z, nt):
    """Exponential-equivalent power: P(single-frequency power > z) = exp(-w)."""
    return -((nt - 3.0) / 2.0) * np.log1p(-2.0 * np.asarray(z, dtype=np.float64) / nt)


def z_of(w, nt):
    return (nt / 2.0) * -np.expm1(-2.0 * np.asarray(w, dtype=np.float64) / (nt - 3.0))


def head(raw, mu, sigma):
    """(m, beta) per pattern."""
    return mu + sigma * raw[:, 0], softplus(raw[:, 1] + BETA_SHIFT)


def quantiles(raw, feat, mu, sigma):
    m, b = head(raw, mu, sigma)
    nt, nf = nt_nf(feat)
    w = np.log(nf)[:, None] + m[:, None] + b[:, None] * G_TAU[None, :]
    return z_of(w, nt[:, None])


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
    return {"X": X, "acts": acts, "Z": Zs, "raw": raw, "q": quantiles(raw, feat, mu, sigma)}


def gumbel_nll(m, beta, w):
    """L = 1/(B R) sum_b sum_r [ln beta_b + u_br + exp(-u_br)], u = (w - m)/beta,
    and dL/dm, dL/dbeta; w [B, R] already has ln Nf removed."""
    B, nR = w.shape
    u = (w - m[:, None]) / beta[:, None]
    e = np.exp(-u)
    L = np.sum(np.log(beta)[:, None] + u + e) / (B * nR)
    dm = np.sum(-(1.0 - e) / beta[:, None], axis=1) / (B * nR)
    db = np.sum(1.0 / beta[:, None] - u * (1.0 - e) / beta[:, None], axis=1) / (B * nR)
    return L, dm, db


def loss_and_grad(p, feat, y, mean, std, mu, sigma, bf=True):
    rnd = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    f = forward(p, feat, mean, std, mu, sigma, bf)
    raw = f["raw"]
    nt, nf = nt_nf(feat)
    w = w_of(y, nt[:, None]) - np.log(nf)[:, None]
    m, b = head(raw, mu, sigma)
    L, dm, db = gumbel_nll(m, b, w)
    dr = np.zeros_like(raw)
    dr[:, 0] = dm * sigma
    dr[:, 1] = db / (1.0 + np.exp(-(raw[:, 1] + BETA_SHIFT)))
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


def fap(raw, feat, mu, sigma, p):
    """P(max >= p) under one member's law, per pattern."""
    m, b = head(raw, mu, sigma)
    nt, nf = nt_nf(feat)
    u = (w_of(p, nt) - np.log(nf) - m) / b
    return -np.expm1(-np.exp(-u))


def fap_sensitivity(raw, feat, mu, sigma, p):
    """d FAP / d m and d FAP / d beta of one member's law at p, per pattern:
    with u = (w(p) - ln Nf - m) / beta and FAP = 1 - exp(-e^{-u}),
    dFAP/du = -e^{-u} exp(-e^{-u}), du/dm = -1/beta, du/dbeta = -u/beta."""
    m, b = head(raw, mu, sigma)
    nt, nf = nt_nf(feat)
    u = (w_of(p, nt) - np.log(nf) - m) / b
    g = np.exp(-u) * np.exp(-np.exp(-u))
    return g / b, g * u / b
