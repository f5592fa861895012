"""MLP deep-ensemble oracle, FP64 numpy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Not part of the paper (which argues for a non-parametric GP, Sec. 1); this is
the learned surrogate that stands beside the GP.  Each member is a
2 -> H -> H -> 1 network with tanh hidden units trained full-batch on the mean
squared error with Adam (Kingma & Ba, 2015).  Readings (also in the design
notes): inputs standardised by the training-set mean and standard deviation;
outputs divided by their RMS; Glorot-uniform weights, zero biases; member k
draws its weights from Philox4x32-10 with key (lo32(seed), hi32(seed)) and
counter (j, k, 2, 0), the parameter p taking word p mod 4 of counter
j = p div 4, mapped to (0,1) as (r + 0.5) / 2^32; ensemble standard deviation
with ddof = 1.

Bootstrap option (the usual remedy for a deep ensemble whose members agree
too readily): member k trains on N points drawn with replacement from the N
training points; draw j is point (r N) >> 32 for the Philox word r of
counter (j div 4, k, 3, 0), word j mod 4, same key.  Its loss is the mean
squared error over that resample, i.e. (1/N) sum_i c_ki r_i^2 with c_ki the
number of times point i was drawn.  Standardisation uses the whole set.

Parameter layout of one member (flat, this order): W1 [H x 2] row-major
(output-major), b1 [H], W2 [H x H], b2 [H], W3 [1 x H], b3 [1].
"""
import numpy as np

from . import md as _md


def n_params(H: int) -> int:
    return H * H + 5 * H + 1


def unpack(theta, H):
    o = 0
    W1 = theta[o:o + 2 * H].reshape(H, 2); o += 2 * H
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + H].reshape(1, H); o += H
    b3 = theta[o:o + 1]
    return W1, b1, W2, b2, W3, b3


def glorot_init(H: int, member: int, seed: int) -> np.ndarray:
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    P = n_params(H)
    words = np.zeros(P, dtype=np.float64)
    for j in range((P + 3) // 4):
        r = _md.philox4x32_10([j, member, 2, 0], key)
        for w in range(4):
            p = 4 * j + w
            if p < P:
                words[p] = (float(r[w]) + 0.5) / 4294967296.0
    theta = np.zeros(P)
    bounds = [(0, 2 * H, np.sqrt(6.0 / (2 + H))),              # W1
              (3 * H, 3 * H + H * H, np.sqrt(6.0 / (2 * H))),  # W2
              (4 * H + H * H, 5 * H + H * H, np.sqrt(6.0 / (H + 1)))]  # W3
    for a, b, lim in bounds:
        theta[a:b] = lim * (2.0 * words[a:b] - 1.0)
    return theta


def bootstrap_counts(N: int, member: int, seed: int) -> np.ndarray:
    """Times each of the N points is drawn in member `member`'s resample."""
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    c = np.zeros(N, dtype=np.int64)
    for j in range((N + 3) // 4):
        r = _md.philox4x32_10([j, member, 3, 0], key)
        for w in range(4):
            if 4 * j + w < N:
                c[(int(r[w]) * N) >> 32] += 1
    return c


def forward(theta, Xs, H):
    W1, b1, W2, b2, W3, b3 = unpack(theta, H)
    h1 = np.tanh(Xs @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    out = h2 @ W3.T + b3
    return out[:, 0], (h1, h2)


def loss_and_grad(theta, Xs, ys, H, w=None):
    """MSE loss and its gradient by hand-written back-propagation; w (per
    point, e.g. bootstrap counts) weights each squared residual, the mean
    still taken over the N points."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, H)
    out, (h1, h2) = forward(theta, Xs, H)
    N = len(ys)
    r = out - ys
    wr = r if w is None else np.asarray(w, dtype=np.float64) * r
    loss = np.mean(wr * r)
    d_out = (2.0 / N) * wr[:, None]                  # N x 1
    gW3 = d_out.T @ h2
    gb3 = d_out.sum(0)
    dz2 = (d_out @ W3) * (1.0 - h2 ** 2)             # N x H
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
    gW1 = dz1.T @ Xs
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


class Ensemble:
    def __init__(self, X, y, members=5, hidden=64, iters=5000, lr=1e-3, seed=0, bootstrap=False):
        X = np.asarray(X, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        self.H = hidden
        self.mu = X.mean(0)
        sd = X.std(0)
        self.sd = np.where(sd > 0, sd, 1.0)
        s = np.sqrt(np.mean(y ** 2))
        self.s_q = s if s > 0 else 1.0
        Xs = (X - self.mu) / self.sd
        ys = y / self.s_q
        self.thetas, self.losses = [], []
        for k in range(members):
            th = glorot_init(hidden, k, seed)
            w = bootstrap_counts(len(ys), k, seed).astype(np.float64) if bootstrap else None
            m = np.zeros_like(th)
            v = np.zeros_like(th)
            loss = None
            for t in range(1, iters + 1):
                loss, g = loss_and_grad(th, Xs, ys, hidden, w)
                th, m, v = adam_step(th, g, m, v, t, lr)
            self.thetas.append(th)
            self.losses.append(loss)

    def member_predict(self, Xq):
        Xs = (np.asarray(Xq, dtype=np.float64) - self.mu) / self.sd
        return np.array([forward(th, Xs, self.H)[0] * self.s_q for th in self.thetas])

    def predict(self, Xq):
        P = self.member_predict(Xq)
        return P.mean(0), P.std(0, ddof=1)
