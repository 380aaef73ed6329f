"""Learned block proposal: the masked-patch convolutional conditional (reference).

The paper only asks for a Monte Carlo estimate over gauge configurations
(Sec. 5.1, sampler unspecified); the learned proposal is an exact
Metropolis-Hastings move on top of it.  A P x P patch of sites (2 P^2 links:
the e1 and e2 link owned by each site) is resampled from a factorised
Bernoulli q(x'|context) whose logits come from a network that sees the link
field around the patch with the patch itself masked out.  Because the mask
hides the patch, q(x'|context) and q(x|context) -- the forward and reverse
proposal probabilities -- come from the same forward pass, and the MH ratio
    N(G') q(x|ctx) / (N(G) q(x'|ctx))
uses the true weight N.

Network (valid 3x3 cross-correlations, window W = P + 8 sites per side, so
four layers shrink it to exactly the P x P patch):
    in  : 2 channels (e1, e2 link of each window site), value 1 - 2k, 0 on patch links
    h1  = tanh(conv(in, W1) + b1)    32 channels, (W-2)^2
    h2  = tanh(conv(h1, W2) + b2)    32 channels, (W-4)^2
    h3  = tanh(conv(h2, W3) + b3)    32 channels, (W-6)^2
    z   = conv(h3, W4) + b4           2 channels, P^2: z[mu][y][x] is the logit of
          link (patch origin + (x, y), mu) having k = 1.
Weights are used rounded to bfloat16 (round to nearest even); biases are float32.
Loss: mean over examples of the binary cross entropy of the patch links.

Parameters are one flat float32 vector in the order W1, b1, W2, b2, W3, b3, W4, b4
(weights [c_out][c_in][dy][dx]).  Patches tile the lattice in P x P blocks;
patch p has origin (P (p mod L/P), P (p div L/P)); its links are ordered
l = 2 (y P + x) + mu.
"""
from __future__ import annotations

import numpy as np

from . import philox

CH = 32
HALO = 4
LAYERS = [(2, CH), (CH, CH), (CH, CH), (CH, 2)]


def n_params() -> int:
    return sum(co * ci * 9 + co for ci, co in LAYERS)


def split(params):
    """Views (W, b) per layer of the flat parameter vector."""
    out = []
    off = 0
    for ci, co in LAYERS:
        w = params[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = params[off:off + co]
        off += co
        out.append((w, b))
    return out


def bf16_round(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).reshape(a.shape)


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights from Philox (counter (index, 0, 0, 9)), zero biases."""
    p = np.zeros(n_params(), np.float32)
    off = 0
    for ci, co in LAYERS:
        cnt = co * ci * 9
        a = np.sqrt(6.0 / (9 * ci + 9 * co))
        x0, _, _, _ = philox.philox_vec(np.arange(off, off + cnt), 0, 0, 9, seed & 0xFFFFFFFF, seed >> 32)
        u = (x0.astype(np.float64) + 0.5) * 2.0 ** -32
        p[off:off + cnt] = ((2.0 * u - 1.0) * a).astype(np.float32)
        off += cnt + co
    return p


def patch_origin(L: int, P: int, p: int):
    return P * (p % (L // P)), P * (p // (L // P))


def window(links_k: np.ndarray, L: int, P: int, p: int) -> np.ndarray:
    """Masked input (2, W, W): 1 - 2k of the e1/e2 link of each window site, 0 on patch links.

    On lattices smaller than the window the periodic images of the patch are
    masked too, so the input never depends on the patch configuration."""
    W = P + 2 * HALO
    ox, oy = patch_origin(L, P, p)
    x = np.zeros((2, W, W), np.float32)
    for wy in range(W):
        for wx in range(W):
            sx, sy = (ox - HALO + wx) % L, (oy - HALO + wy) % L
            s = sy * L + sx
            inside = (sx - ox) % L < P and (sy - oy) % L < P
            for mu in range(2):
                x[mu, wy, wx] = 0.0 if inside else 1.0 - 2.0 * float(links_k[2 * s + mu])
    return x


def patch_links(L: int, P: int, p: int) -> np.ndarray:
    """Lattice link indices of the patch, in patch order l = 2 (y P + x) + mu."""
    ox, oy = patch_origin(L, P, p)
    out = []
    for y in range(P):
        for x in range(P):
            s = ((oy + y) % L) * L + (ox + x) % L
            out += [2 * s, 2 * s + 1]
    return np.array(out)


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Valid 3x3 cross-correlation: out[o, y, x] = b[o] + sum_{c,dy,dx} w[o,c,dy,dx] in[c, y+dy, x+dx]."""
    ci, H, Wd = x.shape
    out = np.zeros((w.shape[0], H - 2, Wd - 2), np.result_type(x, w))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,chw->ohw", w[:, :, dy, dx], x[:, dy:dy + H - 2, dx:dx + Wd - 2])
    return out + b[:, None, None]


def forward(params, x, dtype=np.float64, round_bf16: bool = True):
    """Logits z (2, P, P) and the activations, in dtype, with bf16-rounded weights (unless told not to)."""
    acts = [x.astype(dtype)]
    layers = split(np.asarray(params, np.float32))
    h = acts[0]
    for i, (w, b) in enumerate(layers):
        wq = bf16_round(w) if round_bf16 else w
        pre = conv(h, wq.astype(dtype), b.astype(dtype))
        h = np.tanh(pre) if i < 3 else pre
        acts.append(h)
    return h, acts


def logits_patch_order(z: np.ndarray) -> np.ndarray:
    """z (2, P, P) -> vector in patch link order l = 2 (y P + x) + mu."""
    return np.transpose(z, (1, 2, 0)).reshape(-1)


def bce_loss(z: np.ndarray, y: np.ndarray) -> float:
    """sum_l [softplus(z_l) - y_l z_l] = -sum_l [y log s(z) + (1 - y) log s(-z)]."""
    z = np.asarray(z, np.float64)
    return float(np.sum(np.logaddexp(0.0, z) - y * z))


def loss_and_grad(params, examples, round_bf16: bool = True):
    """Mean BCE over examples [(x (2,W,W), y (2P^2,) in patch order)] and its gradient (float64).

    Back-propagation: dL/dz = sigmoid(z) - y; through a tanh layer the
    pre-activation gradient is (1 - h^2) dL/dh; for out = conv(in, w) + b,
    dL/dw[o,c,dy,dx] = sum_yx dout[o,y,x] in[c,y+dy,x+dx], dL/db[o] = sum_yx dout[o],
    dL/din[c, y+dy, x+dx] += sum_o w[o,c,dy,dx] dout[o,y,x].  The gradient is taken with
    respect to the (unrounded) parameters, treating the bf16 rounding as identity.
    """
    layers = split(np.asarray(params, np.float32))
    grads = [(np.zeros_like(w, np.float64), np.zeros_like(b, np.float64)) for w, b in layers]
    total = 0.0
    for x, y in examples:
        z, acts = forward(params, x, np.float64, round_bf16)
        zl = logits_patch_order(z)
        total += bce_loss(zl, y)
        P = z.shape[1]
        dz = (1.0 / (1.0 + np.exp(-zl)) - y).reshape(P, P, 2).transpose(2, 0, 1)
        dout = dz
        for i in range(3, -1, -1):
            w = (bf16_round(layers[i][0]) if round_bf16 else layers[i][0]).astype(np.float64)
            hin = acts[i]
            H, Wd = dout.shape[1], dout.shape[2]
            for dy in range(3):
                for dx in range(3):
                    grads[i][0][:, :, dy, dx] += np.einsum("ohw,chw->oc", dout, hin[:, dy:dy + H, dx:dx + Wd])
            grads[i][1][:] += dout.sum(axis=(1, 2))
            if i > 0:
                din = np.zeros_like(hin)
                for dy in range(3):
                    for dx in range(3):
                        din[:, dy:dy + H, dx:dx + Wd] += np.einsum("oc,ohw->chw", w[:, :, dy, dx], dout)
                dout = din * (1.0 - hin * hin)          # hin = tanh output of layer i-1
    ne = len(examples)
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads]) / ne
    return total / ne, flat


def adam_step(params, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) in float32; returns new (params, m, v)."""
    g = grad.astype(np.float32)
    m = (b1 * m + (1 - b1) * g).astype(np.float32)
    v = (b2 * v + (1 - b2) * g * g).astype(np.float32)
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = (params - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
    return p, m, v


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-np.asarray(z, np.float64)))


def log_q(z: np.ndarray, y: np.ndarray) -> float:
    """log q(y | context) of a patch configuration y (0/1 per patch link) under logits z."""
    return -bce_loss(z, y)


def propose_p1(z: np.ndarray, y_from: np.ndarray, rho: float) -> np.ndarray:
    """Probability that each patch link is 1 after a proposal with move rate rho: a link keeps its
    value with probability 1 - rho and is otherwise drawn from q(.|context), so
    P(y'_l = 1) = (1 - rho) y_l + rho sigmoid(z_l); rho = 1 is the factorised proposal q(.|context)."""
    return (1.0 - rho) * np.asarray(y_from, np.float64) + rho * sigmoid(z)


def log_q_move(z: np.ndarray, y_to: np.ndarray, y_from: np.ndarray, rho: float) -> float:
    """log q(y_to | y_from, context) of the proposal with move rate rho (see propose_p1), by its
    definition: sum over the patch links of log((1 - rho) [y_to = y_from] + rho q(y_to | context))."""
    s = sigmoid(z)
    y_to = np.asarray(y_to, np.float64)
    q_to = np.where(y_to == 1.0, s, 1.0 - s)
    same = (y_to == np.asarray(y_from, np.float64)).astype(np.float64)
    return float(np.sum(np.log((1.0 - rho) * same + rho * q_to)))


def draw_block(seed: int, chain: int, sweep: int, patch: int, n_links: int):
    """(u_accept, u_links) for a block move: accept word pair at counter (chain, sweep, patch, 2),
    link j's uniform (x + 1/2) 2^-32 from word j mod 4 of counter (chain, sweep, patch, 3 + j div 4)."""
    x0, x1, _, _ = philox.philox4x32_10((chain, sweep, patch, 2), (seed & 0xFFFFFFFF, seed >> 32))
    u_acc = float(philox.uniform_from_words(x0, x1))
    words = []
    for j in range((n_links + 3) // 4):
        words += list(philox.philox4x32_10((chain, sweep, patch, 3 + j), (seed & 0xFFFFFFFF, seed >> 32)))
    u = (np.array(words[:n_links], np.float64) + 0.5) * 2.0 ** -32
    return u_acc, u
