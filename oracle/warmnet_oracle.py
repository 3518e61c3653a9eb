"""Plain FP64 CPU oracle of the learned Krylov warm start.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/`` and nothing else; the
product path never imports it, and it shares no code with the HIP kernels.

What is computed.  The scheme's levels u^{j+1} follow u^j, u^{j-1}, u^{j-2}
closely: for a solution quadratic in t the extrapolation
3(u^j - u^{j-1}) + u^{j-2} is exact, and the L2-1sigma formula (Lemma 1) is
exact for such t-dependence.  The network predicts the remainder.

* Inputs at level j >= 2, with e1 = u^j - u^{j-1} and
  e2 = u^j - 2u^{j-1} + u^{j-2}:
  - channel 0: e1 / s;
  - channel 1: e2 / s, where s is the RMS of e2 over the grid (s = 1 when
    e2 vanishes);
  - channels 2..6: the constants alpha, beta, asinh(q_gamma),
    log1p(q_plus) and log1p(q_minus), with the dimensionless level
    coefficients q_gamma = sigma gamma_j / (h eta_j) and
    q_pm = sigma D_pm,j h^-beta / eta_j.  These are the size of each term of
    sigma L_j (3.3) relative to the diagonal eta_j.
* Network:
  - four 1-D convolutions 7 -> 32 -> 32 -> 32 -> 1, width 5, zero padding;
  - tanh after the first three;
  - weights rounded to bfloat16; the inputs of the two hidden 32 -> 32
    layers (tanh outputs) rounded to bfloat16 too (first to FP32, as the
    device holds them); the input and output layers take their inputs
    unrounded; biases, products and sums in higher precision.  The backward
    pass differentiates that computation with the rounding taken as the
    identity, so the weight gradient uses the rounded inputs.
* Prediction: x0 = 3(u^j - u^{j-1}) + u^{j-2} + y e2.  The correction is
  the network output times the local second difference e2.  It is smooth,
  and it vanishes where the Dirichlet condition of (1.1) fixes u, so it adds
  no grid-scale or boundary content.  The true residual g - A x0, which
  decides whether the guess is used, multiplies such content by up to |A|.
* Loss of one sample: the relative error of the correction,
  sum_p (y_p X1_p - T_p)^2 / (sum_p T_p^2 + n EPS_D), where X1 = e2 / s is
  input channel 1 and T = (u^{j+1} - base) / s is the scaled extrapolation
  error (s cancels).  Zero correction scores about 1 at every level, whatever
  the size of the extrapolation error there.  EPS_D sets where an error
  counts as none: X1 has unit RMS, so it is 1e-6 of the RMS of e2.  A batch's
  loss is the mean over its samples.
* Backward pass: the chain rule written out layer by layer.
* Adam update: Kingma and Ba, "Adam: a method for stochastic optimization"
  (ICLR 2015), Algorithm 1, with bias correction.

Parameter layout (flat vector), layer by layer: W[c_out][c_in][5], then
b[c_out].

Pinned by ``tests/test_oracle_warmnet.py``:
* central finite differences of the forward pass against the backward pass;
* a one-tap kernel acting as a shift;
* exact extrapolation of quadratic-in-t sequences;
* bfloat16 rounding of hand-picked values;
* Adam's first step moving every parameter by lr sign(g).
"""
from __future__ import annotations

import math

import numpy as np

from . import ids_oracle as O

CIN, WIDTH, KS = 7, 32, 5
LAYERS = [(CIN, WIDTH), (WIDTH, WIDTH), (WIDTH, WIDTH), (WIDTH, 1)]  # (c_in, c_out)
HALF = KS // 2
ROUNDED = (1, 2)  # layers whose inputs are rounded to bfloat16 (the hidden ones)


def param_count() -> int:
    return sum(co * ci * KS + co for ci, co in LAYERS)


def unpack(theta: np.ndarray):
    """Flat parameter vector -> [(W (c_out, c_in, KS), b (c_out,)), ...]."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = theta[o:o + co * ci * KS].reshape(co, ci, KS)
        o += co * ci * KS
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits, ties to even),
    returned in float64.  Written from the format's definition: keep the top
    16 bits of the float32 encoding after adding half an ulp (plus the tie
    bit)."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def weights_bf16(theta: np.ndarray) -> np.ndarray:
    """The parameters as the network uses them: weights in bfloat16, biases as given."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    return pack([(bf16_round(W), b.astype(np.float32).astype(np.float64)) for W, b in layers])


def level_features(prob, j: int, eta_j: float, gamma_j: float, dplus_j: float, dminus_j: float) -> np.ndarray:
    """Channels 2..6 at level j (alpha, beta and the three level coefficients
    of sigma L_j relative to eta_j)."""
    s, h, beta = O.sigma_of(prob.alpha), O.mesh_h(prob), prob.beta
    qg = s * gamma_j / (h * eta_j)
    qp = s * dplus_j * h ** (-beta) / eta_j
    qm = s * dminus_j * h ** (-beta) / eta_j
    return np.array([prob.alpha, beta, math.asinh(qg), math.log1p(qp), math.log1p(qm)])


def inputs(u0: np.ndarray, u1: np.ndarray, u2: np.ndarray, feats: np.ndarray):
    """(X (CIN, n), base, s) from u^j, u^{j-1}, u^{j-2} and the level features."""
    e1 = u0 - u1
    e2 = u0 - 2.0 * u1 + u2
    s = math.sqrt(float(np.mean(e2 * e2)))
    if s == 0.0:
        s = 1.0
    n = u0.size
    X = np.empty((CIN, n))
    X[0] = e1 / s
    X[1] = e2 / s
    X[2:] = np.asarray(feats)[:, None]
    base = 3.0 * (u0 - u1) + u2
    return X, base, s


def conv(a: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[co, p] = b[co] + sum_ci sum_k W[co, ci, k] a[ci, p + k - 2], zero outside."""
    ci, n = a.shape
    ap = np.zeros((ci, n + 2 * HALF))
    ap[:, HALF:HALF + n] = a
    out = np.repeat(b[:, None], n, axis=1).astype(np.float64)
    for k in range(KS):
        out += W[:, :, k] @ ap[:, k:k + n]
    return out


def forward(theta: np.ndarray, X: np.ndarray, rnd=bf16_round):
    """Network output y (n,) and the activations needed by backward.  rnd is
    applied to every convolution's input (bfloat16 rounding; the identity
    gives the exact-arithmetic network the chain-rule pin uses)."""
    layers = unpack(theta)
    acts = [X]
    a = X
    for li, (W, b) in enumerate(layers):
        z = conv(rnd(a) if li in ROUNDED else a, W, b)
        a = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(a)
    return a[0], acts


EPS_D = 1e-12  # X1 has unit RMS: corrections within 1e-6 RMS(e2) of the target count as exact


def loss(y: np.ndarray, x1: np.ndarray, t: np.ndarray) -> float:
    """Relative error of the correction y * x1 against t (one sample)."""
    return float(np.sum((y * x1 - t) ** 2) / (np.sum(t * t) + t.size * EPS_D))


def loss_dy(y: np.ndarray, x1: np.ndarray, t: np.ndarray) -> np.ndarray:
    """d loss / d y for one sample."""
    return 2.0 * (y * x1 - t) * x1 / (np.sum(t * t) + t.size * EPS_D)


def backward(theta: np.ndarray, acts, dy: np.ndarray, rnd=bf16_round) -> np.ndarray:
    """Gradient of sum_p dy[p] * y[p] with respect to the parameters (the
    rounding rnd taken as the identity, its output used in the weight
    gradient)."""
    layers = unpack(theta)
    grads = [None] * len(layers)
    dz = dy[None, :].astype(np.float64)  # d/dz of the last (linear) layer
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in = acts[li]
        ci, n = a_in.shape
        ap = np.zeros((ci, n + 2 * HALF))
        ap[:, HALF:HALF + n] = rnd(a_in) if li in ROUNDED else a_in
        dW = np.empty_like(W)
        for k in range(KS):
            dW[:, :, k] = dz @ ap[:, k:k + n].T
        db = dz.sum(axis=1)
        grads[li] = (dW, db)
        if li > 0:
            # d a_in[ci, q] = sum_co sum_k W[co, ci, k] dz[co, q - k + 2]
            dzp = np.zeros((dz.shape[0], n + 2 * HALF))
            dzp[:, HALF:HALF + n] = dz
            da = np.zeros((ci, n))
            for k in range(KS):
                da += W[:, :, k].T @ dzp[:, KS - 1 - k:KS - 1 - k + n]
            dz = da * (1.0 - a_in ** 2)  # tanh'
    return pack(grads)


def loss_and_grad(theta: np.ndarray, samples) -> tuple[float, np.ndarray]:
    """Mean over samples of the relative correction error, and its gradient.
    samples: list of (X, T)."""
    tot, g = 0.0, np.zeros(theta.size)
    for X, t in samples:
        y, acts = forward(theta, X)
        tot += loss(y, X[1], t)
        g += backward(theta, acts, loss_dy(y, X[1], t))
    return tot / len(samples), g / len(samples)


def target(u_next: np.ndarray, base: np.ndarray, s: float) -> np.ndarray:
    return (u_next - base) / s


def predict(theta: np.ndarray, u0, u1, u2, feats) -> np.ndarray:
    X, base, s = inputs(u0, u1, u2, feats)
    y, _ = forward(theta, X)
    return base + y * (u0 - 2.0 * u1 + u2)


def adam_step(theta, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (bias-corrected), returning new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
