"""Plain FP64 CPU oracle of the learned unrolled solver (an extension beyond
the paper: a learned prior stands in for the Hankel IRLS step).

TEST INFRASTRUCTURE ONLY.  Only the test suite may import this module; the
GPU library never calls it and shares no code with it.

What it computes.  The unknown is the slice-unfolded multi-shot k-space x of
Eq. 10 ([L][Ns][N2][N1], complex).  Starting from x_0 = A^H y, each of K
unrolled iterations applies

    z_k     = x_k + s * C(x_k / s)                     (residual prior)
    x_{k+1} = argmin_x ||A x - y||^2 + mu ||x - z_k||^2
            = (A^H A + mu I)^(-1) (A^H y + mu z_k)     (data consistency)

where C is a real CNN on the 2 Ns channels (real and imaginary part of each
shot's k-space) of every slice: five 3 x 3 convolutions (zero padding,
cross-correlation) with ReLU after the first four, weights shared across the
iterations; s = sqrt(mean |A^H y|^2) makes the network see unit-scale data.
The prior acts on k-space because the paper's own prior (Eq. 8-10) is a
shift-invariant relation between neighbouring k-space samples of the shots,
which convolutions over k-space express directly.

Each data-consistency solve is n_cg conjugate-gradient steps warm-started at
z_k (the oracle CG of smsm_oracle).  Training minimises
    loss = ||x_K - x*||^2 / ||x*||^2
against the plain solver's reconstruction x*.  The backward pass treats each
data-consistency solve as the exact inverse: for x = M^-1 (b + mu z),
M = A^H A + mu I (Hermitian), the gradient of a real loss with respect to z
is mu M^-1 g_x, with M^-1 again taken as n_cg CG steps, here from zero.

Two BF16 forms: BF16 weights with exact products (bf16_params), and the
BF16 network (act_bf16: every convolution input rounded to BF16, the
rounding passed straight through in the backward pass).

Pins (tests/test_oracle_learned_pins.py): the convolution against
scipy.signal.correlate2d, every analytic gradient against central finite
differences (with exact solves, where the backward pass is exact), the
data-consistency step against a dense solve, the untrained limit (zero
network: the iteration converges to the SENSE least-squares solution), and
the BF16 network reducing to the plain one on data whose every rounded
quantity is already a BF16 value, with BF16-valued activations otherwise.
"""
import numpy as np

from oracle import smsm_oracle as so


# ---- 3 x 3 convolution layer, [N][C][H][W] real arrays ---------------------

def conv3x3(x, w, b):
    """out[n, o, i, j] = b[o] + sum_{c, a, d} w[o, c, a, d] xp[n, c, i + a, j + d]
    with xp the zero-padded input (one pixel on every side)."""
    n, _, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    out = np.broadcast_to(b[None, :, None, None], (n, w.shape[0], h, wd)).astype(np.float64).copy()
    for a in range(3):
        for d in range(3):
            out += np.einsum('oc,nchw->nohw', w[:, :, a, d], xp[:, :, a:a + h, d:d + wd])
    return out


def conv3x3_backward(x, w, gout):
    """Gradients of sum(gout * conv3x3(x, w, b)) with respect to x, w and b."""
    n, c, h, wd = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    gw = np.zeros_like(w, dtype=np.float64)
    gxp = np.zeros_like(xp, dtype=np.float64)
    for a in range(3):
        for d in range(3):
            gw[:, :, a, d] = np.einsum('nohw,nchw->oc', gout, xp[:, :, a:a + h, d:d + wd])
            gxp[:, :, a:a + h, d:d + wd] += np.einsum('oc,nohw->nchw', w[:, :, a, d], gout)
    gb = gout.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:1 + h, 1:1 + wd], gw, gb


# ---- the network ------------------------------------------------------------

def cnn_forward(x, params, act_bf16=False):
    """params = [(w0, b0), ..., (w4, b4)]; ReLU after every layer but the last.
    Returns the output and the input of every layer (for the backward pass).
    act_bf16: the BF16 network, whose every convolution input (the network
    input and the hidden activations after their ReLU) is rounded to BF16."""
    h = bf16_round(x) if act_bf16 else x
    acts = [h]
    for k, (w, b) in enumerate(params):
        h = conv3x3(h, w, b)
        if k < len(params) - 1:
            h = np.maximum(h, 0.0)
            if act_bf16:
                h = bf16_round(h)
            acts.append(h)
    return h, acts


def cnn_backward(acts, params, gout, act_bf16=False):
    """Gradients with respect to the network input and every (w, b).
    act_bf16: the BF16 network's backward pass (rounding passed straight
    through): the gradient entering each transposed convolution is rounded
    to BF16 as that convolution's input, while the weight and bias gradients
    take the unrounded output gradient and the layer's (rounded) input."""
    grads = [None] * len(params)
    g = gout
    for k in range(len(params) - 1, -1, -1):
        w, _ = params[k]
        gx, gw, gb = conv3x3_backward(acts[k], w, g)
        if act_bf16:
            gx = conv3x3_backward(acts[k], w, bf16_round(g))[0]
        grads[k] = (gw, gb)
        # ReLU of the layer below: the stored activation is its output
        g = gx * (acts[k] > 0.0) if k > 0 else gx
    return g, grads


# ---- k-space <-> channels ---------------------------------------------------

def pack(x, s):
    """Complex [L][Ns][H][W] -> real [L][2 Ns][H][W]: channel 2i is Re x_i / s,
    channel 2i + 1 is Im x_i / s (s = 0, all-zero data: the channels are 0,
    and the prior's term s C(.) vanishes anyway)."""
    L, ns, h, w = x.shape
    f = 1.0 / s if s > 0 else 0.0
    out = np.empty((L, 2 * ns, h, w))
    out[:, 0::2] = x.real * f
    out[:, 1::2] = x.imag * f
    return out


def unpack(c, s):
    return s * (c[:, 0::2] + 1j * c[:, 1::2])


def data_scale(b) -> float:
    return float(np.sqrt(np.mean(np.abs(b) ** 2)))


# ---- unrolled solver --------------------------------------------------------

def dc_solve(apply_aha, b, z, mu: float, n_cg: int, x0=None):
    """n_cg CG steps on (A^H A + mu I) x = b + mu z, from x0 (default z)."""
    return so.cg(lambda v: apply_aha(v) + mu * v, b + mu * z, z if x0 is None else x0, n_cg)


def unrolled_forward(b, apply_aha, params, mu: float, n_unroll: int, n_cg: int, act_bf16=False):
    """x_K and the iterates x_0 .. x_{K-1} (x_0 = b = A^H y)."""
    s = data_scale(b)
    x = b.copy()
    xs = []
    for _ in range(n_unroll):
        xs.append(x)
        c, _ = cnn_forward(pack(x, s), params, act_bf16)
        z = x + unpack(c, s)
        x = dc_solve(apply_aha, b, z, mu, n_cg)
    return x, xs


def loss_value(x, x_target) -> float:
    return float(np.sum(np.abs(x - x_target) ** 2) / np.sum(np.abs(x_target) ** 2))


def unrolled_loss_and_grads(b, apply_aha, params, mu: float, n_unroll: int, n_cg: int, x_target,
                            act_bf16=False):
    """Loss and its gradients with respect to every (w, b) of the network."""
    s = data_scale(b)
    xK, xs = unrolled_forward(b, apply_aha, params, mu, n_unroll, n_cg, act_bf16)
    loss = loss_value(xK, x_target)
    g = 2.0 * (xK - x_target) / np.sum(np.abs(x_target) ** 2)    # d loss / d Re x + i d loss / d Im x
    total = [(np.zeros_like(w, dtype=np.float64), np.zeros_like(bb, dtype=np.float64)) for w, bb in params]
    for k in range(n_unroll - 1, -1, -1):
        wv = so.cg(lambda v: apply_aha(v) + mu * v, g, np.zeros_like(g), n_cg)
        gz = mu * wv
        # z = x + s * unpack(C(pack(x, s))): the network sees x / s and its output is scaled by s
        _, acts = cnn_forward(pack(xs[k], s), params, act_bf16)
        gc = pack(gz, 1.0 / s) if s > 0 else np.zeros_like(acts[0])   # d loss / d output channels: s (Re gz, Im gz)
        gin, grads = cnn_backward(acts, params, gc, act_bf16)
        for j, (gw, gb) in enumerate(grads):
            total[j] = (total[j][0] + gw, total[j][1] + gb)
        g = gz + (unpack(gin, 1.0 / s) if s > 0 else 0.0)   # residual path + d channels / d x = 1 / s
    return loss, total


def bf16_round(w):
    """FP32 values rounded to BF16 (8-bit significand) to nearest, ties to
    even, returned as FP64: the weights the BF16 form of the network uses."""
    bits = np.asarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_params(params):
    """The network's parameters as the BF16 form uses them: weights rounded,
    biases kept."""
    return [(bf16_round(w), np.asarray(b, dtype=np.float64)) for w, b in params]
