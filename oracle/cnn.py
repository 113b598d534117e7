"""Reference for the learned preconditioner stage: a 4-layer 3x3 convolutional
network on the lattice, complex-as-real (4 channels = 2 spins x re/im),
hidden width 32, tanh after the first three layers.

The network is not part of the paper's method; it only proposes an initial
guess for the solves (every solve still runs to its FP64 tolerance, so the
estimator is unchanged).  This module is the plain FP64 forward/backward the
HIP training kernels are checked against.  Nothing in the paper fixes its
values; it is pinned against the mathematics instead: a brute-force
convolution with explicit boundary indices, translation equivariance,
central finite differences of the loss, and Adam's closed-form steps.

Conventions shared with the HIP side
------------------------------------
* fields: float [nb][C][Lt][Lx]; channel 2s = Re psi_s, 2s+1 = Im psi_s.
* padding: periodic in x; in t periodic or antiperiodic (a value fetched
  across the t boundary is multiplied by -1), matching the fermion boundary
  condition; tanh is odd, so every layer is consistent with it.
* conv: out[n][co][t][x] = b[co] + sum_{ci,dt,dx} W[co][ci][dt][dx]
        * in[n][ci][t+dt-1][x+dx-1]    (dt, dx in 0..2)
* parameters packed in one vector: W1 b1 W2 b2 W3 b3 W4 b4 (row-major).
* loss: mean over the batch of ||y - target||^2 / ||target||^2.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (4, 32, 32, 32, 4)


def param_shapes(widths=WIDTHS):
    shapes = []
    for cin, cout in zip(widths[:-1], widths[1:]):
        shapes.append((cout, cin, 3, 3))
        shapes.append((cout,))
    return shapes


def n_params(widths=WIDTHS) -> int:
    return int(sum(np.prod(s) for s in param_shapes(widths)))


def unpack(theta: np.ndarray, widths=WIDTHS):
    out, o = [], 0
    for s in param_shapes(widths):
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def complex_to_channels(v: np.ndarray, Lx: int, Lt: int) -> np.ndarray:
    """[nb][n] complex (dof (t*Lx+x)*2+s) -> [nb][4][Lt][Lx] real."""
    nb = v.shape[0]
    psi = v.reshape(nb, Lt, Lx, 2)
    ch = np.empty((nb, 4, Lt, Lx))
    for s in range(2):
        ch[:, 2 * s] = psi[..., s].real
        ch[:, 2 * s + 1] = psi[..., s].imag
    return ch


def channels_to_complex(ch: np.ndarray) -> np.ndarray:
    nb, _, Lt, Lx = ch.shape
    psi = np.empty((nb, Lt, Lx, 2), dtype=np.complex128)
    for s in range(2):
        psi[..., s] = ch[:, 2 * s] + 1j * ch[:, 2 * s + 1]
    return psi.reshape(nb, -1)


def _shifted(a: np.ndarray, dt: int, dx: int, anti: bool) -> np.ndarray:
    """a[..., t+dt, x+dx] with the lattice boundary conditions."""
    Lt, Lx = a.shape[-2:]
    out = np.roll(a, shift=(-dt, -dx), axis=(-2, -1))
    if anti and dt != 0:
        t = np.arange(Lt)
        crossed = (t + dt >= Lt) | (t + dt < 0)
        out = out * np.where(crossed, -1.0, 1.0)[:, None]
    return out


def conv(inp: np.ndarray, W: np.ndarray, b: np.ndarray, anti: bool) -> np.ndarray:
    nb, cin, Lt, Lx = inp.shape
    cout = W.shape[0]
    out = np.broadcast_to(b[None, :, None, None], (nb, cout, Lt, Lx)).copy()
    for dt in range(3):
        for dx in range(3):
            sh = _shifted(inp, dt - 1, dx - 1, anti)
            out += np.einsum("oc,nctx->notx", W[:, :, dt, dx], sh)
    return out


def conv_backward(inp, W, gout, anti):
    """Gradients of sum(gout * conv(inp)) w.r.t. inp, W and b."""
    gin = np.zeros_like(inp)
    gW = np.zeros_like(W)
    for dt in range(3):
        for dx in range(3):
            sh = _shifted(inp, dt - 1, dx - 1, anti)
            gW[:, :, dt, dx] = np.einsum("notx,nctx->oc", gout, sh)
            contrib = np.einsum("oc,notx->nctx", W[:, :, dt, dx], gout)
            # the adjoint of the shift by (dt-1, dx-1) is the shift back
            gin += _shifted(contrib, -(dt - 1), -(dx - 1), anti)
    gb = gout.sum(axis=(0, 2, 3))
    return gin, gW, gb


def forward(theta: np.ndarray, x: np.ndarray, anti: bool = True, widths=WIDTHS):
    """Returns the output and the activations needed by backward()."""
    params = unpack(theta, widths)
    acts = [x]
    h = x
    nl = len(widths) - 1
    for l in range(nl):
        z = conv(h, params[2 * l], params[2 * l + 1], anti)
        h = np.tanh(z) if l < nl - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grad(theta: np.ndarray, x: np.ndarray, target: np.ndarray, anti: bool = True,
                  widths=WIDTHS):
    y, acts = forward(theta, x, anti, widths)
    nb = x.shape[0]
    diff = y - target
    tn = np.sum(target ** 2, axis=(1, 2, 3))
    loss = float(np.mean(np.sum(diff ** 2, axis=(1, 2, 3)) / tn))
    g = 2.0 * diff / tn[:, None, None, None] / nb
    params = unpack(theta, widths)
    grads = [None] * len(params)
    nl = len(widths) - 1
    for l in reversed(range(nl)):
        if l < nl - 1:
            g = g * (1.0 - acts[l + 1] ** 2)   # through tanh
        gin, gW, gb = conv_backward(acts[l], params[2 * l], g, anti)
        grads[2 * l], grads[2 * l + 1] = gW, gb
        g = gin
    return loss, np.concatenate([q.ravel() for q in grads])


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) with bias-corrected
    moments; ``t`` counts steps from 1.  Returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
