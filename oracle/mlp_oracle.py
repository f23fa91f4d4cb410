"""FP64 CPU reference of the surrogate network (test infrastructure only).

A perceptron with inputs padded to 64 columns, three hidden layers of 256
SiLU units and a linear output padded to 64 columns, and its loss
    L = sum_{r < M, o} wo_o (P_ro - T_ro)^2 / (M sum_o wo_o).
The parameter vector is laid out as the GPU library lays it out:
    W_0[256][64] | b_0[256] | W_1[256][256] | b_1 | W_2[256][256] | b_2 |
    W_3[64][256] | b_3[64]          (weights stored [out][in])

``loss_and_grad(..., bf16=False)`` is the exact FP64 gradient of L
(pinned by central finite differences in the tests).  With ``bf16=True``
the weights, the inputs and the hidden activations are rounded to bfloat16,
as the network stores them; everything else, the back-propagated values
included, stays FP64 (the GPU carries those as high and low bf16 parts,
about 16 significant bits).

Only the tests import this module.
"""
from __future__ import annotations

import numpy as np

PAD = 64
HID = 256
SHAPES = [(HID, PAD), (HID, HID), (HID, HID), (PAD, HID)]


def offsets():
    """(weight offset, bias offset) of each layer in the parameter vector."""
    out, o = [], 0
    for n, k in SHAPES:
        out.append((o, o + n * k))
        o += n * k + n
    return out, o


OFFSETS, NPARAMS = offsets()


def unpack(theta):
    Ws, bs = [], []
    for (n, k), (ow, ob) in zip(SHAPES, OFFSETS):
        Ws.append(theta[ow:ow + n * k].reshape(n, k))
        bs.append(theta[ob:ob + n])
    return Ws, bs


def to_bf16(x):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, X, bf16=False):
    """X [M][64] (already standardised and padded) -> P [M][64], cache."""
    rd = to_bf16 if bf16 else (lambda a: a)
    Ws, bs = unpack(np.asarray(theta, dtype=np.float64))
    Wr = [rd(W) for W in Ws]
    H = [rd(X)]
    Z = []
    for l in range(3):
        z = H[-1] @ Wr[l].T + bs[l]
        Z.append(z)
        H.append(rd(silu(z)))
    P = H[-1] @ Wr[3].T + bs[3]
    return P, (Wr, H, Z)


def loss_and_grad(theta, X, T, wo=None, bf16=False):
    """Loss and its gradient w.r.t. theta; T [M][OUT] with OUT <= 64."""
    M, out = T.shape
    w = np.zeros(PAD)
    w[:out] = 1.0 if wo is None else np.asarray(wo, dtype=np.float64)
    P, (Wr, H, Z) = forward(theta, X, bf16)
    Tp = np.zeros_like(P)
    Tp[:, :out] = T
    D = P - Tp
    D[:, out:] = 0.0
    wsum = w.sum()
    loss = float(np.sum(w[None, :] * D * D) / (M * wsum))
    dZ = 2.0 * w[None, :] * D / (M * wsum)  # dL/dP
    grad = np.zeros(NPARAMS)
    for l in range(3, -1, -1):
        ow, ob = OFFSETS[l]
        n, k = SHAPES[l]
        grad[ow:ow + n * k] = (dZ.T @ H[l]).ravel()
        grad[ob:ob + n] = dZ.sum(0)
        if l > 0:
            dZ = (dZ @ Wr[l]) * dsilu(Z[l - 1])
    return loss, grad
