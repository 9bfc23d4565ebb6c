"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain NumPy forward and backward passes of the small encoder-decoder that
maps (image z, marker distance map d, marker mask) to an initial level set
phi0 = M tanh(o), against which the GPU network's outputs and gradients are
checked.  The backward pass is written out by hand from the chain rule and
is itself pinned by finite differences (tests/test_oracle_pins.py).  With
store=bf16 the same code rounds every value the GPU stores in bfloat16 at
the same point, so that both sides take the ReLU and rounding decisions in
the same precision; the GPU's gradients are compared with that variant, whose
only remaining difference is the order of FP32 versus FP64 accumulation.

Architecture (depth D, widths C_l = base 2^l; every block is two 3x3
convolutions with ReLU, cb(x) = relu(conv_b(relu(conv_a(x))))):
    e_0 = cb(x),        e_l = cb(avgpool2(e_{l-1}))        l = 1..D-1
    d_{D-1} = e_{D-1},  d_l = cb([up2(d_{l+1}) | e_l])     l = D-2..0
    o = w . d_0 + b,        phi0 = M tanh(o)
    t = clip(target / M, -1, 1),  w = pos_weight where t > 0, 1 elsewhere,
    loss = mean(w (softplus(2 o) - o (1 + t)))
(the binary cross-entropy of (1 + tanh o) / 2 against (1 + t) / 2, minimal
at tanh o = t).
conv3 is a 3x3 convolution with zero padding: out[o, y, x] =
sum_{c, ky, kx} W[o, c, ky, kx] in[c, y + ky - 1, x + kx - 1] + b[o].
Parameters in the GPU library's order: the encoder's convolutions (a then b
of level 0, 1, ...), the decoder's (level 0 first), each W [OC][IC][3][3]
then b [OC]; head w [C0], head b [1].
"""
from __future__ import annotations

import numpy as np


def shapes(base: int, depth: int):
    """(IC, OC) of the encoder and decoder convolutions, two per block."""
    C = [base << l for l in range(depth)]
    enc, dec = [], []
    for l in range(depth):
        enc += [(3 if l == 0 else C[l - 1], C[l]), (C[l], C[l])]
    for l in range(depth - 1):
        dec += [(C[l + 1] + C[l], C[l]), (C[l], C[l])]
    return C, enc, dec


def unpack(theta: np.ndarray, base: int, depth: int):
    C, enc, dec = shapes(base, depth)
    out, off = {"enc": [], "dec": []}, 0

    def take(shape):
        nonlocal off
        k = int(np.prod(shape))
        a = theta[off:off + k].reshape(shape)
        off += k
        return a

    for ic, oc in enc:
        out["enc"].append((take((oc, ic, 3, 3)), take((oc,))))
    for ic, oc in dec:
        out["dec"].append((take((oc, ic, 3, 3)), take((oc,))))
    out["hw"] = take((C[0],))
    out["hb"] = take((1,))
    assert off == theta.size
    return out


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv3(x, W, b):
    """x [B, IC, H, W] -> [B, OC, H, W]."""
    B, IC, H, Wd = x.shape
    xp = _pad(x)
    out = np.zeros((B, W.shape[0], H, Wd))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,bchw->bohw", W[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + Wd])
    return out + b[None, :, None, None]


def conv3_grads(x, W, g):
    """Gradients of conv3 for the output gradient g: (dx, dW, db)."""
    B, IC, H, Wd = x.shape
    xp = _pad(x)
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            dW[:, :, ky, kx] = np.einsum("bohw,bchw->oc", g, xp[:, :, ky:ky + H, kx:kx + Wd])
            dxp[:, :, ky:ky + H, kx:kx + Wd] += np.einsum("oc,bohw->bchw", W[:, :, ky, kx], g)
    return dxp[:, :, 1:-1, 1:-1], dW, g.sum(axis=(0, 2, 3))


def avgpool(x):
    B, C, H, W = x.shape
    return x.reshape(B, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def avgpool_grad(g):
    return np.repeat(np.repeat(g, 2, axis=2), 2, axis=3) * 0.25


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=2), 2, axis=3)


def up2_grad(g):
    B, C, H, W = g.shape
    return g.reshape(B, C, H // 2, 2, W // 2, 2).sum(axis=(3, 5))


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64: the
    storage precision of the GPU network's activations, weights and gradients.
    Values are first rounded to float32, as the GPU holds them."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return a


def block(x, Pa, Pb, q=_ident):
    """Two convolutions with ReLU; returns (mid, y, y_stored).  q rounds what
    is stored (weights, activations)."""
    mid = q(np.maximum(conv3(x, q(Pa[0]), Pa[1]), 0.0))
    y = np.maximum(conv3(mid, q(Pb[0]), Pb[1]), 0.0)
    return mid, y, q(y)


def block_grads(x, cache, Pa, Pb, gy, q=_ident):
    """Backward of block(): (gx, (dWa, dba), (dWb, dbb)) for the gradient gy
    of y.  The ReLU derivative is taken from the stored outputs."""
    mid, _, ys = cache
    gy = gy * (ys > 0)
    gmid, dWb, dbb = conv3_grads(mid, q(Pb[0]), gy)
    gmid = q(gmid) * (mid > 0)
    gx, dWa, dba = conv3_grads(x, q(Pa[0]), gmid)
    return q(gx), (dWa, dba), (dWb, dbb)


def forward(theta, x, base, depth, M, store=None):
    """Returns phi0 [B, H, W] and the cache for backward.  store=None is the
    exact FP64 network; store=bf16 rounds where the GPU stores bf16 values
    (input, weights, activations; the head reads the unrounded d_0)."""
    q = store or _ident
    P = unpack(np.asarray(theta, np.float64), base, depth)
    x = q(np.asarray(x, np.float64))
    cache = {"x": x, "enc": [], "e": [], "pool": [], "dec": {}, "cat": {}}
    cur = x
    for l in range(depth):
        c = block(cur, P["enc"][2 * l], P["enc"][2 * l + 1], q)
        cache["enc"].append(c); cache["e"].append(c[2])
        if l < depth - 1:
            cur = q(avgpool(c[2]))
            cache["pool"].append(cur)
    dn = cache["e"][depth - 1]
    for l in range(depth - 2, -1, -1):
        cat = np.concatenate([up2(dn), cache["e"][l]], axis=1)
        c = block(cat, P["dec"][2 * l], P["dec"][2 * l + 1], q)
        dn = c[2]
        cache["cat"][l] = cat; cache["dec"][l] = c
    d0 = cache["dec"][0][1]
    o = np.einsum("c,bchw->bhw", P["hw"], d0) + P["hb"][0]
    cache["o"] = o
    return M * np.tanh(o), cache


def loss_and_grad(theta, x, target, base, depth, M, store=None, pos_weight=1.0):
    """Loss of the forward pass and its gradient with respect to theta (store
    as in forward: None exact, bf16 with the GPU's storage roundings)."""
    q = store or _ident
    P = unpack(np.asarray(theta, np.float64), base, depth)
    _, c = forward(theta, x, base, depth, M, store)
    o = c["o"]
    t = np.clip(np.asarray(target, np.float64) / M, -1.0, 1.0)
    N = o.size
    w = np.where(t > 0, pos_weight, 1.0)
    loss = float((w * (np.logaddexp(0.0, 2.0 * o) - o * (1.0 + t))).mean())
    dO = w * (np.tanh(o) - t) / N
    G = {"enc": [None] * (2 * depth), "dec": [None] * (2 * depth - 2)}
    G["hw"] = np.einsum("bhw,bchw->c", dO, c["dec"][0][1])
    G["hb"] = np.array([dO.sum()])
    gd = q(np.einsum("c,bhw->bchw", P["hw"], dO))
    ge_skip = {}
    for l in range(depth - 1):
        gcat, G["dec"][2 * l], G["dec"][2 * l + 1] = block_grads(
            c["cat"][l], c["dec"][l], P["dec"][2 * l], P["dec"][2 * l + 1], gd, q)
        cu = c["cat"][l].shape[1] - c["e"][l].shape[1]
        ge_skip[l] = gcat[:, cu:]
        gd = q(up2_grad(gcat[:, :cu]))
    ge = gd                                             # gradient of e_{D-1}
    gpool = None
    for l in range(depth - 1, -1, -1):
        if l < depth - 1:
            ge = q(ge_skip[l] + avgpool_grad(gpool))
        xin = c["x"] if l == 0 else c["pool"][l - 1]
        gpool, G["enc"][2 * l], G["enc"][2 * l + 1] = block_grads(
            xin, c["enc"][l], P["enc"][2 * l], P["enc"][2 * l + 1], ge, q)
    flat = []
    for dW, db in G["enc"] + G["dec"]:
        flat += [dW.ravel(), db.ravel()]
    flat += [G["hw"].ravel(), G["hb"].ravel()]
    return loss, np.concatenate(flat)


def param_count(base, depth):
    C, enc, dec = shapes(base, depth)
    return sum(oc * ic * 9 + oc for ic, oc in enc + dec) + C[0] + 1
