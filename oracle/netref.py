"""FP64 reference of the learned preconditioner's network (CPU).

Test infrastructure only (see the package header).  Not part of the paper:
this is the definition of the small U-Net the library trains, written
layer by layer so that the GPU's forward pass and its parameter gradients
can be checked.

Network (per image, channels x height x width, zero padding):
  x0 = r / s, s = RMS(r) (1 if r = 0)
  a1  = relu(conv(x0, L0))          16 ch     a1b = relu(conv(a1, L1))   16 ch
  p1  = avgpool2(a1b)                         a2  = relu(conv(p1, L2))   32 ch
  a2b = relu(conv(a2, L3))          32 ch     p2  = avgpool2(a2b)
  a3  = relu(conv(p2, L4))          64 ch     a3b = relu(conv(a3, L5))   64 ch
  a4  = relu(conv([up2(a3b), a2b], L6)) 32 ch
  a5  = relu(conv([up2(a4), a1b], L7))  16 ch
  y   = conv(a5, L8)[0]                       z = y * s
conv(x, L)[co] = b[co] + sum_{ci, dy, dx} W[co][ci][dy][dx] x[ci][. + dy - 1][. + dx - 1].
Loss: mean over all pixels of the batch of (y - e / s)^2.
Parameter vector: all weights (layer order, [cout][cin][3][3]), then all biases.
"""

import numpy as np

LAYERS = [(1, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (48, 16), (16, 1)]


def unflatten(p):
    p = np.asarray(p, dtype=np.float64)
    Ws, bs, o = [], [], 0
    for cin, cout in LAYERS:
        n = cout * cin * 9
        Ws.append(p[o:o + n].reshape(cout, cin, 3, 3))
        o += n
    for cin, cout in LAYERS:
        bs.append(p[o:o + cout])
        o += cout
    assert o == p.size
    return Ws, bs


def flatten(Ws, bs):
    return np.concatenate([w.ravel() for w in Ws] + [b.ravel() for b in bs])


def conv(x, W, b):
    """3x3 convolution (cross-correlation), zero padding; x [C][H][W]."""
    C, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    out = np.zeros((W.shape[0], H, Wd))
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,chw->ohw", W[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + Wd])
    return out + b[:, None, None]


def conv_backward(x, W, dout):
    """Gradients of sum(dout * conv(x, W, b)) w.r.t. x, W and b."""
    C, H, Wd = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1)))
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            dW[:, :, dy, dx] = np.einsum("ohw,chw->oc", dout, xp[:, dy:dy + H, dx:dx + Wd])
            dxp[:, dy:dy + H, dx:dx + Wd] += np.einsum("oc,ohw->chw", W[:, :, dy, dx], dout)
    return dxp[:, 1:-1, 1:-1], dW, dout.sum(axis=(1, 2))


def pool(x):
    C, H, W = x.shape
    return x.reshape(C, H // 2, 2, W // 2, 2).mean(axis=(2, 4))


def pool_backward(dout):
    return np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dout):
    C, H, W = dout.shape
    return dout.reshape(C, H // 2, 2, W // 2, 2).sum(axis=(2, 4))


def _forward_image(Ws, bs, r):
    s = float(np.sqrt(np.mean(r * r)))
    s = s if s > 0 else 1.0
    t = {"s": s, "x0": (r / s)[None]}
    relu = lambda v: np.maximum(v, 0.0)  # noqa: E731
    t["a1"] = relu(conv(t["x0"], Ws[0], bs[0]))
    t["a1b"] = relu(conv(t["a1"], Ws[1], bs[1]))
    t["p1"] = pool(t["a1b"])
    t["a2"] = relu(conv(t["p1"], Ws[2], bs[2]))
    t["a2b"] = relu(conv(t["a2"], Ws[3], bs[3]))
    t["p2"] = pool(t["a2b"])
    t["a3"] = relu(conv(t["p2"], Ws[4], bs[4]))
    t["a3b"] = relu(conv(t["a3"], Ws[5], bs[5]))
    t["c2"] = np.concatenate([up(t["a3b"]), t["a2b"]])
    t["a4"] = relu(conv(t["c2"], Ws[6], bs[6]))
    t["c1"] = np.concatenate([up(t["a4"]), t["a1b"]])
    t["a5"] = relu(conv(t["c1"], Ws[7], bs[7]))
    t["y"] = conv(t["a5"], Ws[8], bs[8])[0]
    return t


def forward(params, r):
    """z for a batch r [B][H][W] (H, W divisible by 4)."""
    Ws, bs = unflatten(params)
    out = []
    for img in np.asarray(r, dtype=np.float64):
        t = _forward_image(Ws, bs, img)
        out.append(t["y"] * t["s"])
    return np.stack(out)


def loss(params, r, e):
    Ws, bs = unflatten(params)
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    tot = 0.0
    for img, err in zip(r, e):
        t = _forward_image(Ws, bs, img)
        tot += float(((t["y"] - err / t["s"]) ** 2).sum())
    return tot / r.size


def gradients(params, r, e):
    """(loss, d loss / d params) by back-propagation through the layers."""
    Ws, bs = unflatten(params)
    dWs = [np.zeros_like(w) for w in Ws]
    dbs = [np.zeros_like(b) for b in bs]
    r = np.asarray(r, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    N = r.size
    L = 0.0

    def acc(l, x, dout):
        dx, dW, db = conv_backward(x, Ws[l], dout)
        dWs[l] += dW
        dbs[l] += db
        return dx

    for img, err in zip(r, e):
        t = _forward_image(Ws, bs, img)
        d = t["y"] - err / t["s"]
        L += float((d * d).sum())
        dy = (2.0 * d / N)[None]
        da5 = acc(8, t["a5"], dy) * (t["a5"] > 0)
        dc1 = acc(7, t["c1"], da5)
        n4 = t["a4"].shape[0]
        da4 = up_backward(dc1[:n4]) * (t["a4"] > 0)
        da1b_skip = dc1[n4:]
        dc2 = acc(6, t["c2"], da4)
        n3 = t["a3b"].shape[0]
        da3b = up_backward(dc2[:n3]) * (t["a3b"] > 0)
        da2b_skip = dc2[n3:]
        da3 = acc(5, t["a3"], da3b) * (t["a3"] > 0)
        dp2 = acc(4, t["p2"], da3)
        da2b = (pool_backward(dp2) + da2b_skip) * (t["a2b"] > 0)
        da2 = acc(3, t["a2"], da2b) * (t["a2"] > 0)
        dp1 = acc(2, t["p1"], da2)
        da1b = (pool_backward(dp1) + da1b_skip) * (t["a1b"] > 0)
        da1 = acc(1, t["a1"], da1b) * (t["a1"] > 0)
        acc(0, t["x0"], da1)
    return L / N, flatten(dWs, dbs)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    Ws = [rng.standard_normal((co, ci, 3, 3)) * np.sqrt(2.0 / (9 * ci)) for ci, co in LAYERS]
    bs = [rng.standard_normal(co) * 0.1 for ci, co in LAYERS]
    return flatten(Ws, bs)
