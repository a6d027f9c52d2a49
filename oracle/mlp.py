"""Oracle of the learned warm start -- TEST INFRASTRUCTURE.

Plain numpy (float64) versions of the per-cell features, the network
(16 -> 128 -> 128 -> 128, ReLU, softmax over steps 1..m), its cross-entropy
gradient, Adam, the marginal quantisation and (through oracle.c) the seed
sampler.  With ``bf16=True`` the forward and backward products round both
operands to bfloat16 (round to nearest even, from float32) exactly where the
HIP kernels do; with ``bf16=False`` the arithmetic is plain float64 (used by
the finite-difference pin).
"""
import ctypes as C

import numpy as np

D_IN, D_H, D_OUT = 16, 128, 128
SHAPES = [("W1", (D_IN, D_H)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)), ("W3", (D_H, D_OUT)),
          ("b3", (D_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[n], np.float64).reshape(-1) for n, _ in SHAPES])


def bf16(v):
    """float -> float32 -> bfloat16 (round to nearest even) -> float64."""
    f = np.ascontiguousarray(np.asarray(v, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _mm(a, b, rnd):
    if rnd:
        return bf16(a) @ bf16(b)
    return np.asarray(a, np.float64) @ np.asarray(b, np.float64)


def forward(theta, X, msteps, bf16_ops=True):
    """Pre-activations Z1, Z2, logits Z3 and probabilities P (rows x 128)."""
    p = unpack(theta)
    X = np.asarray(X, np.float64)
    Z1 = _mm(X, p["W1"], bf16_ops) + p["b1"]
    Z2 = _mm(np.maximum(Z1, 0), p["W2"], bf16_ops) + p["b2"]
    Z3 = _mm(np.maximum(Z2, 0), p["W3"], bf16_ops) + p["b3"]
    mask = np.arange(D_OUT)[None, :] < np.asarray(msteps)[:, None]
    Zm = np.where(mask, Z3, -np.inf)
    mx = Zm.max(1, keepdims=True)
    e = np.where(mask, np.exp(Zm - mx), 0.0)
    P = e / e.sum(1, keepdims=True)
    return Z1, Z2, Z3, P


def loss_grad(theta, X, msteps, labels, bf16_ops=True):
    """Summed cross-entropy of the label steps and the gradient of the mean."""
    p = unpack(theta)
    X = np.asarray(X, np.float64)
    labels = np.asarray(labels)
    rows = X.shape[0]
    Z1, Z2, Z3, P = forward(theta, X, msteps, bf16_ops)
    loss = float(-np.log(P[np.arange(rows), labels]).sum())
    G3 = P.copy()
    G3[np.arange(rows), labels] -= 1.0
    G3 /= rows
    A1, A2 = np.maximum(Z1, 0), np.maximum(Z2, 0)
    g = {}
    g["W3"] = _mm(A2.T, G3, bf16_ops)
    g["b3"] = G3.sum(0)
    G2 = _mm(G3, p["W3"].T, bf16_ops) * (Z2 > 0)
    g["W2"] = _mm(A1.T, G2, bf16_ops)
    g["b2"] = G2.sum(0)
    G1 = _mm(G2, p["W2"].T, bf16_ops) * (Z1 > 0)
    g["W1"] = _mm(X.T, G1, bf16_ops)
    g["b1"] = G1.sum(0)
    return loss, pack(g)


def adam(theta, m1, m2, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m1 = b1 * m1 + (1 - b1) * grad
    m2 = b2 * m2 + (1 - b2) * grad * grad
    c1, c2 = 1 - b1 ** step, 1 - b2 ** step
    return theta - lr * (m1 / c1) / (np.sqrt(m2 / c2) + eps), m1, m2


def quantize(P, msteps):
    """q = floor(p * 65534) + 1 (in 1..65535) on the float32 probabilities, 0 beyond m."""
    P32 = np.asarray(P, np.float32)
    q = (np.floor(P32 * np.float32(65534.0)) + np.float32(1.0)).astype(np.uint16)
    mask = np.arange(D_OUT)[None, :] < np.asarray(msteps)[:, None]
    return np.where(mask, q, 0).astype(np.uint16)


def features(rows, cols, depot, nofly):
    """16 features per free cell (free-list order)."""
    nofly = np.asarray(nofly, np.uint8).reshape(rows, cols) if nofly is not None else np.zeros((rows, cols), np.uint8)
    free = (nofly == 0)
    i0, j0 = divmod(depot, cols)
    cells = [g for g in range(rows * cols) if g != depot and free.flat[g]]
    m = len(cells)
    side = max(rows, cols)
    den = float(side - 1) if side > 1 else 1.0
    out = np.zeros((m, 16), np.float64)
    for c, g in enumerate(cells):
        i, j = divmod(g, cols)
        out[c, 0], out[c, 1] = i / den, j / den
        out[c, 2], out[c, 3] = (i - i0) / den, (j - j0) / den
        out[c, 4] = np.sqrt((i - i0) ** 2 + (j - j0) ** 2) / (np.sqrt(2.0) * den)
        ring_free, ring_all = np.zeros(9), np.zeros(9)
        nf1 = nf2 = 0
        for a in range(rows):
            for b in range(cols):
                d = max(abs(a - i), abs(b - j))
                if d == 0 or d > 8:
                    continue
                fr = bool(free[a, b])
                nf1 += (not fr) and d == 1
                nf2 += (not fr) and d <= 2
                ring_all[d] += 1
                ring_free[d] += fr
        out[c, 5], out[c, 6] = nf1 / 8.0, nf2 / 24.0
        for r in range(1, 9):
            out[c, 6 + r] = ring_free[r] / ring_all[r] if ring_all[r] else 0.0
        out[c, 15] = m / 99.0
    return out.astype(np.float32)


def sample_seed(q, m, seed, inst, r):
    """Integer seed sampler (oracle.c)."""
    from . import lib
    L = lib()
    if not hasattr(L, "_sample_set"):
        L.orc_sample_seed.argtypes = [C.c_int32, C.POINTER(C.c_uint16), C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.POINTER(C.c_uint8)]
        L.orc_sample_seed.restype = C.c_int32
        L._sample_set = True
    qq = np.ascontiguousarray(q, dtype=np.uint16).reshape(m, 128)
    x = np.zeros(m * m, np.uint8)
    rc = L.orc_sample_seed(m, qq.ctypes.data_as(C.POINTER(C.c_uint16)), seed, inst, r,
                           x.ctypes.data_as(C.POINTER(C.c_uint8)))
    assert rc == 0
    return x
