"""Two-tower entry model, contrastive loss and Adam in NumPy float64
(test infrastructure only).

Model (two-tower score, Preliminaries; projection network of the high-tier
graph section): each tower is a two-layer MLP with ReLU whose output is
L2-normalised, so the score of a query/hub pair is their cosine.

    tower(x) = normalise( W2 . relu(W1 . x + b1) + b2 )

The query tower reads the query vector; the hub tower reads the hub vector
concatenated with its topology features.  Loss: the contrastive objective of
Eq. 2 / Eq. 4 taken query-anchored over all hubs, with the positive inside the
denominator (standard InfoNCE):

    L = (1/B) sum_i [ logsumexp_h(s_ih) - s_i,y_i ],  s_ih = <e_q_i, e_h> / tau

BF16 reading: weights are held as FP32 masters; each matrix product takes its
two operands rounded to bfloat16 (round to nearest even) and accumulates in
higher precision (here FP64).  The operands that are rounded are: the weights,
the tower input, the hidden activation after ReLU and, in the backward pass,
the pre-activation gradients that enter the weight/input products.  Bias adds,
ReLU, normalisation, the logits and softmax stay unrounded.  With
``bf16=False`` every rounding is the identity (used for finite differences).
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 value (ties to even), returned as float64.

    Works from the float64 value: bfloat16 keeps 8 significant bits, so the
    value is rounded at 2**(e-7) where 2**e <= |x| < 2**(e+1)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    m, e = np.frexp(x[nz])            # x = m * 2**e, 0.5 <= |m| < 1
    # 8 significant bits: scale mantissa to [128, 256)
    scaled = m * 256.0
    r = np.round(scaled)              # numpy rounds half to even
    out[nz] = np.ldexp(r, e - 8)
    out[~nz] = x[~nz]
    return out


def _rnd(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def tower_forward(params, x, bf16=True, in_scale=1.0):
    """params = (W1 [h x din], b1 [h], W2 [e x h], b2 [e]) float32 masters;
    the input is multiplied by in_scale (a power of two) before rounding.

    Returns (e_hat [n x e], cache)."""
    W1, b1, W2, b2 = [np.asarray(p, np.float64) for p in params]
    W1r, W2r = _rnd(W1, bf16), _rnd(W2, bf16)
    xr = _rnd(np.asarray(x, np.float64) * in_scale, bf16)
    z1 = xr @ W1r.T + b1
    a1 = np.maximum(z1, 0.0)
    a1r = _rnd(a1, bf16)
    z2 = a1r @ W2r.T + b2
    nrm = np.sqrt(np.sum(z2 * z2, axis=1, keepdims=True))
    e = z2 / nrm
    return e, dict(xr=xr, z1=z1, a1r=a1r, z2=z2, nrm=nrm, e=e, W1r=W1r, W2r=W2r)


def tower_backward(cache, de, bf16=True):
    """Gradient of the tower parameters given dL/d e_hat.  Returns
    (dW1, db1, dW2, db2)."""
    e, nrm = cache["e"], cache["nrm"]
    # d/dz of z/|z|: (de - e <e, de>) / |z|
    dz2 = (de - e * np.sum(e * de, axis=1, keepdims=True)) / nrm
    dz2r = _rnd(dz2, bf16)
    dW2 = dz2r.T @ cache["a1r"]
    db2 = dz2.sum(axis=0)
    da1 = dz2r @ cache["W2r"]
    dz1 = da1 * (cache["z1"] > 0)
    dz1r = _rnd(dz1, bf16)
    dW1 = dz1r.T @ cache["xr"]
    db1 = dz1.sum(axis=0)
    return dW1, db1, dW2, db2


def infonce(eq, eh, labels, tau):
    """Loss and gradients w.r.t. both embedding sets."""
    s = (eq @ eh.T) / tau
    smax = s.max(axis=1, keepdims=True)
    ex = np.exp(s - smax)
    den = ex.sum(axis=1, keepdims=True)
    lse = np.log(den) + smax
    B = eq.shape[0]
    loss = float(np.mean(lse[:, 0] - s[np.arange(B), labels]))
    p = ex / den
    ds = p.copy()
    ds[np.arange(B), labels] -= 1.0
    ds /= B
    deq = ds @ eh / tau
    deh = ds.T @ eq / tau
    return loss, deq, deh, ds


def train_step_grads(qparams, hparams, xq, xh, labels, tau, bf16=True, q_scale=1.0):
    """Full forward/backward of one batch: returns (loss, q grads, h grads,
    eq, eh).  q_scale: the query tower's input scale."""
    eq, cq = tower_forward(qparams, xq, bf16, q_scale)
    eh, ch = tower_forward(hparams, xh, bf16)
    loss, deq, deh, _ = infonce(eq, eh, labels, tau)
    gq = tower_backward(cq, deq, bf16)
    gh = tower_backward(ch, deh, bf16)
    return loss, gq, gh, eq, eh


def hub_contrastive(eh, eq, P: int, N: int, tau: float):
    """Eq. 4 read hub-anchored: hub i (row i of eh) owns query rows
    i*(P+N) .. i*(P+N)+P-1 (its positives) and the next N (its negatives).
    With s_iq = <e_h_i, e_q> / tau and LSE_i over the hub's P + N scores,

        L(V_i) = - sum_{q in pos_i} log softmax_i(q) = P * LSE_i - sum_{pos_i} s_iq,

    and the batch loss is the mean over hubs.  Returns (loss, deh, deq)."""
    Bh = eh.shape[0]
    W = P + N
    loss = 0.0
    deh = np.zeros_like(eh)
    deq = np.zeros_like(eq)
    for i in range(Bh):
        rows = eq[i * W:(i + 1) * W]
        s = rows @ eh[i] / tau
        smax = s.max()
        ex = np.exp(s - smax)
        lse = np.log(ex.sum()) + smax
        loss += P * lse - s[:P].sum()
        ds = P * ex / ex.sum()
        ds[:P] -= 1.0
        ds /= Bh
        deh[i] = ds @ rows / tau
        deq[i * W:(i + 1) * W] = np.outer(ds, eh[i]) / tau
    return loss / Bh, deh, deq


def train_step_grads_hub(qparams, hparams, xq, xh, P, N, tau, bf16=True, q_scale=1.0):
    """Forward/backward of one hub-anchored batch (hub_contrastive): xh holds
    the batch's hub inputs, xq their P + N queries each.  Returns (loss,
    q grads, h grads, eq, eh)."""
    eq, cq = tower_forward(qparams, xq, bf16, q_scale)
    eh, ch = tower_forward(hparams, xh, bf16)
    loss, deh, deq = hub_contrastive(eh, eq, P, N, tau)
    gq = tower_backward(cq, deq, bf16)
    gh = tower_backward(ch, deh, bf16)
    return loss, gq, gh, eq, eh


def adam_update(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on float64 copies; t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    p = p - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


# ---------------------------------------------------------------- Eq. 3 fusion
def fusion_forward(params, p, U, mask, heads: int):
    """Eq. 3 multi-head attention of the hub vector over its topology tokens.

    params = (WQ [m*dk x dp], WK [m*dk x dU], WV [m*dk x dU], WO [dF x m*dk]);
    p [nh x dp] the hub vectors, U [nh x S x dU] the tokens, mask [nh x S]
    (1 = token present).  Head j uses rows j*dk .. j*dk+dk-1 of WQ/WK/WV:
        a_j = softmax_s( <p WQ_j, U_s WK_j> / sqrt(dk) )  over present s
        F   = concat_j( sum_s a_j,s U_s WV_j ) WO^T
    A hub without tokens gets F = 0.  Returns (F [nh x dF], cache)."""
    WQ, WK, WV, WO = [np.asarray(w, np.float64) for w in params]
    p, U = np.asarray(p, np.float64), np.asarray(U, np.float64)
    m = heads
    dk = WQ.shape[0] // m
    q = p @ WQ.T                                  # nh x m*dk
    K = U @ WK.T                                  # nh x S x m*dk
    V = U @ WV.T
    nh, S = U.shape[0], U.shape[1]
    a = np.zeros((nh, m, S))
    O = np.zeros((nh, m * dk))
    for i in range(nh):
        pres = np.asarray(mask[i], bool)
        if not pres.any():
            continue
        for j in range(m):
            sl = slice(j * dk, (j + 1) * dk)
            sc = K[i, :, sl] @ q[i, sl] / np.sqrt(dk)
            sc = np.where(pres, sc, -np.inf)
            e = np.exp(sc - sc[pres].max())
            a[i, j] = e / e.sum()
            O[i, sl] = a[i, j] @ V[i, :, sl]
    F = O @ WO.T
    return F, dict(p=p, U=U, q=q, K=K, V=V, a=a, O=O, WQ=WQ, WK=WK, WV=WV, WO=WO, m=m, dk=dk)


def fusion_backward(cache, dF):
    """Gradients of the four matrices given dL/dF.  Returns (gWQ, gWK, gWV, gWO)."""
    p, U, q, K, V, a, O = (cache[k] for k in ("p", "U", "q", "K", "V", "a", "O"))
    WO, m, dk = cache["WO"], cache["m"], cache["dk"]
    dF = np.asarray(dF, np.float64)
    gWO = dF.T @ O
    dO = dF @ WO                                  # nh x m*dk
    nh, S = U.shape[0], U.shape[1]
    dq = np.zeros_like(q)
    dK = np.zeros_like(K)
    dV = np.zeros_like(V)
    for i in range(nh):
        for j in range(m):
            sl = slice(j * dk, (j + 1) * dk)
            aj = a[i, j]
            dV[i, :, sl] = np.outer(aj, dO[i, sl])
            da = V[i, :, sl] @ dO[i, sl]
            ds = aj * (da - np.dot(aj, da))
            dq[i, sl] = ds @ K[i, :, sl] / np.sqrt(dk)
            dK[i, :, sl] = np.outer(ds, q[i, sl]) / np.sqrt(dk)
    gWQ = dq.T @ p
    gWK = np.einsum("ist,isc->tc", dK, U)
    gWV = np.einsum("ist,isc->tc", dV, U)
    return gWQ, gWK, gWV, gWO


def tower_backward_input(cache, de, bf16=True, in_scale=1.0):
    """dL/d(tower input) given dL/d e_hat (the input's BF16 rounding taken
    as the identity): in_scale * dz1 W1, with dz1 as in tower_backward."""
    e, nrm = cache["e"], cache["nrm"]
    dz2 = (de - e * np.sum(e * de, axis=1, keepdims=True)) / nrm
    dz2r = _rnd(dz2, bf16)
    da1 = dz2r @ cache["W2r"]
    dz1 = da1 * (cache["z1"] > 0)
    dz1r = _rnd(dz1, bf16)
    return in_scale * (dz1r @ cache["W1r"])
