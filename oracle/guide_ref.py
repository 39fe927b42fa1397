"""Reference of the learned path-guiding proposal: network, mixture, loss.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the HIP library never does.

Plain PyTorch CPU code in float64.  The proposal is not part of the paper's
method (its Sec. 3.1 samples the BRDF and the lights); it is the learned
importance sampler the estimator is combined with by one-sample MIS
(Veach 1997, Sec. 9.2.4), trained with the neural-importance-sampling KL
objective (Mueller et al. 2019, Sec. 4).

Network: inputs x = (position normalised to the scene box, shading normal,
outgoing direction, 16-d embedding of the segment), 25 values; four hidden
layers of width 64 with ReLU; 40 outputs, 5 per lobe j:
  mu_j = normalise(y[5j:5j+3]),  kappa_j = min(softplus(y[5j+3]) + 0.01, 1e4),
  weight_j = softmax_j(y[5j+4]).
vMF density on the sphere: kappa / (2 pi (1 - e^{-2 kappa})) e^{kappa (mu.w - 1)}.

Parameter block (float32, as the library stores it): W1 [25][64], b1 [64],
W2, W3, W4 [64][64] with biases [64], W5 [64][40], b5 [40], then the
embedding [S][16].  A layer computes y[n] = b[n] + sum_k x[k] W[k][n].

``bf16=True`` emulates the bfloat16 matrix-core path: the network inputs,
the weights and every hidden activation are rounded to bfloat16 (round to
nearest even), products are accumulated exactly, biases stay float32.  In
the gradient the roundings pass the derivative through unchanged
(straight-through), which is what a bfloat16 backward pass computes.
"""
import numpy as np
import torch

N_IN, N_EMB, N_HID, N_OUT, N_LOBES = 25, 16, 64, 40, 8
N_NET = N_IN * N_HID + N_HID + 3 * (N_HID * N_HID + N_HID) + N_HID * N_OUT + N_OUT   # 16744

_DT = torch.float64


def _bf16(t, straight_through=True):
    r = t.to(torch.float32).to(torch.bfloat16).to(_DT)
    return t + (r - t).detach() if straight_through else r


def unpack(params):
    """Split a parameter block (array or float64 tensor) into layers and embedding."""
    p = params if isinstance(params, torch.Tensor) else torch.as_tensor(np.asarray(params, np.float64))
    off = 0
    layers = []
    for fan_in, fan_out in [(N_IN, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT)]:
        W = p[off:off + fan_in * fan_out].reshape(fan_in, fan_out)
        off += fan_in * fan_out
        b = p[off:off + fan_out]
        off += fan_out
        layers.append((W, b))
    assert off == N_NET
    emb = p[N_NET:].reshape(-1, N_EMB)
    return layers, emb


def network(params, feat, seg, bf16=False):
    """Raw outputs [n, 40] for feature rows feat [n, 9] and segments seg [n]."""
    layers, emb = unpack(params)
    f = torch.as_tensor(np.asarray(feat, np.float64)) if not isinstance(feat, torch.Tensor) else feat
    f = f.to(_DT).reshape(-1, 9)
    x = torch.cat([f.to(torch.float32).to(_DT), emb[torch.as_tensor(np.asarray(seg, np.int64))]], dim=1)
    if bf16:
        x = _bf16(x)
    for li, (W, b) in enumerate(layers):
        Wq = _bf16(W) if bf16 else W
        y = x @ Wq + b
        if li < 4:
            y = torch.relu(y)
            if bf16:
                y = _bf16(y)
        x = y
    return x


def mixture(y):
    """(mu [n,8,3], kappa [n,8], weight [n,8]) from raw outputs y [n, 40]."""
    l = y.reshape(-1, N_LOBES, 5)
    v = l[..., 0:3]
    nv = torch.sqrt((v * v).sum(-1, keepdim=True))
    mu = torch.where(nv > 0, v / torch.where(nv > 0, nv, torch.ones_like(nv)),
                     torch.tensor([0.0, 0.0, 1.0], dtype=_DT))
    kappa = torch.clamp(torch.nn.functional.softplus(l[..., 3]) + 0.01, max=1e4)
    weight = torch.softmax(l[..., 4], dim=-1)
    return mu, kappa, weight


def mixture_flat(y):
    """Per lobe (mu xyz, kappa, weight), [n, 40], the library's layout."""
    mu, kappa, weight = mixture(y)
    return torch.cat([mu, kappa[..., None], weight[..., None]], dim=-1).reshape(-1, N_OUT)


def log_vmf(kappa, c):
    """log of the vMF density at cosine c."""
    return torch.log(kappa) - np.log(2 * np.pi) - torch.log(-torch.expm1(-2 * kappa)) + kappa * (c - 1)


def log_q(mu, kappa, weight, w):
    """log of the mixture density at unit directions w [n, 3]."""
    c = (mu * w[:, None, :]).sum(-1)
    q = (weight * torch.exp(log_vmf(kappa, c))).sum(-1)
    return torch.log(torch.clamp(q, min=1e-30))


def records_split(rec):
    """feat [n,9], seg [n], weight [n], direction [n,3] of records [n,16]."""
    r = np.ascontiguousarray(rec, np.float32)
    feat = np.concatenate([r[:, 0:3], r[:, 4:7], r[:, 8:11]], axis=1).astype(np.float64)
    seg = r[:, 3].view(np.int32).astype(np.int64)
    return feat, seg, r[:, 7].astype(np.float64), r[:, 12:15].astype(np.float64)


def loss(params, rec, bf16=False):
    """-sum_i w_i log q(w_i) / sum_i w_i over records rec [n, 16]; params a float64 tensor."""
    feat, seg, wt, d = records_split(rec)
    y = network(params, feat, seg, bf16=bf16)
    mu, kappa, weight = mixture(y)
    lq = log_q(mu, kappa, weight, torch.as_tensor(d))
    w = torch.as_tensor(wt)
    return -(w * lq).sum() / w.sum()


def loss_grad(params, rec, bf16=False):
    """(loss, gradient [N_NET + 16 S]) by reverse-mode differentiation."""
    p = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    L = loss(p, rec, bf16=bf16)
    L.backward()
    return float(L.detach()), p.grad.numpy().copy()


def loss_grad_mfma(params, rec, round_bf16=True, want_abs=False):
    """(loss, gradient) with the backward pass of the bfloat16 matrix-core
    path: the forward pass as network(bf16=True); the gradient with respect
    to the raw outputs, in float64, is rounded to bfloat16, and so is every
    layer's upstream gradient after the ReLU mask of the layer below;
    weights enter the products rounded to bfloat16 (as in the forward
    pass); products are summed exactly; the embedding gradient (the input
    gradient of the first layer) is not rounded.  With round_bf16=False no
    rounding happens anywhere and the result is the exact gradient of
    loss(bf16=False), which pins the bookkeeping of this manual backward
    against autograd.  want_abs also returns, per parameter, the sum over
    records of the absolute values of the products that make up its
    gradient (how much the gradient is a cancellation)."""
    q = (lambda t: _bf16(t, straight_through=False)) if round_bf16 else (lambda t: t)
    feat, seg, wt, d = records_split(rec)
    p = torch.as_tensor(np.asarray(params, np.float64))
    layers, emb = unpack(p)
    f = torch.as_tensor(feat).to(torch.float32).to(_DT)
    segt = torch.as_tensor(seg)
    x = q(torch.cat([f, emb[segt]], dim=1))
    acts = [x]
    for li, (W, b) in enumerate(layers):
        y = x @ q(W) + b
        if li < 4:
            y = q(torch.relu(y))
            acts.append(y)
        x = y
    Y = x.detach().clone().requires_grad_(True)
    mu, kappa, weight = mixture(Y)
    w = torch.as_tensor(wt)
    L = -(w * log_q(mu, kappa, weight, torch.as_tensor(d))).sum() / w.sum()
    L.backward()
    dz = q(Y.grad)
    gW, gb, aW, ab = [None] * 5, [None] * 5, [None] * 5, [None] * 5
    gemb = torch.zeros_like(emb)
    aemb = torch.zeros_like(emb)
    for l in range(4, -1, -1):
        W, _ = layers[l]
        gb[l] = dz.sum(0)
        gW[l] = acts[l].T @ dz
        ab[l] = dz.abs().sum(0)
        aW[l] = acts[l].abs().T @ dz.abs()
        din = dz @ q(W).T
        if l > 0:
            dz = q(din * (acts[l] > 0).to(_DT))
        else:
            gemb.index_add_(0, segt, din[:, 9:9 + N_EMB])
            aemb.index_add_(0, segt, (dz.abs() @ q(W).abs().T)[:, 9:9 + N_EMB])
    parts, aparts = [], []
    for l in range(5):
        parts += [gW[l].reshape(-1), gb[l]]
        aparts += [aW[l].reshape(-1), ab[l]]
    parts.append(gemb.reshape(-1))
    aparts.append(aemb.reshape(-1))
    if want_abs:
        return float(L.detach()), torch.cat(parts).numpy(), torch.cat(aparts).numpy()
    return float(L.detach()), torch.cat(parts).numpy()

