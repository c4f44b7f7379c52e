"""FP64 CPU reference of the warm-start network (test infrastructure only).

The encoder-decoder is not part of the paper; it predicts the scattered field
``u - u_in`` of the Lippmann-Schwinger solve (eq. u_and_v) from
``(f, Re u_in, Im u_in)`` to start the solver closer to the answer.  This
module evaluates the same architecture, from the same flat parameter vector,
with plain PyTorch CPU float64 operations (``conv2d``, average pooling,
nearest upsampling, concatenation) and obtains gradients by autograd.

Parameter layout (shared with the GPU library): for each convolution in the
order enc1a, enc1b, enc2a, enc2b, enc3a, enc3b, bott_a, bott_b, dec3a, dec3b,
dec2a, dec2b, dec1a, dec1b, head: weights ``[3][3][Cout][Cin]`` then bias
``[Cout]``.  The first layer has ``Cin = 32`` (inputs in channels 0..2) and the
head ``Cout = 32`` (outputs in channels 0..1).

Pinned by: the 3x3 convolution against ``scipy.signal.correlate``; pooling and
upsampling against their definitions; the autograd gradient of the loss
against central finite differences.
"""

from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F


def layer_specs(base=32):
    c1, c2, c3, c4 = base, 2 * base, 4 * base, 8 * base
    return [(32, c1, True), (c1, c1, True), (c1, c2, True), (c2, c2, True), (c2, c3, True), (c3, c3, True),
            (c3, c4, True), (c4, c4, True), (c3 + c4, c3, True), (c3, c3, True), (c2 + c3, c2, True),
            (c2, c2, True), (c1 + c2, c1, True), (c1, c1, True), (c1, 32, False)]


def num_params(base=32):
    return sum(9 * ci * co + co for ci, co, _ in layer_specs(base))


def unpack(params, base=32):
    """Flat vector -> list of (weight [Cout, Cin, 3, 3], bias [Cout]) float64 tensors."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64))
    out, off = [], 0
    for ci, co, _ in layer_specs(base):
        w = p[off:off + 9 * ci * co].reshape(3, 3, co, ci).permute(2, 3, 0, 1).contiguous()
        off += 9 * ci * co
        b = p[off:off + co]
        off += co
        out.append((w, b))
    return out


def conv3x3(x, w, b=None):
    """Cross-correlation with a 3x3 kernel, zero padding 1, NCHW float64."""
    return F.conv2d(x, w, b, padding=1)


def forward(layers, x):
    """x: [B, 32, H, W] float64 input channels; returns the head output [B, 32, H, W]."""
    specs = [s[2] for s in layer_specs(layers[0][0].shape[0])]

    def c(i, t):
        y = conv3x3(t, *layers[i])
        return torch.relu(y) if specs[i] else y

    e1 = c(1, c(0, x))
    e2 = c(3, c(2, F.avg_pool2d(e1, 2)))
    e3 = c(5, c(4, F.avg_pool2d(e2, 2)))
    bt = c(7, c(6, F.avg_pool2d(e3, 2)))
    d3 = c(9, c(8, torch.cat([e3, F.interpolate(bt, scale_factor=2, mode="nearest")], 1)))
    d2 = c(11, c(10, torch.cat([e2, F.interpolate(d3, scale_factor=2, mode="nearest")], 1)))
    d1 = c(13, c(12, torch.cat([e1, F.interpolate(d2, scale_factor=2, mode="nearest")], 1)))
    return c(14, d1)


def make_input(f, u_in, H, W, u_born=None):
    """f: [B, H*W] real; u_in, u_born: [B, H*W] complex -> [B, 32, H, W] float64
    (channels f, Re u_in, Im u_in, Re u_born, Im u_born, zeros)."""
    f = np.asarray(f, dtype=np.float64).reshape(-1, H, W)
    u_in = np.asarray(u_in).reshape(-1, H, W)
    x = np.zeros((f.shape[0], 32, H, W))
    x[:, 0], x[:, 1], x[:, 2] = f, u_in.real, u_in.imag
    if u_born is not None:
        ub = np.asarray(u_born).reshape(-1, H, W)
        x[:, 3], x[:, 4] = ub.real, ub.imag
    return torch.as_tensor(x)


def predict(params, f, u_in, H, W, base=32, u_born=None):
    """u0 = u_in + net(f, u_in, u_born) as a complex numpy array [B, H*W]."""
    with torch.no_grad():
        out = forward(unpack(params, base), make_input(f, u_in, H, W, u_born)).numpy()
    return np.asarray(u_in).reshape(out.shape[0], -1) + (out[:, 0] + 1j * out[:, 1]).reshape(out.shape[0], -1)


def loss_and_grad(params, f, u_in, u, H, W, base=32, u_born=None):
    """Relative-L2 loss (1/B) sum_b ||net_b - (u_b - u_in,b)||^2 / ||u_b - u_in,b||^2 and
    its gradient with respect to the flat parameter vector (autograd, float64)."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    layers, off = [], 0
    for ci, co, _ in layer_specs(base):
        w = p[off:off + 9 * ci * co].reshape(3, 3, co, ci).permute(2, 3, 0, 1)
        off += 9 * ci * co
        layers.append((w, p[off:off + co]))
        off += co
    out = forward(layers, make_input(f, u_in, H, W, u_born))
    B = out.shape[0]
    t = (np.asarray(u) - np.asarray(u_in)).reshape(B, H, W)
    tr, ti = torch.as_tensor(t.real), torch.as_tensor(t.imag)
    e2 = ((out[:, 0] - tr) ** 2 + (out[:, 1] - ti) ** 2).sum((1, 2))
    t2 = (tr ** 2 + ti ** 2).sum((1, 2))
    loss = (e2 / t2).mean()
    loss.backward()
    return float(loss.detach()), p.grad.numpy()
