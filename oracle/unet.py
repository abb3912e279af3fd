"""FP64 CPU reference of the warm-start network (plain PyTorch CPU ops).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` use this module; the product path never imports it,
and it shares no code with the GPU kernels.

The network is not part of the paper (the paper's method is the explicit
phase-field integration); it seeds that integration.  What is computed here
is the plain definition of each layer:

* input channels: glass indicator, log10(dT / 0.2 K), (log10 s - 1.5) / 1.5,
  and five zero channels;
* 3x3x3 convolution, stride 1, zero padding, weights [cout][27][cin] with tap
  index (dz+1)*9 + (dy+1)*3 + (dx+1), followed by ReLU;
* 2x average pooling, nearest 2x upsampling, concatenation [upsampled, skip];
* 1x1 head + sigmoid, zero on glass cells;
* loss: mean over water cells of the squared error; gradients by reverse-mode
  differentiation (torch.autograd) in FP64;
* Adam (Kingma and Ba 2015) with bias correction.

``round_bf16`` rounds to the nearest BF16 value (ties to even), so the same
network can also be evaluated with BF16 storage of weights and activations,
as the matrix-core path stores them.
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np
import torch
import torch.nn.functional as F

# (cin, cout) of the ten convolutions: enc1a, enc1b, enc2a, enc2b, enc3a,
# enc3b, dec2a, dec2b, dec1a, dec1b
LAYERS: List[Tuple[int, int]] = [(8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64),
                                 (96, 32), (32, 32), (48, 16), (16, 16)]


def layout() -> Tuple[List[Tuple[int, int]], int, int, int]:
    """Offsets (weight, bias) of each convolution in the flat vector, the head
    weight and bias offsets and the total length."""
    offs = []
    o = 0
    for cin, cout in LAYERS:
        offs.append((o, o + 27 * cin * cout))
        o += 27 * cin * cout + cout
    return offs, o, o + 16, o + 17


def num_params() -> int:
    return layout()[3]


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 value of each element (round to nearest, ties to even),
    returned as float64.  Inputs must be finite."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (int16) of round_bf16(x)."""
    r = round_bf16(x).astype(np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def from_bf16_bits(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(
        np.float64)


def features(mask: np.ndarray, dT: float, log10_s: float) -> np.ndarray:
    """Network input (8, n3, n2, n1) for a mask (n3, n2, n1), nonzero = glass."""
    m = (np.asarray(mask) != 0).astype(np.float64)
    x = np.zeros((8,) + m.shape)
    x[0] = m
    x[1] = np.log10(dT / 0.2)
    x[2] = (log10_s - 1.5) / 1.5
    return x


def unpack(p) -> Tuple[list, torch.Tensor, torch.Tensor]:
    """[(W (cout, cin, 3, 3, 3), b)] and the head from a flat vector (numpy
    or torch), all float64 torch tensors sharing storage with a torch input."""
    if isinstance(p, np.ndarray):
        p = torch.from_numpy(np.asarray(p, dtype=np.float64))
    offs, hw, hb, _ = layout()
    convs = []
    for (cin, cout), (wo, bo) in zip(LAYERS, offs):
        # [co][tap][ci], tap = kz*9 + ky*3 + kx  ->  (co, ci, kz, ky, kx)
        W = p[wo:wo + 27 * cin * cout].reshape(cout, 3, 3, 3, cin).permute(0, 4, 1, 2, 3)
        convs.append((W, p[bo:bo + cout]))
    return convs, p[hw:hw + 16], p[hb:hb + 1]


def conv3(x: torch.Tensor, W: torch.Tensor, b) -> torch.Tensor:
    """3x3x3 cross-correlation with zero padding; x (cin, n3, n2, n1)."""
    return F.conv3d(x[None], W, b, padding=1)[0]


def pool2(x: torch.Tensor) -> torch.Tensor:
    return F.avg_pool3d(x[None], 2)[0]


def up2(x: torch.Tensor) -> torch.Tensor:
    return x.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2).repeat_interleave(2, dim=3)


def forward(p, mask: np.ndarray, dT: float, log10_s: float, bf16: bool = False,
            return_acts: bool = False):
    """Prediction (n3, n2, n1) as a float64 torch tensor.  bf16=True rounds the
    weights and every stored activation to BF16 like the matrix-core path
    (biases, head and sigmoid stay FP64)."""
    if bf16:
        pn = p.detach().numpy() if isinstance(p, torch.Tensor) else np.asarray(p, np.float64)
        q = pn.copy()
        offs, _, _, _ = layout()
        for (cin, cout), (wo, bo) in zip(LAYERS, offs):
            q[wo:bo] = round_bf16(pn[wo:bo])
        p = q
    convs, hw, hb = unpack(p)
    rnd = (lambda t: torch.from_numpy(round_bf16(t.detach().numpy()))) if bf16 else (lambda t: t)
    x0 = torch.from_numpy(features(mask, dT, log10_s))
    x0 = rnd(x0)

    def cr(i, x):
        W, b = convs[i]
        return rnd(torch.relu(conv3(x, W, b)))

    a1 = cr(0, x0)
    s1 = cr(1, a1)
    p1 = rnd(pool2(s1))
    a2 = cr(2, p1)
    s2 = cr(3, a2)
    p2 = rnd(pool2(s2))
    a3 = cr(4, p2)
    b3 = cr(5, a3)
    c2 = torch.cat([up2(b3), s2], dim=0)
    e2 = cr(6, c2)
    f2 = cr(7, e2)
    c1 = torch.cat([up2(f2), s1], dim=0)
    e1 = cr(8, c1)
    f1 = cr(9, e1)
    z = torch.einsum("c,czyx->zyx", hw, f1) + hb[0]
    water = torch.from_numpy(np.asarray(mask) == 0)
    y = torch.where(water, torch.sigmoid(z), torch.zeros_like(z))
    if return_acts:
        return y, dict(x0=x0, a1=a1, s1=s1, p1=p1, a2=a2, s2=s2, p2=p2, a3=a3, b3=b3, e2=e2,
                       f2=f2, e1=e1, f1=f1)
    return y


def loss_and_grad(p: np.ndarray, mask: np.ndarray, target: np.ndarray, dT: float,
                  log10_s: float) -> Tuple[float, np.ndarray]:
    """Mean squared error over water cells and its gradient (flat, float64)."""
    pt = torch.tensor(np.asarray(p, dtype=np.float64), requires_grad=True)
    y = forward(pt, mask, dT, log10_s)
    water = torch.from_numpy(np.asarray(mask) == 0)
    t = torch.from_numpy(np.asarray(target, dtype=np.float64))
    loss = ((y - t)[water] ** 2).mean()
    loss.backward()
    return float(loss.detach()), pt.grad.numpy().copy()


def loss_value(p: np.ndarray, mask: np.ndarray, target: np.ndarray, dT: float,
               log10_s: float) -> float:
    with torch.no_grad():
        y = forward(np.asarray(p, np.float64), mask, dT, log10_s)
        water = torch.from_numpy(np.asarray(mask) == 0)
        t = torch.from_numpy(np.asarray(target, dtype=np.float64))
        return float(((y - t)[water] ** 2).mean())


def adam(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
         b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (returns new p, m, v); step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def conv3_brute(x: np.ndarray, w: np.ndarray, b) -> np.ndarray:
    """Direct sum of the convolution definition, for tiny inputs:
    x (n3, n2, n1, cin), w (cout, 27, cin) -> (n3, n2, n1, cout)."""
    n3, n2, n1, cin = x.shape
    cout = w.shape[0]
    y = np.zeros((n3, n2, n1, cout))
    for z in range(n3):
        for yy in range(n2):
            for xx in range(n1):
                acc = np.zeros(cout) if b is None else np.array(b, dtype=np.float64)
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            zz, y2, x2 = z + dz, yy + dy, xx + dx
                            if 0 <= zz < n3 and 0 <= y2 < n2 and 0 <= x2 < n1:
                                tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                acc = acc + w[:, tap, :] @ x[zz, y2, x2, :]
                y[z, yy, xx] = acc
    return y


def conv3_cl(x: np.ndarray, w: np.ndarray, b) -> np.ndarray:
    """The convolution on channels-last arrays via the library routine:
    x (n3, n2, n1, cin), w (cout, 27, cin) -> (n3, n2, n1, cout), float64."""
    cout, _, cin = w.shape
    W = torch.from_numpy(np.asarray(w, np.float64)).reshape(cout, 3, 3, 3, cin).permute(
        0, 4, 1, 2, 3)
    X = torch.from_numpy(np.asarray(x, np.float64)).permute(3, 0, 1, 2)
    B = None if b is None else torch.from_numpy(np.asarray(b, np.float64))
    return conv3(X, W, B).permute(1, 2, 3, 0).numpy()


def conv3_cl_grads(x: np.ndarray, w: np.ndarray, dy: np.ndarray) -> Dict[str, np.ndarray]:
    """dx, dw, db of y = conv3(x) + b for an upstream gradient dy, by autograd."""
    X = torch.tensor(np.asarray(x, np.float64), requires_grad=True)
    Wt = torch.tensor(np.asarray(w, np.float64), requires_grad=True)
    cout, _, cin = w.shape
    B = torch.zeros(cout, dtype=torch.float64, requires_grad=True)
    W = Wt.reshape(cout, 3, 3, 3, cin).permute(0, 4, 1, 2, 3)
    Y = conv3(X.permute(3, 0, 1, 2), W, B).permute(1, 2, 3, 0)
    Y.backward(torch.from_numpy(np.asarray(dy, np.float64)))
    return dict(dx=X.grad.numpy(), dw=Wt.grad.numpy(), db=B.grad.numpy())


def nucleus_component(mask: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Water cells (mask == 0) in a face-connected water component that holds
    a water cell with phi > 1/2 (bool array of the mask's shape)."""
    from scipy import ndimage
    water = np.asarray(mask) == 0
    lab, _ = ndimage.label(water, structure=ndimage.generate_binary_structure(3, 1))
    seeds = np.unique(lab[water & (np.asarray(phi) > 0.5)])
    return np.isin(lab, seeds[seeds > 0]) & water
