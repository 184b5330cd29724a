"""Seeded MLP parameters for the neural SDF and colour networks.

Flat FP32 layout shared by every consumer: for each linear layer in order,
the weight matrix ``W [out][in]`` row-major followed by the bias ``b [out]``.

SDF network (IDR/NeuS-style geometric initialisation, so that the untrained
network is close to the SDF of a sphere of radius ``sphere_r`` in normalised
coordinates):
  * hidden layers: ``W ~ N(0, sqrt(2)/sqrt(out))``, ``b = 0``;
  * layer 0 with positional encoding: columns of the sin/cos features are 0;
  * the skip layer: columns that receive the re-injected encoding are 0;
  * output layer: ``W ~ N(sqrt(pi)/sqrt(in), 1e-4)``, ``b = -sphere_r``
    (both negated for an inside-out sphere, as used for indoor scenes).
Colour network: ``W, b ~ U(-1/sqrt(in), 1/sqrt(in))``.
"""
from __future__ import annotations

from dataclasses import dataclass
import numpy as np


@dataclass(frozen=True)
class SdfNet:
    width: int = 256          # hidden width
    n_hidden: int = 8         # hidden (softplus) layers
    pe_freqs: int = 6         # 0 = raw xyz input
    skip_at: int = 4          # layer whose input re-injects the encoding; -1 = none
    n_feat: int = 256         # feature outputs besides f
    beta: float = 100.0       # softplus sharpness
    sphere_r: float = 0.5
    inside_out: bool = False  # SDF ~ r - |x_hat| (the scene surrounds the sphere's centre)

    @property
    def d_in(self):
        return 3 + 6 * self.pe_freqs

    def layer_dims(self):
        """[(in, out)] of every linear layer, output layer last."""
        dims = []
        for l in range(self.n_hidden):
            d_in = self.d_in if l == 0 else self.width
            d_out = self.width - self.d_in if (l + 1) == self.skip_at else self.width
            dims.append((d_in, d_out))
        dims.append((self.width, 1 + self.n_feat))
        return dims

    def n_params(self):
        return sum(i * o + o for i, o in self.layer_dims())


@dataclass(frozen=True)
class ColorNet:
    width: int = 256
    n_hidden: int = 4
    n_feat: int = 256

    @property
    def d_in(self):
        return 9 + self.n_feat   # [p_hat(3), v(3), grad f(3), feat]

    def layer_dims(self):
        dims = []
        for l in range(self.n_hidden):
            dims.append((self.d_in if l == 0 else self.width, self.width))
        dims.append((self.width, 3))
        return dims

    def n_params(self):
        return sum(i * o + o for i, o in self.layer_dims())


def sdf_params(net: SdfNet, seed: int = 42) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    chunks = []
    dims = net.layer_dims()
    for l, (d_in, d_out) in enumerate(dims):
        last = l == len(dims) - 1
        if last:
            W = rng.normal(np.sqrt(np.pi) / np.sqrt(d_in), 1e-4, size=(d_out, d_in))
            b = np.full(d_out, -net.sphere_r)
            if net.inside_out:
                W, b = -W, -b
        else:
            W = rng.normal(0.0, np.sqrt(2.0) / np.sqrt(d_out), size=(d_out, d_in))
            b = np.zeros(d_out)
            if l == 0 and net.pe_freqs > 0:
                W[:, 3:] = 0.0
            if l == net.skip_at:
                W[:, -(net.d_in - 3):] = 0.0
        chunks += [W.ravel(), b]
    return np.concatenate(chunks).astype(np.float32)


def color_params(net: ColorNet, seed: int = 43) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    chunks = []
    for d_in, d_out in net.layer_dims():
        bound = 1.0 / np.sqrt(d_in)
        chunks += [rng.uniform(-bound, bound, size=(d_out, d_in)).ravel(),
                   rng.uniform(-bound, bound, size=d_out)]
    return np.concatenate(chunks).astype(np.float32)


def split_layers(params: np.ndarray, dims):
    """Views (W [out,in], b [out]) of a flat parameter vector."""
    out, k = [], 0
    for d_in, d_out in dims:
        W = params[k:k + d_in * d_out].reshape(d_out, d_in)
        k += d_in * d_out
        b = params[k:k + d_out]
        k += d_out
        out.append((W, b))
    assert k == params.size, (k, params.size)
    return out
