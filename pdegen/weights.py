"""Seeded random parameters for the encoder-processor-decoder GNN.

Shapes follow the architecture of the paper's technical-details appendix
with every MLP made of two Linear layers (ReLU between them), latent and
hidden width h, and n_mp message-passing layers with separate weights:

  node_enc : Lin(1, h)  - ReLU - Lin(h, h)
  edge_enc : Lin(1, h)  - ReLU - Lin(h, h)
  mp{t}.node : Lin(2h, h) - ReLU - Lin(h, h)      input [v_i, m_i]
  mp{t}.edge : Lin(3h, h) - ReLU - Lin(h, h)      input [e_ij, v_i, v_j]
  dec      : Lin(h, h)  - ReLU - Lin(h, 1)
  xdec     : Lin(h, h)  - ReLU - Lin(h, 1)       (optional x_hat_0 head on the
                                                 final node latents)

A Linear layer maps x -> x W + b with W stored [fan_in, fan_out] row-major.
"""
from __future__ import annotations

import numpy as np


def gnn_param_shapes(h: int, n_mp: int, x_head: bool = False) -> list[tuple[str, tuple[int, ...]]]:
    out: list[tuple[str, tuple[int, ...]]] = []

    def mlp(prefix, fin, fout):
        out.extend([(f"{prefix}.W0", (fin, h)), (f"{prefix}.b0", (h,)),
                    (f"{prefix}.W1", (h, fout)), (f"{prefix}.b1", (fout,))])

    mlp("node_enc", 1, h)
    mlp("edge_enc", 1, h)
    for t in range(n_mp):
        mlp(f"mp{t}.node", 2 * h, h)
        mlp(f"mp{t}.edge", 3 * h, h)
    mlp("dec", h, 1)
    if x_head:
        mlp("xdec", h, 1)
    return out


def init_gnn_params(h: int, n_mp: int, seed: int, gain: float = 1.0,
                    zero: bool = False, x_head: bool = False) -> dict[str, np.ndarray]:
    """Uniform(-gain/sqrt(fan_in), gain/sqrt(fan_in)) for weights and biases
    (float64).  zero=True gives all-zero weights and seeded biases."""
    rng = np.random.default_rng(seed)
    params = {}
    shapes = gnn_param_shapes(h, n_mp, x_head)
    for name, shape in shapes:
        fan_in = shape[0] if len(shape) == 2 else None
        if name.endswith(("W0", "W1")):
            bound = gain / np.sqrt(shape[0])
            params[name] = np.zeros(shape) if zero else rng.uniform(-bound, bound, shape)
        else:
            # bias: fan-in of the matching weight
            wname = name[:-2] + "W" + name[-1]
            fin = dict(shapes)[wname][0]
            bound = gain / np.sqrt(fin)
            params[name] = rng.uniform(-bound, bound, shape)
        del fan_in
    return params
