"""The texture decoder MLP in FP64 (oracle).

Paper, Results (implementation): the MLP has hidden layers without bias
terms and ReLU activations. The RGB workloads have a 3-channel head that a
sigmoid maps into (0, 1); the spherical-harmonics appearance (Representation,
Appearance) has a 48-value linear head decoded by oracle.sh. Weights are [out, in] matrices and are
converted exactly from their storage dtype to float64.
"""
from __future__ import annotations

import numpy as np
import torch


def unpack_masks(words, hidden, n_hidden_layers):
    """[S, n_hidden_layers*hidden/32] uint32 bit words -> list of [S, hidden] float64 0/1 masks."""
    words = np.asarray(words).astype(np.uint32).reshape(words.shape[0], n_hidden_layers, hidden // 32)
    bits = (words[:, :, :, None] >> np.arange(32, dtype=np.uint32)[None, None, None, :]) & 1
    bits = bits.reshape(words.shape[0], n_hidden_layers, hidden)
    return [torch.from_numpy(bits[:, i].astype(np.float64)) for i in range(n_hidden_layers)]


def mlp_forward(z, weights, relu_masks=None, head="sigmoid"):
    """sigmoid(W_n ... ReLU(W_1 z)), no biases (head="linear": no sigmoid, for the
    spherical-harmonics head, whose coefficients are decoded by the caller).

    relu_masks (optional, per hidden layer [S, hidden] 0/1) replaces the ReLU
    decision h > 0 by a given one: the layer output is pre * mask. At a
    decision that differs from the natural one the pre-activation is within
    rounding of 0, so the value changes by a rounding-sized amount while the
    gradient follows the given branch."""
    h = z
    last = len(weights) - 1
    for i, w in enumerate(weights):
        h = h @ w.t()
        if i == last:
            h = torch.sigmoid(h) if head == "sigmoid" else h
        elif relu_masks is None:
            h = torch.relu(h)
        else:
            h = h * relu_masks[i]
    return h


def hidden_preactivations(z, weights):
    """Pre-activations W_i h_{i-1} of every hidden layer of the natural network
    (h_0 = z, h_i = ReLU of the i-th pre-activation), as float64 arrays.
    The sign of each is the ReLU decision the exact network takes."""
    h = torch.as_tensor(np.asarray(z), dtype=torch.float64)
    pre = []
    for w in weights[:-1]:
        p = h @ torch.as_tensor(w, dtype=torch.float64).t()
        pre.append(p.numpy())
        h = torch.relu(p)
    return pre
