"""The texture decoder MLP in FP64 (oracle).

Paper, Results (implementation): the MLP has hidden layers without bias
terms and ReLU activations. The workloads used here have a 3-channel RGB
head; a sigmoid maps it into (0, 1). Weights are [out, in] matrices and are
converted exactly from their storage dtype to float64.
"""
from __future__ import annotations

import torch


def mlp_forward(z, weights):
    h = z
    last = len(weights) - 1
    for i, w in enumerate(weights):
        h = h @ w.t()
        h = torch.sigmoid(h) if i == last else torch.relu(h)
    return h
