"""Float64 reference for the cut-set cost model (test infrastructure).

A plain multilayer perceptron: input -> 256 -> 256 -> 256 -> outputs, ReLU after
each hidden layer, mean-squared-error loss over batch and outputs, Adam
(Kingma and Ba, 2015) updates.  Weights are stored [fan_in, fan_out] row-major.
The cost model is not part of the paper; it only ranks candidate cut sets, and
the exact evaluator re-scores every set that is chosen.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


class MLP64:
    def __init__(self, weights: List[np.ndarray], biases: List[np.ndarray]):
        self.W = [np.asarray(w, dtype=np.float64).copy() for w in weights]
        self.b = [np.asarray(b, dtype=np.float64).copy() for b in biases]
        self.m = [np.zeros_like(w) for w in self.W] + [np.zeros_like(b) for b in self.b]
        self.v = [np.zeros_like(w) for w in self.W] + [np.zeros_like(b) for b in self.b]
        self.t = 0

    def forward(self, x: np.ndarray) -> Tuple[np.ndarray, list]:
        acts = [np.asarray(x, dtype=np.float64)]
        h = acts[0]
        L = len(self.W)
        for i in range(L):
            z = h @ self.W[i] + self.b[i]
            h = np.maximum(z, 0.0) if i < L - 1 else z
            acts.append(h)
        return h, acts

    def loss_and_grads(self, x: np.ndarray, y: np.ndarray):
        out, acts = self.forward(x)
        diff = out - y
        loss = float(np.mean(diff * diff))
        g = 2.0 * diff / diff.size            # d loss / d out
        gW = [None] * len(self.W)
        gb = [None] * len(self.W)
        for i in reversed(range(len(self.W))):
            if i < len(self.W) - 1:
                g = g * (acts[i + 1] > 0.0)    # ReLU derivative
            gW[i] = acts[i].T @ g
            gb[i] = g.sum(axis=0)
            g = g @ self.W[i].T
        return loss, gW, gb

    def adam_step(self, gW, gb, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        params = self.W + self.b
        grads = list(gW) + list(gb)
        for k, (p, g) in enumerate(zip(params, grads)):
            self.m[k] = b1 * self.m[k] + (1 - b1) * g
            self.v[k] = b2 * self.v[k] + (1 - b2) * g * g
            mh = self.m[k] / (1 - b1 ** self.t)
            vh = self.v[k] / (1 - b2 ** self.t)
            p -= lr * mh / (np.sqrt(vh) + eps)
