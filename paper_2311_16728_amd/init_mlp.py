"""Learned initialiser for newly densified primitives (Section 3.3.1 creates
them at inactive keypoints; here a small MLP proposes their shape and
appearance, with the heuristic as fallback).

The network, its training step and its inference all run in the library's
kernels (gs_init_mlp_fwd / gs_init_mlp_bwd / gs_init_mlp_adam on the matrix
cores); this module keeps the FP32 master weights, the BF16 copy and the Adam
moments, and marshals arguments.
"""

from __future__ import annotations

import numpy as np
import torch

from . import gs

N_IN, N_IN_PAD, N_HID, N_OUT = 159, 160, 128, 16
N_W = N_HID * N_IN_PAD + N_HID * N_HID + N_OUT * N_HID
N_B = 2 * N_HID + N_OUT
# output columns: log-scale correction (3), quaternion in the camera frame (4),
# opacity logit (1), SH DC correction (3); corrections are relative to the
# heuristic initialiser
N_TARGET = 11


class InitMLP:
    def __init__(self, seed: int = 0, device="cuda"):
        rng = np.random.default_rng(seed)
        fan = np.concatenate([np.full(N_HID * N_IN_PAD, N_IN), np.full(N_HID * N_HID, N_HID),
                              np.full(N_OUT * N_HID, N_HID)])
        w = rng.normal(size=N_W) * np.sqrt(2.0 / fan)        # He initialisation for ReLU
        w[:N_HID * N_IN_PAD].reshape(N_HID, N_IN_PAD)[:, N_IN:] = 0.0
        # small last layer and biases at the heuristic (zero corrections, identity
        # rotation, opacity 0.1): the untrained network reproduces the heuristic
        w[N_HID * N_IN_PAD + N_HID * N_HID:] *= 0.01
        b = np.zeros(N_B)
        b[2 * N_HID + 3] = 1.0
        b[2 * N_HID + 7] = np.log(0.1 / 0.9)
        self.device = device
        self.w = torch.as_tensor(w, dtype=torch.float32, device=device)
        self.b = torch.as_tensor(b, dtype=torch.float32, device=device)
        self.w_bf16 = torch.empty(N_W, dtype=torch.int16, device=device)
        gs.gs_to_bf16(self.w, self.w_bf16)
        self.dw = torch.zeros(N_W, dtype=torch.float32, device=device)
        self.db = torch.zeros(N_B, dtype=torch.float32, device=device)
        self.m = torch.zeros(N_W + N_B, dtype=torch.float32, device=device)
        self.v = torch.zeros(N_W + N_B, dtype=torch.float32, device=device)
        self.step = 0
        self._ws = {}

    def _buffers(self, B):
        if B not in self._ws:
            self._ws[B] = (torch.empty(B, N_OUT, dtype=torch.float32, device=self.device),
                           torch.empty(2 * B * N_HID, dtype=torch.int16, device=self.device))
        return self._ws[B]

    def pack_inputs(self, x: torch.Tensor) -> torch.Tensor:
        """Float [B][k <= 160] features (device) to the zero-padded BF16 [B][160] layout."""
        B = x.shape[0]
        pad = torch.zeros(B, N_IN_PAD, dtype=torch.float32, device=x.device)
        pad[:, :x.shape[1]] = x
        out = torch.empty(B, N_IN_PAD, dtype=torch.int16, device=x.device)
        gs.gs_to_bf16(pad, out)
        return out

    def forward(self, x_bf16: torch.Tensor) -> torch.Tensor:
        y, act = self._buffers(x_bf16.shape[0])
        gs.gs_init_mlp_fwd(self.w_bf16, self.b, x_bf16, y, act)
        return y

    def train_step(self, x_bf16: torch.Tensor, target: torch.Tensor, lr: float = 1e-3,
                   weight: torch.Tensor | None = None) -> float:
        """One Adam step on the mean squared error of the first target.shape[1]
        outputs (optionally weighted per column); returns the loss before the step."""
        B, k = target.shape
        y = self.forward(x_bf16)
        _, act = self._buffers(B)
        diff = y[:, :k] - target
        if weight is not None:
            diff = diff * weight
        loss = float((diff * diff).mean())
        dy = torch.zeros(B, N_OUT, dtype=torch.float32, device=y.device)
        dy[:, :k] = (2.0 / (B * k)) * (diff if weight is None else diff * weight)
        self.dw.zero_()
        self.db.zero_()
        gs.gs_init_mlp_bwd(self.w_bf16, x_bf16, act, dy, self.dw, self.db)
        self.step += 1
        gs.gs_init_mlp_adam(self.w, self.b, self.w_bf16, self.dw, self.db, self.m, self.v, lr, self.step)
        return loss

    def state_dict(self):
        return {"w": self.w.cpu(), "b": self.b.cpu()}

    def load_state_dict(self, sd):
        self.w.copy_(sd["w"])
        self.b.copy_(sd["b"])
        gs.gs_to_bf16(self.w, self.w_bf16)
