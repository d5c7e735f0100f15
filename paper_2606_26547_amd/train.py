"""Model training on the device: majority bundling and retraining epochs.

``fit`` builds the class hypervectors from encoded training rows and then
runs ``epochs`` retraining epochs (the apps' TRAIN_ITERATIONS, Sec. 5): each
epoch predicts every training row with the current model (prepared
matrix-core Hamming search over all dimensions) and applies the
mispredicted-row update of ``hdc_retrain_epoch``.  All device work; the host
only sequences the calls.
"""
from __future__ import annotations

import torch

from . import hdc


def fit(H: torch.Tensor, nbits: int, labels: torch.Tensor, K: int, epochs: int = 0):
    """Returns (C, acc, wrong) with wrong[e] the training rows the model at
    the start of epoch e mispredicts (a device tensor per epoch)."""
    ws = hdc.retrain_workspace(H.shape[0], nbits, K, H.device)
    acc, Cw = hdc.class_acc(H, nbits, labels, K, ws)
    pred = torch.empty(H.shape[0], dtype=torch.int32, device=H.device)
    wrong = []
    for _ in range(epochs):
        hdc.HammingPrepared(Cw, 0, nbits, 1)(H, out=pred)
        w = torch.zeros(1, dtype=torch.int32, device=H.device)
        hdc.retrain_epoch(H, nbits, labels, pred, acc, Cw, w, ws)
        wrong.append(w)
    return Cw, acc, wrong
