"""Trained parameters of the learned initial guess (include/fldnn.h).

The committed file was written by train_guess.py; its JSON sidecar records
the recipe (media, epochs, optimizer), the loss history and the held-out
evaluation.
"""
from __future__ import annotations

import json
import os

import numpy as np

from .train_guess import DEFAULT_WEIGHTS


def load_weights(path=DEFAULT_WEIGHTS):
    """FP32 parameter array (fldnn.h layer order); raises if missing."""
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: train it with "
            "`python -m paper_2503_02764_amd.train_guess`")
    w = np.fromfile(path, dtype="<f4")
    from . import fld
    if w.size != fld.fldnn_param_count():
        raise ValueError(f"{path}: {w.size} parameters, the network has "
                         f"{fld.fldnn_param_count()}")
    return w


def load_record(path=DEFAULT_WEIGHTS):
    with open(os.path.splitext(path)[0] + ".json") as f:
        return json.load(f)
