"""Helpers shared by the GPU tests: media -> C-ABI parameters and tensors."""
import sys

import numpy as np


def announce(msg):
    """Name the case before a GPU step, flushed, so a crash log shows it."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def params_for(m, **kw):
    from paper_2503_02764_amd.solver import make_params
    args = dict(ndim=m.ndim, n=m.n[: m.ndim], dx=m.dx[: m.ndim], bc=m.bc,
                c=m.c, a_rad=m.a_rad, gamma=m.gamma, gas_const=m.gas_const,
                limiter=m.limiter, face_mean=m.face_mean, rtol=m.rtol)
    args.update(kw)
    return make_params(**args)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))
