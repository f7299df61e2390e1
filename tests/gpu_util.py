"""Helpers shared by the GPU tests: move a synthetic problem to the device."""
import numpy as np
import torch

import paper_1602_02070_amd as cp


def dev_problem(P, dtype=torch.float64):
    d = dict(
        Lr=cp.Graph.from_scipy(P.Lr), Lc=cp.Graph.from_scipy(P.Lc),
        Lr_til=cp.Graph.from_scipy(P.Lr_til), Lc_til=cp.Graph.from_scipy(P.Lc_til),
        om_r=torch.from_numpy(P.omega_r).cuda(), om_c=torch.from_numpy(P.omega_c).cuda(),
        Ytil=torch.from_numpy(P.Ytil).to(dtype).cuda(),
    )
    return d


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def host(t):
    return t.detach().double().cpu().numpy()


_VIDEO = {}


def video_problem():
    """The video-shaped workload (20480 x 4096, full data kept), generated once
    per test session and shared by the modules that need it."""
    if "P" not in _VIDEO:
        import synth
        _VIDEO["P"] = synth.cfg3_video(0, keep_full=True)
    return _VIDEO["P"]
