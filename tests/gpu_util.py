"""Helpers shared by the GPU tests (comparison metrics, tensor transfer, problem setup)."""
import numpy as np


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(gpu, ref, c=1.0):
    """Max error of E, F, T scaled like the parity metric: |dE|/max|E|, |dF|/(c max E), |dT|/max|T|."""
    gpu, ref = np.asarray(gpu), np.asarray(ref)
    sE = max(np.abs(ref[0]).max(), 1e-300)
    sT = max(np.abs(ref[3]).max(), 1e-300)
    eE = np.abs(gpu[0] - ref[0]).max() / sE
    eF = np.abs(gpu[1:3] - ref[1:3]).max() / (c * sE)
    eT = np.abs(gpu[3] - ref[3]).max() / sT
    return max(eE, eF, eT)


def field_err(gpu, ref, scale):
    return np.abs(np.asarray(gpu) - np.asarray(ref)).max() / scale


def announce(*args):
    print("[gpu-case]", *args, flush=True)
