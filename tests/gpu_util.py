"""Helpers shared by the GPU tests: move a synthetic instance to the device."""

import numpy as np
import torch

import paper_1703_10973_amd as pk

DEV = torch.device("cuda", 0)


def to_dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def problem_from(ctx, inst):
    con, row, col, val = inst.triplets()
    return pk.Problem(ctx, inst.n, inst.m, to_dev(con, torch.int32), to_dev(row, torch.int32),
                      to_dev(col, torch.int32), to_dev(val))


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))
