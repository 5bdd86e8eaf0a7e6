"""Helpers for the GPU parity tests (marshalling only)."""
import numpy as np


def to_dev(a):
    import torch
    return torch.from_numpy(np.asfortranarray(a)).to(torch.device("cuda", 0))


def to_host(t):
    return t.detach().cpu().numpy()


def projector():
    import paper_1912_02767_amd as psdp
    return psdp.Projector(0)
