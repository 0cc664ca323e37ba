"""Helpers shared by the GPU parity tests (not collected: no test_ prefix)."""
import numpy as np
import torch


def u32_to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def dev_to_u32(t):
    return t.cpu().numpy().view(np.uint32)


def f32_to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def say(msg):
    print(msg, flush=True)
