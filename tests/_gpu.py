"""Helpers shared by the GPU tests: seeded chains on the device, error
measures, and a flushed progress line before every GPU step."""
import sys

import numpy as np
import torch

from paper_2003_05286_amd import binding as sdq

DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def relF(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_cache = {}


def dev_tensor(a):
    key = id(a)
    if key not in _cache:
        _cache[key] = (a, torch.from_numpy(np.ascontiguousarray(a)).to(DEV))
    return _cache[key][1]


def chains_of(instances):
    return [sdq.Chain(dev_tensor(i.expk), torch.from_numpy(np.ascontiguousarray(i.field)).to(DEV),
                      i.alpha, i.k, dev_tensor(i.expk_inv)) for i in instances]
