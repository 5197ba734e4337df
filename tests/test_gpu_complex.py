"""Complex UDT (sdq_udt_complex): U, D and T against the oracle's complex
pivoted QR on the same seeded matrices, n = 1 .. 64, ragged batches, extreme
scales, real input, a zero column, a batch larger than the grid; the limits."""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl
from _gpu import DEV, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sdq.Context(0)


def relf(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def cmats(count, n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * (rng.normal(size=(count, n, n)) + 1j * rng.normal(size=(count, n, n)))


def check(ctx, W, sample=None):
    Wd = torch.from_numpy(np.ascontiguousarray(W)).to(DEV)
    u, d, t = ctx.udt_complex(Wd)
    torch.cuda.synchronize()
    u, d, t = u.cpu().numpy(), d.cpu().numpy(), t.cpu().numpy()
    worst = 0.0
    for b in (range(W.shape[0]) if sample is None else sample):
        Uo, Do, To = oracle.udt_complex(W[b])
        e = max(relf(u[b], Uo), relf(d[b], Do), relf(t[b], To))
        worst = max(worst, e)
    return worst


@pytest.mark.parametrize("n,count", [(1, 3), (2, 3), (7, 5), (16, 3), (33, 4), (64, 3)])
def test_complex_udt_matches_oracle(ctx, n, count):
    W = cmats(count, n, wl.BASE_SEED + 1800 + n)
    say(f"[gpu] sdq_udt_complex n={n} count={count}")
    e = check(ctx, W)
    say(f"[gpu]   worst relF {e:.2e}")
    assert e <= 1e-10


@pytest.mark.parametrize("scale", [1e-150, 1e150])
def test_complex_udt_extreme_scales(ctx, scale):
    W = cmats(2, 24, wl.BASE_SEED + 1850, scale)
    say(f"[gpu] sdq_udt_complex n=24 scale={scale:g}")
    assert check(ctx, W) <= 1e-10


def test_complex_udt_real_input_and_zero_column(ctx):
    rng = np.random.default_rng(wl.BASE_SEED + 1860)
    W = np.stack([rng.normal(size=(20, 20)) + 0j, cmats(1, 20, wl.BASE_SEED + 1861)[0]])
    W[1][:, 5] = 0.0
    say("[gpu] sdq_udt_complex n=20: real matrix, matrix with a zero column")
    assert check(ctx, W) <= 1e-10
    Wd = torch.from_numpy(W).to(DEV)
    _, d, _ = ctx.udt_complex(Wd)
    assert d[1, -1].item() == 0.0


def test_complex_udt_batch_beyond_the_grid(ctx):
    # more matrices than resident workgroups: the grid-stride loop
    W = cmats(1100, 64, wl.BASE_SEED + 1870)
    say("[gpu] sdq_udt_complex n=64 count=1100 (sampled)")
    assert check(ctx, W, sample=[0, 1, 511, 512, 513, 1023, 1099]) <= 1e-10


def test_complex_udt_limits(ctx):
    say("[gpu] sdq_udt_complex at n = 65 -> SDQ_EUNSUPPORTED; count = 0 -> OK")
    with pytest.raises(sdq.SdqError) as e:
        ctx.udt_complex(torch.zeros(1, 65, 65, dtype=torch.complex128, device=DEV))
    assert e.value.status == sdq.SDQ_EUNSUPPORTED
    u, d, t = ctx.udt_complex(torch.zeros(0, 8, 8, dtype=torch.complex128, device=DEV))
    assert u.shape == (0, 8, 8)
