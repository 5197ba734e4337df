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


def test_complex_udt_rejects_a_non_square_batch(ctx):
    say("[gpu] sdq_udt_complex binding: [count, n, m] with m != n -> ValueError")
    for shape in ((2, 8, 4), (2, 4, 8), (8, 8)):
        with pytest.raises(ValueError):
            ctx.udt_complex(torch.zeros(*shape, dtype=torch.complex128, device=DEV))


def test_complex_udt_graded_benchmark_batch(ctx):
    # the benchmark's inputs: columns graded over 30 decades, random order
    W = wl.complex_batch(96, 64)
    say("[gpu] sdq_udt_complex on the graded benchmark batch, n=64 count=96 (sampled)")
    assert check(ctx, W, sample=range(0, 96, 5)) <= 1e-10
    W = wl.complex_batch(40, 37, seed=wl.BASE_SEED + 1880)
    say("[gpu] sdq_udt_complex on a graded batch, n=37 count=40")
    assert check(ctx, W) <= 1e-10


def _near_dependent(count, n, rank, noise, seed):
    rng = np.random.default_rng(seed)

    def g(*s):
        return rng.normal(size=s) + 1j * rng.normal(size=s)
    out = []
    for _ in range(count):
        A = g(n, rank) @ g(rank, n)
        for j in range(rank, n, 5):
            A[:, j] = A[:, (j * 7) % rank] * (1.0 + 1e-9 * rng.normal())
        out.append(A + noise * g(n, n))
    return np.stack(out)


@pytest.mark.parametrize("n,rank,noise", [(32, 4, 1e-7), (64, 6, 1e-11)])
def test_complex_udt_near_dependent_columns(ctx, n, rank, noise):
    """Nearly dependent columns drive downdated norms below the
    Drmac-Bujanovic guard, so the exact norm recompute runs.  Unique parts:
    the leading `rank` rows of T and columns of U (well-determined) against
    the oracle; D against the oracle to the accuracy the noise level leaves;
    reconstruction and unitarity of the GPU's own factors."""
    import scipy.linalg as sl
    W = _near_dependent(3, n, rank, noise, wl.BASE_SEED + 1890 + n)
    Wd = torch.from_numpy(np.ascontiguousarray(W)).to(DEV)
    say(f"[gpu] sdq_udt_complex near-dependent columns n={n} rank={rank} noise={noise:g}")
    u, d, t = ctx.udt_complex(Wd)
    torch.cuda.synchronize()
    u, d, t = u.cpu().numpy(), d.cpu().numpy(), t.cpu().numpy()
    for b in range(W.shape[0]):
        Uo, Do, To = oracle.udt_complex(W[b])
        nW = np.linalg.norm(W[b])
        assert np.all(np.abs(d[b] - Do) <= 1e-6 * Do + 1e-13 * nW), b
        dl = np.abs(np.diag(sl.qr(W[b], pivoting=True)[1]))
        assert np.all(np.abs(d[b] - dl) <= 1e-6 * dl + 1e-13 * nW), b
        assert relf(u[b][:, :rank], Uo[:, :rank]) <= 1e-10
        assert relf(t[b][:rank], To[:rank]) <= 1e-10
        assert np.linalg.norm(u[b] @ (d[b][:, None] * t[b]) - W[b]) <= 1e-13 * n * nW
        assert np.linalg.norm(u[b].conj().T @ u[b] - np.eye(n)) <= 1e-13 * n
