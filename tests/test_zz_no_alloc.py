"""sdq_greens_noalloc (the entry point for callers that cannot allocate)
against sdq_greens, called through the C ABI on the same seeded chains: two
calls in a row, the second with a smaller batch, each at the parity bar
(relative Frobenius <= 1e-10 per G, log|det| to 1e-12 relative, equal signs
and statuses); its size and shape limits."""
import numpy as np
import pytest
import torch

from _gpu import DEV, chains_of, relF, say
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sdq.Context(0)


def _batch(seed, spec):
    out = []
    for i, (L, beta, flav) in enumerate(spec):
        out += wl.hubbard_ising(L, beta, 1, flav, seed=seed + i)
    return out


def _compare(ctx, insts, label):
    ch = chains_of(insts)
    cnt = len(ch)
    g_ref, ld_ref, sg_ref, st_ref = ctx.greens(ch)
    gs = [torch.full((c.n, c.n), float("nan"), dtype=torch.float64, device=DEV) for c in ch]
    ld = torch.full((cnt,), float("nan"), dtype=torch.float64, device=DEV)
    sg = torch.zeros(cnt, dtype=torch.float64, device=DEV)
    st = torch.full((cnt,), 7, dtype=torch.int32, device=DEV)
    say(f"[gpu] sdq_greens_noalloc: {label}: {cnt} chains, n = {sorted({c.n for c in ch})}")
    ctx.greens_noalloc(ch, gs, ld, sg, st)
    torch.cuda.synchronize()
    assert torch.equal(st.cpu(), st_ref.cpu()) and (st.cpu() == 0).all()
    ldh, ldr = ld.cpu().numpy(), ld_ref.cpu().numpy()
    worst = 0.0
    for a in range(cnt):
        e = relF(gs[a].cpu().numpy(), g_ref[a].cpu().numpy())
        worst = max(worst, e)
        assert e <= 1e-10, (label, a, e)
        assert abs(ldh[a] - ldr[a]) <= 1e-12 * max(1.0, abs(ldr[a])), (label, a)
    assert torch.equal(sg.cpu(), sg_ref.cpu())
    say(f"[gpu]   max relF against sdq_greens = {worst:.2e}")


def test_noalloc_matches_greens_twice_then_smaller():
    ctx = sdq.Context(0)
    # several size classes (n = 16 .. 121, ragged tiles) and both flavours
    big = _batch(wl.BASE_SEED + 3000, [(4, 10.0, 2), (6, 5.0, 2), (8, 10.0, 2), (10, 4.0, 1),
                                        (11, 2.0, 1), (8, 40.0, 2), (7, 3.0, 1)])
    big += wl.hubbard_ising(8, 20.0, 24, 2, seed=wl.BASE_SEED + 3100)
    _compare(ctx, big, "first call")
    small = _batch(wl.BASE_SEED + 3200, [(4, 2.0, 1), (6, 1.0, 1), (3, 1.5, 1)])
    _compare(ctx, small, "second call, smaller batch")
    _compare(ctx, big[:5], "third call")
    ctx.close()


def test_noalloc_limits(ctx):
    I = wl.hubbard_ising(8, 1.0, 1, 1, seed=wl.BASE_SEED + 3300)[0]
    ch = chains_of([I])[0]
    # more than the fixed scratch holds: rejected with its size, nothing enqueued
    many = [ch] * 2000
    ld = torch.zeros(len(many), dtype=torch.float64, device=DEV)
    st = torch.zeros(len(many), dtype=torch.int32, device=DEV)
    say("[gpu] sdq_greens_noalloc with 2000 chains of n = 64 -> SDQ_EINVAL")
    with pytest.raises(sdq.SdqError) as e:
        ctx.greens_noalloc(many, [None] * len(many), ld, ld.clone(), st)
    assert e.value.status == sdq.SDQ_EINVAL and "MiB" in str(e.value)
    J = wl.hubbard_ising(12, 1.0, 1, 1, seed=wl.BASE_SEED + 3301)[0]
    say("[gpu] sdq_greens_noalloc with n = 144 -> SDQ_EUNSUPPORTED")
    with pytest.raises(sdq.SdqError) as e:
        ctx.greens_noalloc(chains_of([J]), [None], ld[:1], ld[1:2], st[:1])
    assert e.value.status == sdq.SDQ_EUNSUPPORTED
    # the context still works afterwards
    _compare(ctx, [I], "after the rejected calls")
