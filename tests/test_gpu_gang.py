"""Chains with 128 < n <= 1024 (the gang kernels: a chain spread over
several workgroups, one LDS column slab each) against the CPU oracle.

Shapes follow the paper's Hubbard workloads on L = 12 (n = 144) and L = 16
(n = 256) square lattices with the Hirsch field, plus a continuous field for
the gradient; the same tolerance as the single-workgroup kernels.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl
from _gpu import DEV, chains_of, relF, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    say("[gpu] creating sdq context on cuda:0")
    return sdq.Context(0)

TOL_G = 1e-10
TOL_LD = 1e-12


def test_gang_udt_graded_columns(ctx):
    """UDT (Sec. 4.2.2) of random matrices with columns graded over 16
    decades, n = 144 and 256: the factors equal the oracle's (no pivot ties)
    and reconstruct the input."""
    rng = np.random.default_rng(wl.BASE_SEED + 700)
    for n, cnt in ((144, 3), (256, 2)):
        W = rng.standard_normal((cnt, n, n)) * np.logspace(-8, 8, n)[None, None, :]
        say(f"[gpu] sdq_udt n={n} count={cnt}")
        u, d, t = ctx.udt(torch.from_numpy(W).to(DEV))
        torch.cuda.synchronize()
        u, d, t = u.cpu().numpy(), d.cpu().numpy(), t.cpu().numpy()
        for a in range(cnt):
            U, D, T = oracle.udt(W[a])
            assert relF(u[a], U) <= 1e-12, (n, a, relF(u[a], U))
            assert np.max(np.abs(d[a] / D - 1)) <= 1e-12
            assert relF(t[a], T) <= 1e-12, (n, a, relF(t[a], T))
            rec = (u[a] * d[a][None, :]) @ t[a]
            assert relF(rec, W[a]) <= 1e-13


@pytest.mark.parametrize("L,beta,count", [(12, 10.0, 3), (16, 4.0, 2)])
def test_gang_greens(ctx, L, beta, count):
    insts = wl.hubbard_ising(L, beta, count, 1, seed=wl.BASE_SEED + 710 + L)
    say(f"[gpu] sdq_greens n={L * L} m={insts[0].m} count={count}")
    gs, ld, sg, st = ctx.greens(chains_of(insts))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    for a, I in enumerate(insts):
        G, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
        assert relF(gs[a].cpu().numpy(), G) <= TOL_G, (a, relF(gs[a].cpu().numpy(), G))
        assert abs(ld[a].item() - ldo) <= TOL_LD * abs(ldo), (a, ld[a].item(), ldo)
        assert sg[a].item() == sgo


def test_gang_tdisp(ctx):
    insts = wl.hubbard_ising(12, 10.0, 2, 1, seed=wl.BASE_SEED + 720)
    ls = [0, 1, 9, 10, 11, 37, 50, 99, 100]
    say(f"[gpu] sdq_greens_tdisp n=144 m=100 l={ls}")
    gts, gs, ld, sg, st = ctx.greens_tdisp(chains_of(insts), ls)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    for a, I in enumerate(insts):
        G, ldo, _ = oracle.greens(I.expk, I.field, I.alpha, I.k)
        assert relF(gs[a].cpu().numpy(), G) <= TOL_G
        gt = gts[a].cpu().numpy()
        for idx, l in enumerate(ls):
            ref = oracle.greens_tdisp(I.expk, I.expk_inv, I.field, I.alpha, I.k, l)
            assert relF(gt[idx], ref) <= TOL_G, (a, l, relF(gt[idx], ref))


def test_gang_grad(ctx):
    insts = wl.hubbard_continuous(12, 2.0, 2, seed=wl.BASE_SEED + 730)
    say(f"[gpu] sdq_logdet_grad n=144 m={insts[0].m}")
    grads, ld, sg, st = ctx.logdet_grad(chains_of(insts))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    for a, I in enumerate(insts):
        ref = oracle.logdet_grad(I.expk, I.field, I.alpha, I.k, list(range(1, I.m + 1)))
        g = grads[a].cpu().numpy()
        for l in range(I.m):
            assert relF(g[l], ref[l]) <= TOL_G, (a, l + 1, relF(g[l], ref[l]))
        _, ldo, _ = oracle.greens(I.expk, I.field, I.alpha, I.k)
        assert abs(ld[a].item() - ldo) <= TOL_LD * abs(ldo)
