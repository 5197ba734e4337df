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


def ring_instance(n, beta, seed, k=10):
    """A periodic ring of n sites (the 1-D model of Sec. 3) with the Hirsch
    field: any n, so that the last 16-wide tile is ragged."""
    e, ei = wl.expk_pair(wl.chain_hopping_matrix(n), 0.1)
    m = int(round(beta / 0.1))
    rng = wl.rng_streams(seed, 1)[0]
    return wl.Instance(n, m, k, wl.hirsch_lambda(4.0, 0.1), wl.ising_field(rng, m, n), e, ei, 0.1,
                       f"ring{n}_b{beta:g}")


@pytest.mark.parametrize("n", [129, 200])
def test_gang_ragged_sizes(ctx, n):
    insts = [ring_instance(n, 4.0, wl.BASE_SEED + 740 + n), ring_instance(n, 2.0, wl.BASE_SEED + 741 + n, k=7)]
    say(f"[gpu] sdq_greens ragged n={n}")
    gs, ld, sg, st = ctx.greens(chains_of(insts))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all(), st
    for a, I in enumerate(insts):
        G, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
        assert relF(gs[a].cpu().numpy(), G) <= TOL_G, (a, relF(gs[a].cpu().numpy(), G))
        assert abs(ld[a].item() - ldo) <= TOL_LD * max(1.0, abs(ldo))
        assert sg[a].item() == sgo


def test_gang_n1024_one_block(ctx):
    """One L = 32 chain (n = 1024, the largest supported size) at beta = 1
    (one stabilization block), against the oracle."""
    I = wl.hubbard_ising(32, 1.0, 1, 1, seed=wl.BASE_SEED + 750)[0]
    say("[gpu] sdq_greens n=1024 m=10")
    gs, ld, sg, st = ctx.greens(chains_of([I]))
    torch.cuda.synchronize()
    assert st.item() == 0
    G, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
    assert relF(gs[0].cpu().numpy(), G) <= TOL_G
    assert abs(ld.item() - ldo) <= TOL_LD * abs(ldo)
    assert sg.item() == sgo


def test_gang_chain_udt(ctx):
    """The stabilized chain's final U, D, T (Sec. 4.1) at n = 144 equal the
    oracle's factors (same pivots, same reflector signs)."""
    insts = wl.hubbard_ising(12, 3.0, 2, 1, seed=wl.BASE_SEED + 760)
    say("[gpu] sdq_chain_udt n=144 m=30")
    u, d, t = ctx.chain_udt(chains_of(insts))
    torch.cuda.synchronize()
    for a, I in enumerate(insts):
        U, D, T = oracle.chain(I.expk, I.expk_inv, I.field, I.alpha, I.k, 0, 1, I.m)
        assert relF(u[a].cpu().numpy(), U) <= 1e-10
        assert np.max(np.abs(d[a].cpu().numpy() / D - 1)) <= 1e-10
        assert relF(t[a].cpu().numpy(), T) <= 1e-10


def test_gang_tdisp_n256(ctx):
    insts = wl.hubbard_ising(16, 4.0, 1, 2, seed=wl.BASE_SEED + 770)
    ls = [0, 5, 20, 33, 40]
    say(f"[gpu] sdq_greens_tdisp n=256 m=40 l={ls}")
    gts, gs, ld, sg, st = ctx.greens_tdisp(chains_of(insts), ls)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for a, I in enumerate(insts):
        gt = gts[a].cpu().numpy()
        for idx, l in enumerate(ls):
            ref = oracle.greens_tdisp(I.expk, I.expk_inv, I.field, I.alpha, I.k, l)
            assert relF(gt[idx], ref) <= TOL_G, (a, l, relF(gt[idx], ref))


def test_gang_grad_with_handle(ctx):
    """sdq_logdet keeping its forward stages, then the gradient from that
    handle: same result as the gradient that recomputes them."""
    insts = wl.hubbard_continuous(12, 2.0, 2, seed=wl.BASE_SEED + 780)
    ch = chains_of(insts)
    say("[gpu] sdq_logdet(keep) + sdq_logdet_grad(handle) n=144")
    ld0, _, st0, h = ctx.logdet(ch, keep=True)
    g1, ld1, _, st1 = ctx.logdet_grad(ch, handle=h)
    g2, ld2, _, _ = ctx.logdet_grad(ch)
    torch.cuda.synchronize()
    ctx.release(h)
    assert (st0.cpu().numpy() == 0).all() and (st1.cpu().numpy() == 0).all()
    for a in range(len(insts)):
        assert torch.equal(g1[a], g2[a])
    assert torch.equal(ld0, ld1) and torch.equal(ld1, ld2)


def test_gang_large_config_sampled(ctx):
    """The large-instance shape (L = 16, beta = 40, M = 400, k = 10) on 8
    chains x 2 flavours in one call with G(tau, 0) at every 10th slice: two
    chains against the oracle at sampled tau, every chain against the
    boundary identities G(0,0) = G and G(beta,0) = 1 - G."""
    insts = wl.hubbard_ising(16, 40.0, 8, 2, seed=wl.BASE_SEED + 4)
    ls = list(range(0, 401, 10))
    say(f"[gpu] sdq_greens_tdisp n=256 m=400, {len(insts)} chains, {len(ls)} taus")
    gts, gs, ld, sg, st = ctx.greens_tdisp(chains_of(insts), ls)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    eye = np.eye(256)
    for a in range(len(insts)):
        g = gs[a].cpu().numpy()
        gt = gts[a]
        assert relF(gt[0].cpu().numpy(), g) <= TOL_G
        assert relF(gt[-1].cpu().numpy(), eye - g) <= TOL_G
    for a, checks in ((0, (0, 200)), (15, (150,))):
        I = insts[a]
        G, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
        assert relF(gs[a].cpu().numpy(), G) <= TOL_G
        assert abs(ld[a].item() - ldo) <= TOL_LD * abs(ldo)
        assert sg[a].item() == sgo
        for l in checks:
            ref = oracle.greens_tdisp(I.expk, I.expk_inv, I.field, I.alpha, I.k, l)
            assert relF(gts[a][ls.index(l)].cpu().numpy(), ref) <= TOL_G, (a, l)


def test_gang_n1024_beta40_all_tau():
    """The large-instance shape with its L = 32 chain: n = 1024, beta = 40
    (M = 400, k = 10), G(tau_l, 0) at every l = 0..400 in one call.  The oracle
    cannot run at this size, so the check is on relations that hold exactly:
    G(0,0) = G and G(beta,0) = 1 - G (both routes computed independently of
    each other), and G(tau_20,0) (computed directly from the stage pair at
    tau = 20 slices) = B_20 G(tau_19,0) (propagated nine slices from tau = 10)."""
    ctx = sdq.Context(0)
    I = wl.hubbard_ising(32, 40.0, 1, 1, seed=wl.BASE_SEED + 790)[0]
    ls = list(range(0, 401))
    say("[gpu] sdq_greens_tdisp n=1024 m=400, all 401 tau")
    gts, gs, ld, sg, st = ctx.greens_tdisp(chains_of([I]), ls)
    torch.cuda.synchronize()
    assert st.item() == 0
    g = gs[0].cpu().numpy()
    g0 = gts[0][0].cpu().numpy()
    gb = gts[0][400].cpu().numpy()
    g19 = gts[0][19].cpu().numpy()
    g20 = gts[0][20].cpu().numpy()
    assert np.isfinite(ld.item()) and sg.item() in (-1.0, 1.0)
    e0, eb = relF(g0, g), relF(gb, np.eye(1024) - g)
    b20 = I.expk * np.exp(I.alpha * I.field[19])[None, :]
    ep = relF(b20 @ g19, g20)
    say(f"[gpu]   relF: G(0,0) vs G {e0:.2e}, G(beta,0) vs 1-G {eb:.2e}, B_20 G(19) vs G(20) {ep:.2e}")
    assert e0 <= TOL_G and eb <= TOL_G and ep <= TOL_G
    ctx.close()
