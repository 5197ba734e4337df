"""Chains of dense slices (sdq_greens_dense, generalized slices): G, log|det|
and sign against the oracle's same chain on the same dense matrices, for the
Hubbard slices written out (also against the library's own Hubbard path) and
for non-symmetric perturbed slices, at N = 16, 36, 64 and 100 up to
beta = 40; G(tau,0) at stage boundaries and inside blocks, also with a short
last block; the limits."""
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
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def slices_for(L, beta, seed, perturb):
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), 0.1)
    lam = wl.hirsch_lambda(4.0, 0.1)
    m, n = int(round(beta / 0.1)), L * L
    rng = np.random.default_rng(seed)
    f = 2.0 * rng.integers(0, 2, (m, n)) - 1.0
    B = np.stack([E * np.exp(lam * f[l])[None, :] for l in range(m)])
    if perturb:
        B = np.stack([B[l] @ (np.eye(n) + perturb * rng.normal(size=(n, n))) for l in range(m)])
    return E, Ei, lam, f, B


@pytest.mark.parametrize("L,beta,perturb", [(4, 10.0, 0.0), (4, 40.0, 0.0), (8, 10.0, 0.0), (8, 40.0, 0.0),
                                            (4, 40.0, 0.02), (6, 20.0, 0.02), (8, 20.0, 0.02),
                                            (10, 10.0, 0.02)])
def test_dense_greens_matches_oracle(ctx, L, beta, perturb):
    E, Ei, lam, f, B = slices_for(L, beta, wl.BASE_SEED + 1600 + L + int(beta), perturb)
    Bd = torch.from_numpy(B).to(DEV)
    say(f"[gpu] sdq_greens_dense L={L} beta={beta} perturbation={perturb}")
    gs, ld, sg, st = ctx.greens_dense([Bd], 10)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    Go, ldo, sgo = oracle.greens_dense(B, 10)
    e = relf(gs[0].cpu().numpy(), Go)
    say(f"[gpu]   relF vs oracle {e:.2e}; log det {ld[0].item():.10g} (oracle {ldo:.10g})")
    assert e <= 1e-10
    assert abs(ld[0].item() - ldo) <= 1e-12 * max(1.0, abs(ldo)) and sg[0].item() == sgo
    if perturb == 0.0:
        # the same chain through the Hubbard path of the library
        ch = [sdq.Chain(torch.from_numpy(E).to(DEV), torch.from_numpy(f).to(DEV), lam, 10)]
        gh, ldh, _, _ = ctx.greens(ch)
        torch.cuda.synchronize()
        assert relf(gs[0].cpu().numpy(), gh[0].cpu().numpy()) <= 1e-10


def test_dense_limits():
    c = sdq.Context(0)
    B = torch.zeros(10, 144, 144, dtype=torch.float64, device=DEV)
    say("[gpu] sdq_greens_dense at n = 144 and with the SVD stabilizer -> SDQ_EUNSUPPORTED")
    with pytest.raises(sdq.SdqError) as e:
        c.greens_dense([B], 10)
    assert e.value.status == sdq.SDQ_EUNSUPPORTED
    c.set_stabilizer(sdq.STAB_SVD)
    with pytest.raises(sdq.SdqError) as e:
        c.greens_dense([torch.zeros(10, 16, 16, dtype=torch.float64, device=DEV)], 10)
    assert e.value.status == sdq.SDQ_EUNSUPPORTED


@pytest.mark.parametrize("L,beta,perturb", [(4, 40.0, 0.0), (4, 40.0, 0.02), (8, 20.0, 0.02), (10, 10.0, 0.02)])
def test_dense_tdisp_matches_oracle(ctx, L, beta, perturb):
    E, Ei, lam, f, B = slices_for(L, beta, wl.BASE_SEED + 1650 + L + int(beta), perturb)
    m = B.shape[0]
    # stage boundaries and l inside blocks (propagation over the dense slices)
    ls = sorted({0, 3, 10, 19, m // 2, m // 2 + 7, m - 10, m - 1, m})
    Bd = torch.from_numpy(B).to(DEV)
    say(f"[gpu] sdq_greens_tdisp_dense L={L} beta={beta} perturbation={perturb} l={ls}")
    gts, gs, ld, _, st = ctx.greens_tdisp_dense([Bd], 10, ls)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    Go, ldo, _ = oracle.greens_dense(B, 10)
    assert relf(gs[0].cpu().numpy(), Go) <= 1e-10
    for j, l in enumerate(ls):
        Ao = oracle.greens_tdisp_dense(B, 10, l)
        e = relf(gts[0][j].cpu().numpy(), Ao)
        say(f"[gpu]   l={l}: relF {e:.2e}")
        assert e <= 1e-10


@pytest.mark.parametrize("n,m,k", [(16, 25, 10), (36, 7, 3), (64, 1, 1)])
def test_dense_tdisp_ragged_blocks(ctx, n, m, k):
    """m not a multiple of k (a short last block), every l from 0 to m."""
    rng = np.random.default_rng(wl.BASE_SEED + 1700 + n + m)
    B = np.stack([1.2 * np.eye(n) + (0.5 / np.sqrt(n)) * rng.normal(size=(n, n)) for _ in range(m)])
    ls = list(range(m + 1))
    say(f"[gpu] sdq_greens_tdisp_dense n={n} m={m} k={k} l=0..{m}")
    gts, gs, _, _, st = ctx.greens_tdisp_dense([torch.from_numpy(B).to(DEV)], k, ls)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    worst = 0.0
    for j, l in enumerate(ls):
        worst = max(worst, relf(gts[0][j].cpu().numpy(), oracle.greens_tdisp_dense(B, k, l)))
    say(f"[gpu]   worst relF {worst:.2e}")
    assert worst <= 1e-10


def test_dense_tdisp_rejects_l_beyond_m(ctx):
    B = torch.zeros(20, 16, 16, dtype=torch.float64, device=DEV)
    say("[gpu] sdq_greens_tdisp_dense at l = 21 > m -> SDQ_EINVAL")
    with pytest.raises(sdq.SdqError) as e:
        ctx.greens_tdisp_dense([B], 10, [21])
    assert e.value.status == sdq.SDQ_EINVAL
