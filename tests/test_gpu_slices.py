"""The symmetric Trotter slice of Sec. 2, B_l = H diag(v_l) H with
H = exp(-dtau K / 2), through the library: G and G(tau,0) for the slices
E diag(v_l) (E = H^2), mapped by sdq_similarity with left = H^{-1},
right = H, against the oracle's chain of symmetric slices (multiplied out in
that form); log|det| and sign directly.  Plus sdq_similarity itself against
numpy on random batches larger than its grid."""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl
from _gpu import DEV, chains_of, relF, say

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    return sdq.Context(0)


def halves(L, dtau=0.1):
    K = wl.hopping_matrix(L)
    H, Hi = wl.expk_pair(K, dtau / 2)
    return H, Hi


@pytest.mark.parametrize("L,beta", [(4, 40.0), (6, 10.0), (8, 40.0)])
def test_symmetric_slices_greens(ctx, L, beta):
    insts = wl.hubbard_ising(L, beta, 1, 2, seed=wl.BASE_SEED + 980 + L)
    H, Hi = halves(L)
    say(f"[gpu] symmetric slices: sdq_greens + sdq_similarity, L={L} beta={beta}")
    gs, ld, sg, st = ctx.greens(chains_of(insts))
    ctx.similarity(gs, torch.from_numpy(Hi).to(DEV), torch.from_numpy(H).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for a, I in enumerate(insts):
        G, ldo, sgo = oracle.greens_sym(H, I.field, I.alpha, I.k)
        assert relF(gs[a].cpu().numpy(), G) <= TOL, (a, relF(gs[a].cpu().numpy(), G))
        assert abs(ld[a].item() - ldo) <= 1e-12 * abs(ldo) and sg[a].item() == sgo


def test_symmetric_slices_tdisp(ctx):
    insts = wl.hubbard_ising(8, 40.0, 2, 1, seed=wl.BASE_SEED + 990)
    H, Hi = halves(8)
    ls = list(range(0, 401, 10))
    say(f"[gpu] symmetric slices: sdq_greens_tdisp + sdq_similarity, L=8 beta=40, {len(ls)} tau")
    gts, _, _, _, st = ctx.greens_tdisp(chains_of(insts), ls, want_g=False)
    ctx.similarity(gts, torch.from_numpy(Hi).to(DEV), torch.from_numpy(H).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for a, I in enumerate(insts):
        for l in (0, 10, 130, 200, 400):
            ref = oracle.greens_tdisp_sym(H, Hi, I.field, I.alpha, I.k, l)
            got = gts[a][ls.index(l)].cpu().numpy()
            assert relF(got, ref) <= TOL, (a, l, relF(got, ref))


@pytest.mark.parametrize("n,count", [(37, 3000), (128, 1500)])
def test_similarity_random_batches(ctx, n, count):
    rng = np.random.default_rng(wl.BASE_SEED + 995 + n)
    A = rng.standard_normal((count, n, n))
    Lm, Rm = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    say(f"[gpu] sdq_similarity n={n} count={count}")
    t = torch.from_numpy(A).to(DEV)
    ctx.similarity([t], torch.from_numpy(Lm).to(DEV), torch.from_numpy(Rm).to(DEV))
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    ref = Lm @ A @ Rm
    err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
    assert err.max() <= 1e-14, err.max()


def test_similarity_argument_errors(ctx):
    big = torch.zeros(144, 144, dtype=torch.float64, device=DEV)
    say("[gpu] sdq_similarity n=144 -> SDQ_EUNSUPPORTED")
    with pytest.raises(sdq.SdqError) as e:
        ctx.similarity([big.clone()], big, big)
    assert e.value.status == sdq.SDQ_EUNSUPPORTED
    m = torch.zeros(16, 16, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        ctx.similarity([torch.zeros(8, 8, dtype=torch.float64, device=DEV)], m, m)
