"""Local-update sweeps (sdq_local_sweep: single-site flips accepted on the
determinant ratio, Sec. 2) against the oracle run as plain sequential
Metropolis in the same site order with every ratio computed from scratch as
exp(sum_f log|det(1+B'_f)| - log|det(1+B_f)|) by the oracle's stabilized
chain (no wrapping, no rank-one updates): the final fields and the accepted
counts must be identical."""
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


def oracle_sweep(E, field, alphas, k, u):
    f = field.copy()
    m, n = f.shape
    ld = [oracle.greens(E, f, a, k)[1] for a in alphas]
    acc = 0
    for l in range(m):
        for i in range(n):
            g = f.copy()
            g[l, i] = -g[l, i]
            ldn = [oracle.greens(E, g, a, k)[1] for a in alphas]
            p = np.exp(sum(ldn) - sum(ld))
            assert abs(u[l, i] - p) > 1e-9, "a decision within rounding of its threshold"
            if u[l, i] < p:
                f, ld, acc = g, ldn, acc + 1
    return f, acc


# L = 3, 4: one wave per chain; L = 6, 8, 10 (N = 36, 64, 100): several waves
# exchanging columns through LDS, ragged last tiles at N = 36 and 100
@pytest.mark.parametrize("L,beta,k,nf,chains", [(4, 2.0, 10, 2, 3), (4, 4.0, 10, 2, 2),
                                                (4, 2.5, 10, 2, 2), (3, 3.0, 7, 1, 2),
                                                (4, 10.0, 10, 2, 1), (6, 1.5, 5, 2, 1),
                                                (8, 1.0, 10, 2, 2), (8, 1.5, 5, 2, 1),
                                                (10, 0.5, 5, 2, 1)])
def test_local_sweep_matches_sequential_metropolis(ctx, L, beta, k, nf, chains):
    dtau, U = 0.1, 4.0
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), dtau)
    lam = wl.hirsch_lambda(U, dtau)
    m, n = int(round(beta / dtau)), L * L
    rng = np.random.default_rng(wl.BASE_SEED + 1100 + 10 * L + int(beta))
    F0 = 2.0 * rng.integers(0, 2, (chains, m, n)) - 1.0
    u = rng.uniform(0.0, 1.0, (chains, m, n))
    alphas = (lam, -lam) if nf == 2 else (lam,)
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    Fd = torch.from_numpy(F0).to(DEV)
    ch = [sdq.Chain(E_d, Fd[c], a, k, Ei_d) for c in range(chains) for a in alphas]
    say(f"[gpu] sdq_local_sweep L={L} beta={beta} k={k} nf={nf} chains={chains}")
    acc, st = ctx.local_sweep(ch, nf, torch.from_numpy(u).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    Fg, accg = Fd.cpu().numpy(), acc.cpu().numpy()
    for c in range(chains):
        fo, ao = oracle_sweep(E, F0[c], alphas, k, u[c])
        say(f"[gpu]   chain {c}: accepted {accg[c]} (oracle {ao}) of {m * n}")
        assert accg[c] == ao
        assert np.array_equal(Fg[c], fo)


def check_decisions_in_parallel(E, F0, Fg, alphas, k, u, threads=16):
    """Every site is visited once per sweep, so the sites whose sign changed
    are exactly the accepted flips, and the field before each proposal is
    known from the decisions before it.  Each decision is then checked on its
    own against the oracle's ratio exp(sum_f log|det(1+B'_f)| -
    log|det(1+B_f)|) (one oracle log|det| per flavour and proposal, in
    parallel).  If every decision agrees, the library followed the sequential
    Metropolis path exactly."""
    import concurrent.futures as cf
    m, n = F0.shape
    acc = (Fg != F0)
    states = []
    f = F0.copy()
    for l in range(m):
        for i in range(n):
            g = f.copy()
            g[l, i] = -g[l, i]
            states.append(g)
            if acc[l, i]:
                f = g
    assert np.array_equal(f, Fg)

    def ld_of(fld):
        return sum(oracle.greens(E, fld, a, k)[1] for a in alphas)

    with cf.ThreadPoolExecutor(threads) as ex:
        ldp = list(ex.map(ld_of, states))
    cur = ld_of(F0)
    t = 0
    for l in range(m):
        for i in range(n):
            p = np.exp(ldp[t] - cur)
            assert abs(u[l, i] - p) > 1e-9, "a decision within rounding of its threshold"
            assert bool(u[l, i] < p) == bool(acc[l, i]), (l, i, u[l, i], p)
            if acc[l, i]:
                cur = ldp[t]
            t += 1
    return int(acc.sum())


@pytest.mark.parametrize("L,beta,k", [(8, 4.0, 10), (6, 6.0, 10)])
def test_local_sweep_longer_chains(ctx, L, beta, k):
    """The benchmark's lattice (N = 64) at beta = 4 (M = 40, four blocks of
    wrapping and recomputation) and N = 36 at beta = 6, both flavours."""
    dtau, U = 0.1, 4.0
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), dtau)
    lam = wl.hirsch_lambda(U, dtau)
    m, n = int(round(beta / dtau)), L * L
    rng = np.random.default_rng(wl.BASE_SEED + 1200 + L)
    F0 = 2.0 * rng.integers(0, 2, (1, m, n)) - 1.0
    u = rng.uniform(0.0, 1.0, (1, m, n))
    alphas = (lam, -lam)
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    Fd = torch.from_numpy(F0).to(DEV)
    ch = [sdq.Chain(E_d, Fd[0], a, k, Ei_d) for a in alphas]
    say(f"[gpu] sdq_local_sweep L={L} beta={beta} k={k}, decisions checked against the oracle")
    acc, st = ctx.local_sweep(ch, 2, torch.from_numpy(u).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    na = check_decisions_in_parallel(E, F0[0], Fd[0].cpu().numpy(), alphas, k, u[0])
    say(f"[gpu]   accepted {na} of {m * n}")
    assert acc.cpu().numpy()[0] == na


def test_local_sweep_then_greens(ctx):
    """After a sweep the field is a valid configuration: the library's G of
    the updated field equals the oracle's, and a second sweep from there
    again matches sequential Metropolis."""
    L, beta, k = 4, 3.0, 10
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), 0.1)
    lam = wl.hirsch_lambda(4.0, 0.1)
    m, n = 30, 16
    rng = np.random.default_rng(wl.BASE_SEED + 1150)
    F0 = 2.0 * rng.integers(0, 2, (1, m, n)) - 1.0
    u1, u2 = rng.uniform(0.0, 1.0, (1, m, n)), rng.uniform(0.0, 1.0, (1, m, n))
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    Fd = torch.from_numpy(F0).to(DEV)
    ch = [sdq.Chain(E_d, Fd[0], a, k, Ei_d) for a in (lam, -lam)]
    say("[gpu] two sdq_local_sweep calls, then sdq_greens")
    ctx.local_sweep(ch, 2, torch.from_numpy(u1).to(DEV))
    ctx.local_sweep(ch, 2, torch.from_numpy(u2).to(DEV))
    gs, _, _, st = ctx.greens(ch)
    torch.cuda.synchronize()
    f1, _ = oracle_sweep(E, F0[0], (lam, -lam), k, u1[0])
    f2, _ = oracle_sweep(E, f1, (lam, -lam), k, u2[0])
    assert np.array_equal(Fd[0].cpu().numpy(), f2)
    G, _, _ = oracle.greens(E, f2, lam, k)
    assert np.linalg.norm(gs[0].cpu().numpy() - G) <= 1e-10 * np.linalg.norm(G)


def test_local_sweep_argument_errors(ctx):
    E, Ei = wl.expk_pair(wl.hopping_matrix(4), 0.1)
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    f1 = torch.ones(20, 16, dtype=torch.float64, device=DEV)
    f2 = torch.ones(20, 16, dtype=torch.float64, device=DEV)
    u = torch.zeros(1, 20, 16, dtype=torch.float64, device=DEV)
    say("[gpu] sdq_local_sweep with flavours on different fields -> SDQ_EINVAL")
    with pytest.raises(sdq.SdqError) as e:
        ctx.local_sweep([sdq.Chain(E_d, f1, 0.5, 10, Ei_d), sdq.Chain(E_d, f2, -0.5, 10, Ei_d)], 2, u)
    assert e.value.status == sdq.SDQ_EINVAL
