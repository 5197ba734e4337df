"""Hybrid Monte Carlo trajectories of a continuous field (sdq_hmc): the
energy change, the accept decision and the end field against the same
leapfrog trajectory taken with the oracle's gradient and log|det| (every
slice's G from the oracle's stabilized chain), the start field restored
exactly on rejection, and the leapfrog's second-order energy error (halving
the step at a fixed trajectory length divides |dH| by about four)."""
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


def oracle_trajectory(E, phi0, alphas, k, eps, nsteps, inv_var, mom):
    """Leapfrog with the oracle's gradient; returns (end field, dH, log|det| at
    the start and at the end per flavour)."""
    m = phi0.shape[0]
    ls = np.arange(1, m + 1, dtype=np.int32)

    def force(phi):
        F = inv_var * phi
        for a in alphas:
            F = F - oracle.logdet_grad(E, phi, a, k, ls)
        return F

    def logdets(phi):
        return np.array([oracle.greens(E, phi, a, k)[1] for a in alphas])

    phi = phi0.copy()
    p = mom - 0.5 * eps * force(phi)
    for s in range(1, nsteps + 1):
        phi = phi + eps * p
        p = p - (eps if s < nsteps else 0.5 * eps) * force(phi)
    ld0, ld1 = logdets(phi0), logdets(phi)
    h0 = 0.5 * inv_var * np.sum(phi0 ** 2) + 0.5 * np.sum(mom ** 2) - ld0.sum()
    h1 = 0.5 * inv_var * np.sum(phi ** 2) + 0.5 * np.sum(p ** 2) - ld1.sum()
    return phi, h1 - h0, ld0, ld1


def setup(L, beta, chains, nf, seed, dtau=0.1, g=1.0):
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), dtau)
    m, n = int(round(beta / dtau)), L * L
    rng = np.random.default_rng(seed)
    phi0 = rng.normal(0.0, 1.0, (chains, m, n))
    mom = rng.normal(0.0, 1.0, (chains, m, n))
    alphas = (dtau * g,) if nf == 1 else (dtau * g, -dtau * g)
    return E, Ei, phi0, mom, alphas


def run_gpu(ctx, E, Ei, phi0, alphas, k, eps, nsteps, inv_var, mom, u):
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    Fd = torch.from_numpy(phi0.copy()).to(DEV)
    ch = [sdq.Chain(E_d, Fd[c], a, k, Ei_d) for c in range(phi0.shape[0]) for a in alphas]
    acc, dh, ld, sg, st = ctx.hmc(ch, len(alphas), eps, nsteps, inv_var, torch.from_numpy(mom).to(DEV),
                                  torch.from_numpy(u).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    return Fd.cpu().numpy(), acc.cpu().numpy(), dh.cpu().numpy(), ld.cpu().numpy()


@pytest.mark.parametrize("L,beta,k,nf,chains,eps,nsteps", [(4, 2.0, 10, 1, 3, 0.05, 4),
                                                           (4, 2.0, 10, 2, 2, 0.05, 3),
                                                           (6, 1.5, 5, 2, 1, 0.04, 3)])
def test_hmc_matches_oracle_trajectory(ctx, L, beta, k, nf, chains, eps, nsteps):
    E, Ei, phi0, mom, alphas = setup(L, beta, chains, nf, wl.BASE_SEED + 1400 + 10 * L + nf)
    inv_var = 1.0
    ref = [oracle_trajectory(E, phi0[c], alphas, k, eps, nsteps, inv_var, mom[c]) for c in range(chains)]
    # accept every chain but the last, which gets u just above exp(-dH) when
    # that is below 1 (a rejection), else just below it
    u = np.array([min(0.5, 0.5 * np.exp(-r[1])) for r in ref])
    dl = ref[-1][1]
    u[-1] = np.exp(-dl) * (1.0 + 1e-6) if dl > 1e-5 else min(0.999, np.exp(-dl) * (1.0 - 1e-6))
    say(f"[gpu] sdq_hmc L={L} beta={beta} nf={nf} chains={chains} eps={eps} nsteps={nsteps}")
    phi1, acc, dh, ld = run_gpu(ctx, E, Ei, phi0, alphas, k, eps, nsteps, inv_var, mom, u)
    for c in range(chains):
        phi_o, dh_o, ld0, ld1 = ref[c]
        take = np.log(u[c]) < -dh_o
        say(f"[gpu]   chain {c}: dH {dh[c]:.6e} (oracle {dh_o:.6e}), accepted {acc[c]} (oracle {int(take)})")
        assert abs(dh[c] - dh_o) <= 1e-9 * max(1.0, abs(dh_o))
        assert acc[c] == int(take)
        if take:
            assert np.linalg.norm(phi1[c] - phi_o) <= 1e-10 * np.linalg.norm(phi_o)
            ref_ld = ld1
        else:
            assert np.array_equal(phi1[c], phi0[c])
            ref_ld = ld0
        # the start field comes back bit for bit on rejection (log det to the
        # usual 1e-12); an accepted end field agrees with the oracle's
        # trajectory to 1e-10 only, and its log det to the same order
        tol = 1e-10 if take else 1e-12
        for f in range(len(alphas)):
            assert abs(ld[c * len(alphas) + f] - ref_ld[f]) <= tol * max(1.0, abs(ref_ld[f]))


def test_hmc_energy_error_is_second_order(ctx):
    L, beta, k, chains = 4, 2.0, 10, 8
    E, Ei, phi0, mom, alphas = setup(L, beta, chains, 2, wl.BASE_SEED + 1450)
    u = np.full(chains, 0.5)
    say("[gpu] sdq_hmc at eps = 0.04 x 5 and 0.02 x 10 (same trajectory length)")
    _, _, dh1, _ = run_gpu(ctx, E, Ei, phi0, alphas, k, 0.04, 5, 1.0, mom, u)
    _, _, dh2, _ = run_gpu(ctx, E, Ei, phi0, alphas, k, 0.02, 10, 1.0, mom, u)
    r = np.mean(np.abs(dh2)) / np.mean(np.abs(dh1))
    say(f"[gpu]   mean |dH| {np.mean(np.abs(dh1)):.3e} -> {np.mean(np.abs(dh2)):.3e} (ratio {r:.3f})")
    assert 0.15 < r < 0.4


def test_hmc_argument_errors(ctx):
    E, Ei = wl.expk_pair(wl.hopping_matrix(4), 0.1)
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    f1 = torch.zeros(20, 16, dtype=torch.float64, device=DEV)
    mom = torch.zeros(1, 20, 16, dtype=torch.float64, device=DEV)
    u = torch.full((1,), 0.5, dtype=torch.float64, device=DEV)
    say("[gpu] sdq_hmc with nsteps = 0 -> SDQ_EINVAL")
    with pytest.raises(sdq.SdqError) as e:
        ctx.hmc([sdq.Chain(E_d, f1, 0.1, 10, Ei_d)], 1, 0.01, 0, 1.0, mom, u)
    assert e.value.status == sdq.SDQ_EINVAL
