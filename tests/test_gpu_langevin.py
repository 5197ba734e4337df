"""Langevin steps of a continuous field (sdq_langevin): the force and the
updated field against the same Euler-Maruyama step taken with the oracle's
gradient (d log|det(1 + B)| / d phi = alpha (1 - G_l)_ii at every slice, each
G_l from the oracle's stabilized chain, no wrapping), the log|det| of the
field before the step, and the field-independent case alpha = 0, where the
step reduces to the Ornstein-Uhlenbeck update of the Gaussian weight."""
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


# L = 12 (N = 144) takes the gradient through the gang kernels
@pytest.mark.parametrize("L,beta,k,nf,chains", [(4, 2.0, 10, 1, 3), (4, 2.0, 10, 2, 2),
                                                (6, 1.5, 5, 2, 1), (8, 2.0, 10, 1, 2),
                                                (12, 1.0, 10, 1, 1)])
def test_langevin_matches_oracle_step(ctx, L, beta, k, nf, chains):
    dtau, g, eps, inv_var = 0.1, 1.0, 0.01, 1.0
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), dtau)
    m, n = int(round(beta / dtau)), L * L
    rng = np.random.default_rng(wl.BASE_SEED + 1300 + 10 * L + nf)
    phi0 = rng.normal(0.0, 1.0, (chains, m, n))
    eta = rng.normal(0.0, 1.0, (chains, m, n))
    alphas = (dtau * g,) if nf == 1 else (dtau * g, -dtau * g)
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    Fd = torch.from_numpy(phi0.copy()).to(DEV)
    ch = [sdq.Chain(E_d, Fd[c], a, k, Ei_d) for c in range(chains) for a in alphas]
    say(f"[gpu] sdq_langevin L={L} beta={beta} k={k} nf={nf} chains={chains}")
    frc, ld, sg, st = ctx.langevin(ch, nf, eps, inv_var, torch.from_numpy(eta).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    phi1, F_g, ld_g = Fd.cpu().numpy(), frc.cpu().numpy(), ld.cpu().numpy()
    ls = np.arange(1, m + 1, dtype=np.int32)
    for c in range(chains):
        F = inv_var * phi0[c]
        for f, a in enumerate(alphas):
            F = F - oracle.logdet_grad(E, phi0[c], a, k, ls)
            ldo = oracle.greens(E, phi0[c], a, k)[1]
            assert abs(ld_g[c * nf + f] - ldo) <= 1e-12 * max(1.0, abs(ldo))
        want = phi0[c] - eps * F + np.sqrt(2.0 * eps) * eta[c]
        e_f = relf(F_g[c], F)
        e_p = np.abs(phi1[c] - want).max() / (eps * np.abs(F).max())
        say(f"[gpu]   chain {c}: relF(force) {e_f:.2e}, field error / max step {e_p:.2e}")
        assert e_f <= 1e-10
        assert e_p <= 1e-10


def test_langevin_without_coupling_is_ornstein_uhlenbeck(ctx):
    """alpha = 0: det(1 + B) does not depend on the field, the gradient is
    exactly zero and phi' = phi - eps inv_var phi + sqrt(2 eps) eta."""
    L, m, k, eps, inv_var = 4, 20, 10, 0.05, 2.0
    E, Ei = wl.expk_pair(wl.hopping_matrix(L), 0.1)
    rng = np.random.default_rng(wl.BASE_SEED + 1350)
    phi0 = rng.normal(0.0, 1.0, (2, m, L * L))
    eta = rng.normal(0.0, 1.0, (2, m, L * L))
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    Fd = torch.from_numpy(phi0.copy()).to(DEV)
    ch = [sdq.Chain(E_d, Fd[c], 0.0, k, Ei_d) for c in range(2)]
    say("[gpu] sdq_langevin with alpha = 0")
    frc, _, _, st = ctx.langevin(ch, 1, eps, inv_var, torch.from_numpy(eta).to(DEV))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(frc.cpu().numpy(), inv_var * phi0)
    want = phi0 - eps * inv_var * phi0 + np.sqrt(2.0 * eps) * eta
    assert np.abs(Fd.cpu().numpy() - want).max() <= 1e-15 * np.abs(want).max()


def test_langevin_argument_errors(ctx):
    E, Ei = wl.expk_pair(wl.hopping_matrix(4), 0.1)
    E_d, Ei_d = torch.from_numpy(E).to(DEV), torch.from_numpy(Ei).to(DEV)
    f1 = torch.zeros(20, 16, dtype=torch.float64, device=DEV)
    f2 = torch.zeros(20, 16, dtype=torch.float64, device=DEV)
    eta1 = torch.zeros(1, 20, 16, dtype=torch.float64, device=DEV)
    say("[gpu] sdq_langevin with flavours on different fields / eps <= 0 -> SDQ_EINVAL")
    with pytest.raises(sdq.SdqError) as e:
        ctx.langevin([sdq.Chain(E_d, f1, 0.1, 10, Ei_d), sdq.Chain(E_d, f2, -0.1, 10, Ei_d)], 2, 0.01, 1.0,
                     eta1)
    assert e.value.status == sdq.SDQ_EINVAL
    with pytest.raises(sdq.SdqError) as e:
        ctx.langevin([sdq.Chain(E_d, f1, 0.1, 10, Ei_d)], 1, 0.0, 1.0, eta1)
    assert e.value.status == sdq.SDQ_EINVAL
