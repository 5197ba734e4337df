"""Chains of complex slices (sdq_greens_complex, App. B): G, log|det(1+B)|
and the phase of det(1+B) against the oracle's complex chain on the same
seeded slices (relative Frobenius <= 1e-10 for G, log|det| to 1e-12
relative, phase to 1e-10), against the closed form of an imaginary chemical
potential, against the real path on real slices; ragged sizes, a mixed
batch, a batch beyond the grid, the limits."""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl
from _gpu import DEV, relF, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return sdq.Context(0)


def cslices(L, beta, seed, phase_amp=0.3, nonsym=0.0):
    """B_l = E diag(exp(lambda s_l + i phi_l)), optionally with a complex
    non-symmetric perturbation of E (the oracle pins use the same recipe)."""
    inst = wl.hubbard_ising(L, beta, 1, 1, seed=seed)[0]
    rng = np.random.default_rng(seed + 1)
    phi = rng.uniform(-phase_amp, phase_amp, inst.field.shape)
    E = inst.expk.astype(complex)
    if nonsym:
        E = E + nonsym * (rng.standard_normal(E.shape) + 1j * rng.standard_normal(E.shape))
    return np.stack([E * np.exp(inst.alpha * inst.field[q] + 1j * phi[q])[None, :] for q in range(inst.m)])


def run(ctx, sls, ks):
    dev = [torch.from_numpy(np.ascontiguousarray(s)).to(DEV) for s in sls]
    gs, ld, ph, st = ctx.greens_complex(dev, ks)
    torch.cuda.synchronize()
    return [g.cpu().numpy() for g in gs], ld.cpu().numpy(), ph.cpu().numpy(), st.cpu().numpy()


def check(ctx, sls, ks, label):
    say(f"[gpu] sdq_greens_complex: {label}: {len(sls)} chains, n = {sorted({s.shape[1] for s in sls})}")
    gs, ld, ph, st = run(ctx, sls, ks)
    worst = 0.0
    for a, (sl, k) in enumerate(zip(sls, ks)):
        G, ldo, pho = oracle.greens_complex(sl, k)
        e = relF(gs[a], G)
        worst = max(worst, e)
        assert st[a] == 0, (label, a)
        assert e <= 1e-10, (label, a, e)
        assert abs(ld[a] - ldo) <= 1e-12 * max(1.0, abs(ldo)), (label, a, ld[a], ldo)
        assert abs(ph[a] - pho) <= 1e-10, (label, a, ph[a], pho)
    say(f"[gpu]   max relF = {worst:.2e}")


@pytest.mark.parametrize("L,beta,k", [(4, 10.0, 10), (4, 40.0, 10), (6, 10.0, 10), (8, 40.0, 10), (3, 4.0, 7)])
def test_complex_chain_matches_oracle(ctx, L, beta, k):
    sls = [cslices(L, beta, wl.BASE_SEED + 5000 + 10 * L + c) for c in range(3)]
    check(ctx, sls, [k] * 3, f"L={L} beta={beta} k={k}")


def test_complex_chain_nonsymmetric_slices(ctx):
    sls = [cslices(4, 4.0, wl.BASE_SEED + 5100 + c, nonsym=0.02) for c in range(2)]
    check(ctx, sls, [7, 7], "non-symmetric complex slices, k = 7 (ragged last block)")


def test_complex_chain_imaginary_chemical_potential(ctx):
    """B_l = e^{i theta} E (U = 0): closed form G = V diag(1/(1 + e^{iM theta -
    beta eps})) V^T and det(1 + B) = prod (1 + e^{iM theta - beta eps})."""
    L, beta, theta = 4, 40.0, 0.0071
    K = wl.hopping_matrix(L)
    m = 400
    E, _ = wl.expk_pair(K, 0.1)
    sl = np.stack([np.exp(1j * theta) * E.astype(complex)] * m)
    say("[gpu] sdq_greens_complex: imaginary chemical potential, L=4 beta=40")
    gs, ld, ph, st = run(ctx, [sl], [10])
    eps, V = np.linalg.eigh(K)
    z = np.exp(1j * m * theta - beta * eps)
    assert st[0] == 0
    assert relF(gs[0], (V / (1.0 + z)) @ V.T) <= 1e-10
    assert abs(ld[0] - np.sum(np.log(np.abs(1.0 + z)))) <= 1e-12 * abs(ld[0])
    assert abs(ph[0] - np.prod((1.0 + z) / np.abs(1.0 + z))) <= 1e-10


def test_complex_chain_of_real_slices_matches_the_real_path(ctx):
    inst = wl.hubbard_ising(8, 20.0, 1, 1, seed=wl.BASE_SEED + 5200)[0]
    sl = np.stack([inst.expk * np.exp(inst.alpha * inst.field[q])[None, :] for q in range(inst.m)])
    say("[gpu] sdq_greens_complex on real slices vs sdq_greens_dense")
    gs, ld, ph, st = run(ctx, [sl.astype(complex)], [10])
    gr, ldr, sgr, str_ = ctx.greens_dense([torch.from_numpy(sl).to(DEV)], 10)
    torch.cuda.synchronize()
    assert st[0] == 0 and str_.item() == 0
    assert np.abs(gs[0].imag).max() <= 1e-12 * np.abs(gs[0]).max()
    assert relF(gs[0].real, gr[0].cpu().numpy()) <= 1e-10
    assert abs(ld[0] - ldr.item()) <= 1e-12 * abs(ldr.item())
    assert abs(ph[0] - sgr.item()) <= 1e-12


def test_complex_chain_mixed_batch_and_beyond_the_grid(ctx):
    sls, ks = [], []
    for c, (L, beta, k) in enumerate([(4, 2.0, 5), (6, 3.0, 10), (8, 4.0, 10), (5, 1.3, 4), (7, 2.0, 10)]):
        sls.append(cslices(L, beta, wl.BASE_SEED + 5300 + c))
        ks.append(k)
    check(ctx, sls, ks, "mixed sizes and lengths")
    # more chains than resident workgroups (grid-stride), sampled
    base = [cslices(4, 1.0, wl.BASE_SEED + 5400 + c) for c in range(4)]
    many = [base[c % 4] for c in range(300)]
    say("[gpu] sdq_greens_complex: 300 chains (sampled)")
    gs, ld, ph, st = run(ctx, many, [5] * 300)
    assert (st == 0).all()
    for a in (0, 1, 255, 256, 257, 299):
        G, ldo, pho = oracle.greens_complex(many[a], 5)
        assert relF(gs[a], G) <= 1e-10 and abs(ph[a] - pho) <= 1e-10


def test_complex_chain_limits_and_status(ctx):
    say("[gpu] sdq_greens_complex: n = 65 -> SDQ_EUNSUPPORTED; k = 0 -> SDQ_EINVAL; a NaN -> SDQ_ERANGE")
    big = torch.zeros(2, 65, 65, dtype=torch.complex128, device=DEV)
    with pytest.raises(sdq.SdqError) as e:
        ctx.greens_complex([big], 1)
    assert e.value.status == sdq.SDQ_EUNSUPPORTED
    sl = cslices(4, 1.0, wl.BASE_SEED + 5500)
    with pytest.raises(sdq.SdqError) as e:
        ctx.greens_complex([torch.from_numpy(sl).to(DEV)], 0)
    assert e.value.status == sdq.SDQ_EINVAL
    with pytest.raises(ValueError):
        ctx.greens_complex([torch.zeros(3, 4, 5, dtype=torch.complex128, device=DEV)], 1)
    bad = sl.copy()
    bad[3, 2, 1] = np.nan
    gs, ld, ph, st = run(ctx, [sl, bad], [5, 5])
    assert st.tolist() == [0, sdq.SDQ_ERANGE]
