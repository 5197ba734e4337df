"""LogDet1pB: the torch.autograd.Function over sdq_logdet / sdq_logdet_grad.

Checks that autograd returns the adjoint gradient alpha (1 - G_l)_ii of every
field entry (against the library call and the oracle), that a repeated
backward works, and that one Langevin-style field update decreases
|log det| along the gradient as first-order theory predicts."""
import numpy as np
import pytest
import torch

import oracle
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl
from _gpu import DEV, relF, say

pytestmark = pytest.mark.gpu


def test_autograd_matches_adjoint_and_oracle():
    insts = wl.hubbard_continuous(4, 4.0, 3, seed=wl.BASE_SEED + 800)
    I0 = insts[0]
    E = torch.from_numpy(I0.expk).to(DEV)
    Ei = torch.from_numpy(I0.expk_inv).to(DEV)
    field = torch.from_numpy(np.stack([I.field for I in insts])).to(DEV).requires_grad_(True)
    say("[gpu] LogDet1pB forward/backward, L=4 beta=4, 3 chains")
    ld, sg = sdq.LogDet1pB.apply(field, E, Ei, I0.alpha, I0.k)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=DEV)
    (ld * w).sum().backward(retain_graph=True)
    g1 = field.grad.clone()
    field.grad = None
    (ld * w).sum().backward()  # second backward recomputes the stages
    assert torch.equal(field.grad, g1)
    for a, I in enumerate(insts):
        ref = oracle.logdet_grad(I.expk, I.field, I.alpha, I.k, list(range(1, I.m + 1)))
        assert relF(g1[a].cpu().numpy() / w[a].item(), ref) <= 1e-10
        _, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
        assert abs(ld[a].item() - ldo) <= 1e-12 * abs(ldo)
        assert sg[a].item() == sgo


def test_autograd_langevin_step_first_order():
    """f <- f - eps grad: log det changes by -eps |grad|^2 to first order."""
    I = wl.hubbard_continuous(4, 4.0, 1, seed=wl.BASE_SEED + 801)[0]
    E = torch.from_numpy(I.expk).to(DEV)
    Ei = torch.from_numpy(I.expk_inv).to(DEV)
    field = torch.from_numpy(I.field[None]).to(DEV).requires_grad_(True)
    say("[gpu] LogDet1pB Langevin step")
    ld, _ = sdq.LogDet1pB.apply(field, E, Ei, I.alpha, I.k)
    ld.sum().backward()
    g = field.grad.detach()
    for eps in (1e-4, 1e-5):
        with torch.no_grad():
            ld2, _ = sdq.LogDet1pB.apply(field - eps * g, E, Ei, I.alpha, I.k)
        pred = -eps * float((g * g).sum())
        got = float(ld2.sum() - ld.detach().sum())
        assert abs(got - pred) <= 5e-2 * abs(pred), (eps, got, pred)
