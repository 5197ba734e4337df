"""Block products before the sweep (k_prod, tile classes 7 .. 9): every
block of k slices multiplied out first, all blocks of all chains at once,
then the stabilized sweep over the products with one factorization each
(Sec. 4.1).  The context's setting SDQ_BLOCK_PRODUCTS (read at creation)
forces the path on (1) or off (0); both are compared with the oracle at the
chains' own k (relative Frobenius <= 1e-10 for G, log|det| to 1e-12
relative, sign exact) and with each other, on n = 100, 121, 144, a ragged
last block, k = 1 (blocks of one slice: no product in k_prod) and k = m (one
block), in one mixed call with n <= 64 chains that never take the path."""
import os

import numpy as np
import pytest
import torch

import oracle
from _gpu import chains_of, relF, say
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_G = 1e-10
TOL_LD = 1e-12


def context_with(mode):
    old = os.environ.get("SDQ_BLOCK_PRODUCTS")
    os.environ["SDQ_BLOCK_PRODUCTS"] = str(mode)
    try:
        return sdq.Context(0)
    finally:
        if old is None:
            del os.environ["SDQ_BLOCK_PRODUCTS"]
        else:
            os.environ["SDQ_BLOCK_PRODUCTS"] = old


def chains():
    out = []
    for c, (L, beta, k) in enumerate([(10, 10.0, 10), (11, 2.0, 1), (12, 4.3, 10), (12, 2.0, 20), (8, 4.0, 10),
                                      (10, 4.0, 7)]):
        I = wl.hubbard_ising(L, beta, 1, 1, k=k, seed=wl.BASE_SEED + 7100 + c)[0]
        out.append(I)
    return out


@pytest.fixture(scope="module")
def results():
    insts = chains()
    res = {}
    for mode in (1, 0):
        ctx = context_with(mode)
        ctx.set_profiling(True)
        say(f"[gpu] sdq_greens, SDQ_BLOCK_PRODUCTS={mode}: n = {[I.n for I in insts]}, "
            f"m = {[I.m for I in insts]}, k = {[I.k for I in insts]}")
        gs, ld, sg, st = ctx.greens(chains_of(insts))
        torch.cuda.synchronize()
        prod = ctx.kernel_stats("prod")[0]
        res[mode] = ([g.cpu().numpy() for g in gs], ld.cpu().numpy(), sg.cpu().numpy(), st.cpu().numpy(), prod)
        ctx.close()
    return insts, res


@pytest.mark.parametrize("mode", [1, 0])
def test_block_products_match_oracle(results, mode):
    insts, res = results
    gs, ld, sg, st, prod = res[mode]
    # the path ran exactly when forced on: one launch per tile class 7, 8, 9
    assert prod == (3 if mode == 1 else 0), prod
    assert (st == 0).all()
    for a, I in enumerate(insts):
        G, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
        e = relF(gs[a], G)
        say(f"[gpu]   mode {mode} n={I.n} m={I.m} k={I.k}: relF {e:.2e}")
        assert e <= TOL_G, (a, e)
        assert abs(ld[a] - ldo) <= TOL_LD * abs(ldo), (a, ld[a], ldo)
        assert sg[a] == sgo


def test_block_products_agree_with_the_sequential_sweep(results):
    insts, res = results
    for a, I in enumerate(insts):
        e = relF(res[1][0][a], res[0][0][a])
        assert e <= 2 * TOL_G, (a, e)
        if I.n <= 64:  # never on the path: the same kernels, bit for bit
            assert np.array_equal(res[1][0][a], res[0][0][a])


def test_block_products_auto_mode_and_status():
    """Auto (the default): only the class of the longest chain takes the
    path (here n = 144 at m = 43 against n = 100, 121 at m = 100, 20); a NaN
    in that chain's field gives SDQ_ERANGE for it alone."""
    ctx = sdq.Context(0)
    ctx.set_profiling(True)
    insts = chains()[:3]
    bad = insts[2]
    field = bad.field.copy()
    field[5, 7] = np.nan
    insts[2] = wl.Instance(bad.L, bad.m, bad.k, bad.alpha, field, bad.expk, bad.expk_inv)
    say("[gpu] sdq_greens, auto block products, a NaN field in the n = 144 chain")
    gs, ld, sg, st = ctx.greens(chains_of(insts))
    torch.cuda.synchronize()
    assert ctx.kernel_stats("prod")[0] == 1
    assert ctx.kernel_stats("prod/nt9")[0] == 1
    assert st.cpu().tolist() == [0, 0, sdq.SDQ_ERANGE]
    G, _, _ = oracle.greens(insts[0].expk, insts[0].field, insts[0].alpha, insts[0].k)
    assert relF(gs[0].cpu().numpy(), G) <= TOL_G
    ctx.close()
