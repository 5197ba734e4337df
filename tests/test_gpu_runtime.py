"""Runtime features through the C ABI on the GPU: HIP graph replay and the
autotuner.  Graph replays are checked one by one against the eager result,
with the test's own eager work and synchronizations between them."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from _gpu import chains_of, relF, say
from paper_2003_05286_amd import binding as sdq
from paper_2003_05286_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_graph_replay_matches_eager():
    say("[gpu] graph replay: L=6 beta=10, 8 chains, G + G(tau,0)")
    ctx = sdq.Context(0)
    insts = wl.hubbard_ising(6, 10.0, 4, 2, seed=wl.BASE_SEED + 700)
    ch = chains_of(insts)
    ls = [0, 10, 35, 60, 100]
    gts0, gs0, ld0, sg0, st0 = ctx.greens_tdisp(ch, ls)
    torch.cuda.synchronize()
    ctx.set_graphs(True)
    import ctypes
    inst_arr = ctx._instances(ch)
    larr = (ctypes.c_int32 * len(ls))(*ls)
    gts = [torch.empty_like(g) for g in gts0]
    gs = [torch.empty_like(g) for g in gs0]
    ld = torch.empty_like(ld0)
    sg = torch.empty_like(sg0)
    st = torch.empty_like(st0)
    gp, g2 = ctx._ptr_array(gts), ctx._ptr_array(gs)
    for rep in range(4):
        for t in gts + gs:
            t.zero_()          # eager work between replays
        ld.zero_()
        junk = torch.randn(1000, device="cuda").sum()  # unrelated eager kernels
        torch.cuda.synchronize()
        say(f"[gpu]   replay {rep}")
        ctx._chk(ctx.lib.sdq_greens_tdisp(ctx.h, inst_arr, len(ch), 0, larr, len(ls), gp, g2,
                                          ctypes.c_void_p(ld.data_ptr()), ctypes.c_void_p(sg.data_ptr()),
                                          ctypes.c_void_p(st.data_ptr())))
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a in range(len(ch)):
            assert torch.equal(gts[a], gts0[a]), (rep, a)
            assert torch.equal(gs[a], gs0[a]), (rep, a)
        assert torch.equal(ld, ld0) and torch.equal(sg, sg0) and torch.equal(st, st0)
    ctx.set_graphs(False)
    ctx.close()


def test_autotune_cache_and_parity(tmp_path):
    path = str(tmp_path / "tune.jsonl")
    ctx = sdq.Context(0)
    say("[gpu] sdq_tune n = 36, 64")
    ctx.tune([36, 64], path)
    lines = [json.loads(l) for l in open(path)]
    assert {l["n"] for l in lines} == {36, 64}
    assert all(l["variant"] in (0, 1, 4, 5) and l["blocks_per_cu"] in (0, 1) for l in lines)
    # a second call reads the cache and adds nothing
    ctx.tune([36, 64], path)
    assert len(open(path).read().splitlines()) == 2
    for L, beta in ((6, 10.0), (8, 20.0)):
        insts = wl.hubbard_ising(L, beta, 2, 1, seed=wl.BASE_SEED + 710 + L)
        gs, ld, sg, st = ctx.greens(chains_of(insts))
        torch.cuda.synchronize()
        for a, I in enumerate(insts):
            G, ldo, sgo = oracle.greens(I.expk, I.field, I.alpha, I.k)
            assert relF(gs[a].cpu().numpy(), G) <= 1e-10
            assert abs(ld[a].item() - ldo) <= 1e-12 * abs(ldo)
    ctx.close()


def test_graph_mode_with_gang_chains_runs_directly():
    """A batch with an n > 128 chain (cooperative launches) in graph mode is
    launched directly; repeated calls equal the eager result."""
    ctx = sdq.Context(0)
    insts = wl.hubbard_ising(12, 2.0, 1, 1, seed=wl.BASE_SEED + 720) + \
        wl.hubbard_ising(4, 2.0, 1, 1, seed=wl.BASE_SEED + 721)
    ch = chains_of(insts)
    say("[gpu] graph mode, mixed n = 144 and 16")
    gs0, ld0, _, st0 = ctx.greens(ch)
    torch.cuda.synchronize()
    ctx.set_graphs(True)
    for rep in range(3):
        gs, ld, _, st = ctx.greens(ch)
        torch.cuda.synchronize()
        for a in range(len(ch)):
            assert torch.equal(gs[a], gs0[a]), (rep, a)
        assert torch.equal(ld, ld0) and (st.cpu().numpy() == 0).all()
    ctx.set_graphs(False)
    ctx.close()


def test_tune_accepts_large_sizes(tmp_path):
    """Sizes above 128 have one kernel: accepted, nothing timed or cached."""
    path = str(tmp_path / "tune.jsonl")
    ctx = sdq.Context(0)
    say("[gpu] sdq_tune n = 16, 144")
    ctx.tune([16, 144], path)
    lines = [json.loads(l) for l in open(path)]
    assert [l["n"] for l in lines] == [16]
    ctx.close()


def test_gang_status_flags_nonfinite_field():
    ctx = sdq.Context(0)
    I = wl.hubbard_ising(12, 2.0, 1, 1, seed=wl.BASE_SEED + 722)[0]
    f = I.field.copy()
    f[5, 17] = np.nan
    I2 = wl.Instance(I.L, I.m, I.k, I.alpha, f, I.expk, I.expk_inv)
    say("[gpu] gang sdq_greens with a NaN in the field")
    _, _, _, st = ctx.greens(chains_of([I, I2]))
    torch.cuda.synchronize()
    assert st.cpu().numpy().tolist() == [0, sdq.SDQ_ERANGE]
    ctx.close()


def test_graph_mode_consumers_match_eager():
    """Local sweeps, Langevin steps and HMC trajectories in graph mode (each
    plan captured and replayed, the library's tables copied outside the
    graphs) give bitwise the same fields as eager launches, twice in a row."""
    say("[gpu] graph mode: local sweep, Langevin step, HMC trajectory vs eager (L=4, beta=2)")
    E, Ei = wl.expk_pair(wl.hopping_matrix(4), 0.1)
    lam = wl.hirsch_lambda(4.0, 0.1)
    rng = np.random.default_rng(wl.BASE_SEED + 750)
    F0 = 2.0 * rng.integers(0, 2, (2, 20, 16)) - 1.0
    P0 = rng.normal(0.0, 1.0, (2, 20, 16))
    u = [torch.from_numpy(rng.uniform(0.0, 1.0, (2, 20, 16))).cuda() for _ in range(2)]
    eta = [torch.from_numpy(rng.normal(0.0, 1.0, (2, 20, 16))).cuda() for _ in range(2)]
    uh = [torch.from_numpy(rng.uniform(0.0, 1.0, 2)).cuda() for _ in range(2)]
    E_d, Ei_d = torch.from_numpy(E).cuda(), torch.from_numpy(Ei).cuda()
    results = []
    for graphs in (False, True):
        ctx = sdq.Context(0)
        ctx.set_graphs(graphs)
        Fl = torch.from_numpy(F0.copy()).cuda()
        Pl = torch.from_numpy(P0.copy()).cuda()
        Ph = torch.from_numpy(P0.copy()).cuda()
        loc = [sdq.Chain(E_d, Fl[c], a, 10, Ei_d) for c in range(2) for a in (lam, -lam)]
        lan = [sdq.Chain(E_d, Pl[c], 0.1, 10, Ei_d) for c in range(2)]
        hmc = [sdq.Chain(E_d, Ph[c], 0.1, 10, Ei_d) for c in range(2)]
        for rep in range(2):
            ctx.local_sweep(loc, 2, u[rep])
            ctx.langevin(lan, 1, 0.01, 1.0, eta[rep])
            ctx.hmc(hmc, 1, 0.05, 3, 1.0, eta[rep], uh[rep])
            torch.randn(1000, device="cuda").sum()  # unrelated eager work between calls
        torch.cuda.synchronize()
        results.append((Fl.cpu().numpy(), Pl.cpu().numpy(), Ph.cpu().numpy()))
        ctx.close()
    for a, b in zip(results[0], results[1]):
        assert np.array_equal(a, b)
