"""Benchmark: batched stabilized Green's functions on one MI355X.

Workload (one "step"): 512 Hubbard chains, L = 8 (N = 64 sites), beta = 40
(M = 400 slices, dtau = 0.1), U = 4, k = 10: 256 seeded Ising fields x both
spin flavours.  Every step computes, for every chain, the equal-time G, its
log|det(1 + B)| and sign, and G(tau_l, 0) at l = 10, 20, ..., 400 (40
matrices per chain), in one batched call (forward + backward stabilized
sweeps, then the time-displaced inversions).  Inputs are resident in HBM
before the timed region.

Printed: one JSON line with the throughput (chains per second, each chain
with its G and 40 G(tau,0)), the roofline of the dominant kernel measured
with HIP events over the timed region, and the CPU oracle timed on a bounded
sample on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12   # MI355X dense FP64 matrix, FLOP/s
PEAK_HBM = 8.0e12          # bytes/s


def sweep_flops(n, m, k):
    """Algorithmic flops of one stabilized sweep: 2N^3 per slice product and
    (4/3 + 4/3 + 1) N^3 per stabilization (pivoted QR, forming Q, T update)."""
    nb = math.ceil(m / k)
    return (2.0 * m + nb * 11.0 / 3.0) * n ** 3


def pair_flops(n, n_direct, n_prop):
    """Time-displaced inversions: per direct tau two products (4N^3), pivoted
    QR of the middle matrix (4/3 N^3), Q^T applied to N right-hand sides
    (2N^3), triangular solve (N^3) and the final product (2N^3); 2N^3 per
    propagated slice."""
    return n_direct * (4.0 + 4.0 / 3.0 + 2.0 + 1.0 + 2.0) * n ** 3 + n_prop * 2.0 * n ** 3


def grad_flops(n, m, k):
    """Gradient per chain: at each checkpoint the product T1 T2^T (2N^3), a
    pivoted QR (4/3 N^3), Q formation (4/3 N^3), two products (4N^3), the
    equal-time inversion (about 16/3 N^3); then 4N^3 per wrapped slice."""
    nb = (m + k - 1) // k
    return nb * (2.0 + 4.0 / 3.0 + 4.0 / 3.0 + 4.0 + 16.0 / 3.0) * n ** 3 + (m - nb) * 4.0 * n ** 3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-sample", type=int, default=16, help="chains in the CPU sample")
    ap.add_argument("--scale", type=float, default=1.0, help="fraction of the 512 chains (tests only)")
    ap.add_argument("--profile-only", action="store_true",
                    help="time the batched step only (no equal-time / per-chain extras); for profiler runs")
    ap.add_argument("--workload", default="hubbard_L8_b40_batch512",
                    choices=["hubbard_L8_b40_batch512", "hubbard_L4_b10_single", "hubbard_uneven_batch512",
                             "hubbard_L8_b40_metropolis256", "hubbard_L8_b40_local256",
                             "hubbard_L8_b20_phi_batch128", "hubbard_L8_b20_phi_langevin128",
                             "hubbard_L8_b20_phi_hmc128", "hubbard_L8_b40_dense128",
                             "hubbard_L16_b40_batch128", "hubbard_L32_b40_single",
                             "udt_complex_n64_batch4096", "hubbard_L8_b40_complex128"],
                    help="the default is the headline workload; the others time the same library "
                         "on the single small chain (latency of one G), the mixed-size batch "
                         "(equal-time G), the continuous-field batch (log|det| + gradient), the "
                         "L=16 batch and the L=32 chain (G + G(tau,0) at every slice)")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the step from a captured HIP graph (sdq_set_graphs)")
    ap.add_argument("--scheme", default="loh", choices=["loh", "plain"],
                    help="inversion scheme of the time-displaced workloads: Loh's split (default) or "
                         "the single-decomposition inv_sum, which also reports its deviation from "
                         "the split scheme at every tau")
    ap.add_argument("--stab", default="qr", choices=["qr", "svd"],
                    help="stabilizer of the sweeps: the pivoted QR (default) or the one-sided Jacobi SVD "
                         "(n <= 80); the roofline keeps the QR method's flop count, so with the SVD it "
                         "reads as the rate of the QR-equivalent work")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported "
              f"(the path would shard by independent chains, each GPU taking a share)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2003_05286_amd import binding as sdq
    from paper_2003_05286_amd import workloads as wl

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy: {args.calib_copy_mib} MiB read, {args.calib_copy_mib} MiB written",
              file=sys.stderr, flush=True)
        del src, dst
    if args.workload == "udt_complex_n64_batch4096":
        return run_udt_complex(args, dev, sdq, wl)
    if args.workload == "hubbard_L8_b40_complex128":
        return run_greens_complex(args, dev, sdq, wl)
    W = wl.workload(args.workload, scale=args.scale)
    insts = W.instances
    l_list = W.l_list or []
    kind = {"hubbard_L8_b40_batch512": "tdisp", "hubbard_L16_b40_batch128": "tdisp",
            "hubbard_L32_b40_single": "tdisp", "hubbard_L4_b10_single": "greens",
            "hubbard_uneven_batch512": "greens", "hubbard_L8_b20_phi_batch128": "grad",
            "hubbard_L8_b40_metropolis256": "metropolis",
            "hubbard_L8_b40_local256": "local",
            "hubbard_L8_b20_phi_langevin128": "langevin",
            "hubbard_L8_b20_phi_hmc128": "hmc",
            "hubbard_L8_b40_dense128": "dense"}[args.workload]
    n, m, k = insts[0].n, insts[0].m, insts[0].k
    cnt = len(insts)
    plain = args.scheme == "plain"
    if plain and kind != "tdisp":
        raise SystemExit("bench: --scheme plain applies to the time-displaced workloads")
    scheme = sdq.SCHEME_PLAIN if plain else sdq.SCHEME_LOH
    print(f"[bench] {W.name}: {cnt} chains, n={sorted({I.n for I in insts})}, m={m}, k={k}, "
          f"{len(l_list)} G(tau,0) each", file=sys.stderr, flush=True)

    # inputs resident in HBM before timing (instances share their operator and
    # field tensors where the workload shares them)
    dcache = {}

    def dev_of(a):
        if id(a) not in dcache:
            dcache[id(a)] = torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        return dcache[id(a)]

    chains = [sdq.Chain(dev_of(I.expk), dev_of(I.field), I.alpha, I.k, dev_of(I.expk_inv)) for I in insts]
    ctx = sdq.Context(0)
    if args.stab == "svd":
        ctx.set_stabilizer(sdq.STAB_SVD)
    if args.graphs:
        ctx.set_graphs(True)
    # outputs preallocated once
    import ctypes
    inst_arr = ctx._instances(chains, need_inv=(kind in ("grad", "langevin", "hmc") or plain))
    ls = (ctypes.c_int32 * max(len(l_list), 1))(*l_list)
    gts = [torch.empty(len(l_list), I.n, I.n, dtype=torch.float64, device=dev) for I in insts] \
        if kind in ("tdisp", "dense") else []
    gs = [torch.empty(I.n, I.n, dtype=torch.float64, device=dev) for I in insts] \
        if kind not in ("grad", "langevin", "hmc") else []
    grads = [torch.empty(I.m, I.n, dtype=torch.float64, device=dev) for I in insts] if kind == "grad" else []
    ld = torch.empty(cnt, dtype=torch.float64, device=dev)
    sg = torch.empty(cnt, dtype=torch.float64, device=dev)
    st = torch.empty(cnt, dtype=torch.int32, device=dev)
    gt_ptrs = ctx._ptr_array(gts) if gts else None
    g_ptrs = ctx._ptr_array(gs) if gs else None
    gr_ptrs = ctx._ptr_array(grads) if grads else None
    vp = lambda t: ctypes.c_void_p(t.data_ptr())

    if kind == "metropolis":
        # both flavours of a chain share its field: current fields in one
        # tensor, proposals (the spins of one random time slice flipped) in
        # another, dS = 0 for the Hirsch field
        assert all(insts[2 * c].field is insts[2 * c + 1].field for c in range(cnt // 2))
        C = cnt // 2
        Fc = torch.from_numpy(np.stack([insts[2 * c].field for c in range(C)])).to(dev)
        Fp = torch.empty_like(Fc)
        cur_ch, prop_ch = [], []
        for c in range(C):
            for I in (insts[2 * c], insts[2 * c + 1]):
                cur_ch.append(sdq.Chain(dev_of(I.expk), Fc[c], I.alpha, I.k, dev_of(I.expk_inv)))
                prop_ch.append(sdq.Chain(dev_of(I.expk), Fp[c], I.alpha, I.k, dev_of(I.expk_inv)))
        ci, pi = ctx._instances(cur_ch), ctx._instances(prop_ch)
        ld_m, sg_m, _, _ = ctx.logdet(cur_ch)
        dS = torch.zeros(C, dtype=torch.float64, device=dev)
        acc = torch.zeros(C, dtype=torch.int32, device=dev)
        idx = torch.arange(C, device=dev)
        mgen = torch.Generator(device=dev)
        mgen.manual_seed(wl.BASE_SEED + 2000)
        acc_sum = torch.zeros(C, dtype=torch.int64, device=dev)

    if kind == "langevin":
        # one Langevin step of every chain's field per step (Gaussian weight
        # of unit variance, step 0.01); the normal numbers are drawn on the
        # device per step
        Fl = torch.from_numpy(np.stack([I.field for I in insts])).to(dev)
        lg_ch = [sdq.Chain(dev_of(I.expk), Fl[c], I.alpha, I.k, dev_of(I.expk_inv)) for c, I in enumerate(insts)]
        lgi = ctx._instances(lg_ch, need_inv=True)
        ngen = torch.Generator(device=dev)
        ngen.manual_seed(wl.BASE_SEED + 2200)
        nbuf = torch.empty(cnt, m, n, dtype=torch.float64, device=dev)
        frc = torch.empty(cnt, m, n, dtype=torch.float64, device=dev)

    if kind == "dense":
        # the slices E diag(exp(alpha f_l)) of every chain written out as
        # dense matrices on the device (input preparation, not timed)
        dense_t = [(dev_of(I.expk)[None, :, :] * torch.exp(I.alpha * dev_of(I.field))[:, None, :]).contiguous()
                   for I in insts]
        dense_arr = (sdq._DenseInstance * cnt)()
        for i, t in enumerate(dense_t):
            dense_arr[i] = sdq._DenseInstance(n, m, k, 0, t.data_ptr())
    HMC_EPS, HMC_STEPS = 0.05, 10
    if kind == "hmc":
        # one trajectory of every chain per step; momenta and uniform numbers
        # drawn on the device per step
        Fh = torch.from_numpy(np.stack([I.field for I in insts])).to(dev)
        hm_ch = [sdq.Chain(dev_of(I.expk), Fh[c], I.alpha, I.k, dev_of(I.expk_inv)) for c, I in enumerate(insts)]
        hmi = ctx._instances(hm_ch, need_inv=True)
        hgen = torch.Generator(device=dev)
        hgen.manual_seed(wl.BASE_SEED + 2300)
        mbuf = torch.empty(cnt, m, n, dtype=torch.float64, device=dev)
        ubuf_h = torch.empty(cnt, dtype=torch.float64, device=dev)
        acc = torch.zeros(cnt, dtype=torch.int32, device=dev)
        acc_sum = torch.zeros(cnt, dtype=torch.int64, device=dev)
        dHb = torch.empty(cnt, dtype=torch.float64, device=dev)

    if kind == "local":
        # one sweep of single-site flips over every chain's field (both
        # flavours share it); uniform numbers drawn on the device per step
        assert all(insts[2 * c].field is insts[2 * c + 1].field for c in range(cnt // 2))
        C = cnt // 2
        Fc = torch.from_numpy(np.stack([insts[2 * c].field for c in range(C)])).to(dev)
        loc_ch = []
        for c in range(C):
            for I in (insts[2 * c], insts[2 * c + 1]):
                loc_ch.append(sdq.Chain(dev_of(I.expk), Fc[c], I.alpha, I.k, dev_of(I.expk_inv)))
        li = ctx._instances(loc_ch, need_inv=True)
        acc = torch.zeros(C, dtype=torch.int32, device=dev)
        acc_sum = torch.zeros(C, dtype=torch.int64, device=dev)
        ugen = torch.Generator(device=dev)
        ugen.manual_seed(wl.BASE_SEED + 2100)
        ubuf = torch.empty(C, m, n, dtype=torch.float64, device=dev)

    def step():
        if kind == "dense":
            ctx._chk(ctx.lib.sdq_greens_tdisp_dense(ctx.h, dense_arr, cnt, ls, len(l_list), gt_ptrs, g_ptrs,
                                                    vp(ld), vp(sg), vp(st)))
        elif kind == "hmc":
            mbuf.normal_(generator=hgen)
            ubuf_h.uniform_(generator=hgen)
            ctx._chk(ctx.lib.sdq_hmc(ctx.h, hmi, cnt, 1, HMC_EPS, HMC_STEPS, 1.0, vp(mbuf), vp(ubuf_h), vp(ld),
                                     vp(sg), vp(acc), vp(dHb), vp(st)))
            acc_sum.add_(acc)
        elif kind == "langevin":
            nbuf.normal_(generator=ngen)
            ctx._chk(ctx.lib.sdq_langevin(ctx.h, lgi, cnt, 1, 0.01, 1.0, vp(nbuf), vp(frc), vp(ld), vp(sg),
                                          vp(st)))
        elif kind == "local":
            ubuf.uniform_(generator=ugen)
            ctx._chk(ctx.lib.sdq_local_sweep(ctx.h, li, C, 2, vp(ubuf), vp(acc), vp(st)))
            acc_sum.add_(acc)
        elif kind == "metropolis":
            Fp.copy_(Fc)
            rows = torch.randint(0, m, (C,), device=dev, generator=mgen)
            Fp[idx, rows] *= -1.0
            u = torch.rand(C, device=dev, dtype=torch.float64, generator=mgen).clamp_min_(1e-300)
            ctx._chk(ctx.lib.sdq_metropolis(ctx.h, ci, pi, C, 2, vp(dS), vp(u), vp(ld_m), vp(sg_m), vp(acc),
                                            vp(st)))
            acc_sum.add_(acc)
        elif kind == "tdisp":
            ctx._chk(ctx.lib.sdq_greens_tdisp(ctx.h, inst_arr, cnt, scheme, ls, len(l_list),
                                              gt_ptrs, g_ptrs, vp(ld), vp(sg), vp(st)))
        elif kind == "greens":
            ctx._chk(ctx.lib.sdq_greens(ctx.h, inst_arr, cnt, sdq.SCHEME_LOH, g_ptrs, vp(ld), vp(sg), vp(st)))
        else:
            ctx._chk(ctx.lib.sdq_logdet_grad(ctx.h, ctypes.c_uint64(0), inst_arr, cnt, gr_ptrs,
                                             vp(ld), vp(sg), vp(st)))

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    if int((st != 0).sum().item()) != 0 and not plain:
        raise SystemExit("bench: nonzero status after warmup")

    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_times = "HIP events around each launch inside the timed region"
    if args.graphs and kind in ("tdisp", "greens", "grad", "dense"):
        # the kernel nodes of a replayed graph carry no events: the kernels'
        # own times come from as many eager steps right after the timed region
        ctx.set_profiling(False)
        ctx.set_graphs(False)
        ctx.set_profiling(True)
        for i in range(args.steps):
            step()
        torch.cuda.synchronize()
        ctx.set_graphs(True)
        kernel_times = "HIP events around each launch of as many eager steps after the timed graph replays"
    names = ctx.kernel_names()
    per_class = {}
    for nm in names:
        if "/nt" in nm:
            nl, ms = ctx.kernel_stats(nm)
            per_class[nm] = (nl, ms)
    n_sw, ms_sw = ctx.kernel_stats("sweep")
    # block products (k_prod) carry the slice products of the classes that
    # use them: their time counts with the sweep's
    n_pr, ms_pr = ctx.kernel_stats("prod")
    n_pa, ms_pa = ctx.kernel_stats("grad" if kind in ("grad", "langevin", "hmc") else "pair")
    n_eq, ms_eq = ctx.kernel_stats("equal")
    n_lo, ms_lo = ctx.kernel_stats("local")
    n_bs, ms_bs = ctx.kernel_stats("bstart")
    n_lv, ms_lv = ctx.kernel_stats("langevin")
    ctx.set_profiling(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step; sweep {ms_sw / max(n_sw, 1):.3f} ms x "
          f"{n_sw}, pair {ms_pa / max(n_pa, 1):.3f} ms x {n_pa}", file=sys.stderr, flush=True)
    status_ok = int((st != 0).sum().item()) == 0
    n_bad = int((st != 0).sum().item())

    sweeps_per_chain = 1 if kind in ("greens", "metropolis") else 2  # local: backward + rebuilt forward
    f_sweep = sum(sweeps_per_chain * sweep_flops(I.n, I.m, I.k) for I in insts)
    if plain:
        f_sweep = sum(plain_sweep_flops(I.n, I.m, I.k, l_list) for I in insts)
        n_direct = sum(1 for l in l_list if l % k == 0 or l == m)
        f_pair = sum(plain_pair_flops(I.n, n_direct, len(l_list) - n_direct) for I in insts)
    elif kind in ("tdisp", "dense"):
        # l a multiple of k (or m) is a direct inversion, the others propagate
        n_direct = sum(1 for l in l_list if l % k == 0 or l == m)
        f_pair = sum(pair_flops(I.n, n_direct, len(l_list) - n_direct) for I in insts)
    elif kind in ("grad", "langevin", "hmc"):
        f_pair = sum(grad_flops(I.n, I.m, I.k) for I in insts)
    else:
        f_pair = 0.0
    f_equal = sum((4.0 / 3.0 + 2.0 + 1.0 + 2.0) * I.n ** 3 for I in insts)
    # the step's sweep flops over the step's summed sweep-launch time: equal
    # to flops per launch over the mean launch time when a step launches the
    # sweep once, and still the kernel's own rate when a step launches it
    # several times (one launch per size class, or per block of a local
    # sweep); launches of different classes may overlap in wall time
    sweep_launches_per_step = n_sw / max(args.steps, 1)
    sweep_avg_s = (ms_sw + ms_pr) / max(args.steps, 1) * 1e-3
    if kind == "local":
        # one backward sweep and nb-1 single-block forward rebuilds per step
        f_sweep = sum(2.0 * sweep_flops(I.n, I.m, I.k) for I in insts)
    pair_avg_s = ms_pa / max(args.steps, 1) * 1e-3
    evals = HMC_STEPS + 1 if kind == "hmc" else 1  # gradient evaluations per step
    f_sweep_step, f_pair_step = evals * f_sweep, evals * f_pair
    # per size class: launches and device time per step, algorithmic flops,
    # rate (the sweeps of a class: its chains' sweep flops)
    classes = {}
    for nm, (nl, ms) in sorted(per_class.items()):
        kname, nt = nm.split("/nt")
        nt = int(nt)
        members = [I for I in insts if (I.n + 15) // 16 == nt]
        row = {"launches_per_step": nl / max(args.steps, 1), "ms_per_step": ms / max(args.steps, 1),
               "chains": len(members), "n": sorted({I.n for I in members})}
        if kname == "sweep" and not plain:
            spc = 1 if kind in ("greens", "metropolis") else 2
            fl = evals * sum(spc * sweep_flops(I.n, I.m, I.k) for I in members)
            row["flops_per_step"] = fl
            # with the class's block products, if it has them
            ms_all = (ms + per_class.get(f"prod/nt{nt}", (0, 0.0))[1]) / max(args.steps, 1)
            if ms_all * max(args.steps, 1) > ms:
                row["ms_per_step_with_block_products"] = ms_all
            row["tflops"] = fl / (ms_all * 1e-3) / 1e12 if ms > 0 else None
            row["frac_fp64_peak"] = fl / (ms_all * 1e-3) / PEAK_FP64_MFMA if ms > 0 else None
        classes[nm] = row
    achieved = f_sweep_step / sweep_avg_s if sweep_avg_s > 0 else 0.0
    total_flops = f_sweep + f_pair + f_equal
    if kind == "hmc":
        # HMC_STEPS + 1 gradient evaluations per trajectory, log|det| at two
        total_flops = (HMC_STEPS + 1) * (f_sweep + f_pair) + 2 * f_equal

    eq_rate = per_inst_rate = scheme_check = None
    if plain:
        scheme_check = plain_vs_loh(ctx, chains, l_list, gts, torch)
    if not args.profile_only and kind == "tdisp" and not plain:
        # equal-time only, same batch (one forward sweep per chain)
        ctx.greens(chains)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            ctx.greens(chains)
        torch.cuda.synchronize()
        eq_rate = cnt * args.steps / (time.perf_counter() - t2)

        # plain per-instance form on the same GPU: one chain per call, looped
        sub = chains[: min(32, cnt)]
        for c in sub[:2]:
            ctx.greens_tdisp([c], l_list)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for c in sub:
            ctx.greens_tdisp([c], l_list)
        torch.cuda.synchronize()
        per_inst_rate = len(sub) / (time.perf_counter() - t3)

    if args.workload == "hubbard_L8_b40_batch512":
        metric = "stabilized Green's functions/sec (FP64, L=8, beta=40, batched)"
        if plain:
            metric = "stabilized Green's functions/sec (FP64, L=8, beta=40, batched, inv_sum)"
        unit = "chains/s (each: G + 40 G(tau,0))"
    elif kind == "tdisp":
        metric = f"stabilized Green's functions/sec (FP64, {W.name})"
        unit = f"chains/s (each: G + {len(l_list)} G(tau,0))"
    elif kind == "greens":
        metric = f"equal-time Green's functions/sec (FP64, {W.name})"
        unit = "chains/s (each: G, log|det|, sign)"
    elif kind == "local":
        metric = "local-update sweeps/sec (FP64, L=8, beta=40, 256 chains x 2 flavours)"
        unit = ("chain sweeps/s (each: M x N = 25600 single-flip proposals with both flavours' "
                "determinant ratios, rank-one updates, wrapping and per-block recomputation)")
    elif kind == "metropolis":
        metric = "global Metropolis updates/sec (FP64, L=8, beta=40, 256 chains x 2 flavours)"
        unit = ("chain updates/s (each: the stabilized log|det(1+B)| of both flavours of a proposed "
                "field, one time slice flipped, and the accept step)")
    elif kind == "dense":
        metric = "stabilized Green's functions/sec of dense-slice chains (FP64, L=8, beta=40, 128 chains)"
        unit = "chains/s (each: G + 40 G(tau,0); slices read as dense matrices)"
    elif kind == "hmc":
        metric = "HMC trajectories/sec (FP64, L=8, beta=20, 128 chains, continuous field)"
        unit = (f"chain trajectories/s (each: {HMC_STEPS} leapfrog steps of {HMC_EPS}, {HMC_STEPS + 1} "
                "evaluations of log|det| and its adjoint gradient, the Metropolis test on the energy)")
    elif kind == "langevin":
        metric = "Langevin steps/sec (FP64, L=8, beta=20, 128 chains, continuous field)"
        unit = ("chain steps/s (each: log|det| and its adjoint gradient over all M x N field entries, "
                "then phi <- phi - eps dS/dphi + sqrt(2 eps) eta)")
    else:
        metric = f"log|det| + adjoint gradients/sec (FP64, {W.name})"
        unit = "chains/s (each: log|det| and its gradient over all M x N field entries)"
    value = (cnt // 2 if kind in ("metropolis", "local") else cnt) / (ms_step * 1e-3)
    higher = True
    if args.workload == "hubbard_L4_b10_single":
        # one small chain: a latency, not a throughput
        metric = "equal-time Green's function latency (FP64, L=4, beta=10, one chain)"
        unit = "us per G (one sdq_greens call: G, log|det|, sign)"
        value, higher = ms_step * 1e3, False
    betas = sorted({round(I.m * I.dtau, 6) for I in insts})
    out = {
        "metric": metric,
        "value": value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": higher,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": W.name, "chains": cnt, "n": sorted({I.n for I in insts}),
                   "m": sorted({I.m for I in insts}), "k": k, "beta": betas, "dtau": 0.1,
                   "l_list": (f"{l_list[0]},{l_list[1]},...,{l_list[-1]}" if len(l_list) > 2 else l_list),
                   "scheme": args.scheme, "stabilizer": args.stab},
        "roofline": {"kernel": "sweep", "bound": "mfma", "achieved": achieved / 1e12,
                     "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_MFMA,
                     # (the counters were taken on the default scheme and stabilizer)
                     "traffic": measured_traffic() if (args.workload == "hubbard_L8_b40_batch512" and not plain
                                                       and args.stab == "qr") else None,
                     "flops_per_step": f_sweep_step, "launches_per_step": sweep_launches_per_step,
                     "device_ms_per_step": sweep_avg_s * 1e3,
                     "block_products_ms_per_step": ms_pr / max(args.steps, 1),
                     "flops_per_launch": f_sweep_step / max(sweep_launches_per_step, 1e-30),
                     "launch_ms": ms_sw / max(n_sw, 1)},
        "pair_kernel": {"launches_per_step": n_pa / max(args.steps, 1), "device_ms_per_step": pair_avg_s * 1e3,
                        "flops_per_step": f_pair_step,
                        "achieved_tflops": (f_pair_step / pair_avg_s / 1e12) if pair_avg_s > 0 else None},
        "equal_kernel": {"launch_ms": ms_eq / max(n_eq, 1)},
        "classes": classes,
        "graphs": bool(args.graphs),
        "kernel_times": kernel_times,
        "step_tflops": total_flops / (ms_step * 1e-3) / 1e12,
        "green_matrices_per_s": (cnt * (1 + len(l_list)) / (ms_step * 1e-3))
        if kind in ("tdisp", "greens") else None,
        "equal_time_only_per_s": eq_rate,
        "per_instance_loop_per_s": per_inst_rate,
        "status_ok": status_ok,
    }
    if kind == "metropolis":
        out["acceptance"] = float(acc_sum.sum().item()) / (C * (args.warmup + args.steps))
    if kind == "hmc":
        out["acceptance"] = float(acc_sum.sum().item()) / (cnt * (args.warmup + args.steps))
    if kind == "local":
        out["acceptance"] = float(acc_sum.sum().item()) / (C * m * n * (args.warmup + args.steps))
        # algorithmic flops of the local kernels per step: per flavour the
        # block-start G (about 20 N^3 per block, as in the gradient; its own
        # launch), 4 N^3 per wrap, 2 N^2 per accepted flip
        flips = float(acc_sum.sum().item()) / (args.warmup + args.steps)
        nbk = (m + k - 1) // k
        f_local = C * 2 * (nbk * 20.0 + (m - nbk) * 4.0) * n ** 3 + flips * 2 * 2.0 * n ** 2
        ms_both = (ms_lo + ms_bs) / max(args.steps, 1)
        out["local_kernel"] = {"launches_per_step": (n_lo + n_bs) / max(args.steps, 1),
                               "ms_per_step": ms_both,
                               "block_start_ms_per_step": ms_bs / max(args.steps, 1),
                               "flops_per_step": f_local,
                               "achieved_tflops": f_local / (ms_both * 1e-3) / 1e12 if ms_both > 0 else None}
    if kind == "langevin":
        # the update itself: read phi, the gradient and the noise, write phi
        # and the force (5 x 8 B per entry)
        b_upd = 5 * 8.0 * sum(I.m * I.n for I in insts)
        ms_u = ms_lv / max(n_lv, 1)
        out["langevin_kernel"] = {"launches_per_step": n_lv / max(args.steps, 1), "launch_ms": ms_u,
                                  "bytes_per_launch": b_upd,
                                  "achieved_gbs": b_upd / (ms_u * 1e-3) / 1e9 if ms_u > 0 else None}
    if scheme_check is not None:
        scheme_check["chains_flagged_nonfinite"] = n_bad
        out["scheme_check"] = scheme_check

    if not args.no_cpu and kind == "metropolis":
        out["cpu_baseline"] = cpu_baseline_metropolis(insts, args.cpu_sample)
    if not args.no_cpu and kind == "local":
        out["cpu_baseline"] = cpu_baseline_local(insts)
    if not args.no_cpu and kind == "langevin":
        out["cpu_baseline"] = cpu_baseline_langevin(insts, 2)
    if not args.no_cpu and kind == "dense":
        out["cpu_baseline"] = cpu_baseline_dense(insts, 4, l_list)
    if not args.no_cpu and kind == "hmc":
        out["cpu_baseline"] = cpu_baseline_langevin(insts, 1, HMC_STEPS + 1)
    if not args.no_cpu and args.workload == "hubbard_L8_b40_batch512" and not plain and args.stab == "qr":
        out["cpu_baseline"] = cpu_baseline(insts, l_list, args.cpu_sample)
    if not args.no_cpu and args.workload == "hubbard_L4_b10_single":
        out["cpu_baseline"] = cpu_baseline_single(insts[0])
    if not args.no_cpu and args.workload == "hubbard_uneven_batch512":
        out["cpu_baseline"] = cpu_baseline_uneven(insts)
    if not args.no_cpu and args.workload == "hubbard_L8_b20_phi_batch128":
        out["cpu_baseline"] = cpu_baseline_langevin(insts, 2)
        out["cpu_baseline"]["unit"] = "chains/s (each: log|det| and its gradient)"
    if not args.no_cpu and args.workload == "hubbard_L16_b40_batch128":
        out["cpu_baseline"] = cpu_baseline_tdisp_sampled(insts[0], l_list, [1, 200, 400], len(insts))
    if not args.no_cpu and args.workload == "hubbard_L32_b40_single":
        out["cpu_baseline"] = cpu_baseline_n1024(insts[0], l_list)
    if "cpu_baseline" in out:
        out["cpu_baseline"].update(host_cpu()[0])
    # release the context's device memory, streams and graphs while the HIP
    # runtime (and a profiler, if attached) is still up
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(out), flush=True)


def udt_complex_flops(n):
    """Real flops of one complex UDT: the Householder QR (16/3 n^3) and the
    formation of Q (16/3 n^3); a complex multiply-add is 8 real flops."""
    return 32.0 / 3.0 * n ** 3


def run_udt_complex(args, dev, sdq, wl):
    """Complex UDT of 4096 graded complex 64 x 64 matrices per step (the
    decomposition complex slices need, Sec. 4.2.2 / App. B)."""
    import numpy as np
    import torch

    count, n = 4096, 64
    Wh = wl.complex_batch(count, n)
    Wd = torch.from_numpy(Wh).to(dev)
    ctx = sdq.Context(0)
    print(f"[bench] udt_complex_n64_batch4096: {count} complex matrices, n={n}", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        u, d, t = ctx.udt_complex(Wd)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        u, d, t = ctx.udt_complex(Wd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_k, ms_k = ctx.kernel_stats("udt_complex")
    ctx.set_profiling(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    launch_s = ms_k / max(n_k, 1) * 1e-3
    flops = count * udt_complex_flops(n)
    # the FP64 vector peak (256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz)
    peak_valu = 78.6e12
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step; kernel {launch_s * 1e3:.3f} ms x {n_k}",
          file=sys.stderr, flush=True)
    ok = bool(torch.isfinite(d).all().item())
    out = {
        "metric": "complex UDT factorizations/sec (FP64, n=64, 4096 per batch)",
        "value": count / (ms_step * 1e-3),
        "unit": "matrices/s (each: complex pivoted QR, U, D, T)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "udt_complex_n64_batch4096", "matrices": count, "n": n,
                   "inputs": "complex Gaussian columns scaled over 30 decades, random column order"},
        "roofline": {"kernel": "udt_complex", "bound": "alu", "achieved": flops / launch_s / 1e12,
                     "peak": peak_valu / 1e12, "unit": "TFLOP/s", "frac": flops / launch_s / peak_valu,
                     "traffic": None, "flops_per_launch": flops, "launch_ms": launch_s * 1e3,
                     "bytes_per_launch": count * n * n * 16 * 3 + count * n * 8},
        "status_ok": ok,
    }
    if not args.no_cpu:
        import oracle
        threads = host_cpu()[1]
        sample = [Wh[b] for b in range(count)]
        print(f"[bench] cpu oracle: {len(sample)} complex UDTs on {threads} threads", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(oracle.udt_complex, sample))
        dt = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": len(sample) / dt, "unit": "matrices/s", "cores": threads,
                               "kind": "oracle", "sample": f"all 4096 matrices; {dt:.1f} s wall"}
        c1 = time.perf_counter()
        for W1 in sample[:256]:
            oracle.udt_complex(W1)
        d1 = time.perf_counter() - c1
        out["cpu_baseline"]["one_core"] = {"value": 256 / d1, "sample": f"256 matrices on one thread; {d1:.1f} s"}
        out["cpu_baseline"].update(host_cpu()[0])
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(out), flush=True)


def complex_chain_flops(n, m, k):
    """Real flops of one chain of complex slices: 8 n^3 per complex slice
    product, per stabilization the complex QR and Q (16/3 + 16/3) n^3 and the
    T update (4 n^3), and the inversion (elimination 8/3 n^3, the n
    right-hand sides 8 n^3)."""
    nb = math.ceil(m / k)
    return (8.0 * m + nb * (32.0 / 3.0 + 4.0) + 8.0 / 3.0 + 8.0) * n ** 3


def run_greens_complex(args, dev, sdq, wl):
    """Equal-time G, log|det| and phase of 128 chains of complex slices,
    L = 8 (N = 64), beta = 40 (M = 400), k = 10 (App. B's complex slices)."""
    import numpy as np
    import torch

    L, beta, chains, k = 8, 40.0, max(1, int(round(128 * args.scale))), 10
    E, lam, s, phi = wl.complex_hubbard(L, beta, chains)
    m, n = s.shape[1], s.shape[2]
    Ed = torch.from_numpy(E).to(dev).to(torch.complex128)
    # the dense slices, formed on the device (input preparation, not timed)
    sls = []
    for c in range(chains):
        v = torch.exp(torch.from_numpy(lam * s[c] + 1j * phi[c]).to(dev))  # [m, n]
        sls.append((Ed[None, :, :] * v[:, None, :]).contiguous())
    torch.cuda.synchronize()
    ctx = sdq.Context(0)
    print(f"[bench] hubbard_L8_b40_complex128: {chains} chains of complex slices, n={n}, m={m}, k={k}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        gs, ld, ph, st = ctx.greens_complex(sls, k)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        gs, ld, ph, st = ctx.greens_complex(sls, k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_k, ms_k = ctx.kernel_stats("greens_complex")
    ctx.set_profiling(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    launch_s = ms_k / max(n_k, 1) * 1e-3
    flops = chains * complex_chain_flops(n, m, k)
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step; kernel {launch_s * 1e3:.3f} ms x {n_k}",
          file=sys.stderr, flush=True)
    ok = bool((st == 0).all().item())
    out = {
        "metric": "stabilized Green's functions/sec of complex-slice chains (FP64, L=8, beta=40, 128 chains)",
        "value": chains / (ms_step * 1e-3),
        "unit": "chains/s (each: complex G, log|det|, phase)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "hubbard_L8_b40_complex128", "chains": chains, "n": n, "m": m, "k": k,
                   "slices": "E diag(exp(lambda s + i phi)), s = +-1, phi ~ U(-0.3, 0.3), dense complex"},
        "roofline": {"kernel": "greens_complex", "bound": "mfma", "achieved": flops / launch_s / 1e12,
                     "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s", "frac": flops / launch_s / PEAK_FP64_MFMA,
                     "traffic": None, "flops_per_launch": flops, "launch_ms": launch_s * 1e3},
        "status_ok": ok,
    }
    if not args.no_cpu:
        import oracle
        threads = host_cpu()[1]
        sample = list(range(min(chains, 128)))
        host = [np.ascontiguousarray(sls[c].cpu().numpy()) for c in sample]
        print(f"[bench] cpu oracle: {len(host)} chains on {threads} threads", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda h: oracle.greens_complex(h, k), host))
        dt = time.perf_counter() - c0
        c1 = time.perf_counter()
        for h in host[:2]:
            oracle.greens_complex(h, k)
        d1 = time.perf_counter() - c1
        out["cpu_baseline"] = {"value": len(host) / dt, "unit": "chains/s", "cores": threads, "kind": "oracle",
                               "sample": f"{len(host)} of the chains; {dt:.1f} s wall",
                               "one_core": {"value": 2 / d1, "sample": f"2 chains on one thread; {d1:.1f} s"}}
        out["cpu_baseline"].update(host_cpu()[0])
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(out), flush=True)


def plain_sweep_flops(n, m, k, l_list):
    """Sweeps of the single-decomposition G(tau,0): one forward sweep for the
    equal-time G, and for every stage pair j with an output the chains
    B_1^{-1}...B_{tau_j}^{-1} (ceil(tau_j/k) blocks) and B_m...B_{tau_j+1}
    (nb - j blocks), at (2 slices + 11/3) N^3 per block as in sweep_flops."""
    nb = math.ceil(m / k)
    js = sorted({nb if l == m else l // k for l in l_list})
    blocks = 0
    for j in js:
        tau = min(j * k, m)
        blocks += math.ceil(tau / k) + (nb - j)
    per_block = (2.0 * k + 11.0 / 3.0) * n ** 3
    return sweep_flops(n, m, k) + blocks * per_block


def plain_pair_flops(n, n_direct, n_prop):
    """inv_sum per direct tau: X_R^{-1} by pivoted QR (4/3 + 2 + 1) N^3, the
    products X_L X_R^{-1} and U_L^T U_R (4N^3), pivoted QR of the middle
    matrix with its solve (4/3 + 2 + 1) N^3 and the final product (2N^3);
    2N^3 per propagated slice."""
    return n_direct * (2 * (4.0 / 3.0 + 2.0 + 1.0) + 4.0 + 2.0) * n ** 3 + n_prop * 2.0 * n ** 3


def plain_vs_loh(ctx, chains, l_list, gts_plain, torch):
    """Relative Frobenius deviation of the single-decomposition G(tau,0) from
    Loh's split scheme on the same batch, per tau over all chains (Sec. 6.2:
    inv_sum fails around beta/2)."""
    from paper_2003_05286_amd import binding as sdq
    gl, _, _, _, st = ctx.greens_tdisp(chains, l_list, want_g=False, scheme=sdq.SCHEME_LOH)
    torch.cuda.synchronize()
    dev = torch.stack([torch.linalg.matrix_norm(gp - g) / torch.linalg.matrix_norm(g)
                       for gp, g in zip(gts_plain, gl)])  # [chains][n_l]
    dev = torch.nan_to_num(dev, nan=float("inf")).cpu().numpy()
    import numpy as np
    half = l_list.index(max(l_list) // 2) if (max(l_list) // 2) in l_list else len(l_list) // 2
    return {"relF_vs_loh_max_per_l": {str(l): float(dev[:, i].max()) for i, l in enumerate(l_list)},
            "tau_half": {"l": l_list[half], "max": float(dev[:, half].max()),
                         "median": float(np.median(dev[:, half])), "min": float(dev[:, half].min())},
            "loh_status_ok": bool((st == 0).all().item())}


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    or None if the kernel source changed since the counters were taken."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2003_05286_amd", "csrc", "sdq_device.hpp")
    prof = os.path.join(ROOT, "profiles", "hbm_counters_hubbard_L8_b40_batch512.md")
    try:
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        text = open(prof).read()
    except OSError:
        return None
    if h not in text:
        return None
    m = re.search(r"bench traffic line: sweep ([0-9.eE+-]+)", text)
    return float(m.group(1)) if m else None


def cpu_baseline_local(insts, nsites=1024):
    """The oracle's local update as it stands (the ratio of one flip from two
    stabilized log|det| per flavour), on a bounded sample of `nsites` flips of
    one chain on the host threads, scaled to chain sweeps (M x N flips)."""
    import numpy as np
    import oracle

    I0, I1 = insts[0], insts[1]
    m, n = I0.field.shape
    rng = np.random.default_rng(2)
    jobs = []
    for _ in range(nsites):
        f = I0.field.copy()
        f[rng.integers(0, m), rng.integers(0, n)] *= -1.0
        jobs += [(I0, f), (I1, f)]
    threads = host_cpu()[1]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda j: oracle.greens(j[0].expk, j[1], j[0].alpha, j[0].k), jobs))
    dt = time.perf_counter() - t0
    return {"value": nsites / dt / (m * n), "unit": "chain sweeps/s", "cores": threads, "kind": "oracle",
            "sample": f"{nsites} flips of one chain (2 flavours, one oracle log|det| each), {dt:.1f} s "
                      f"wall, scaled to {m * n} flips per sweep"}


def cpu_baseline_dense(insts, nchains, l_list):
    """The oracle as it stands on a bounded sample: `nchains` dense-slice
    chains (their slices written out on the host), each with its G and all
    G(tau_l, 0), one oracle call per host thread."""
    import numpy as np
    import oracle

    threads = host_cpu()[1]
    sample = insts[:nchains]
    dense = [np.ascontiguousarray(I.expk[None, :, :] * np.exp(I.alpha * I.field)[:, None, :]) for I in sample]
    jobs = [(d, None) for d in dense] + [(d, l) for d in dense for l in l_list]
    k = sample[0].k
    print(f"[bench] cpu oracle: {len(jobs)} dense-slice calls on {threads} threads", file=sys.stderr, flush=True)

    def run(job):
        d, l = job
        return oracle.greens_dense(d, k) if l is None else oracle.greens_tdisp_dense(d, k, l)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, jobs))
    dt = time.perf_counter() - t0
    return {"value": len(sample) / dt, "unit": f"chains/s (each: G + {len(l_list)} G(tau,0))", "cores": threads,
            "kind": "oracle", "sample": f"{len(sample)} of the 128 chains; {dt:.1f} s wall"}


def cpu_baseline_langevin(insts, nchains, nevals=1):
    """The oracle as it stands, on a bounded sample: `nevals` gradients of each
    of `nchains` chains (every slice's G from its stabilized chain, the slices
    of a chain split over the host threads) and the step's update; for a
    trajectory (nevals > 1) the log|det| at its ends is not timed (it is
    small beside the gradients)."""
    import numpy as np
    import oracle

    threads = host_cpu()[1]
    print(f"[bench] cpu oracle: {nevals} gradient(s) of each of {nchains} chain(s) on {threads} threads",
          file=sys.stderr, flush=True)
    rng = np.random.default_rng(7)
    t0 = time.perf_counter()
    for I in insts[:nchains]:
        parts = [p for p in np.array_split(np.arange(1, I.m + 1, dtype=np.int32), threads) if len(p)]
        for _ in range(nevals):
            with cf.ThreadPoolExecutor(threads) as ex:
                g = np.concatenate(list(ex.map(lambda ls: oracle.logdet_grad(I.expk, I.field, I.alpha, I.k, ls),
                                               parts)))
        eta = rng.normal(size=I.field.shape)
        _ = I.field - 0.01 * (I.field - g) + np.sqrt(0.02) * eta
    dt = time.perf_counter() - t0
    what = "steps" if nevals == 1 else "trajectories"
    return {"value": nchains / dt, "unit": f"chain {what}/s", "cores": threads, "kind": "oracle",
            "sample": f"{nchains} of the 128 chains, each: {nevals} x the oracle's gradient over all "
                      f"{insts[0].m} x {insts[0].n} entries and the update; {dt:.1f} s wall"}


def cpu_baseline_metropolis(insts, nchains):
    """The oracle on the same step for a bounded sample: `nchains` chains,
    each: log|det(1+B)| of both flavours of a field with one time slice
    flipped (the decision itself is negligible), one oracle call per thread."""
    import numpy as np
    import oracle

    rng = np.random.default_rng(1)
    jobs = []
    for c in range(min(nchains, len(insts) // 2)):
        f = insts[2 * c].field.copy()
        f[rng.integers(0, f.shape[0])] *= -1.0
        for I in (insts[2 * c], insts[2 * c + 1]):
            jobs.append((I, f))
    threads = host_cpu()[1]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda j: oracle.greens(j[0].expk, j[1], j[0].alpha, j[0].k), jobs))
    dt = time.perf_counter() - t0
    return {"value": (len(jobs) // 2) / dt, "unit": "chain updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(jobs) // 2} chains x 2 flavours of the batch, one oracle log|det| per "
                      f"flavour of a proposed field; {dt:.1f} s wall"}


def cpu_baseline(insts, l_list, nchains):
    """The oracle as it stands, on a bounded sample: `nchains` chains, each
    with its G and all G(tau_l, 0), spread over the host cores (one oracle
    call per thread; the C oracle releases the GIL)."""
    import oracle

    sample = insts[:nchains]
    jobs = []
    for I in sample:
        jobs.append(("g", I, 0))
        for l in l_list:
            jobs.append(("t", I, l))
    threads = host_cpu()[1]

    def run(job):
        kind, I, l = job
        if kind == "g":
            oracle.greens(I.expk, I.field, I.alpha, I.k)
        else:
            oracle.greens_tdisp(I.expk, I.expk_inv, I.field, I.alpha, I.k, l)

    print(f"[bench] cpu oracle: {len(jobs)} calls on {threads} threads", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, jobs))
    dt = time.perf_counter() - t0
    # one core: the first chain of the sample, serially
    one = [j for j in jobs if j[1] is sample[0]]
    t1 = time.perf_counter()
    for j in one:
        run(j)
    d1 = time.perf_counter() - t1
    return {"value": len(sample) / dt, "unit": "chains/s (each: G + 40 G(tau,0))", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(sample)} of the 512 chains, each: oracle G plus oracle G(tau_l,0) for all "
                      f"{len(l_list)} l; {dt:.1f} s wall",
            "one_core": {"value": 1.0 / d1, "sample": f"1 chain (G + {len(l_list)} G(tau,0)) on one thread; "
                                                      f"{d1:.1f} s"}}


def host_cpu():
    """The host's CPU as the baselines use it: ({nproc, affinity, cpu_model},
    threads).  The baselines run on the CPUs this process may use, at most 16
    (the host share that comes with one GPU)."""
    nproc = os.cpu_count() or 1
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = nproc
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": nproc, "affinity": aff, "cpu_model": model}, max(1, min(16, aff))


def cpu_baseline_single(I, reps=40):
    """The oracle's G, log|det|, sign of the one chain, on one thread."""
    import oracle
    oracle.greens(I.expk, I.field, I.alpha, I.k)
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.greens(I.expk, I.field, I.alpha, I.k)
    dt = (time.perf_counter() - t0) / reps
    return {"value": dt * 1e6, "unit": "us per G", "cores": 1, "kind": "oracle",
            "sample": f"the chain itself, {reps} calls on one thread"}


def cpu_baseline_uneven(insts, nchains=24):
    """The oracle's G of a bounded sample of the mixed-size batch (every
    21st chain, so sizes and lengths are represented), on the host threads,
    scaled to chains per second; one core: the first 4 of them."""
    import oracle
    threads = host_cpu()[1]
    sample = insts[::max(1, len(insts) // nchains)][:nchains]

    def run(I):
        oracle.greens(I.expk, I.field, I.alpha, I.k)

    print(f"[bench] cpu oracle: {len(sample)} chains on {threads} threads", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, sample))
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    for I in sample[:4]:
        run(I)
    d1 = time.perf_counter() - t1
    return {"value": len(sample) / dt, "unit": "chains/s (each: G, log|det|, sign)", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(sample)} chains of the batch (every {max(1, len(insts) // nchains)}th, n = "
                      f"{sorted({I.n for I in sample})}); {dt:.1f} s wall",
            "one_core": {"value": 4 / d1, "sample": f"the first 4 of them on one thread; {d1:.1f} s"}}


def cpu_baseline_tdisp_sampled(I, l_list, l_sample, nchains):
    """The oracle on one chain: its G and G(tau_l, 0) at the sampled l, one
    call per thread; scaled (labelled extrapolation) to one chain with all of
    l_list, as chains per second.  The oracle builds each G(tau_l, 0) from
    scratch, so its cost per l is about the same for every l."""
    import oracle
    threads = host_cpu()[1]
    jobs = [None] + list(l_sample)

    def run(l):
        if l is None:
            oracle.greens(I.expk, I.field, I.alpha, I.k)
        else:
            oracle.greens_tdisp(I.expk, I.expk_inv, I.field, I.alpha, I.k, l)

    print(f"[bench] cpu oracle: G + {len(l_sample)} G(tau,0) of one n={I.n} chain on {threads} threads",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, jobs))
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    run(l_sample[0])
    d1 = time.perf_counter() - t1
    per_chain = d1 * (1 + len(l_list))  # serial cost of one chain, extrapolated
    return {"value": min(threads, 1 + len(l_list)) / per_chain, "unit": f"chains/s (each: G + {len(l_list)} G(tau,0))",
            "cores": threads, "kind": "oracle",
            "sample": f"one chain: G and G(tau_l,0) at l = {l_sample} ({dt:.1f} s wall on {threads} threads); "
                      f"one G(tau,0) on one thread took {d1:.1f} s; extrapolated to {1 + len(l_list)} "
                      f"matrices per chain with the threads working on separate matrices",
            "extrapolated": True,
            "one_core": {"value": 1.0 / per_chain, "sample": "extrapolated from the one-thread G(tau,0)"}}


def cpu_baseline_n1024(I, l_list):
    """The oracle at N = 1024 is far beyond a bounded sample (each of its
    G(tau_l, 0) multiplies out both chains again: about 400 slice products of
    2 N^3 flops).  Timed here: one slice product and one UDT of the oracle at
    this N on one thread (one slice of the chain and one stabilization), then
    scaled to the oracle's work for G plus all G(tau_l, 0) (extrapolation)."""
    import numpy as np
    import oracle
    n, m, k = I.n, I.m, I.k
    rng = np.random.default_rng(3)
    W = rng.standard_normal((n, n))
    print(f"[bench] cpu oracle: one slice product and one UDT at n={n}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    oracle.chain(I.expk, I.expk_inv, I.field[:1], I.alpha, 1, 0, 1, 1)
    t_slice_udt = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.udt(W)
    t_udt = time.perf_counter() - t1
    t_slice = max(t_slice_udt - t_udt, 0.0)
    nb = (m + k - 1) // k
    # oracle work: G (m slices, nb UDTs) and per l the two chains (m slices,
    # about nb + 1 UDTs) and the inversion (a few UDT-sized factorizations)
    per_chain = (1 + len(l_list)) * (m * t_slice + (nb + 3) * t_udt)
    return {"value": 1.0 / per_chain, "unit": f"chains/s (each: G + {len(l_list)} G(tau,0))", "cores": 1,
            "kind": "oracle",
            "sample": f"one slice product ({t_slice:.1f} s) and one UDT ({t_udt:.1f} s) at n={n} on one thread, "
                      f"scaled to {1 + len(l_list)} matrices x ({m} slices + {nb + 3} UDTs)",
            "extrapolated": True}


if __name__ == "__main__":
    main()
