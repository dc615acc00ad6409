"""Benchmark: solves/s to 1e-9 relative residual on a 32^3 x 64 twisted-mass
lattice, chosen (multi-RHS mixed precision) vs plain (FP64 CG), and the HBM
throughput of the multi-RHS half-lattice Dslash.

One step = one pass of the hot path over one batch: a Z4 noise vector with
12 spin-colour dilutions generated on the GPU, even-odd source preparation,
12 right-hand sides solved together by CG on the normal equations with FP16
spinor and link storage, FP32 arithmetic and FP64 reliable updates to a
1e-9 full-system residual, odd reconstruction, FP64 true-residual check, and
the one-end loop contraction 2 i eps sum_x s^dag gamma5 Gamma_n s for the 16
Gamma at every time slice.  Inputs (gauge field) are resident in HBM before
timing; the noise is generated inside the step.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dslash-reps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--cpu-full-solve", action="store_true",
                    help="also run one 32^3x64 oracle solve to 1e-9 to completion (minutes of CPU time)")
    ap.add_argument("--no-ptc", action="store_true",
                    help="skip the learned-preconditioner comparison on 32^3x64")
    ap.add_argument("--ptc-pairs", type=int, default=4096)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the momentum, TSM/HPE, time-dilution and uneven-batch legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the workload (one 32^3x64 lattice, noise vectors "
              "solved in batches) is measured on a single MI355X; --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1309_2256_amd as P
    import synth as S

    dev = "cuda:0"
    cfg = S.CONFIGS["c3"]
    L, kappa, eps = cfg["L"], cfg["kappa"], cfg["two_kappa_mu"]
    V = int(np.prod(L))
    seed_noise = S.NOISE_SEEDS["c3"]
    t0 = time.time()
    U = S.gauge_links(L, cfg["eps_links"], cfg["seed"])
    print("[bench] gauge field %s generated in %.1fs" % (str(L), time.time() - t0),
          file=sys.stderr, flush=True)
    ctx = P.Context(L, kappa, eps)
    ctx.set_gauge(torch.from_numpy(U).to(dev))
    torch.cuda.synchronize()

    nrhs = 12
    chosen = P.solve_params(tol=1e-9, maxiter=100000, solver=P.TM_CG_MIXED,
                            inner_prec=P.TM_F16, delta=0.1, check_every=8)

    def loop_params(noise_index):
        p = P.tm_loop_params()
        p.seed, p.n_hp, p.n_lp = seed_noise, 1, 0
        p.noise_offset = noise_index
        p.dilution = P.TM_DIL_SPIN_COLOUR
        p.estimators = P.TM_EST_ONE_END
        p.mu_sign = 1
        p.hp = chosen
        return p

    def step(k):
        loops, _, st, status = ctx.loops(loop_params(k))
        assert status == P.TM_OK and st.max_res_hp <= 1e-9, (status, st.max_res_hp)
        return loops, st

    for k in range(args.warmup):
        step(k)
        print("[bench] warmup step %d done" % k, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        loops, st = step(args.warmup + k)
        stats.append(st)
        print("[bench] step %d: %d solves, %d iterations, max residual %.2e, %.2fs"
              % (k, st.n_solves_hp, st.iters_hp, st.max_res_hp, st.seconds),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n_solves = sum(s.n_solves_hp for s in stats)
    value = n_solves / elapsed
    chosen_iters = sum(s.iters_hp for s in stats) / n_solves

    # the same chosen solve with the configuration's stated link precision:
    # FP32 links (all 18 parameters) with FP16 spinors
    ctx.set_half_spinor_links(P.TM_F32)
    step(args.warmup + args.steps)  # warm (tuning of the FP32-link kernels)
    torch.cuda.synchronize()
    tf = time.perf_counter()
    fst = [step(args.warmup + args.steps + 1 + k)[1] for k in range(args.steps)]
    torch.cuda.synchronize()
    f32_elapsed = time.perf_counter() - tf
    ctx.set_half_spinor_links(P.TM_F16)
    f32_links = {"solves_per_s": sum(q.n_solves_hp for q in fst) / f32_elapsed,
                 "iters_per_solve": sum(q.iters_hp for q in fst) / sum(q.n_solves_hp for q in fst),
                 "max_res": max(q.max_res_hp for q in fst),
                 "what": "the chosen solve with FP32 links (18 parameters) and FP16 spinors, "
                         "the configuration's stated precision; same steps as value"}
    print("[bench] chosen solve with FP32 links: %.2f solves/s" % f32_links["solves_per_s"],
          file=sys.stderr, flush=True)

    # plain: FP64 CG, one right-hand side at a time (the first dilution of
    # noise 0), median of three timed solves
    b = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device=dev)
    eta12 = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    ctx.noise(eta12, seed_noise, 0, P.TM_DIL_SPIN_COLOUR)
    b.copy_(eta12[:1])
    del eta12
    x = torch.zeros_like(b)
    ctx.solve(x, b, 1, P.solve_params(tol=1e-9, solver=P.TM_CG_F64))  # warm
    plain_times = []
    for _ in range(3):
        x.zero_()
        torch.cuda.synchronize()
        tp = time.perf_counter()
        _, pst = ctx.solve(x, b, 1, P.solve_params(tol=1e-9, solver=P.TM_CG_F64))
        torch.cuda.synchronize()
        plain_times.append(time.perf_counter() - tp)
    plain_time = float(np.median(plain_times))
    plain_value = 1.0 / plain_time
    plain_iters = pst[0].iters
    print("[bench] plain FP64 solve: %d iterations, residual %.2e, %s s"
          % (plain_iters, pst[0].true_rel_res, ["%.3f" % v for v in plain_times]), file=sys.stderr, flush=True)
    del x, b

    # dominant kernel: 12-RHS half-lattice Dslash R^-1 H (FP16 spinors and
    # links, FP32 arithmetic), the form the chosen solver launches, timed with
    # HIP events on the stream it is launched on (torch's current stream)
    vh = V // 2
    nb = ctx.half_numel(P.TM_F16, nrhs)
    bufs = [torch.randn(nb // 2, dtype=torch.float16, device=dev) * 0.1 for _ in range(2)]
    outb = torch.empty(nb, dtype=torch.uint8, device=dev)
    ctx.set_link_format(LINK_PARAMS)  # the library default, stated for the byte count
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def time_half(link_prec, reps):
        for _ in range(10):
            ctx.dslash(outb, bufs[0], nrhs, P.TM_RINV_HOP_OE, 1, P.TM_F16, link_prec)
        torch.cuda.synchronize()
        ev0.record()
        for r in range(reps):
            ctx.dslash(outb, bufs[r % 2], nrhs, P.TM_RINV_HOP_OE, 1, P.TM_F16, link_prec)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps

    dslash_s = time_half(P.TM_F16, args.dslash_reps)
    dslash_f32_s = time_half(P.TM_F32, args.dslash_reps)
    # algorithmic bytes per output site and RHS (one read of the input field,
    # one write of the output, the 8 links of a site shared by the 12 RHS):
    #   reference model, FP32 links (18 parameters) / FP16 spinors:
    #     48 + 48 + 8 * 72 / 12 = 144 B
    #   this kernel's format, binary16 links with 12 parameters:
    #     48 + 48 + 8 * (LINK_PARAMS / 2) * 4 / 12 = 112 B
    ref_bytes = vh * nrhs * (48 + 48 + 8 * 72 / nrhs)
    own_bytes = vh * nrhs * (48 + 48 + 8 * (LINK_PARAMS // 2) * 4 / nrhs)
    achieved = ref_bytes / dslash_s / 1e9
    del bufs, outb

    # the other Dslash forms the solvers run: FP64 1 RHS (plain solve and
    # reliable updates), FP16 1 RHS (low-precision TSM solves without dilution)
    def time_dslash(prec, n, reps=100):
        nbytes = ctx.half_numel(prec, n)
        dt_ = torch.float64 if prec == P.TM_F64 else torch.float16
        ins = [torch.randn(nbytes // dt_.itemsize, dtype=dt_, device=dev) * 0.1 for _ in range(2)]
        o = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        for _ in range(10):
            ctx.dslash(o, ins[0], n, P.TM_RINV_HOP_OE, 1, prec)
        torch.cuda.synchronize()
        ev0.record()
        for r in range(reps):
            ctx.dslash(o, ins[r % 2], n, P.TM_RINV_HOP_OE, 1, prec)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps

    dslash_cases = {}
    for name, prec, n, site_rhs_bytes, fmt in (
            ("fp64_1rhs_12param_links", P.TM_F64, 1, 192 + 192 + 8 * 6 * 16, 12),
            ("fp64_1rhs_8param_links", P.TM_F64, 1, 192 + 192 + 8 * 4 * 16, 8),
            ("fp16_1rhs_12param_links", P.TM_F16, 1, 48 + 48 + 8 * 6 * 4, 12)):
        ctx.set_link_format(fmt)
        t_s = time_dslash(prec, n)
        b_ = vh * n * site_rhs_bytes
        dslash_cases[name] = {"us": t_s * 1e6, "algorithmic_bytes": b_,
                              "algorithmic_tb_s": b_ / t_s / 1e12, "frac_of_8tb_s": b_ / t_s / 8e12}
    ctx.set_link_format(LINK_PARAMS)
    dslash_cases["fp16_12rhs_12param_links"] = {
        "us": dslash_s * 1e6, "algorithmic_bytes": own_bytes, "algorithmic_tb_s": own_bytes / dslash_s / 1e12,
        "frac_of_8tb_s": own_bytes / dslash_s / 8e12}
    dslash_cases["fp16_12rhs_fp32_18param_links"] = {
        "us": dslash_f32_s * 1e6, "algorithmic_bytes": ref_bytes, "algorithmic_tb_s": ref_bytes / dslash_f32_s / 1e12,
        "frac_of_8tb_s": ref_bytes / dslash_f32_s / 8e12}

    # plain FP64 solve with 8-parameter links (same source, same process)
    ctx.set_link_format(8)
    b8 = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device=dev)
    e12 = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    ctx.noise(e12, seed_noise, 0, P.TM_DIL_SPIN_COLOUR)
    b8.copy_(e12[:1])
    del e12
    x8 = torch.zeros_like(b8)
    ctx.solve(x8, b8, 1, P.solve_params(tol=1e-9, solver=P.TM_CG_F64))  # warm
    t8 = []
    for _ in range(3):
        x8.zero_()
        torch.cuda.synchronize()
        tp = time.perf_counter()
        _, p8 = ctx.solve(x8, b8, 1, P.solve_params(tol=1e-9, solver=P.TM_CG_F64))
        torch.cuda.synchronize()
        t8.append(time.perf_counter() - tp)
    ctx.set_link_format(LINK_PARAMS)
    plain_8param = {"solves_per_s": 1.0 / float(np.median(t8)), "iters": p8[0].iters,
                    "true_rel_res": p8[0].true_rel_res}
    del x8, b8

    # practical streaming ceiling (and the calibration kernel for the HBM
    # byte counters): a device-to-device copy of 1 GiB each way
    csrc = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(10):
        cdst.copy_(csrc)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * csrc.numel() * 4 / (ev0.elapsed_time(ev1) / 1e3 / 10) / 1e9
    del csrc, cdst

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, S, L, kappa, eps, U, seed_noise, plain_iters)

    out = {
        "metric": "solves/s to 1e-9 rel. residual, 32^3x64 (plain vs chosen); Dslash HBM TB/s",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "32^3x64 twisted-mass Wilson, kappa 0.1245, 2 kappa mu 0.0014, links "
                        "exp(i 0.15 H) seed 103; per step 1 Z4 noise x 12 spin-colour "
                        "dilutions solved together (FP16 spinors, 12-parameter binary16 links, FP32 arithmetic, "
                        "FP64 reliable updates) to 1e-9, one-end loop contraction",
            "lattice": list(L), "rhs_per_step": nrhs, "parallelism": "single GPU",
        },
        "plain_solves_per_s": plain_value,
        "plain_seconds": plain_times,
        "plain_iters": plain_iters,
        "plain_8param_links": plain_8param,
        "chosen_fp32_links": f32_links,
        "chosen_iters_per_solve": chosen_iters,
        "speedup_vs_plain": value / plain_value,
        "dslash_tb_s": achieved / 1e3,
        "dslash_cases": dslash_cases,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_dslash (R_oo^-1 H_oe, 12 RHS, FP16 spinors, 12-parameter binary16 links, "
                      "autotuned RHS tile)",
            "avg_launch_us": dslash_s * 1e6,
            "bytes_model": "achieved and frac: reference bytes, 144 B per site-RHS (FP32 links with 18 "
                           "parameters, FP16 spinors) x 12 RHS x V/2 = %.3f GB per launch; own_*: the "
                           "bytes this kernel's format needs, 112 B per site-RHS (binary16 links, 12 "
                           "parameters) = %.3f GB" % (ref_bytes / 1e9, own_bytes / 1e9),
            "algorithmic_bytes_per_launch": ref_bytes,
            "own_bytes_per_launch": own_bytes, "own_achieved": own_bytes / dslash_s / 1e9,
            "own_frac": own_bytes / dslash_s / 1e9 / HBM_PEAK_GBS,
            "fp32_links_kernel_us": dslash_f32_s * 1e6,
            "fp32_links_kernel_frac": ref_bytes / dslash_f32_s / 1e9 / HBM_PEAK_GBS,
            "copy_gb_s": copy_gbs, "frac_of_copy": achieved / copy_gbs,
        },
        "cpu_baseline": cpu,
    }
    traffic = dslash_traffic(own_bytes, ref_bytes)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic["bytes"]
        out["roofline"]["traffic_source"] = traffic["source"]
        out["roofline"]["kernel"] = traffic["kernel"]
    if not args.no_extra:
        out["momentum_c3"] = momentum_leg(P, torch, dev, ctx, L, nrhs)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    if not args.no_extra:
        out["tsm_hpe_c2"] = tsm_leg(P, S, torch, dev)
        out["uneven_batch_c4"] = batch_leg(P, S, torch, dev)
        out["time_dilution_c2"] = time_dilution_leg(P, S, torch, dev)
    if not args.no_ptc:
        out["ptc_c5"] = ptc_leg(args, P, S, torch, dev)
    print(json.dumps(out), flush=True)


def momentum_leg(P, torch, dev, ctx, L, nrhs, p2max=9, reps=3):
    """Momentum projection on 32^3x64: standard and one-end loops of 12
    resident right-hand sides (complex128 fields) for every momentum with
    |n|^2 <= 9, against the per-slice (p = 0 only) contraction; and the
    paper's full loop output, 160 insertions (16 local + 64 one-derivative,
    one-end and generalised one-end) at the same momenta."""
    V = int(np.prod(L))
    g = torch.Generator(device=dev)
    g.manual_seed(7)
    eta = torch.randn((nrhs, V, 4, 3), dtype=torch.complex128, device=dev, generator=g)
    sol = torch.randn((nrhs, V, 4, 3), dtype=torch.complex128, device=dev, generator=g)
    est = P.TM_EST_STD | P.TM_EST_ONE_END
    n_mom = len(P.momenta(p2max))
    res = {"workload": "32^3x64, %d RHS, STD + one-end loops, %d momenta (|n|^2 <= %d); "
                       "160 insertions: one-end + generalised one-end, local + one-derivative"
                       % (nrhs, n_mom, p2max)}
    est160 = P.TM_EST_ONE_END | P.TM_EST_GEN_ONE_END
    for name, fn in (("per_slice", lambda: ctx.contract(eta, sol, nrhs, est)),
                     ("momentum", lambda: ctx.contract_momentum(eta, sol, nrhs, est, p2max)),
                     ("insertions160", lambda: ctx.contract_momentum(eta, sol, nrhs, est160, p2max,
                                                                    derivative=1))):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[name + "_ms"] = (time.perf_counter() - t) / reps * 1e3
    print("[bench/momentum] per-slice %.1f ms, %d momenta %.1f ms, 160 insertions x %d momenta "
          "%.1f ms" % (res["per_slice_ms"], n_mom, res["momentum_ms"], n_mom,
                       res["insertions160_ms"]), file=sys.stderr, flush=True)
    del eta, sol
    torch.cuda.empty_cache()
    return res


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(args, S, L, kappa, eps, U, seed_noise, plain_iters):
    """The FP64 oracle on the host cores (a reported baseline, not the
    target), on a bounded sample: per-CG-iteration time of the 32^3x64 solve
    at all threads and at one thread, scaled to the iteration count of the
    plain GPU solve; a full oracle solve of the 4^3x8 lattice; CG iterations
    of the 16^3x32 lattice."""
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    O.set_threads(threads)
    eta = O.noise_z4(L, seed_noise, 0)
    src = np.zeros_like(eta)
    src[:, 0, 0] = eta[:, 0, 0]  # first spin-colour dilution, as the plain GPU solve

    def per_iter(n_threads, k):
        O.set_threads(n_threads)
        tc = time.perf_counter()
        O.cgnr_iterations(L, kappa, eps, -1, U, src, 1)
        t1 = time.perf_counter() - tc
        tc = time.perf_counter()
        O.cgnr_iterations(L, kappa, eps, -1, U, src, 1 + k)
        t2 = time.perf_counter() - tc
        return (t2 - t1) / k, max(t1 - (t2 - t1) / k, 0.0), t1 + t2

    it_all, setup, t_all = per_iter(threads, args.cpu_iters)
    it_one, _, t_one = per_iter(1, 1)
    O.set_threads(threads)
    cpu_solve_s = setup + plain_iters * it_all
    tc = time.perf_counter()
    O.hop(L, kappa, -1, U, src)
    hop_s = time.perf_counter() - tc
    small = {}
    cf = S.CONFIGS["c1"]
    Uc = S.gauge_links(cf["L"], cf["eps_links"], cf["seed"])
    ec = O.noise_z4(cf["L"], S.NOISE_SEEDS["c1"], 0)
    tc = time.perf_counter()
    _, its, res = O.cgnr(cf["L"], cf["kappa"], cf["two_kappa_mu"], -1, Uc, ec, 1e-9)
    dt_c = time.perf_counter() - tc
    small["c1"] = {"lattice": list(cf["L"]), "iterations": int(its), "seconds": dt_c,
                   "solves_per_s": 1.0 / dt_c, "residual": float(res)}
    cf = S.CONFIGS["c2"]
    Uc = S.gauge_links(cf["L"], cf["eps_links"], cf["seed"])
    ec = O.noise_z4(cf["L"], S.NOISE_SEEDS["c2"], 0)
    tc = time.perf_counter()
    O.cgnr_iterations(cf["L"], cf["kappa"], cf["two_kappa_mu"], -1, Uc, ec, 1)
    ta = time.perf_counter() - tc
    tc = time.perf_counter()
    O.cgnr_iterations(cf["L"], cf["kappa"], cf["two_kappa_mu"], -1, Uc, ec, 6)
    tb = time.perf_counter() - tc
    small["c2"] = {"lattice": list(cf["L"]), "per_iteration_s": (tb - ta) / 5}
    model, nproc = cpu_info()
    full = None
    if args.cpu_full_solve:
        tc = time.perf_counter()
        _, its, res = O.cgnr(L, kappa, eps, -1, U, src, 1e-9)
        full = {"seconds": time.perf_counter() - tc, "iterations": int(its), "true_rel_res": float(res),
                "threads": threads}
        print("[bench] oracle 32^3x64 solve to 1e-9: %d iterations, %.1fs" % (its, full["seconds"]),
              file=sys.stderr, flush=True)
    return {"value": 1.0 / cpu_solve_s, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "nproc": nproc,
            "per_iteration_s": it_all, "per_iteration_s_1thread": it_one,
            "solves_per_s_1thread": 1.0 / (setup * threads + plain_iters * it_one),
            "full_lattice_hop_s": hop_s, "small_lattices": small, "full_solve": full,
            "sample": "FP64 oracle CGNR on the even-odd system, same source and lattice as the plain GPU "
                      "solve; %d + %d CG iterations timed at %d threads (%.1fs) and 1 + 1 at one thread "
                      "(%.1fs): %.2f s and %.2f s per iteration, scaled to the %d iterations the plain "
                      "FP64 GPU solve needed for 1e-9" % (1, 1 + args.cpu_iters, threads, t_all, t_one,
                                                          it_all, it_one, plain_iters)}


def make_context(P, S, torch, dev, name):
    cfg = S.CONFIGS[name]
    U = torch.from_numpy(S.gauge_links(cfg["L"], cfg["eps_links"], cfg["seed"])).to(dev)
    c = P.Context(cfg["L"], cfg["kappa"], cfg["two_kappa_mu"])
    c.set_gauge(U)
    torch.cuda.synchronize()
    return c, cfg


def tsm_leg(P, S, torch, dev):
    """Truncated Solver Method with the Hopping Parameter Expansion on the
    16^3x32 lattice: 64 Z4 volume noises (seed 202) without dilution, all 64
    solved to 1e-2 (low precision, no reliable update), the first 4 also to
    1e-9 (mixed CG); standard and HPE loops at every time slice.  Reports
    the cost of a high- and of a low-precision solve (the paper's
    high/low cost ratio) for FP16 and FP32 low-precision storage."""
    ctx, cfg = make_context(P, S, torch, dev, "c2")
    res = {"workload": "16^3x32, links exp(i 0.2 H) seed 102, kappa 0.124, 2 kappa mu 0.0028; "
                       "64 Z4 noises (seed 202), 4 high-precision (mixed CG to 1e-9) + 64 "
                       "low-precision (to 1e-2) solves; STD + HPE loops"}
    for name, lprec in (("lp_fp16", P.TM_F16), ("lp_fp32", P.TM_F32)):
        p = P.tm_loop_params()
        p.seed, p.n_hp, p.n_lp = S.NOISE_SEEDS["c2"], 4, 60
        p.dilution, p.estimators, p.mu_sign = P.TM_DIL_NONE, P.TM_EST_STD | P.TM_EST_HPE, 1
        p.hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
        p.lp = P.solve_params(tol=1e-2, solver=P.TM_CG_LOW, inner_prec=lprec)
        ctx.loops(p)  # warm (tuning, buffers)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, st, status = ctx.loops(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        it_hp, it_lp = st.iters_hp / st.n_solves_hp, st.iters_lp / st.n_solves_lp
        res[name] = {"seconds": dt, "n_solves_hp": st.n_solves_hp, "n_solves_lp": st.n_solves_lp,
                     "iters_per_hp_solve": it_hp, "iters_per_lp_solve": it_lp,
                     "hp_lp_iteration_ratio": it_hp / it_lp, "max_res_hp": st.max_res_hp,
                     "max_res_lp": st.max_res_lp, "status": status}
        print("[bench/tsm] %s: %d HP (%.0f it) + %d LP (%.1f it) solves in %.2fs"
              % (name, st.n_solves_hp, it_hp, st.n_solves_lp, it_lp, dt), file=sys.stderr, flush=True)
    ctx.close()
    return res


def time_dilution_leg(P, S, torch, dev):
    """Time dilution with coherent sources on 16^3x32 (the paper's strategy
    for heavier quarks): one Z4 noise (seed 202) split into 4 sources on the
    slices t = o (mod 4) (8 slices apart) x 12 spin-colour components, 48
    mixed-CG solves to 1e-9 in batches of 12, STD + HPE loops with the
    single-time-slice contraction; against the same noise as volume sources
    (12 solves)."""
    ctx, cfg = make_context(P, S, torch, dev, "c2")
    res = {"workload": "16^3x32, links exp(i 0.2 H) seed 102, kappa 0.124, 2 kappa mu 0.0028; 1 Z4 "
                       "noise x 12 spin-colour, time dilution period 4 (48 sources) vs volume "
                       "sources (12); mixed CG to 1e-9; STD + HPE loops"}
    for name, period in (("period4", 4), ("volume", 0)):
        p = P.tm_loop_params()
        p.seed, p.n_hp, p.n_lp = S.NOISE_SEEDS["c2"], 1, 0
        p.dilution, p.estimators, p.mu_sign = P.TM_DIL_SPIN_COLOUR, P.TM_EST_STD | P.TM_EST_HPE, 1
        p.t_period = period
        p.hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
        ctx.loops(p)  # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, st, status = ctx.loops(p)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        res[name] = {"seconds": dt, "n_solves": st.n_solves_hp,
                     "iters_per_solve": st.iters_hp / st.n_solves_hp, "max_res": st.max_res_hp,
                     "solves_per_s": st.n_solves_hp / dt, "status": status}
        print("[bench/tdil] %s: %d solves (%.0f it) in %.2fs" % (name, st.n_solves_hp,
              st.iters_hp / st.n_solves_hp, dt), file=sys.stderr, flush=True)
    ctx.close()
    return res


def batch_leg(P, S, torch, dev):
    """Uneven batch: 8^3x16 / 12^3x24 / 16^3x32 lattices with 4 / 2 / 1 Z4
    noises x 12 spin-colour dilutions (48 / 24 / 12 right-hand sides), mixed
    CG to 1e-9 and standard + one-end loops, solved as one batch (the
    library's timed choice between the persistent kernel and the graph of
    multi-instance launches; each form also forced and timed) and, for
    comparison, lattice by lattice."""
    names = ("c4a", "c4b", "c4c")
    ctxs = [make_context(P, S, torch, dev, n)[0] for n in names]
    hp = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)

    def lp_of(k, n_hp):
        p = P.tm_loop_params()
        p.seed, p.n_hp, p.n_lp = 1040 + k, n_hp, 0
        p.dilution, p.estimators, p.mu_sign = P.TM_DIL_SPIN_COLOUR, P.TM_EST_STD | P.TM_EST_ONE_END, 1
        p.hp = hp
        return p
    plist = [lp_of(k, n) for k, n in enumerate((4, 2, 1))]

    def timed_batch(form):
        # form: None = the library's timed choice, "1" persistent kernel, "0" graph
        old = os.environ.get("TM_BATCH_PERSIST")
        if form is not None:
            os.environ["TM_BATCH_PERSIST"] = form
        try:
            batch = P.Batch(ctxs)
        finally:
            if form is not None:
                if old is None:
                    os.environ.pop("TM_BATCH_PERSIST")
                else:
                    os.environ["TM_BATCH_PERSIST"] = old
        batch.loops(plist)  # warm (and, for the timed choice, one group of each form)
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st, _ = batch.loops(plist)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        batch.close()
        return dt, st
    tb, bst = timed_batch(None)
    tp, _ = timed_batch("1")
    tg, _ = timed_batch("0")
    for c, p in zip(ctxs, plist):
        c.loops(p)  # warm
    torch.cuda.synchronize()
    t = time.perf_counter()
    sst = [c.loops(p)[2] for c, p in zip(ctxs, plist)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t
    n = sum(q.n_solves_hp for q in bst)
    ok = all(q.max_res_hp <= 1e-9 for q in bst) and all(q.max_res_hp <= 1e-9 for q in sst)
    for c in ctxs:
        c.close()
    print("[bench/batch] %d solves: batch %.3fs, lattice by lattice %.3fs" % (n, tb, ts),
          file=sys.stderr, flush=True)
    return {"workload": "8^3x16 / 12^3x24 / 16^3x32 (links 0.3/0.2/0.15, seeds 1041-1043, kappa "
                        "0.124, 2 kappa mu 0.005), 48/24/12 RHS, mixed CG to 1e-9, STD + one-end loops",
            "solves": n, "all_verified": ok, "batch_seconds": tb, "batch_solves_per_s": n / tb,
            "persistent_kernel_seconds": tp, "graph_seconds": tg,
            "sequential_seconds": ts, "sequential_solves_per_s": n / ts, "speedup": ts / tb,
            "iters": [q.iters_hp for q in bst]}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dslash_rinv_hop_12rhs_fp16_c3_traffic.json")
LINK_PARAMS = 12  # binary16 link format of the timed Dslash (two rows stored)


def dslash_traffic(own_bytes, ref_bytes):
    """HBM bytes per launch of the timed Dslash from the committed counter
    summary (FETCH_SIZE x its copy calibration + WRITE_SIZE x its), or None
    when the kernel source has changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    src = open(os.path.join(ROOT, "paper_1309_2256_amd", "csrc", "dslash.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["dslash_hip_sha256"]:
        return None
    b = (rec["fetch_kib_per_dispatch"] * rec["fetch_factor"] +
         rec["write_kib_per_dispatch"] * rec["write_factor"]) * 1024
    return {"bytes": b, "kernel": rec["kernel"],
            "source": os.path.relpath(TRAFFIC_FILE, ROOT) + " (%.2f x own bytes, %.2f x reference bytes)" % (
                b / own_bytes, b / ref_bytes)}


def ptc_leg(args, P, S, torch, dev):
    """Learned preconditioner on the 32^3x64 lattice with 16^3x32-lattice
    physics (links exp(i 0.2 H), kappa 0.124, 2 kappa mu 0.0028).  Training
    on the 16^3x32 lattice of the same physics (the network is a local
    stencil, its weights carry over to any volume): pairs from the mixed CG's
    own iterates (Z4 spin-colour-diluted sources, (b - M x_k, x* - x_k) at
    k = 8, 16, 32, 64, BF16 store), residual loss |M N(r) - r|^2 / |r|^2,
    Adam, from the second-order hopping expansion.  Then all 24 right-hand
    sides (2 noises x 12) solved to 1e-9 on 32^3x64 by mixed CG (12 per call)
    and by FGMRES(16) with the trained network on the matrix cores (BF16),
    with the trained network in FP32, with the analytic start, and without
    a network."""
    def log(msg):
        print("[bench/ptc] " + msg, file=sys.stderr, flush=True)

    def make(name):
        return make_context(P, S, torch, dev, name)

    res = {}
    c2, cfg2 = make("c2")
    V2 = int(np.prod(cfg2["L"]))
    iters = [8, 16, 32, 64]
    n_src = max(args.ptc_pairs // (12 * len(iters)), 1)
    c2.ptc_pairs_reserve(n_src * 12 * len(iters), P.TM_BF16)
    eta = torch.zeros((12, V2, 4, 3), dtype=torch.complex128, device=dev)
    mixed = P.solve_params(tol=1e-9, solver=P.TM_CG_MIXED, inner_prec=P.TM_F16)
    t0 = time.perf_counter()
    npairs = 0
    for k in range(n_src):
        c2.noise(eta, 9000, k, P.TM_DIL_SPIN_COLOUR)
        npairs += c2.ptc_pairs_from_solve(eta, 12, mixed, iters)
    torch.cuda.synchronize()
    res["pairs"] = npairs
    res["pairs_iterations"] = iters
    res["pairs_seconds"] = time.perf_counter() - t0
    log("%d iterate pairs in %.1fs" % (npairs, res["pairs_seconds"]))
    del eta
    c2.ptc_init_hopping(nc=12, mu_sign=1, seed=1, noise=1e-3)
    W1h, W2h = c2.ptc_get_weights(12)
    st, _ = c2.ptc_train(epochs=2, batch=16, lr=1e-3, seed=3, loss=P.TM_PTC_LOSS_RESIDUAL, mu_sign=1)
    res["train"] = {"loss": "residual |M N(r) - r|^2 / |r|^2", "steps": st.steps, "batch": 16, "epochs": 2,
                    "loss_first_epoch": st.loss_first, "loss_last_epoch": st.loss_last, "seconds": st.seconds}
    log("trained: loss %.4f -> %.4f in %.1fs" % (st.loss_first, st.loss_last, st.seconds))
    W1t, W2t = c2.ptc_get_weights(12)
    c2.close()
    del c2
    torch.cuda.empty_cache()

    c5, cfg5 = make("c5")
    V5 = int(np.prod(cfg5["L"]))
    b = torch.zeros((12, V5, 4, 3), dtype=torch.complex128, device=dev)
    x = torch.zeros_like(b)

    def run24(name, params):
        tot, n_ok, its, worst, fb = 0.0, 0, [], 0.0, 0
        for k in range(2):
            c5.noise(b, 505, k, P.TM_DIL_SPIN_COLOUR)
            x.zero_()
            torch.cuda.synchronize()
            t = time.perf_counter()
            status, stats = c5.solve(x, b, 12, params, allow_noconv=True)
            torch.cuda.synchronize()
            tot += time.perf_counter() - t
            n_ok += sum(1 for s_ in stats if s_.true_rel_res <= 1e-9)
            its += [s_.iters for s_ in stats]
            worst = max(worst, max(s_.true_rel_res for s_ in stats))
            fb += sum(s_.fallback for s_ in stats)
        r = {"rhs": 24, "verified": n_ok, "solves_per_s": n_ok / tot, "iters_mean": float(np.mean(its)),
             "max_true_rel_res": worst, "seconds": tot, "fallbacks": fb}
        log("%s: %d/24 verified, %.1f iterations, %.2fs" % (name, n_ok, r["iters_mean"], tot))
        return r

    res["mixed_cg"] = run24("mixed CG", mixed)
    res["plain_cg_f64"] = run24("plain FP64 CG", P.solve_params(tol=1e-9, solver=P.TM_CG_F64))
    fg = dict(tol=1e-9, check_every=16, maxiter=3000)
    c5.ptc_set_weights(W1t, W2t)
    c5.ptc_set_arith(P.TM_BF16)
    res["fgmres_ptc_trained_bf16"] = run24("FGMRES(16)+network (trained, BF16 matrix cores)",
                                           P.solve_params(solver=P.TM_FGMRES_PTC, **fg))
    c5.ptc_set_arith(P.TM_F32)
    res["fgmres_ptc_trained_f32"] = run24("FGMRES(16)+network (trained, FP32)",
                                          P.solve_params(solver=P.TM_FGMRES_PTC, **fg))
    c5.ptc_set_weights(W1h, W2h)
    res["fgmres_ptc_hopping_init"] = run24("FGMRES(16)+network (hopping-expansion weights)",
                                           P.solve_params(solver=P.TM_FGMRES_PTC, **fg))
    res["fgmres_no_net"] = run24("FGMRES(16) without network", P.solve_params(solver=P.TM_FGMRES, **fg))
    res["workload"] = ("32^3x64, links exp(i 0.2 H) seed 105, kappa 0.124, 2 kappa mu 0.0028; "
                       "Z4 noise seed 505, 2 noises x 12 spin-colour dilutions = 24 RHS per solver, "
                       "12 per call; network trained on 16^3x32 of the same physics")
    c5.close()
    return res


if __name__ == "__main__":
    main()
