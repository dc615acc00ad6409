"""Benchmark: solves/s to 1e-9 relative residual on a 32^3 x 64 twisted-mass
lattice, chosen (multi-RHS mixed precision) vs plain (FP64 CG), and the HBM
throughput of the multi-RHS half-lattice Dslash.

One step = one pass of the hot path over one batch: a Z4 noise vector with
12 spin-colour dilutions generated on the GPU, even-odd source preparation,
12 right-hand sides solved together by CG on the normal equations with FP16
spinor storage / FP32 links and arithmetic and FP64 reliable updates to a
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
    ap.add_argument("--dslash-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
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

    # plain: FP64 CG, one right-hand side at a time (the first dilution of noise 0)
    b = torch.zeros((1, V, 4, 3), dtype=torch.complex128, device=dev)
    eta12 = torch.zeros((12, V, 4, 3), dtype=torch.complex128, device=dev)
    ctx.noise(eta12, seed_noise, 0, P.TM_DIL_SPIN_COLOUR)
    b.copy_(eta12[:1])
    del eta12
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    _, pst = ctx.solve(x, b, 1, P.solve_params(tol=1e-9, solver=P.TM_CG_F64))
    torch.cuda.synchronize()
    plain_time = time.perf_counter() - tp
    plain_value = 1.0 / plain_time
    plain_iters = pst[0].iters
    print("[bench] plain FP64 solve: %d iterations, residual %.2e, %.2fs"
          % (plain_iters, pst[0].true_rel_res, plain_time), file=sys.stderr, flush=True)
    del x, b

    # dominant kernel: 12-RHS half-lattice Dslash R^-1 H (FP16 spinors, FP32 links)
    vh = V // 2
    nb = ctx.half_numel(P.TM_F16, nrhs)
    bufs = [torch.randn(nb // 2, dtype=torch.float16, device=dev) * 0.1 for _ in range(2)]
    outb = torch.empty(nb, dtype=torch.uint8, device=dev)
    for _ in range(3):
        ctx.dslash(outb, bufs[0], nrhs, P.TM_RINV_HOP_OE, 1, P.TM_F16)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for r in range(args.dslash_reps):
        ctx.dslash(outb, bufs[r % 2], nrhs, P.TM_RINV_HOP_OE, 1, P.TM_F16)
    ev1.record()
    torch.cuda.synchronize()
    dslash_s = ev0.elapsed_time(ev1) / 1e3 / args.dslash_reps
    # compulsory bytes per output site and RHS: 8 neighbour spinors are one
    # read of the input field (12 complex FP16 = 48 B), one output write
    # (48 B), 8 FP32 links per site (576 B) shared by 12 RHS (48 B)
    bytes_per_site_rhs = 48 + 48 + 8 * 9 * 8 / nrhs
    alg_bytes = vh * nrhs * bytes_per_site_rhs
    achieved = alg_bytes / dslash_s / 1e9
    del bufs, outb

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
        import oracle as O
        eta = O.noise_z4(L, seed_noise, 0)
        src = np.zeros_like(eta)
        src[:, 0, 0] = eta[:, 0, 0]  # first spin-colour dilution, as the plain GPU solve
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        tc = time.perf_counter()
        O.cgnr_iterations(L, kappa, eps, -1, U, src, 1)
        t1 = time.perf_counter() - tc
        tc = time.perf_counter()
        O.cgnr_iterations(L, kappa, eps, -1, U, src, 1 + args.cpu_iters)
        t2 = time.perf_counter() - tc
        per_iter = (t2 - t1) / args.cpu_iters
        setup = max(t1 - per_iter, 0.0)
        cpu_solve_s = setup + plain_iters * per_iter
        cpu = {"value": 1.0 / cpu_solve_s, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": "FP64 oracle CGNR on the even-odd system, same source and lattice; "
                         "%d + %d CG iterations timed (%.1fs), %.2fs per iteration, scaled "
                         "to the %d iterations the plain FP64 GPU solve needed for 1e-9"
                         % (1, 1 + args.cpu_iters, t1 + t2, per_iter, plain_iters)}

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
                        "dilutions solved together (FP16 spinors, FP32 links and arithmetic, "
                        "FP64 reliable updates) to 1e-9, one-end loop contraction",
            "lattice": list(L), "rhs_per_step": nrhs, "parallelism": "single GPU",
        },
        "plain_solves_per_s": plain_value,
        "plain_iters": plain_iters,
        "chosen_iters_per_solve": chosen_iters,
        "speedup_vs_plain": value / plain_value,
        "dslash_tb_s": achieved / 1e3,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "k_dslash<h2,float2,float,2,0,0> (R_oo^-1 H_oe, 12 RHS)",
            "avg_launch_us": dslash_s * 1e6, "algorithmic_bytes_per_launch": alg_bytes,
            "copy_gb_s": copy_gbs, "frac_of_copy": achieved / copy_gbs,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
