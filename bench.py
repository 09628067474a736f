"""Benchmark of the MPS lattice Boltzmann step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload vascular128]

A step is one full D3Q19 MPS-LBM step (moments, 1/rho, variational
products, BGK sums, streaming, open faces, bounce-back, all roundings) on
the synthetic workload, inputs resident in HBM.  The default workload is
the 128^3 branching-tube configuration at chi = 128 with BF16X3
contractions (the largest configuration of the target that one GPU runs
whole); the 64^3 porous medium at chi = 64 (FP32), the 256^3 Taylor-Green
vortex on D3Q15 at chi = 128 and the 128^3 pin array (tensor-product mask,
ramped inlet, Delta p / p_0 over the inflow region) at chi = 128 are timed
as extra fields.  Prints one JSON line.
"""
import argparse
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MPS-LBM steps/s & equiv. MLUPS at fixed chi vs plain FP64 path; MFMA util"

# MI355X published peaks
PEAK = {"hbm_gbs": 8000.0, "fp64_tflops": 78.6, "fp32_tflops": 157.3, "bf16_tflops": 2500.0}


def make_case(name):
    import workloads as WL
    if name == "porous64":
        # 64^3 random spheres (radius 4-8, 30 % solid), pressure-driven in x,
        # chi = 64, FP32 (the structured porous medium configuration)
        return WL.case_porous(n=6, chi=64, tau=0.6, tol=1e-8, precision="fp32")
    if name == "porous32":
        return WL.case_porous(n=5, chi=32, tau=0.6, tol=1e-8, precision="fp32")
    if name == "channel16":
        return WL.case_channel()
    if name == "tgv256":
        # Taylor-Green vortex of Sections 4.1 / 5.1: 256^3, Re 800,
        # Ma = 0.1 / c_s, D3Q15, chi = 128, BF16X3 contractions
        return WL.case_tgv(n=8, chi=128, re=800.0, tol=1e-8, precision="bf16x3")
    if name == "pinfin128":
        # pin array (8^3 layout of 16^3 pins, mask as their tensor product),
        # inlet ramped as u_0 (1 - e^(-1.5 t)) with t in flow-through times
        # L / u_0 = 128 / 0.02 steps, chi = 128, BF16X3
        c = WL.case_pinfin(n=7, l=3, chi=128, tau=0.56, u_in=0.02, tol=1e-8,
                           precision="bf16x3")
        c.face_profile = {0: ((0.0, 1.0, 1.5, 0.0, 0.0, 0.0), 0.02 / 128.0)}
        return c
    if name == "vascular128":
        # 128^3 branching tube tree, velocity inlet 0.02 / pressure outlet,
        # chi = 128, contractions on BF16 MFMA with three-term operand
        # splitting and FP32 accumulation (FP32 storage and factorisations)
        return WL.case_vascular(n=7, chi=128, tau=0.55, tol=1e-8, precision="bf16x3")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(case, roundings_per_step, products_per_step, budget_s=20.0):
    """The CPU oracle (FP64 numpy MPS path) timed on a bounded sample of the
    workload: roundings of sums of two MPS and variational products at the
    workload's bond profile (bond min(chi, 8^k, 8^(n-k))), repeated for
    about budget_s; the step rate is extrapolated with the per-step counts
    of roundings and products the library reports for the same workload."""
    import numpy as np
    from oracle import mps as M
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    rng = np.random.default_rng(2512)
    n, chi = case.n, case.chi
    b = [1] + [min(chi, 8 ** k, 8 ** (n - k)) for k in range(1, n)] + [1]

    def rand_mps():
        return [rng.standard_normal((b[k], 8, b[k + 1])) / 8.0 for k in range(n)]

    x, y = rand_mps(), rand_mps()
    t_round, k_round = 0.0, 0
    t_prod, k_prod = 0.0, 0
    t_start = time.perf_counter()
    while time.perf_counter() - t_start < budget_s or k_round == 0 or k_prod == 0:
        t0 = time.perf_counter()
        M.round_mps(M.add(x, y), chi, case.tol)
        t_round += time.perf_counter() - t0
        k_round += 1
        t0 = time.perf_counter()
        M.hadamard_variational(x, y)
        t_prod += time.perf_counter() - t0
        k_prod += 1
    per_step = roundings_per_step * t_round / k_round + products_per_step * t_prod / k_prod
    return {"value": 1.0 / per_step, "unit": "steps/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{k_round} roundings (sum of two MPS, bonds {b[1:-1]}) and {k_prod} "
                      f"variational products of the CPU FP64 MPS oracle on {case.name}, "
                      f"scaled by {roundings_per_step} roundings + {products_per_step} "
                      f"products per step (initialisation excluded)"}


def batched_rate(case, count, stream, steps):
    """Domain-steps/s of `count` domains of the workload (the same geometry
    generator with different seeds) held by one handle and advanced
    together; one untimed step first."""
    import dataclasses
    import torch
    import workloads as WL
    from paper_2512_07615_amd import mps_lbm as L
    cases = [case]
    for k in range(1, count):
        if case.name.startswith("porous"):
            cases.append(WL.case_porous(n=case.n, chi=case.chi, tau=case.tau, tol=case.tol,
                                        precision=case.precision, seed=2514 + 100 * k))
        else:
            cases.append(dataclasses.replace(case))
    b = L.BatchSimulation(cases, hip_stream=stream.cuda_stream)
    b.step(1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    b.close()
    return {"domains": count, "steps": steps, "ms_per_step": ms,
            "domain_steps_per_s": count * 1000.0 / ms,
            "equiv_mlups": count * case.N ** 3 * 1000.0 / ms / 1e6}


def c4_rate(stream, steps, progress):
    """48 seeded domains of mixed size (32^3 to 128^3), bond dimension (32 to
    128) and policy (FP32, BF16X3) in one handle: the groups of equal shape
    run as batched engines on streams of their own, and the whole step is
    replayed as one HIP graph.  Returns domain-steps/s and the groups."""
    import torch
    import workloads as WL
    from paper_2512_07615_amd import mps_lbm as L
    cases = WL.c4_cases()
    t0 = time.time()
    b = L.BatchSimulation(cases, hip_stream=stream.cuda_stream)
    torch.cuda.synchronize()
    init_s = time.time() - t0
    progress(f"c4: 48 domains initialised in {init_s:.1f} s")
    b.capture()            # one eager step, then the next one recorded
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nonfinite = sum(b.observables(d).nonfinite for d in range(len(cases)))
    b.close()
    groups = sorted({(c.n, c.chi, c.precision) for c in cases})
    cells = sum(c.N ** 3 for c in cases)
    return {"domains": len(cases), "groups": len(groups), "steps": steps, "ms_per_step": ms,
            "domain_steps_per_s": len(cases) * 1000.0 / ms,
            "equiv_mlups": cells * 1000.0 / ms / 1e6, "init_s": init_s,
            "hip_graph": True, "nonfinite": nonfinite}


def stored_traffic(kind, workload):
    """HBM bytes per launch of the roofline kernel from the committed
    rocprofv3 counter summary (profiles/<workload>_<kind>_hbm_traffic.md),
    when it exists and the kernel's sources still hash to what was
    measured; else None."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", f"{workload}_{kind}_hbm_traffic.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(source_sha256|traffic_bytes_per_launch): (\S+)$", text, re.M))
    h = hashlib.sha256()
    for f in ("paper_2512_07615_amd/csrc/linalg.h", "paper_2512_07615_amd/csrc/common.h"):
        h.update(open(os.path.join(root, f), "rb").read())
    if fields.get("source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def roofline(kind, ks, prec):
    """Roofline entry of the timed kernel class from its event-timed launches
    and device-counted algorithmic flops."""
    avg_ms = ks.total_ms / max(ks.launches, 1)
    flops_per_launch = ks.flops / max(ks.launches, 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    if kind == "prodgemm":
        bound = "mfma"
        peak = {"fp32": PEAK["fp32_tflops"], "bf16": PEAK["bf16_tflops"],
                "bf16x3": PEAK["bf16_tflops"]}.get(prec, PEAK["fp64_tflops"])
    else:
        # FP64 vector ALU: 256 CUs x 2.4 GHz x 128 FP64 flops/clock/CU
        bound, peak = "alu", PEAK["fp64_tflops"]
    return {"bound": bound, "kernel": kind, "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
            "launches": ks.launches, "avg_launch_ms": avg_ms,
            "flops_per_launch": flops_per_launch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="vascular128")
    ap.add_argument("--extra-workload", default="porous64,tgv256,pinfin128",
                    help="also time these workloads' steps (comma-separated; empty = skip)")
    ap.add_argument("--extra-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--graph-steps", type=int, default=3,
                    help="steps timed as HIP graph replays")
    ap.add_argument("--batch", type=int, default=0,
                    help="also time this many domains of the workload advanced together "
                         "(0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--c4-steps", type=int, default=2,
                    help="graph-replayed steps of the 48 mixed domains (0 = skip)")
    ap.add_argument("--mfma-steps", type=int, default=2,
                    help="steps timed for the MFMA utilisation of the product GEMMs")
    ap.add_argument("--no-graph", action="store_true",
                    help="issue the step kernel by kernel instead of replaying a HIP graph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain elementwise copy of 256 MiB three times (the "
                         "reference for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default split-K shares instead of tuning them after the "
                         "warm-up steps")
    ap.add_argument("--predictor-steps", type=int, default=3,
                    help="steps timed with the rank-predicted randomized truncation "
                         "(0 = skip; FP32/BF16 workloads)")
    ap.add_argument("--roofline-kernel", default="jacobi",
                    choices=["jacobi", "householder", "prodgemm", "cholesky"])
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (N=1); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2512_07615_amd import mps_lbm as L

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    case = make_case(args.workload)
    stream = torch.cuda.Stream()
    if args.copy_calibration:
        # y = x * 1 over 256 MiB of FP32: reads and writes 256 MiB per launch
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y
        progress("copy calibration: 3 launches of 256 MiB read + 256 MiB written")
    t_init = time.perf_counter()
    sim = L.Simulation(case, hip_stream=stream.cuda_stream)
    progress(f"{case.name}: initialised in {time.perf_counter() - t_init:.1f} s")
    for _ in range(args.warmup):
        sim.step(1)
        torch.cuda.synchronize()
        progress("warm-up step done")
    torch.cuda.synchronize()
    tuned = 0
    if not args.no_autotune and args.warmup > 0:
        tuned = sim.autotune()
        progress(f"autotuned {tuned} contraction classes")
    kind = {"jacobi": L.K_JACOBI, "householder": L.K_HOUSEHOLDER,
            "prodgemm": L.K_PRODGEMM, "cholesky": L.K_CHOLESKY}[args.roofline_kernel]
    sim.kernel_timing(kind)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        sim.step(1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    progress(f"timed {args.steps} steps: {ms:.1f} ms/step")
    ks = sim.kernel_stats()
    obs = sim.observables()
    sps = 1000.0 / ms
    N3 = case.N ** 3
    out = {
        "metric": METRIC, "value": sps, "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64", "bf16": "bf16-mfma/f32",
                  "bf16x3": "bf16x3-mfma/f32"}[case.precision],
        "data": "synthetic",
        "config": {"workload": case.name, "n": case.n, "chi": case.chi, "tau": case.tau,
                   "tol": case.tol, "geometry": case.meta,
                   "equiv_mlups": N3 * sps / 1e6, "max_bond": obs.max_bond,
                   "mask_bond": obs.mask_bond, "mask_trunc_err": obs.mask_trunc_err,
                   "roundings_per_step": obs.roundings, "products_per_step": obs.products,
                   "jacobi_sweeps_mean": obs.jacobi_sweeps,
                   "jacobi_sweeps_wide": obs.jacobi_sweeps_wide,
                   "jacobi_cols_wide": obs.jacobi_cols_wide,
                   "jacobi_sweep_limit_hits": obs.svd_failures,
                   "lds_bytes": obs.lds_bytes, "autotuned_classes": tuned,
                   "compression": obs.compression, "face_trunc_err": obs.face_trunc_err,
                   "inverse_density": "taylor2, FP64 island"},
    }
    out["roofline"] = roofline(args.roofline_kernel, ks, case.precision)
    out["roofline"]["traffic"] = stored_traffic(args.roofline_kernel, args.workload)
    out["roofline"]["share_of_step"] = ks.total_ms / (ms * args.steps)
    if args.mfma_steps > 0:
        # MFMA utilisation of the product contractions, timed the same way
        sim.kernel_timing(L.K_PRODGEMM)
        e0.record(stream)
        for _ in range(args.mfma_steps):
            sim.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        mms = e0.elapsed_time(e1) / args.mfma_steps
        kp = sim.kernel_stats()
        out["roofline_mfma"] = roofline("prodgemm", kp, case.precision)
        out["roofline_mfma"]["share_of_step"] = kp.total_ms / (mms * args.mfma_steps)
        if case.precision == "bf16x3":
            # achieved counts one useful product per multiply-add; the
            # matrix cores run six BF16 products for each (three-term split)
            rm = out["roofline_mfma"]
            rm["mfma_products_per_useful"] = 6
            rm["matrix_core_frac"] = 6 * rm["frac"]
    if not args.no_graph and args.graph_steps > 0:
        # the same step recorded once as a HIP graph and replayed (the timed
        # region above issues it kernel by kernel, with per-launch events)
        sim.kernel_timing(L.K_NONE)
        sim.capture()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.graph_steps):
            sim.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / args.graph_steps
        out["config"]["hip_graph_steps_per_s"] = 1000.0 / gms
        progress(f"graph replay: {gms:.1f} ms/step")
    sim.close()
    if args.predictor_steps > 0 and case.precision != "fp64":
        # the same workload with the rank predictor on: two steps to seed the
        # predictions, then timed steps; acceptance counts are totals
        simp = L.Simulation(case, hip_stream=stream.cuda_stream, rank_predictor=1)
        for _ in range(2):
            simp.step(1)
        torch.cuda.synchronize()
        o0 = simp.observables()
        e0.record(stream)
        for _ in range(args.predictor_steps):
            simp.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / args.predictor_steps
        o1 = simp.observables()
        att = o1.rs_attempted - o0.rs_attempted
        out["config"]["rank_predictor"] = {
            "steps_per_s": 1000.0 / pms, "speedup": ms / pms,
            "sketches_per_step": att / args.predictor_steps,
            "accepted_frac": (o1.rs_accepted - o0.rs_accepted) / att if att else 0.0,
            "max_bond": o1.max_bond}
        simp.close()
        progress(f"rank predictor: {pms:.1f} ms/step")
    if args.fp64_steps > 0 and case.precision != "fp64":
        sim64 = L.Simulation(case, precision="fp64", hip_stream=stream.cuda_stream)
        sim64.step(1)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.fp64_steps):
            sim64.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1) / args.fp64_steps
        out["config"]["fp64_steps_per_s"] = 1000.0 / ms64
        out["config"]["speedup_vs_fp64_path"] = ms64 / ms
        sim64.close()
        progress(f"FP64 policy: {ms64:.1f} ms/step")
    if args.batch > 0:
        out["config"]["batched"] = batched_rate(case, args.batch, stream, args.batch_steps)
    if args.c4_steps > 0:
        out["config"]["c4_mixed_domains"] = c4_rate(stream, args.c4_steps, progress)
        progress(f"c4: {out['config']['c4_mixed_domains']['ms_per_step']:.0f} ms per step")
    extras = [w for w in (args.extra_workload or "").split(",") if w and w != args.workload]
    if extras and args.extra_steps > 0:
        out["config"]["extra"] = []
    for wname in (extras if args.extra_steps > 0 else []):
        xc = make_case(wname)
        progress(f"{xc.name}: init")
        xs = L.Simulation(xc, hip_stream=stream.cuda_stream)
        if wname == "pinfin128":
            # Delta p / p_0 over the inflow region of Section 4.2 (x < 2 L / 256,
            # y, z < L / 2)
            xs.set_region((0, 0, 0), (1, 64, 64), 1.0)
        xs.step(1)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.extra_steps):
            xs.step(1)
        e1.record(stream)
        torch.cuda.synchronize()
        xms = e0.elapsed_time(e1) / args.extra_steps
        xo = xs.observables()
        rec = {"workload": xc.name, "precision": xc.precision, "lattice": f"D3Q{xc.lattice}",
               "chi": xc.chi, "steps_per_s": 1000.0 / xms, "ms_per_step": xms,
               "equiv_mlups": xc.N ** 3 * 1000.0 / xms / 1e6,
               "mask_bond": xo.mask_bond, "max_bond": xo.max_bond,
               "compression": xo.compression, "steps_taken": int(xo.step)}
        if wname == "tgv256":
            rec["e_kin"] = xs.kinetic_energy()
        if wname == "pinfin128":
            rec["dp_p0_inflow"] = xo.dp_p0
        xs.close()
        out["config"]["extra"].append(rec)
        progress(f"{xc.name}: {xms:.1f} ms/step")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, obs.roundings, obs.products)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
