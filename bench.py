"""Throughput of the adaptive Hessian-sketch ridge solver on one MI355X.

Default workload (one "step"): the 2^21 x 8192 FP32 problem (64 GiB) A = G
diag(sigma) V^T with sigma_i = 1/i, G i.i.d. N(0, 1/n), V Haar, b = A x_pl +
0.1 xi (seed 5), solved by Algorithm 1 (SRHT, rho = 0.1, FP64 factor and
control) to the decrement tolerance, once at nu^2 = 1e-2 and once at nu^2 =
1e-4, one solve after the other on one stream.

The reported value is the learned form with BF16 sketches (features, MLP
prediction of the starting m, then Algorithm 1 with the doubling rule as the
fallback).  Beside it: the plain method (FP32 sketch, m from 1) on the same
problem in the same process (--plain-steps steps), the roofline of the gradient
pass (one more step with every gradient launch bracketed by HIP events on its
stream) and of the SRHT at the learned starting sizes.  Inputs are resident in
HBM before timing.  Every timed solve is judged afterwards by the oracle's
streamed certificate, an upper bound on delta(x)/delta(0) from one FP64 pass over
the stored A (verified when <= 1e-6), and the oracle's direct solve is timed on
a row sample of the same problem.

Other workloads (--workload): c2 (65536 x 1024), c3 (precision form), c4a (nu
grid), c4b (uneven batch), path, dual, refreshed, sparse.

Prints one JSON line: the throughput, the dominant kernel's roofline (live HIP
events; traffic from the counter passes when given) and the oracle's CPU rate.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N, D = 65536, 1024
NU2S = (1e-2, 1e-4)
HBM_PEAK_GBS = 8000.0


def with_error_roots(obj):
    """Every relative prediction error field (delta(x)/delta(0), a squared norm
    ratio) gets its square root beside it as <key>_sqrt, at any depth."""
    if isinstance(obj, dict):
        out = {}
        for k, v in obj.items():
            out[k] = with_error_roots(v)
            if "rel_pred_err" in k and not k.endswith("_sqrt") and k + "_sqrt" not in obj:
                if isinstance(v, (int, float)):
                    out[k + "_sqrt"] = math.sqrt(max(v, 0.0))
                elif isinstance(v, dict) and all(isinstance(x, (int, float)) for x in v.values()):
                    out[k + "_sqrt"] = {kk: math.sqrt(max(x, 0.0)) for kk, x in v.items()}
        return out
    if isinstance(obj, list):
        return [with_error_roots(v) for v in obj]
    return obj


def emit(line):
    print(json.dumps(with_error_roots(line)))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--workers", type=int, default=8,
                    help="worker streams for the uneven batch (c4b)")
    ap.add_argument("--graph-steps", action="store_true",
                    help="batched solves replay each job's queued steps from HIP graphs")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", default="polyak", choices=["polyak", "gd"])
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--mode", default="learned-bf16",
                    choices=["learned-bf16", "learned-single", "plain"],
                    help="learned-bf16: the step's solves batched (the value); learned-single: "
                         "the same solves one at a time; plain: FP32 sketch, m from 1")
    ap.add_argument("--model", default=None, help="learned-start model (.npz)")
    ap.add_argument("--skip-plain", action="store_true",
                    help="do not time the plain method beside the learned form")
    ap.add_argument("--plain-child", action="store_true",
                    help="c2: time the plain comparison in a child process of its own "
                         "instead of this one (after the learned regions)")
    ap.add_argument("--plain-steps", type=int, default=3,
                    help="c5: timed steps of the plain FP32 comparison (at most --steps)")
    ap.add_argument("--workload", default="c5",
                    choices=["c2", "c3", "c4a", "c4b", "c5", "path", "dual", "refreshed",
                             "sparse"],
                    help="c5 (default): learned+BF16 against plain FP32 on the 2^21x8192 "
                         "evaluation problem; c2: the 65536x1024 problem; c3: the 2^20x4096 precision "
                         "form; c4a: 64 nu^2 on one 2^18x2048 problem; c4b: 256 uneven "
                         "problems, batched; path: the warm-started regularization path "
                         "nu = 10^0..10^-4 on one 65536x1024 problem; dual: the "
                         "underdetermined 1024x65536 problem through the dual; refreshed: "
                         "fixed vs refreshed sketches at a fixed m on the headline problem; "
                         "sparse: 2^20x1024 CSR (1.5%% dense) with the CountSketch")
    ap.add_argument("--path-modes", default="path_warm_f32,path_warm_bf16,cold_f32",
                    help="path workload: the modes to time (the first listed is the value)")
    ap.add_argument("--skip-persistent", action="store_true",
                    help="c4a: do not time the grid's persistent form (its cooperative launch)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 256 MiB device-to-device copy first (a counter "
                         "reference for HBM traffic measurements)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_grad_partial_65536x1024_f32_traffic.txt")
TRAFFIC_FILE_C5 = os.path.join(ROOT, "profiles", "k_grad_wide_2p21x8192_f32_traffic.txt")
# the two-job pass (a pair's shared gradient) at 2^21 x 8192
TRAFFIC_FILE_C5_TWO = os.path.join(ROOT, "profiles",
                                   "k_grad_wide_two_2p21x8192_f32_traffic.txt")
# counter summaries of the BF16 SRHT at 2^21 x 8192, per sketch size
SRHT_TRAFFIC_FILES_C5 = {m: os.path.join(ROOT, "profiles", f"k_srht_2p21x8192_m{m}_bf16_traffic.txt")
                         for m in (512, 4096)}
CSRC = os.path.join(ROOT, "paper_2006_05874_amd", "csrc")
GRAD_SOURCES = [os.path.join(CSRC, f) for f in ("k_gradient.hip", "rs_device.hpp")]
SRHT_SOURCES = [os.path.join(CSRC, f) for f in ("k_srht.hip", "rs_device.hpp")]


def recorded_traffic_all(path, sources):
    """HBM bytes per launch of each kernel of a committed counter summary
    ({kernel: bytes}), or None when the kernel sources changed since the counters
    were taken."""
    try:
        text = open(path).read()
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in sources)).hexdigest()
    except OSError:
        return None
    out, kernel, src_sha = {}, None, None
    for line in text.splitlines():
        if ": " not in line or line.startswith("#"):
            continue
        k, v = (x.strip() for x in line.split(": ", 1))
        if k == "kernel_source_sha256":
            src_sha = v
        elif k == "kernel":
            kernel = v
        elif k == "traffic_bytes_per_launch" and kernel:
            out[kernel] = float(v)
    if src_sha != sha or not out:
        return None
    return out


def recorded_traffic(path=TRAFFIC_FILE, sources=GRAD_SOURCES):
    """HBM bytes per gradient launch from a committed counter summary, or None."""
    t = recorded_traffic_all(path, sources)
    return next(iter(t.values())) if t else None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        return max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:
        return os.cpu_count() or 1


def plain_in_child(args):
    """The plain FP32 method (m from 1) on the same problem, timed by this script in
    a child process of its own (this process waits, idle, for it); the same-process
    comparison measures the same (171.7 against 171.2 solves/s on the MI355X)."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "c2", "--mode", "plain",
           "--steps",
           str(args.steps), "--warmup", str(args.warmup), "--no-cpu-baseline", "--variant",
           args.variant, "--check-every", str(args.check_every)]
    print("[bench] plain FP32 comparison in its own process", file=sys.stderr, flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"plain comparison run failed with status {r.returncode}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": d["value"], "unit": "solves/s", "ms_per_step": d["ms_per_step"],
            "verified": d["verified"], "rel_pred_err": d["rel_pred_err"], "solve": d["solve"],
            "dtype": "f32 sketch", "m_init": 1, "process": "own (same script, --mode plain)"}


def cpu_baseline(A, b):
    """The oracle's direct solve x* = (A^T A + nu^2 I)^-1 A^T b in FP64, timed on
    the host: the full problem, one solve per nu^2, repeated while under ~20 s."""
    from oracle import ridge
    A64 = A.astype(np.float64)
    b64 = b.astype(np.float64)
    solves = 0
    t0 = time.perf_counter()
    while True:
        for nu2 in NU2S:
            ridge.solve_direct(A64, b64, nu2)
            solves += 1
        if time.perf_counter() - t0 > 10.0 or solves >= 8:
            break
    dt = time.perf_counter() - t0
    return {"value": solves / dt, "unit": "solves/s", "cores": blas_threads(), "kind": "oracle",
            "sample": f"oracle direct FP64 Cholesky solve of the full {N}x{D} problem, "
                      f"{solves} solves over nu^2 in {list(NU2S)}"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "c3":
        return run_c3(args)
    if args.workload == "c4b":
        return run_c4b(args)
    if args.workload == "c4a":
        return run_c4a(args)
    if args.workload == "c5":
        return run_c5(args)
    if args.workload == "path":
        return run_path(args)
    if args.workload == "dual":
        return run_dual(args)
    if args.workload == "refreshed":
        return run_refreshed(args)
    if args.workload == "sparse":
        return run_sparse(args)
    return run_c2(args)


def run_c2(args):
    """The 65536 x 1024 problem (sigma_i = 1/i) at nu^2 = 1e-2 and 1e-4: the learned
    form's two solves per step batched over two worker streams (the value), the
    same solves one at a time, and the plain method in a process of its own."""
    import torch

    from paper_2006_05874_amd import rs
    from synth import config_c2

    torch.cuda.set_device(0)
    probs = {nu2: config_c2(nu2=nu2, seed=0) for nu2 in NU2S}
    # the same A and b for both nu^2 (the generator ignores nu^2)
    p0 = probs[NU2S[0]]
    A = rs.padded(N, D, dtype=torch.float32)
    A.copy_(torch.from_numpy(p0.A))
    b = torch.from_numpy(p0.b).cuda()
    torch.cuda.synchronize()
    # the gradient pass's shape and grid, tuned on this problem (both k used)
    plans = {k: rs.rs_gradient_autotune(A, b, k=k) for k in (1, 2)}

    model = None
    if args.mode in ("learned-bf16", "learned-single"):
        from paper_2006_05874_amd import learned
        path = args.model or learned.MODEL_PATH
        if not os.path.exists(path):
            print(json.dumps({"error": f"no learned-start model at {path}; train one with "
                              "python -m paper_2006_05874_amd.learned, or pass --mode plain"}))
            sys.exit(2)
        model = learned.load_model(path)[:3]

    def solve(nu2, mode):
        if mode == "plain":
            return rs.rs_adaptive_solve(A, b, nu2, kind="srht", variant=args.variant,
                                        sketch_dtype="f32", check_every=args.check_every)
        params, mu, sd = model
        return rs.rs_learned_solve(A, b, nu2, params, mu, sd, kind="srht", variant=args.variant,
                                   sketch_dtype="bf16", check_every=args.check_every)

    def step_batched():
        params, mu, sd = model
        res = rs.rs_learned_solve_batch([(A, b, nu2) for nu2 in NU2S], params, mu, sd,
                                        kind="srht", variant=args.variant, sketch_dtype="bf16",
                                        check_every=args.check_every, workers=len(NU2S),
                                        graph_steps=args.graph_steps)
        return [(nu2, x, info) for nu2, (x, info) in zip(NU2S, res)]

    def timed(mode, profile):
        """mode: "plain" or "learned" (single solves, one after another) or
        "learned-batched" (each step's solves as one batch over worker streams)."""
        def one_step():
            if mode == "learned-batched":
                return step_batched()
            return [(nu2,) + tuple(solve(nu2, mode)) for nu2 in NU2S]
        for _ in range(args.warmup):
            one_step()
        torch.cuda.synchronize()
        if profile:
            rs.rs_profile_enable(True)
            rs.rs_profile_read()                       # clear
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        t0 = time.perf_counter()
        out = []
        for _ in range(args.steps):
            out.extend(one_step())
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = (0, 0.0)
        if profile:
            rs.rs_profile_enable(False)
            prof = rs.rs_profile_read()
        return out, ev0.elapsed_time(ev1), wall, prof

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    solves = args.steps * len(NU2S)
    main_mode = args.mode
    main = {"plain": "plain", "learned-single": "learned"}.get(main_mode, "learned-batched")
    # value: the timed steps as the library runs them; roofline: the same steps
    # again with every gradient launch timed by HIP events (timing costs about 4%
    # of the step, so it gets a timed region of its own)
    # the one-at-a-time learned solves first: after a batch the process's host
    # round trips were seen to run slower at times (the GPU kernels unchanged)
    sres = None
    iso_launches, iso_ms = 0, 0.0
    if main_mode == "learned-bf16" and not args.skip_plain:
        sres, sms, _, _ = timed("learned", profile=False)
        ires, _, _, (iso_launches, iso_ms) = timed("learned", profile=True)
    results, ms_total, wall, _ = timed(main, profile=False)
    ms_per_step = ms_total / args.steps
    value = solves / (ms_total / 1e3)
    rres, rms, _, (launches, grad_ms) = timed(main, profile=True)

    # verification against the oracle (FP64 direct solve of the stored problem),
    # after every timed region: the host BLAS threads it wakes stay off the timing
    from oracle import ridge
    A64 = p0.A.astype(np.float64)
    G = A64.T @ A64
    Atb = A64.T @ p0.b.astype(np.float64)
    xstar = {nu2: ridge.solve_direct_from_gram(G, Atb, nu2) for nu2 in NU2S}

    def verify(results):
        rels, infos = {}, {}
        for nu2 in NU2S:
            H = G + nu2 * np.eye(D)
            worst = 0.0
            for (nu, x, info) in results:
                if nu == nu2:
                    worst = max(worst, ridge.relative_error(H, x.cpu().numpy(), xstar[nu2]))
                    infos[nu2] = info
            rels[nu2] = worst
        ok = all(r <= 1e-6 for r in rels.values()) and all(
            i["status"] == "ok" for _, _, i in results)
        keys = ("m_final", "doublings", "steps", "grad_passes", "accepted_polyak", "accepted_gd")
        summary = {str(k): {kk: infos[k][kk] for kk in keys} for k in NU2S}
        for k in NU2S:
            if "m_init" in infos[k]:
                summary[str(k)]["m_init"] = infos[k]["m_init"]
        return ok, rels, summary

    ok, rels, solve_summary = verify(results)
    rok, _, _ = verify(rres)
    ok = ok and rok
    del results, rres
    if sres is not None:
        iok, _, _ = verify(ires)
        del ires
    seq = None
    if sres is not None:
        sok, srels, _ = verify(sres)
        del sres
        seq = {"value": round(solves / (sms / 1e3), 3), "unit": "solves/s",
               "ms_per_step": round(sms / args.steps, 3), "verified": sok and iok,
               "rel_pred_err": {str(k): v for k, v in srels.items()}}

    # roofline of the dominant kernel: the gradient pass over A
    alg_bytes = N * D * 4 + N * 4
    def roofline(n_launch, ms, region):
        us = ms / max(n_launch, 1) * 1e3
        ach = alg_bytes / (us / 1e6) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic else None, "algorithmic_bytes": alg_bytes,
                "kernel": "k_grad_partial (A^T(AX-b) pass, 2 RHS)",
                "avg_launch_us": round(us, 2), "launches": n_launch, "region": region}

    traffic = recorded_traffic()
    timing = ("each gradient launch timed by its own HIP start/stop events "
              "(hipExtLaunchKernelGGL) on its stream")
    roof_main = roofline(launches, grad_ms, "the timed steps repeated, " + timing)
    roof_main["profiled_ms_per_step"] = round(rms / args.steps, 3)
    roof_iso = None
    if seq is not None and iso_launches:
        roof_iso = roofline(iso_launches, iso_ms,
                            "the learned + BF16 solves one at a time, repeated, " + timing +
                            "; no other stream's kernels beside the pass")
    # the roofline reported is the kernel's own (solves one at a time); in the
    # batched steps two streams share HBM, which lengthens each launch
    roof = roof_iso if roof_iso is not None else roof_main
    line = {
        "metric": ("ridge solves/s to 1e-6 rel. pred. error, learned+BF16 vs plain FP32; HBM GB/s"
                   if main_mode != "plain" else
                   "ridge solves/s to 1e-6 rel. pred. error (plain FP32 IHS, SRHT)"),
        "value": round(value, 3), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 sketch / f32 gradient / f64 factor" if main_mode != "plain" else "f32",
        "data": "synthetic (seeded low-rank-decay A = G diag(1/i) V^T)",
        "config": {"workload": f"{N}x{D} FP32, sigma_i=1/i, nu^2 in {list(NU2S)}, SRHT rho=0.1, "
                               + {"learned-bf16": "learned m_init, BF16 sketch, the step's "
                                                  "solves batched over 2 streams",
                                  "learned-single": "learned m_init, BF16 sketch, one solve "
                                                    "at a time",
                                  "plain": "m_init=1, FP32 sketch"}[main_mode]
                               + f", {args.variant}, 2 solves per step",
                   "mode": main_mode,
                   "gradient_plan_k2": list(plans[2]),
                   "n": N, "d": D, "parallelism": "single GPU"},
        "verified": ok,
        "rel_pred_err": {str(k): v for k, v in rels.items()},
        "solve": solve_summary,
        "wall_s": round(wall, 3),
        "roofline": roof,
    }
    if seq is not None:
        line["learned_bf16_one_at_a_time"] = seq
    if roof_iso is not None:
        line["roofline_overlapped"] = roof_main
    # the plain method in a process of its own, once this one's timed work is done
    # (this one stays idle meanwhile)
    if main_mode == "learned-bf16" and not args.skip_plain:
        torch.cuda.synchronize()
        if not args.plain_child:
            pres, pms, _, _ = timed("plain", profile=False)
            pok, prels, psum = verify(pres)
            plain = {"value": round(solves / (pms / 1e3), 3), "unit": "solves/s",
                     "ms_per_step": round(pms / args.steps, 3), "verified": pok,
                     "rel_pred_err": {str(k): v for k, v in prels.items()}, "solve": psum,
                     "dtype": "f32 sketch", "m_init": 1, "process": "same"}
        else:
            plain = plain_in_child(args)
        line["plain_fp32"] = plain
        line["speedup_vs_plain_fp32"] = round(value / plain["value"], 3)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p0.A, p0.b)
    emit(line)


def oracle_gram_chunks(A_dev, b_dev, rows=65536):
    """FP64 Gram A^T A and A^T b of a device problem, accumulated on the host in
    row chunks (the oracle's definition, summed chunk by chunk)."""
    n, d = A_dev.shape
    G = np.zeros((d, d))
    Atb = np.zeros(d)
    for r0 in range(0, n, rows):
        Ac = A_dev[r0:r0 + rows].cpu().numpy().astype(np.float64)
        bc = b_dev[r0:r0 + rows].cpu().numpy().astype(np.float64)
        G += Ac.T @ Ac
        Atb += Ac.T @ bc
        print(f"[oracle] Gram rows {min(n, r0 + rows)}/{n}", file=sys.stderr, flush=True)
    return G, Atb


def run_c3(args):
    """Precision form on the 2^20 x 4096 FP32 problem (sigma_i = exp(-i/400),
    nu^2 = 1e-3 sigma_1^2): SRHT sketches in FP32, BF16 and FP8-E4M3; each solve's
    relative prediction error against the oracle's FP64 solution."""
    import torch
    from oracle import ridge
    from paper_2006_05874_amd import rs
    from synth import make_problem_torch, spectrum
    n, d = 1 << 20, 4096
    sig = spectrum("exp", d, 400.0)
    nu2 = 1e-3 * float(sig[0]) ** 2
    torch.cuda.set_device(0)
    A0, b, _ = make_problem_torch(n, d, sig, 0.1, 3, "cuda")
    A = rs.padded(n, d, dtype=torch.float32)
    A.copy_(A0)
    del A0
    torch.cuda.synchronize()
    for k in (1, 2):
        rs.rs_gradient_autotune(A, b, k=k)
    print(f"[c3] problem ready", file=sys.stderr, flush=True)
    from paper_2006_05874_amd import learned
    params, mu, sd, _ = learned.load_model(args.model or learned.MODEL_PATH)
    res, xs_dev = {}, {}
    for dt in ("f32", "bf16", "fp8", "learned_bf16"):
        if dt == "learned_bf16":
            solve = lambda: rs.rs_learned_solve(A, b, nu2, params, mu, sd, sketch_dtype="bf16",
                                                raise_on_error=False)
        else:
            solve = lambda: rs.rs_adaptive_solve(A, b, nu2, sketch_dtype=dt,
                                                 raise_on_error=False)
        solve()                                                   # warm-up
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        outs = [solve() for _ in range(args.steps)]
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        x, info = outs[-1]
        xs_dev[dt] = [o[0] for o in outs]
        res[dt] = {"solves_per_s": round(1e3 / ms, 3), "ms_per_solve": round(ms, 3),
                   "status": info["status"], "m_final": info["m_final"],
                   "doublings": info["doublings"], "grad_passes": info["grad_passes"]}
        if "m_init" in info:
            res[dt]["m_init"] = info["m_init"]
        print(f"[c3] {dt}: {res[dt]}", file=sys.stderr, flush=True)
    roof = gradient_roofline(
        rs, lambda: rs.rs_adaptive_solve(A, b, nu2, sketch_dtype="bf16", raise_on_error=False),
        n * d * 4 + n * 4, "k_grad_partial (A^T(AX-b) pass)", "one more BF16 solve")
    # the oracle's FP64 solution, after every timed region
    print(f"[c3] oracle Gram on the host", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    G, Atb = oracle_gram_chunks(A, b)
    xs = ridge.solve_direct_from_gram(G, Atb, nu2)
    H = G + nu2 * np.eye(d)
    oracle_s = time.perf_counter() - t0
    for dt, xl in xs_dev.items():
        res[dt]["rel_pred_err"] = max(ridge.relative_error(H, x.cpu().numpy(), xs) for x in xl)
    base = res["f32"]["solves_per_s"]
    line = {"metric": "ridge solves/s to 1e-6 rel. pred. error, precision form",
            "value": res["bf16"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": res["bf16"]["ms_per_solve"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16 sketch / f32 gradient / f64 factor", "data": "synthetic",
            "config": {"workload": f"{n}x{d} FP32, sigma_i=exp(-i/400), nu^2=1e-3 sigma_1^2, "
                                   "SRHT rho=0.1, m from 1", "n": n, "d": d},
            "verified": all(r["rel_pred_err"] <= 1e-6 and r["status"] == "ok"
                            for r in res.values()),
            "per_dtype": res, "speedup_bf16_vs_f32": round(res["bf16"]["solves_per_s"] / base, 3),
            "speedup_fp8_vs_f32": round(res["fp8"]["solves_per_s"] / base, 3),
            "speedup_learned_bf16_vs_f32": round(res["learned_bf16"]["solves_per_s"] / base, 3),
            "roofline": roof,
            "cpu_baseline": {"value": round(1.0 / oracle_s, 5), "unit": "solves/s",
                             "cores": blas_threads(), "kind": "oracle",
                             "sample": f"one oracle direct FP64 solve of the full {n}x{d} "
                                       f"problem (Gram accumulated from row blocks read back "
                                       f"from the device, Cholesky): {oracle_s:.1f} s"}}
    emit(line)


def oracle_gradient_bound(A_dev, b_dev, x, nu2, rows=32768):
    """The oracle's FP64 gradient g = A^T (A x - b) + nu^2 x at a device solution,
    streamed from the device in row blocks, and the bound it gives on the relative
    prediction error: delta(x) = g^T H^-1 g / 2 <= |g|^2 / (2 nu^2) and
    delta(0) = (A^T b)^T H^-1 (A^T b) / 2 >= |A^T b|^2 / (2 (|A|_F^2 + nu^2))."""
    n, d = A_dev.shape
    xh = x.cpu().numpy().astype(np.float64)
    g = np.zeros(d)
    atb = np.zeros(d)
    fro = 0.0
    for r0 in range(0, n, rows):
        Ac = A_dev[r0:r0 + rows].cpu().numpy().astype(np.float64)
        bc = b_dev[r0:r0 + rows].cpu().numpy().astype(np.float64)
        g += Ac.T @ (Ac @ xh - bc)
        atb += Ac.T @ bc
        fro += float(np.sum(Ac * Ac))
        if (r0 // rows) % 16 == 0:
            print(f"[oracle] gradient rows {min(n, r0 + rows)}/{n}", file=sys.stderr, flush=True)
    g += nu2 * xh
    bound = (g @ g / nu2) * (fro + nu2) / (atb @ atb)
    return float(bound), float(np.linalg.norm(g) / np.linalg.norm(atb))


C5_N, C5_D = 1 << 21, 8192
C5_NU2S = (1e-2, 1e-4)
C5_SEED = 5


def c5_certify(A_dev, b_dev, X, nu2s, rows=32768, k=256):
    """The oracle's streamed certificate of every solution (columns of X, with
    their nu^2): row blocks of the stored A and b read back from the device; per
    point an upper bound on delta(x) / delta(0).  Identical points are judged once."""
    from oracle.certify import StreamedCertificate
    n, d = A_dev.shape
    keys = [(nu, x.tobytes()) for nu, x in zip(nu2s, X.T)]
    uniq = {}
    for key in keys:
        uniq.setdefault(key, len(uniq))
    cols = [None] * len(uniq)
    for (nu, xb), j in uniq.items():
        cols[j] = (nu, np.frombuffer(xb, dtype=np.float64))
    C = StreamedCertificate(d, np.stack([c[1] for c in cols], axis=1), k=k)
    t0 = time.perf_counter()
    for r0 in range(0, n, rows):
        C.add(A_dev[r0:r0 + rows].cpu().numpy(), b_dev[r0:r0 + rows].cpu().numpy())
        if (r0 // rows) % 8 == 0:
            print(f"[oracle] certificate rows {min(n, r0 + rows)}/{n} "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    res = C.bounds(np.array([c[0] for c in cols]))
    return [res[uniq[key]] for key in keys], len(uniq), k


def run_c5(args):
    """The metric's configuration: the learned form with BF16 SRHT sketches against
    the plain method (FP32 sketch, m from 1) on the 2^21 x 8192 FP32 evaluation
    problem (64 GiB; sigma_i = 1/i, G ~ N(0, 1/n), V Haar, b = A x_pl + 0.1 xi,
    seed 5).  One step = the solve at nu^2 = 1e-2 and the solve at nu^2 = 1e-4
    (nominal effective dimensions 15.2 and 155), each to the default decrement
    tolerance.  The value is the learned form with the step's two solves batched
    (rs_learned_solve_batch: the two jobs share A and b, so they run as a pair on
    two worker streams, with one features pass and one gradient pass per common
    step for both); the same solves one at a time on one stream and the plain
    method are timed beside it.  Every timed solve is
    judged afterwards by the oracle's streamed certificate (an upper bound on
    delta(x) / delta(0) from one FP64 pass over the stored A)."""
    import torch
    from paper_2006_05874_amd import learned, rs
    from synth import make_problem_torch, spectrum
    n, d = C5_N, C5_D
    torch.cuda.set_device(0)
    print(f"[c5] generating the {n}x{d} problem on the device", file=sys.stderr, flush=True)
    A, b, _ = make_problem_torch(n, d, spectrum("poly", d, 1.0), 0.1, C5_SEED, "cuda")
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    plans = {k: rs.rs_gradient_autotune(A, b, k=k) for k in (1, 2)}
    print(f"[c5] problem ready; gradient plans {plans}", file=sys.stderr, flush=True)
    path = args.model or learned.MODEL_PATH
    params, mu, sd, _ = learned.load_model(path)

    def solve(nu2, mode):
        if mode == "plain":
            return rs.rs_adaptive_solve(A, b, nu2, kind="srht", variant=args.variant,
                                        sketch_dtype="f32", check_every=args.check_every,
                                        raise_on_error=False)
        return rs.rs_learned_solve(A, b, nu2, params, mu, sd, kind="srht", variant=args.variant,
                                   sketch_dtype="bf16", check_every=args.check_every,
                                   raise_on_error=False)

    def batch():
        return rs.rs_learned_solve_batch([(A, b, nu2) for nu2 in C5_NU2S], params, mu, sd,
                                         kind="srht", variant=args.variant, sketch_dtype="bf16",
                                         check_every=args.check_every, workers=len(C5_NU2S),
                                         raise_on_error=False)

    def one_step(mode):
        if mode == "batched":
            return [(nu2, x, info) for nu2, (x, info) in zip(C5_NU2S, batch())]
        return [(nu2,) + tuple(solve(nu2, mode)) for nu2 in C5_NU2S]

    def timed(mode, steps, warmup):
        for _ in range(warmup):
            one_step(mode)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        t0 = time.perf_counter()
        out = []
        for s in range(steps):
            out += one_step(mode)
        ev1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print(f"[c5] {mode}: {steps} steps in {wall:.2f} s", file=sys.stderr, flush=True)
        return out, ev0.elapsed_time(ev1), wall

    main_mode = {"plain": "plain", "learned-single": "learned"}.get(args.mode, "batched")
    single = None
    if main_mode == "batched":
        # the same solves one at a time on one stream, timed first
        sres, sms, _ = timed("learned", args.steps, args.warmup)
        single = {"steps": args.steps, "warmup": args.warmup, "ms_per_step": sms / args.steps,
                  "value": args.steps * len(C5_NU2S) / (sms / 1e3), "res": sres}
    results, ms_total, wall = timed(main_mode, args.steps, args.warmup)
    solves = args.steps * len(C5_NU2S)
    value = solves / (ms_total / 1e3)
    free_b, total_b = torch.cuda.mem_get_info()
    print(f"[c5] device memory in use {(total_b - free_b) / 2 ** 30:.1f} of "
          f"{total_b / 2 ** 30:.1f} GiB", file=sys.stderr, flush=True)
    plain = None
    if main_mode != "plain" and not args.skip_plain:
        # the comparison: fewer steps (each plain solve walks the doubling ladder)
        psteps = max(1, min(args.steps, args.plain_steps))
        pres, pms, _ = timed("plain", psteps, 1)
        plain = {"steps": psteps, "warmup": 1, "ms_per_step": pms / psteps,
                 "value": psteps * len(C5_NU2S) / (pms / 1e3), "res": pres}

    # roofline of the dominant kernel: one more step of the timed form with every
    # gradient pass timed by HIP events on its stream (algorithmic bytes per launch:
    # A and b once, also for a pair's shared pass)
    grad_bytes = n * d * 4 + n * 4
    kname = "k_grad_wide / k_grad_partial (A^T(AX-b) pass over 64 GiB, tuned plan)"
    kname_two = ("k_grad_wide_two (a pair's shared A^T(AX-b) pass: both solves' two "
                 "candidates in one read of the 64 GiB A)")
    roof_single = None
    if main_mode == "batched":
        roof = gradient_roofline(rs, lambda: one_step("batched"), grad_bytes, kname_two,
                                 "one more batched step (the pair's passes; a pass after "
                                 "one job has stopped runs alone)")
        tt = recorded_traffic(TRAFFIC_FILE_C5_TWO, GRAD_SOURCES)
        if tt and list(plans[2])[0] == 512:
            roof["traffic"] = round(tt)
            roof["traffic_source"] = (os.path.relpath(TRAFFIC_FILE_C5_TWO, ROOT) + " (two-job "
                                      "pass, FETCH_SIZE + WRITE_SIZE scaled by a 256 MiB copy)")
        roof_single = gradient_roofline(rs, lambda: one_step("learned"), grad_bytes, kname,
                                        "one more step, its solves one at a time")
    else:
        roof = gradient_roofline(rs, lambda: one_step(main_mode), grad_bytes, kname,
                                 "one more step")
    traffic = recorded_traffic(TRAFFIC_FILE_C5, GRAD_SOURCES)
    rk2 = roof_single if roof_single is not None else roof
    if traffic and list(plans[2])[0] == 512:
        rk2["traffic"] = round(traffic)
        rk2["traffic_source"] = ("profiles/k_grad_wide_2p21x8192_f32_traffic.txt (k = 2 pass, "
                                 "FETCH_SIZE + WRITE_SIZE scaled by a 256 MiB copy)")
    # the SRHT at the sketch size each learned solve started from (BF16 output),
    # timed by events around the call on its stream
    srht = {}
    for nu2, _, info in results[:len(C5_NU2S)]:
        m = int(info.get("m_init", info["m_final"]))
        sdt = "bf16" if main_mode in ("learned", "batched") else "f32"
        rs.rs_sketch_srht(A, m, sa_dtype=sdt)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record()
        for r in range(reps):
            rs.rs_sketch_srht(A, m, sketch_id=r + 1, sa_dtype=sdt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = n * d * 4 + m * d * (2 if sdt == "bf16" else 4)
        ach = alg / (ms / 1e3) / 1e9
        srht[str(nu2)] = {"bound": "hbm", "m": m, "sa_dtype": sdt, "ms_per_sketch": round(ms, 3),
                          "algorithmic_bytes": alg, "achieved": round(ach, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                          "region": f"{reps} calls of rs_sketch_srht (selection, both passes), "
                                    "HIP events around them on the stream"}
        tf = SRHT_TRAFFIC_FILES_C5.get(m) if sdt == "bf16" else None
        st = recorded_traffic_all(tf, SRHT_SOURCES) if tf else None
        if st:
            srht[str(nu2)]["traffic"] = round(sum(st.values()))
            srht[str(nu2)]["traffic_source"] = (os.path.relpath(tf, ROOT) + " (both passes, "
                                                "FETCH_SIZE + WRITE_SIZE scaled by a 256 MiB "
                                                "copy)")

    # where a solve's GPU time goes: one more step per mode with the phases timed by
    # HIP events inside the library (sketches, Grams and factors, the rest)
    phases = {}
    rs.set_phase_timing(True)
    for mode in (["learned" if main_mode == "batched" else main_mode]
                 + (["plain"] if plain is not None else [])):
        for nu2 in C5_NU2S:
            _, inf = solve(nu2, mode)
            phases.setdefault(mode, {})[str(nu2)] = {
                "ms_sketch": round(inf["ms_sketch"], 2), "ms_factor": round(inf["ms_factor"], 2),
                "ms_iterate": round(inf["ms_iterate"], 2), "m_final": inf["m_final"],
                "doublings": inf["doublings"], "grad_passes": inf["grad_passes"]}
    rs.set_phase_timing(False)

    # the oracle's certificate of every timed solve, after the timed work
    pts = [(nu2, x, info, "main") for nu2, x, info in results]
    if single is not None:
        pts += [(nu2, x, info, "single") for nu2, x, info in single["res"]]
    if plain is not None:
        pts += [(nu2, x, info, "plain") for nu2, x, info in plain["res"]]
    X = np.stack([x.cpu().numpy().astype(np.float64) for _, x, _, _ in pts], axis=1)
    bounds, nuniq, kny = c5_certify(A, b, X, [p[0] for p in pts])

    def summary(which):
        rel, infos = {}, {}
        ok = True
        for (nu2, x, info, w), (up, lo, ratio) in zip(pts, bounds):
            if w != which:
                continue
            rel[str(nu2)] = max(rel.get(str(nu2), 0.0), ratio)
            infos[str(nu2)] = info
            ok = ok and ratio <= 1e-6 and info["status"] == "ok"
        keys = ("m_final", "doublings", "steps", "grad_passes", "accepted_polyak", "accepted_gd")
        sol = {k: {kk: v[kk] for kk in keys} for k, v in infos.items()}
        for k, v in infos.items():
            if "m_init" in v:
                sol[k]["m_init"] = v["m_init"]
        return ok, rel, sol

    ok, rel, sol = summary("main")

    # the oracle's direct solve on a bounded sample: the FP64 Gram of the first 2^15
    # rows (linear in the rows: scaled by n / 2^15) and the d x d Cholesky solve
    from oracle import ridge
    rows = 1 << 15
    As = A[:rows].cpu().numpy().astype(np.float64)
    bs = b[:rows].cpu().numpy().astype(np.float64)
    t0 = time.perf_counter()
    Gs = As.T @ As
    cs = As.T @ bs
    t_gram = time.perf_counter() - t0
    t0 = time.perf_counter()
    ridge.solve_direct_from_gram(Gs, cs, C5_NU2S[0])
    t_solve = time.perf_counter() - t0
    del As, bs, Gs
    t_full = t_gram * n / rows + t_solve
    cpu = {"value": round(1.0 / t_full, 6), "unit": "solves/s", "cores": blas_threads(),
           "kind": "oracle",
           "sample": f"the oracle's direct FP64 solve on the first {rows} rows: Gram "
                     f"{t_gram:.1f} s (scaled by {n}/{rows}) + Cholesky solve {t_solve:.1f} s"}
    learned_form = main_mode in ("learned", "batched")
    dtype = "bf16 sketch / f32 gradient / f64 factor" if learned_form else "f32"
    line = {
        "metric": "ridge solves/s to 1e-6 rel. pred. error, learned+BF16 vs plain FP32; HBM GB/s",
        "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_total / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic (seeded low-rank-decay A = G diag(1/i) V^T, generated on the device)",
        "config": {"workload": f"{n}x{d} FP32 (64 GiB), sigma_i=1/i, nu^2 in {list(C5_NU2S)}, "
                               "SRHT rho=0.1, "
                               + ("learned m_init, BF16 sketch" if learned_form
                                  else "m_init=1, FP32 sketch")
                               + f", {args.variant}, 2 solves per step, "
                               + ("batched as a pair on 2 worker streams (shared features "
                                  "and gradient passes)" if main_mode == "batched"
                                  else "one stream"),
                   "mode": main_mode, "n": n, "d": d,
                   "gradient_plan_k2": list(plans[2]), "parallelism": "single GPU"},
        "verified": ok,
        "rel_pred_err_bound": rel,
        "rel_pred_err_bound_sqrt": {k: math.sqrt(v) for k, v in rel.items()},
        "certificate": f"oracle/certify.py: upper bound on delta(x)/delta(0) from one FP64 pass "
                       f"over the stored A (Nystrom k={kny}); {nuniq} distinct solutions judged",
        "solve": sol, "wall_s": round(wall, 3),
        "roofline": roof, "srht_roofline": srht,
        "phases_ms": phases,
    }
    if roof_single is not None:
        line["roofline_one_at_a_time"] = roof_single
    if single is not None:
        sok, srel, ssol = summary("single")
        line["learned_bf16_one_at_a_time"] = {
            "value": round(single["value"], 4), "unit": "solves/s", "steps": single["steps"],
            "warmup": single["warmup"], "ms_per_step": round(single["ms_per_step"], 3),
            "verified": sok, "rel_pred_err_bound": srel, "solve": ssol}
    if plain is not None:
        pok, prel, psol = summary("plain")
        line["plain_fp32"] = {"value": round(plain["value"], 4), "unit": "solves/s",
                              "steps": plain["steps"], "warmup": plain["warmup"],
                              "ms_per_step": round(plain["ms_per_step"], 3), "verified": pok,
                              "rel_pred_err_bound": prel, "solve": psol,
                              "dtype": "f32 sketch", "m_init": 1, "process": "same"}
        line["speedup_vs_plain_fp32"] = round(value / plain["value"], 3)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu
    emit(line)


def run_c4a(args):
    """64 values of nu^2 (log-spaced in [1e-6, 1]) on one 2^18 x 2048 FP32 problem
    (sigma_i = i^-0.8): the nu-grid solver (shared level sketches, batched
    factors, multi-RHS gradients; BF16 sketches) against 64 plain single solves
    (FP32 sketch, m from 1).  Sampled nu checked against the oracle."""
    import torch
    from oracle import ridge
    from paper_2006_05874_amd import rs
    from synth import config_c4a_nu2, make_c4a_problem
    torch.cuda.set_device(0)
    A0, b = make_c4a_problem("cuda")
    n, d = A0.shape
    A = rs.padded(n, d, dtype=torch.float32)
    A.copy_(A0)
    del A0
    nus = list(config_c4a_nu2())
    torch.cuda.synchronize()
    print("[c4a] problem ready", file=sys.stderr, flush=True)

    def grid(persistent=False):
        X, infos = rs.rs_solve_nu_grid(A, b, nus, sketch_dtype="bf16", raise_on_error=False,
                                       persistent=persistent)
        return [(X[k], infos[k]) for k in range(len(nus))]

    def seq():
        return [rs.rs_adaptive_solve(A, b, nu, sketch_dtype="f32", raise_on_error=False)
                for nu in nus]

    out = {}
    # the grid's persistent form (each window of steps one cooperative launch) runs
    # the same arithmetic: its solutions must equal the default form's bit for bit
    modes = [("grid_bf16", grid), ("grid_bf16_persistent", lambda: grid(True)),
             ("sequential_plain_f32", seq)]
    if args.skip_persistent:
        modes.pop(1)
    for name, fn in modes:
        fn()
        torch.cuda.synchronize()
        rs.rs_profile_enable(name == "grid_bf16")
        rs.rs_profile_read()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        launches, gms = rs.rs_profile_read()
        rs.rs_profile_enable(False)
        out[name] = {"solves_per_s": round(len(nus) / sec, 2), "s_per_grid": round(sec, 4),
                     "res": res}
        if name == "grid_bf16":
            out[name]["mr_gradient_launches"] = launches
            out[name]["mr_gradient_ms_total"] = round(gms, 3)
        print(f"[c4a] {name}: {len(nus) / sec:.1f} solves/s", file=sys.stderr, flush=True)
    # the multi-RHS gradient passes of the timed grid solves (timed by HIP events):
    # each running nu adds its candidates as columns, 4 n d flops per column
    gres = out["grid_bf16"]["res"]
    same = None if args.skip_persistent else all(
        torch.equal(x0, x1) and i0["events"] == i1["events"]
        for (x0, i0), (x1, i1) in zip(gres, out["grid_bf16_persistent"]["res"]))
    cols = sum(2 * i["grad_passes"] - 1 for _, i in gres) * args.steps
    gms = out["grid_bf16"]["mr_gradient_ms_total"]
    tfl = 4.0 * n * d * cols / (gms / 1e3) / 1e12 if gms > 0 else 0.0
    roof = {"bound": "mfma", "achieved": round(tfl, 2), "peak": 157.3, "unit": "TFLOP/s",
            "frac": round(tfl / 157.3, 4), "traffic": None,
            "algorithmic_flops": 4.0 * n * d * cols / max(out["grid_bf16"]["mr_gradient_launches"],
                                                          1),
            "kernel": "k_mr_resid + k_mr_atr (multi-RHS gradient, FP32 matrix cores)",
            "avg_launch_us": round(gms / max(out["grid_bf16"]["mr_gradient_launches"], 1) * 1e3,
                                   2),
            "launches": out["grid_bf16"]["mr_gradient_launches"],
            "region": "the timed grid solves; each pass timed from its first kernel's start to "
                      "its second's stop by HIP events; columns counted from every nu's passes"}
    t0 = time.perf_counter()
    G, Atb = oracle_gram_chunks(A, b)
    ridge.solve_direct_from_gram(G, Atb, nus[0])
    oracle_s = time.perf_counter() - t0
    worst = {k: 0.0 for k in out}
    for k in (0, 16, 32, 48, 63):
        xs = ridge.solve_direct_from_gram(G, Atb, nus[k])
        H = G + nus[k] * np.eye(d)
        for name in out:
            worst[name] = max(worst[name], ridge.relative_error(
                H, out[name]["res"][k][0].cpu().numpy(), xs))
    for name in out:
        res = out[name].pop("res")
        out[name]["not_ok"] = sum(i["status"] != "ok" for _, i in res)
        out[name]["sampled_worst_rel_pred_err"] = worst[name]
        out[name]["m_final"] = [i["m_final"] for _, i in res]
    line = {"metric": "ridge solves/s to 1e-6 rel. pred. error, nu grid on one A",
            "value": out["grid_bf16"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1,
            "ms_per_step": round(out["grid_bf16"]["s_per_grid"] * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16 sketch / f32 gradient / f64 factor", "data": "synthetic",
            "config": {"workload": f"{n}x{d} FP32, sigma_i=i^-0.8, 64 nu^2 log-spaced in "
                                   "[1e-6, 1], SRHT fresh, m from 1", "n": n, "d": d},
            "verified": all(v["sampled_worst_rel_pred_err"] <= 1e-6 and v["not_ok"] == 0
                            for v in out.values()),
            "modes": out, "roofline": roof,
            "cpu_baseline": {"value": round(1.0 / oracle_s, 4), "unit": "solves/s",
                             "cores": blas_threads(), "kind": "oracle",
                             "sample": f"one oracle direct FP64 solve of the full {n}x{d} "
                                       f"problem (Gram from row blocks read back from the "
                                       f"device, Cholesky): {oracle_s:.1f} s"},
            "speedup_vs_sequential_plain_f32": round(
                out["grid_bf16"]["solves_per_s"] / out["sequential_plain_f32"]["solves_per_s"], 3),
            "persistent_identical_to_launches": same}
    emit(line)


def run_path(args):
    """The regularization path nu = 10^0 .. 10^-4 (decreasing) on one 65536 x 1024
    FP32 problem (sigma_i = 1/i), each solve stopped at eps = 1e-10 measured from
    the origin: the path solver (warm starts, sketch size carried over, nested
    sketches with one transformed A) against the same five solves run cold (x = 0,
    m from 1, fresh sketches).  Every solution is checked against the oracle."""
    import torch
    from oracle import ridge
    from paper_2006_05874_amd import rs
    from synth import config_path_nu2, make_path_problem
    torch.cuda.set_device(0)
    A0, b = make_path_problem("cuda")
    n, d = A0.shape
    A = rs.padded(n, d, dtype=torch.float32)
    A.copy_(A0)
    del A0
    nus = list(config_path_nu2())
    tol = 1e-10
    torch.cuda.synchronize()
    print("[path] problem ready", file=sys.stderr, flush=True)

    def path(sd):
        def fn():
            X, infos = rs.rs_solve_path(A, b, nus, sketch_dtype=sd, tol=tol,
                                        raise_on_error=False)
            return [(X[k], infos[k]) for k in range(len(nus))]
        return fn

    def cold():
        return [rs.rs_adaptive_solve(A, b, nu, sketch_dtype="f32", tol=tol,
                                     raise_on_error=False) for nu in nus]

    modes = {"path_warm_f32": path("f32"), "path_warm_bf16": path("bf16"), "cold_f32": cold}
    names = args.path_modes.split(",")
    out = {}
    for name in names:
        fn = modes[name]
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        out[name] = {"solves_per_s": round(len(nus) / sec, 2), "ms_per_path": round(sec * 1e3, 3),
                     "res": res}
        print(f"[path] {name}: {sec * 1e3:.2f} ms per path", file=sys.stderr, flush=True)
    roof = gradient_roofline(rs, path("f32"), n * d * 4 + n * 4,
                             "k_grad_partial (A^T(AX-b) pass)", "one more path_warm_f32 path")
    G, Atb = oracle_gram_chunks(A, b)
    A64 = A.cpu().numpy().astype(np.float64)
    b64 = b.cpu().numpy().astype(np.float64)
    cpu = oracle_rate([lambda nu=nu: ridge.solve_direct(A64, b64, nu) for nu in nus],
                      f"oracle direct FP64 Cholesky solves of the full {n}x{d} problem at the "
                      "path's nu^2 (the oracle's path itself forms dense Hadamard sketches)")
    del A64
    for name in out:
        res = out[name].pop("res")
        worst = 0.0
        for k, nu2 in enumerate(nus):
            xs = ridge.solve_direct_from_gram(G, Atb, nu2)
            worst = max(worst, ridge.relative_error(G + nu2 * np.eye(d), res[k][0].cpu().numpy(),
                                                    xs))
        out[name]["worst_rel_pred_err"] = worst
        out[name]["not_ok"] = sum(i["status"] != "ok" for _, i in res)
        out[name]["m_final"] = [i["m_final"] for _, i in res]
        out[name]["grad_passes"] = [i["grad_passes"] for _, i in res]
        out[name]["doublings"] = [i["doublings"] for _, i in res]
    best = names[0]
    line = {"metric": "ridge solves/s along a regularization path (eps = 1e-10 rel. pred. error)",
            "value": out[best]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": out[best]["ms_per_path"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 gradient / f32 sketch / f64 factor", "data": "synthetic",
            "config": {"workload": f"{n}x{d} FP32, sigma_i=1/i, path nu^2 in "
                                   f"{[float(v) for v in nus]} "
                                   "(decreasing), warm starts, SRHT nested, eps=1e-10",
                       "n": n, "d": d},
            "verified": all(v["worst_rel_pred_err"] <= 1e-9 and v["not_ok"] == 0
                            for v in out.values()),
            "roofline": roof, "cpu_baseline": cpu,
            "modes": out}
    if "cold_f32" in out:
        line["speedup_vs_cold_f32"] = round(out[best]["solves_per_s"]
                                            / out["cold_f32"]["solves_per_s"], 3)
    emit(line)


def run_dual(args):
    """The underdetermined case: 1024 x 65536 FP32 (the transpose of the headline
    shape), sigma_i = 1/i, nu^2 in {1e-2, 1e-4}, solved through the dual problem
    (A^T formed once per solve, Algorithm 1 on it, x = A^T z), FP32 and BF16
    sketches, m from 1, eps = 1e-10 on the dual decrement.  Every solution is
    checked against the oracle's direct dual solve mapped to x."""
    import torch
    from paper_2006_05874_amd import rs
    from synth import make_dual_problem
    torch.cuda.set_device(0)
    A0, b = make_dual_problem("cuda")
    n, d = A0.shape
    A = rs.padded(n, d, dtype=torch.float32)
    A.copy_(A0)
    del A0
    nus = [1e-2, 1e-4]
    tol = 1e-10
    torch.cuda.synchronize()
    print("[dual] problem ready", file=sys.stderr, flush=True)
    out = {}
    for sd in ("f32", "bf16"):
        def fn():
            return [rs.rs_adaptive_solve_dual(A, b, nu, sketch_dtype=sd, tol=tol,
                                              raise_on_error=False) for nu in nus]
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        out[f"dual_{sd}"] = {"solves_per_s": round(len(nus) / sec, 2),
                             "ms_per_solve": round(sec * 1e3 / len(nus), 3), "res": res}
        print(f"[dual] {sd}: {len(nus) / sec:.1f} solves/s", file=sys.stderr, flush=True)
    roof = gradient_roofline(
        rs, lambda: [rs.rs_adaptive_solve_dual(A, b, nu, sketch_dtype="f32", tol=tol,
                                               raise_on_error=False) for nu in nus],
        d * n * 4 + d * 4, "k_grad_partial over A^T (the dual's A A^T z pass)",
        "the dual_f32 solves repeated")
    # oracle: z* = (A A^T + nu^2 I)^-1 b in FP64 on the host, x* = A^T z*
    from oracle import ridge
    A64 = A.cpu().numpy().astype(np.float64)
    b64 = b.cpu().numpy().astype(np.float64)
    cpu = oracle_rate([lambda nu=nu: A64.T @ ridge.solve_dual_direct(A64, b64, nu) for nu in nus],
                      f"oracle direct FP64 dual solves z* = (A A^T + nu^2 I)^-1 b, x* = A^T z* "
                      f"of the full {n}x{d} problem")
    K = A64 @ A64.T
    for name in out:
        res = out[name].pop("res")
        worst = 0.0
        for k, nu2 in enumerate(nus):
            zs = np.linalg.solve(K + nu2 * np.eye(n), b64)
            xs = A64.T @ zs
            e = res[k][0].cpu().numpy() - xs
            delta = np.sum((A64 @ e) ** 2) + nu2 * np.sum(e ** 2)
            worst = max(worst, delta / (np.sum((A64 @ xs) ** 2) + nu2 * np.sum(xs ** 2)))
        out[name]["worst_rel_pred_err"] = worst
        out[name]["not_ok"] = sum(i["status"] != "ok" for _, _, i in res)
        out[name]["m_final"] = [i["m_final"] for _, _, i in res]
        out[name]["grad_passes"] = [i["grad_passes"] for _, _, i in res]
    best = "dual_f32"
    line = {"metric": "ridge solves/s to 1e-6 rel. pred. error, underdetermined (dual) form",
            "value": out[best]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1,
            "ms_per_step": round(out[best]["ms_per_solve"] * len(nus), 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 gradient / f32 sketch / f64 factor", "data": "synthetic",
            "config": {"workload": f"{n}x{d} FP32 (n < d), sigma_i=1/i, nu^2 in {nus}, dual "
                                   "problem, SRHT fresh, m from 1, eps=1e-10 (dual)",
                       "n": n, "d": d},
            "verified": all(v["worst_rel_pred_err"] <= 1e-6 and v["not_ok"] == 0
                            for v in out.values()),
            "roofline": roof, "cpu_baseline": cpu,
            "modes": out}
    emit(line)


def gradient_roofline(rs, fn, alg_bytes, kernel, region):
    """Repeat fn with every gradient pass timed by HIP events on its own stream
    (rs_profile_enable); the roofline of the pass from its average duration."""
    import torch
    torch.cuda.synchronize()
    rs.rs_profile_enable(True)
    rs.rs_profile_read()
    fn()
    torch.cuda.synchronize()
    rs.rs_profile_enable(False)
    n, ms = rs.rs_profile_read()
    us = ms / max(n, 1) * 1e3
    ach = alg_bytes / (us / 1e6) / 1e9 if us > 0 else 0.0
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "algorithmic_bytes": int(alg_bytes), "kernel": kernel, "avg_launch_us": round(us, 2),
            "launches": n, "region": region + "; each pass timed by its own HIP start/stop "
                                              "events; no counter passes taken for this workload"}


def oracle_rate(calls, sample, budget_s=10.0):
    """The oracle's direct solves timed on the host: the calls in turn, repeated while
    under budget_s (at least one)."""
    done = 0
    t0 = time.perf_counter()
    while True:
        for c in calls:
            c()
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": round(done / dt, 4), "unit": "solves/s", "cores": blas_threads(),
            "kind": "oracle", "sample": f"{sample}; {done} solves in {dt:.1f} s"}


def run_refreshed(args):
    """Ablation of the fixed embedding: on the 65536 x 1024 headline problem at
    nu^2 = 1e-2 and a fixed sketch size m (the final m of a plain run, 512), the
    IHS with a new sketch and factor every step against Algorithm 1 started at
    that m (one sketch, step tests), for the SRHT and the Gaussian embedding and
    both update variants, to eps = 1e-10.  Every solution is checked against the
    oracle's direct solve."""
    import torch
    from oracle import ridge
    from paper_2006_05874_amd import rs
    from synth import config_c2
    torch.cuda.set_device(0)
    p = config_c2(nu2=1e-2, seed=0)
    n, d = p.A.shape
    A = rs.padded(n, d, dtype=torch.float32)
    A.copy_(torch.from_numpy(p.A))
    b = torch.from_numpy(p.b).cuda()
    m, tol = 512, 1e-10
    xs = ridge.solve_direct(p.A.astype(np.float64), p.b.astype(np.float64), p.nu2)
    H = ridge.hessian(p.A.astype(np.float64), p.nu2)
    print("[refreshed] problem ready", file=sys.stderr, flush=True)
    out = {}
    for kind in ("srht", "gaussian"):
        for variant in ("gd", "polyak"):
            def refreshed():
                x, rh, i = rs.rs_refreshed_ihs(A, b, p.nu2, m, kind=kind, variant=variant,
                                               tol=tol, raise_on_error=False)
                return x, i

            def fixed():
                return rs.rs_adaptive_solve(A, b, p.nu2, kind=kind, variant=variant, m_init=m,
                                            tol=tol, raise_on_error=False)
            for name, fn in (("refreshed", refreshed), ("fixed", fixed)):
                fn()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(args.steps):
                    x, info = fn()
                torch.cuda.synchronize()
                sec = (time.perf_counter() - t0) / args.steps
                out[f"{kind}_{variant}_{name}"] = {
                    "ms_per_solve": round(sec * 1e3, 3), "steps": info["steps"],
                    "m_final": info["m_final"], "doublings": info.get("doublings", 0),
                    "status": info["status"],
                    "rel_pred_err": ridge.relative_error(H, x.cpu().numpy(), xs)}
                print(f"[refreshed] {kind} {variant} {name}: {sec * 1e3:.2f} ms, "
                      f"{info['steps']} steps", file=sys.stderr, flush=True)
    roof = gradient_roofline(
        rs, lambda: rs.rs_refreshed_ihs(A, b, p.nu2, m, kind="srht", variant="gd", tol=tol,
                                        raise_on_error=False),
        n * d * 4 + n * 4, "k_grad_partial (A^T(AX-b) pass)", "one more SRHT gd refreshed solve")
    A64, b64 = p.A.astype(np.float64), p.b.astype(np.float64)
    cpu = oracle_rate([lambda: ridge.solve_direct(A64, b64, p.nu2)],
                      f"oracle direct FP64 Cholesky solve of the full {n}x{d} problem")
    best = "srht_gd_refreshed"
    line = {"metric": "ridge solves/s to eps = 1e-10, refreshed-embedding IHS (ablation)",
            "value": round(1e3 / out[best]["ms_per_solve"], 2), "unit": "solves/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": out[best]["ms_per_solve"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 gradient / f32 sketch / f64 factor", "data": "synthetic",
            "config": {"workload": f"{n}x{d} FP32, sigma_i=1/i, nu^2=1e-2, fixed m={m}, "
                                   "refreshed vs fixed sketch, eps=1e-10", "n": n, "d": d},
            "verified": all(v["rel_pred_err"] <= 1e-8 and v["status"] == "ok"
                            for v in out.values()),
            "roofline": roof, "cpu_baseline": cpu,
            "modes": out}
    emit(line)


def run_sparse(args):
    """Sparse A: 2^20 x 1024 CSR, 16 power-law column draws per row (about 15.8M
    stored entries, 1.5% dense), nu^2 = 0.1 (d_e about 105), eps = 1e-10: Algorithm 1
    with the CountSketch (FP32 and BF16 sketches) against the dense SRHT solver on
    the same matrix stored densely (4 GiB).  Every solution is checked against the
    oracle's direct solve from the sparse Gram."""
    import scipy.sparse as sp
    import torch
    from oracle import ridge
    from paper_2006_05874_amd import rs
    from synth import config_sparse
    torch.cuda.set_device(0)
    (rowptr, col, val, b), nu2 = config_sparse()
    n, d = rowptr.size - 1, 1024
    rp, cl, vl, bd = (torch.from_numpy(a).cuda() for a in (rowptr, col, val, b))
    tol = 1e-10
    print("[sparse] problem ready", file=sys.stderr, flush=True)
    out = {}

    def csr(sd):
        return lambda: rs.rs_adaptive_solve_csr(rp, cl, vl, d, bd, nu2, sketch_dtype=sd, tol=tol,
                                                raise_on_error=False)

    modes = [("count_f32", csr("f32")), ("count_bf16", csr("bf16"))]
    Ad = rs.padded(n, d, dtype=torch.float32)
    Ad.zero_()
    rows = torch.repeat_interleave(torch.arange(n, device="cuda"), rp[1:] - rp[:-1])
    Ad[rows, cl.long()] = vl
    del rows
    modes.append(("dense_srht_f32", lambda: rs.rs_adaptive_solve(Ad, bd, nu2, sketch_dtype="f32",
                                                                 tol=tol, raise_on_error=False)))
    for name, fn in modes:
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            x, info = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        out[name] = {"solves_per_s": round(1.0 / sec, 2), "ms_per_solve": round(sec * 1e3, 3),
                     "m_final": info["m_final"], "grad_passes": info["grad_passes"],
                     "status": info["status"], "x": x.cpu().numpy()}
        print(f"[sparse] {name}: {sec * 1e3:.2f} ms, m = {info['m_final']}", file=sys.stderr,
              flush=True)
    nnz = int(rowptr[-1])
    # per pass (2 right-hand sides): indices and values twice (rows, then columns),
    # rowptr and b, the residuals written once and read once
    roof = gradient_roofline(rs, csr("f32"), 2 * nnz * (4 + 4) + n * (8 + 4) + 2 * n * 2 * 8,
                             "sparse gradient pass (k_csr_resid .. k_csc_finish)",
                             "one more count_f32 solve")
    A = sp.csr_matrix((val.astype(np.float64), col, rowptr), shape=(n, d))
    b64 = b.astype(np.float64)

    def direct():
        Gs = (A.T @ A).toarray()
        return ridge.solve_direct_from_gram(Gs, A.T @ b64, nu2)
    cpu = oracle_rate([direct], f"oracle direct FP64 solve from the sparse Gram of the full "
                                f"{n}x{d} CSR problem (scipy sparse product, Cholesky)")
    G = (A.T @ A).toarray()
    xs = ridge.solve_direct_from_gram(G, A.T @ b.astype(np.float64), nu2)
    for v in out.values():
        v["rel_pred_err"] = ridge.relative_error(G + nu2 * np.eye(d), v.pop("x"), xs)
    best = "count_f32"
    line = {"metric": "ridge solves/s to eps = 1e-10, sparse A with the CountSketch",
            "value": out[best]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1, "ms_per_step": out[best]["ms_per_solve"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32 values / f32 sketch / f64 gradient and factor", "data": "synthetic",
            "config": {"workload": f"{n}x{d} CSR, nnz={int(rowptr[-1])}, power-law columns "
                                   f"(alpha 0.8), nu^2={nu2}, CountSketch fresh, m from 1, "
                                   "eps=1e-10", "n": n, "d": d, "nnz": int(rowptr[-1])},
            "verified": all(v["rel_pred_err"] <= 1e-8 and v["status"] == "ok"
                            for v in out.values()),
            "roofline": roof, "cpu_baseline": cpu,
            "modes": out,
            "speedup_vs_dense_srht_f32": round(out[best]["solves_per_s"]
                                               / out["dense_srht_f32"]["solves_per_s"], 3)}
    emit(line)


def run_c4b(args):
    """256 independent problems (n = 2^U{12..16}, d = U{128..1024}, sigma_i =
    0.95^i, nu^2 = 1e-3): learned-start batched solves over worker streams with
    BF16 sketches (the value), the same batch starting at m = 1, and the problems
    solved one after another by the plain method (FP32 sketch).  Every solution is
    checked against the oracle's direct solve."""
    import torch
    from oracle import ridge
    from paper_2006_05874_amd import rs
    from synth import config_c4b_specs, make_c4b_problem
    torch.cuda.set_device(0)
    specs = config_c4b_specs()
    probs = []
    for sp in specs:
        A0, b = make_c4b_problem(sp, "cuda")
        A = rs.padded(sp["n"], sp["d"], dtype=torch.float32)
        A.copy_(A0)
        probs.append((A, b, sp["nu2"]))
    del A0
    torch.cuda.synchronize()
    print(f"[c4b] {len(probs)} problems ready", file=sys.stderr, flush=True)

    from paper_2006_05874_amd import learned
    params, mu, sd, _ = learned.load_model(args.model or learned.MODEL_PATH)

    def run_learned():
        return rs.rs_learned_solve_batch(probs, params, mu, sd, sketch_dtype="bf16",
                                         workers=args.workers, graph_steps=args.graph_steps,
                                         raise_on_error=False)

    def run_batch():
        return rs.rs_solve_batch(probs, sketch_dtype="bf16", workers=args.workers,
                                 graph_steps=args.graph_steps, raise_on_error=False)

    def run_seq():
        return [rs.rs_adaptive_solve(A, b, nu2, sketch_dtype="f32", raise_on_error=False)
                for A, b, nu2 in probs]

    out = {}
    for name, fn in (("learned_bf16_batched", run_learned), ("batched_bf16", run_batch),
                     ("sequential_plain_f32", run_seq)):
        fn()                                   # warm-up (allocations)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = fn()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        out[name] = {"solves_per_s": round(len(probs) / sec, 2), "s_per_batch": round(sec, 4),
                     "res": res}
        print(f"[c4b] {name}: {len(probs) / sec:.1f} solves/s", file=sys.stderr, flush=True)
    # the gradient passes of one more learned batch, each timed by HIP events; the
    # bytes of a problem's pass are n d 4 + n 4
    torch.cuda.synchronize()
    rs.rs_profile_enable(True)
    rs.rs_profile_read()
    pres = run_learned()
    torch.cuda.synchronize()
    rs.rs_profile_enable(False)
    nl, gms = rs.rs_profile_read()
    tot = sum(info["grad_passes"] * (A.shape[0] * A.shape[1] * 4 + A.shape[0] * 4)
              for (A, _, _), (_, info) in zip(probs, pres))
    ach = tot / (gms / 1e3) / 1e9 if gms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "algorithmic_bytes": int(tot), "kernel": "k_grad_partial (every problem's passes)",
            "avg_launch_us": round(gms / max(nl, 1) * 1e3, 2), "launches": nl,
            "region": "one more learned batch; each pass timed by its own HIP start/stop "
                      "events on its worker stream (passes of different streams overlap, so "
                      "this is the bytes-weighted rate of a pass, not the device's total)"}
    # oracle check of the last batch of each kind
    worst = {k: 0.0 for k in out}
    bad = {k: 0 for k in out}
    oracle_s = 0.0
    for i, (A, b, nu2) in enumerate(probs):
        A64 = A.cpu().numpy().astype(np.float64)
        b64 = b.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        Gm = A64.T @ A64
        xs = ridge.solve_direct_from_gram(Gm, A64.T @ b64, nu2)
        oracle_s += time.perf_counter() - t0
        H = Gm + nu2 * np.eye(Gm.shape[0])
        for k in out:
            x, info = out[k]["res"][i]
            worst[k] = max(worst[k], ridge.relative_error(H, x.cpu().numpy(), xs))
            bad[k] += info["status"] != "ok"
    for k in out:
        del out[k]["res"]
        out[k]["worst_rel_pred_err"] = worst[k]
        out[k]["not_ok"] = bad[k]
    line = {"metric": "ridge solves/s to 1e-6 rel. pred. error, batched uneven problems",
            "value": out["learned_bf16_batched"]["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
            "steps": args.steps, "warmup": 1,
            "ms_per_step": round(out["learned_bf16_batched"]["s_per_batch"] * 1e3, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16 sketch / f32 gradient / f64 factor", "data": "synthetic",
            "config": {"workload": "256 problems, n=2^U{12..16}, d=U{128..1024}, "
                                   f"sigma_i=0.95^i, nu^2=1e-3, SRHT, {args.workers} worker streams, "
                                   "learned start + BF16 sketches, one host thread per worker"
                                   + (", steps replayed from HIP graphs" if args.graph_steps
                                      else ""),
                       "graph_steps": bool(args.graph_steps)},
            "verified": all(v["worst_rel_pred_err"] <= 1e-6 and v["not_ok"] == 0
                            for v in out.values()),
            "modes": out, "roofline": roof,
            "cpu_baseline": {"value": round(len(probs) / oracle_s, 3), "unit": "solves/s",
                             "cores": blas_threads(), "kind": "oracle",
                             "sample": f"the oracle's direct FP64 solves of all {len(probs)} "
                                       f"problems: {oracle_s:.1f} s"},
            "speedup_vs_sequential_plain_f32": round(
                out["learned_bf16_batched"]["solves_per_s"] /
                out["sequential_plain_f32"]["solves_per_s"], 3)}
    emit(line)


if __name__ == "__main__":
    main()
