"""Time single hot-path calls of librs on one GPU (also the program the counter
and kernel-trace summaries under profiles/ are taken from).

  python -m paper_2006_05874_amd.kernel_bench gradient --n N --d D --k K --reps R
  python -m paper_2006_05874_amd.kernel_bench srht --n N --d D --m M --sa bf16 --reps R
  python -m paper_2006_05874_amd.kernel_bench gaussian --n N --d D --m M --sa bf16 --reps R
  python -m paper_2006_05874_amd.kernel_bench pair --n N --d D --reps R

pair: one learned + BF16 batch of two solves on A, b (nu^2 = 1e-2 and 1e-4), which
runs as a pair: its features pass (k_srht_p1_two) also forms the first sketches'
first pass; the line gives the whole batch and N D 4 bytes.

A is N x D FP32 with i.i.d. N(0, 1/N) entries and b N(0, 1), drawn on the device
(the values do not change the traffic of either pass).  Each call is timed by HIP
events on the stream; the line printed per call gives milliseconds and the
algorithmic bytes over that time (gradient: N D 4 + N 4 per pass, A and b read
once; SRHT: N D 4 + M D s, A read once and SA written; Gaussian: also 2 M N D flops,
printed as TFLOP/s).  --copy-calibration first
runs one 256 MiB device-to-device copy, the reference for HBM counters.
"""
import argparse
import sys

import torch

from . import rs


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["gradient", "gradient2", "srht", "gaussian", "pair"])
    ap.add_argument("--n", type=int, default=1 << 21)
    ap.add_argument("--d", type=int, default=8192)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--m", type=int, default=2048)
    ap.add_argument("--sa", default="bf16", choices=["f32", "bf16", "fp8"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if a.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, d = a.n, a.d
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    A = rs.padded(n, d, dtype=torch.float32)
    for r0 in range(0, n, 1 << 16):
        A[r0:r0 + (1 << 16)].normal_(0.0, n ** -0.5, generator=gen)
    b = torch.randn(n, device="cuda", generator=gen)
    torch.cuda.synchronize()
    if a.what == "gradient":
        X = torch.randn(a.k, d, dtype=torch.float64, device="cuda", generator=gen)
        if not a.no_tune:
            print("plan", rs.rs_gradient_autotune(A, b, k=a.k), flush=True)
        call = lambda: rs.rs_gradient(A, b, 0.01, X)
        alg = n * d * 4 + n * 4
    elif a.what == "gradient2":
        # two problems on the same A and b, two columns each, in one read of A
        X0 = torch.randn(2, d, dtype=torch.float64, device="cuda", generator=gen)
        X1 = torch.randn(2, d, dtype=torch.float64, device="cuda", generator=gen)
        if not a.no_tune:
            print("plan", rs.rs_gradient_autotune(A, b, k=2), flush=True)
        call = lambda: rs.rs_gradient_two(A, b, (0.01, 0.0001), X0, X1)
        alg = n * d * 4 + n * 4
    elif a.what == "pair":
        from . import learned
        for k in (1, 2):
            print("plan", k, rs.rs_gradient_autotune(A, b, k=k), flush=True)
        params, mu, sd, _ = learned.load_model(learned.MODEL_PATH)
        call = lambda: rs.rs_learned_solve_batch([(A, b, 1e-2), (A, b, 1e-4)], params, mu, sd,
                                                 sketch_dtype="bf16", workers=2)
        alg = n * d * 4
    else:
        es = {"f32": 4, "bf16": 2, "fp8": 1}[a.sa]
        sid = [0]
        sketch = rs.rs_sketch_srht if a.what == "srht" else rs.rs_sketch_gaussian

        def call():
            sid[0] += 1
            return sketch(A, a.m, sketch_id=sid[0], sa_dtype=a.sa)
        alg = n * d * 4 + a.m * d * es
    call()
    torch.cuda.synchronize()
    for r in range(a.reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        extra = (f", {2.0 * a.m * n * d / ms / 1e9:.1f} TFLOP/s" if a.what == "gaussian" else "")
        print(f"{a.what} n={n} d={d} rep {r}: {ms:.3f} ms, {alg / ms / 1e6:.1f} GB/s algorithmic"
              + extra, flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
