"""Training and use of the learned starting sketch size.

  python -m paper_2006_05874_amd.learned generate --count N --first P --out FILE
  python -m paper_2006_05874_amd.learned train --data F1 [F2 ...] --out MODEL
  python -m paper_2006_05874_amd.learned evaluate --model MODEL --count N --out FILE

Training problems (problem p uses seed 10^6 + p):
  with odds 4:1 either n = 2^U{12..18}, d = U{64..2048} or the wide family
  d = U{2049..8192}, n = 2^U{14..17} (n >= 2d); a third, tall family
  (problem p uses seed 2 10^6 + p) has n = 2^U{19..21}, d = U{64..1024}.
  Singular values either
  exponential sigma_i = r^i, r ~ U[0.9, 0.999], or power law sigma_i = i^-alpha,
  alpha ~ U[0.5, 2] (even odds); nu^2 = sigma_1^2 * 10^U[-6, 0]; b = A x_pl +
  0.1 xi.  A is generated on the device (synth.make_problem_torch).
Label: log2 of the final sketch size of a plain run (fresh SRHT, FP32 sketch,
m from 1).  Features: rs_features with the same seed.  Training runs on the GPU
with rs_mlp_forward / rs_mlp_backward / rs_mlp_adam_step (MSE, Adam, batch 256,
80/20 split); the parameters kept are those of the epoch with the lowest
validation error.  The output offset (m_init = 2^floor(y + offset)) is then
chosen on separate held-out problems (p >= 10^5) by total solve time.  Every
number the model sees comes from the library's kernels.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MODEL_PATH = os.path.join(HERE, "models", "m_init_mlp.npz")


def problem_spec(p, seed_base=10 ** 6):
    rng = np.random.default_rng(seed_base + p)
    if rng.random() < 0.8:
        n = 2 ** int(rng.integers(12, 19))
        d = int(rng.integers(64, 2049))
    else:
        n = 2 ** int(rng.integers(14, 18))
        d = int(rng.integers(2049, 8193))
    if rng.random() < 0.5:
        kind, rate = "geom", float(rng.uniform(0.9, 0.999))
    else:
        kind, rate = "poly", float(rng.uniform(0.5, 2.0))
    nu2_rel = 10.0 ** float(rng.uniform(-6.0, 0.0))
    return {"p": p, "seed": seed_base + p, "n": n, "d": d, "kind": kind, "rate": rate,
            "nu2": nu2_rel}   # sigma_1 = 1 for both families


def tall_spec(p, seed_base=2 * 10 ** 6):
    """The tall family: n = 2^U{19..21}, d = U{64..1024}, the same spectra and nu^2."""
    rng = np.random.default_rng(seed_base + p)
    n = 2 ** int(rng.integers(19, 22))
    d = int(rng.integers(64, 1025))
    if rng.random() < 0.5:
        kind, rate = "geom", float(rng.uniform(0.9, 0.999))
    else:
        kind, rate = "poly", float(rng.uniform(0.5, 2.0))
    nu2_rel = 10.0 ** float(rng.uniform(-6.0, 0.0))
    return {"p": p, "seed": seed_base + p, "n": n, "d": d, "kind": kind, "rate": rate,
            "nu2": nu2_rel, "family": "tall"}


FAMILIES = {"mixed": problem_spec, "tall": tall_spec}


def make_device_problem(spec, device="cuda"):
    import torch
    from synth import spectrum
    from synth.problems import make_problem_torch
    from . import rs
    sig = spectrum(spec["kind"], spec["d"], spec["rate"])
    A0, b, _ = make_problem_torch(spec["n"], spec["d"], sig, 0.1, spec["seed"], device)
    A = rs.padded(spec["n"], spec["d"], dtype=torch.float32)
    A.copy_(A0)
    del A0
    return A, b


def generate(count, first, out, log_every=100, max_seconds=None, family="mixed"):
    """Features and labels of problems first .. first + count - 1 of a family,
    saved to out every log_every problems; stops early (after a whole problem)
    once max_seconds have passed."""
    import torch
    from . import rs
    rows = []
    t0 = time.time()
    for p in range(first, first + count):
        if max_seconds is not None and time.time() - t0 > max_seconds:
            print(f"[generate] time budget reached after {p - first} problems", flush=True)
            break
        spec = FAMILIES[family](p)
        A, b = make_device_problem(spec)
        f = rs.rs_features(A, spec["nu2"], seed=spec["seed"])
        t1 = time.time()
        x, info = rs.rs_adaptive_solve(A, b, spec["nu2"], kind="srht", sketch_dtype="f32",
                                       seed=spec["seed"], raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.time() - t1
        rows.append({**spec, "features": f.cpu().numpy().tolist(), "m_final": info["m_final"],
                     "status": info["status"], "passes": info["grad_passes"],
                     "solve_s": dt})
        del A, b, x
        if (p - first + 1) % log_every == 0:
            print(f"[generate] {p - first + 1}/{count} problems, {time.time() - t0:.1f}s",
                  flush=True)
            _save_rows(rows, out)
    _save_rows(rows, out)
    return rows


def _save_rows(rows, out):
    ok = [r for r in rows if r["status"] == "ok"]
    np.savez(out, features=np.array([r["features"] for r in ok], dtype=np.float32),
             label=np.array([math.log2(r["m_final"]) for r in ok], dtype=np.float32),
             meta=json.dumps(rows))


def load_data(paths):
    F, L = [], []
    for path in paths:
        z = np.load(path, allow_pickle=False)
        F.append(z["features"])
        L.append(z["label"])
    return np.concatenate(F), np.concatenate(L)


def _he_init(seed):
    """W ~ N(0, 2 / fan_in), biases 0 (flat layout of include/rs.h)."""
    rng = np.random.default_rng(seed)
    th = np.zeros(18817, dtype=np.float32)
    th[0:2048] = rng.standard_normal(2048) * math.sqrt(2.0 / 16)
    th[2176:18560] = rng.standard_normal(16384) * math.sqrt(2.0 / 128)
    th[18688:18816] = rng.standard_normal(128) * math.sqrt(1.0 / 128)
    return th


def train(F, L, epochs=300, batch=256, lr=1e-3, seed=0, log_every=25, val_frac=0.2,
          select_every=5):
    """Train on the GPU with the library's kernels.  The validation error is taken
    every select_every epochs and the parameters of the lowest one are kept.
    Returns (params, mu, sd, history, selected) with selected = {"epoch",
    "val_mse", "train_mse"} of the kept parameters."""
    import torch
    from . import rs
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(L))
    nval = int(len(L) * val_frac)
    val, tr = idx[:nval], idx[nval:]
    mu = F[tr].mean(0).astype(np.float32)
    sd = (F[tr].std(0) + 1e-3).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    P = dev(_he_init(seed))
    P[18816] = float(L[tr].mean())
    M, V = torch.zeros_like(P), torch.zeros_like(P)
    mud, sdd = dev(mu), dev(sd)
    Ftr, Ltr = dev(F[tr].astype(np.float32)), dev(L[tr].astype(np.float32))
    Fva, Lva = dev(F[val].astype(np.float32)), dev(L[val].astype(np.float32))
    hist = []
    step = 0
    best, best_p = None, P.clone()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(len(tr))).cuda()
        for b0 in range(0, len(tr) - batch + 1, batch):
            sel = perm[b0:b0 + batch]
            step += 1
            _, C = rs.rs_mlp_forward(P, Ftr[sel], mud, sdd, cache=True)
            G, loss = rs.rs_mlp_backward(P, C, Ltr[sel])
            rs.rs_mlp_adam_step(P, G, M, V, step, lr=lr)
        last = ep == epochs - 1
        if (ep + 1) % select_every == 0 or (ep + 1) % log_every == 0 or last:
            ytr = rs.rs_mlp_forward(P, Ftr, mud, sdd)
            yva = rs.rs_mlp_forward(P, Fva, mud, sdd)
            mtr = float(torch.mean((ytr - Ltr) ** 2))
            mva = float(torch.mean((yva - Lva) ** 2))
            if best is None or mva < best["val_mse"]:
                best = {"epoch": ep + 1, "val_mse": mva, "train_mse": mtr}
                best_p.copy_(P)
            if (ep + 1) % log_every == 0 or last:
                hist.append({"epoch": ep + 1, "train_mse": mtr, "val_mse": mva})
                print(f"[train] epoch {ep + 1} train mse {mtr:.4f} val mse {mva:.4f}", flush=True)
    print(f"[train] kept epoch {best['epoch']} (val mse {best['val_mse']:.4f})", flush=True)
    return best_p.cpu().numpy(), mu, sd, hist, best


def save_model(path, params, mu, sd, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=params.astype(np.float32), mu=mu, sd=sd, meta=json.dumps(meta))


def load_model(path=MODEL_PATH):
    import torch
    z = np.load(path, allow_pickle=False)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return dev(z["params"]), dev(z["mu"]), dev(z["sd"]), json.loads(str(z["meta"]))


def evaluate(model_path, count, first, out, offsets=(0.0,), log_every=50, family="mixed"):
    """Held-out problems: plain (m from 1, FP32 sketch) against the learned start
    with each bias offset (added to the output bias: m_init = 2^floor(y + off)).
    Records each solve's time, final m, passes and status."""
    import torch
    from . import rs
    params, mu, sd, _ = load_model(model_path)
    rows = []
    for p in range(first, first + count):
        spec = FAMILIES[family](p)
        A, b = make_device_problem(spec)
        res = {**spec}
        for mode in ["plain"] + [f"learned{o:+.2f}" for o in offsets]:
            th = params
            if mode != "plain":
                th = params.clone()
                th[OFF_B3] += float(mode[len("learned"):])
            torch.cuda.synchronize()
            t1 = time.time()
            if mode == "plain":
                x, info = rs.rs_adaptive_solve(A, b, spec["nu2"], seed=spec["seed"],
                                               raise_on_error=False)
            else:
                x, info = rs.rs_learned_solve(A, b, spec["nu2"], th, mu, sd, seed=spec["seed"],
                                              raise_on_error=False)
            torch.cuda.synchronize()
            res[mode] = {"s": time.time() - t1, "m_final": info["m_final"],
                         "passes": info["grad_passes"], "status": info["status"],
                         "m_init": info.get("m_init", 1), "doublings": info["doublings"]}
        rows.append(res)
        del A, b
        if (p - first + 1) % log_every == 0:
            print(f"[evaluate] {p - first + 1}/{count}", flush=True)
    summary = summarize(rows)
    with open(out, "w") as f:
        json.dump({"summary": summary, "rows": rows}, f)
    return rows, summary


def summarize(rows):
    modes = [k for k in rows[0] if k == "plain" or k.startswith("learned")]
    out = {}
    for k in modes:
        t = np.array([r[k]["s"] for r in rows])
        out[k] = {"total_s": float(t.sum()), "median_s": float(np.median(t)),
                  "mean_doublings": float(np.mean([r[k]["doublings"] for r in rows])),
                  "mean_passes": float(np.mean([r[k]["passes"] for r in rows])),
                  "not_ok": int(sum(r[k]["status"] != "ok" for r in rows))}
    base = out["plain"]["total_s"]
    for k in modes:
        out[k]["speedup_total"] = base / out[k]["total_s"]
    return out


OFF_B3 = 18816


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("generate")
    g.add_argument("--count", type=int, required=True)
    g.add_argument("--first", type=int, default=0)
    g.add_argument("--out", required=True)
    g.add_argument("--max-seconds", type=float, default=None)
    g.add_argument("--log-every", type=int, default=100)
    g.add_argument("--family", default="mixed", choices=sorted(FAMILIES))
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--out", default=MODEL_PATH)
    t.add_argument("--epochs", type=int, default=300)
    e = sub.add_parser("evaluate")
    e.add_argument("--model", default=MODEL_PATH)
    e.add_argument("--count", type=int, default=200)
    e.add_argument("--first", type=int, default=10 ** 5)
    e.add_argument("--offsets", type=float, nargs="+", default=[0.0])
    e.add_argument("--out", required=True)
    e.add_argument("--family", default="mixed", choices=sorted(FAMILIES))
    f = sub.add_parser("finalize", help="fold the chosen offset into the output bias")
    f.add_argument("--model", required=True)
    f.add_argument("--eval", required=True)
    f.add_argument("--out", default=MODEL_PATH)
    a = ap.parse_args()
    if a.cmd == "generate":
        generate(a.count, a.first, a.out, log_every=a.log_every, max_seconds=a.max_seconds,
                 family=a.family)
    elif a.cmd == "train":
        F, L = load_data(a.data)
        params, mu, sd, hist, sel = train(F, L, epochs=a.epochs)
        save_model(a.out, params, mu, sd, {"problems": int(len(L)), "history": hist,
                                           "selected": sel,
                                           "data": [os.path.basename(x) for x in a.data]})
        print(f"saved {a.out}", flush=True)
    elif a.cmd == "evaluate":
        _, summary = evaluate(a.model, a.count, a.first, a.out, offsets=a.offsets,
                              family=a.family)
        print(json.dumps(summary, indent=1), flush=True)
    else:
        summary = json.load(open(a.eval))["summary"]
        best = max((k for k in summary if k.startswith("learned")),
                   key=lambda k: summary[k]["speedup_total"])
        off = float(best[len("learned"):])
        z = np.load(a.model, allow_pickle=False)
        params = z["params"].copy()
        params[OFF_B3] += off
        meta = json.loads(str(z["meta"]))
        meta["output_offset"] = off
        meta["evaluation"] = summary
        save_model(a.out, params, z["mu"], z["sd"], meta)
        print(f"offset {off:+.2f} -> {a.out}", flush=True)


if __name__ == "__main__":
    main()
