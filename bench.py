#!/usr/bin/env python3
"""Benchmark: SGD updates/s of s-step (communication-avoiding) SGD on one MI355X.

Workload (the dense FP32 configuration): X is 2^20 x 2048 FP32 with N(0, 1/2048)
entries and 205 seeded columns scaled x10, labels sign(Xw) with 5% flips,
b = 64, lambda = 1e-5, seed 42. One "step" is one outer iteration of the
method: sample s*b rows, Gram + margins, s residual corrections, one update
(s SGD updates). `value` is SGD updates per second over the K timed steps of
one fused launch (inputs already resident in HBM).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--s 16] [--dtype f32]

Prints one JSON line. `--sweep` adds a per-s table; `--eta-sweep` runs the
step-size selection (one epoch of plain SGD per candidate); `--no-cpu` skips
the CPU-oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Step size of the dense FP32 workload, chosen by the one-epoch plain-SGD sweep
# over powers of two (bench.py --eta-sweep); reused for every s and precision.
ETA_C2 = 2.0
LAMBDA_C2 = 1e-5
B_C2 = 64
SEED = 42

PEAK = {  # MI355X published dense peaks
    "hbm_GBps": 8000.0,
    "f32_TFLOPs": 157.3, "bf16_TFLOPs": 2500.0, "f16_TFLOPs": 2500.0, "fp8_TFLOPs": 5000.0,
    "f64_TFLOPs": 78.6,
}
DT_NAME = {"f32": 0, "bf16": 1, "f16": 2, "fp8": 3}
DT_BYTES = {"f32": 4, "bf16": 2, "f16": 2, "fp8": 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def outer_flops(b: int, s: int, n: int) -> float:
    """Algorithmic flops of one outer iteration: strict block-lower Gram
    s(s-1) b^2 n, margins 2 s b n, update 2 s b n, corrections b^2 s (s-1)."""
    return s * (s - 1) * b * b * n + 4.0 * s * b * n + b * b * s * (s - 1)


def outer_bytes(b: int, s: int, n: int, e: int) -> float:
    """Algorithmic HBM bytes of one outer iteration: the sampled rows once,
    x read and written, indices and labels."""
    return s * b * n * e + 8.0 * n + 8.0 * s * b + (4.0 * s * b if e == 1 else 0.0)


def gram_flops(b: int, s: int, n: int) -> float:
    return s * (s - 1) * b * b * n


def paper_ai(b: int, s: int, n: int, e: int) -> float:
    """The paper's roofline arithmetic intensity convention (Fig. 5):
    2 (sb)^2 n / (2 sb n e + 4 (sb)^2)."""
    sb = s * b
    return 2.0 * sb * sb * n / (2.0 * sb * n * e + 4.0 * sb * sb)


class Workload:
    def __init__(self, m: int, n: int, seed: int = SEED, with_test: bool = False):
        from workloads import dense_c2
        t = time.perf_counter()
        self.p = dense_c2(seed, m=m, n=n, m_test=(m // 4 if with_test else 1))
        log(f"[bench] generated X {m}x{n} fp32 in {time.perf_counter() - t:.1f}s")
        self.m, self.n = m, n


def upload(cg, wl: Workload, dtype: str):
    import torch
    Xd = torch.from_numpy(wl.p.X).to("cuda")
    y = torch.from_numpy(wl.p.y).to("cuda")
    if dtype == "f32":
        return cg.dense_matrix(Xd), y, Xd
    stored, scale = cg.casgd_quantize(Xd, DT_NAME[dtype])
    del Xd
    torch.cuda.synchronize()
    return cg.dense_matrix(stored, scale, n=wl.n), y, stored


def timed_fit(cg, X, y, n, b, s, eta, lam, K, W, opts_kw):
    """Warm up W outer iterations, then time K in one launch with HIP events
    on the stream the kernels run on. Returns (ms, x, ws)."""
    import torch
    stream = torch.cuda.current_stream()
    x = torch.zeros(n, device="cuda")
    o = cg.opts(**opts_kw)
    ws = cg.workspace(cg.casgd_workspace_size(X, b, s))
    if W > 0:
        cg.casgd_fit(X, y, x, eta, lam, b, s, SEED, 0, W, opts=o, ws=ws, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    cg.casgd_fit(X, y, x, eta, lam, b, s, SEED, W, K, opts=o, ws=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    cg.casgd_check(ws)
    return e0.elapsed_time(e1), x, ws


def gram_roofline(cg, X, n, b, s, dtype, reps=20):
    """Average duration of the standalone Gram kernel (one launch per outer
    iteration), timed with HIP events over `reps` launches."""
    import torch
    if s < 2:
        return None
    stream = torch.cuda.current_stream()
    sb = s * b
    G = torch.zeros(sb, sb, device="cuda")
    ws = cg.workspace(cg.casgd_workspace_size(X, b, s))
    for h in range(3):
        cg.casgd_gram_margin(X, None, b, s, SEED, h, G=G, ws=ws, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for h in range(reps):
        cg.casgd_gram_margin(X, None, b, s, SEED, h, G=G, ws=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    fl = gram_flops(b, s, n)
    peak = PEAK[f"{dtype}_TFLOPs"]
    ach = fl / (ms * 1e-3) / 1e12
    return {"kernel": "k_gram (one launch: zero-counters + Gram tiles)", "bound": "mfma",
            "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 4), "us_per_launch": round(ms * 1e3, 3),
            "flops_per_launch": fl,
            "paper_convention_TFLOPs": round(2.0 * sb * sb * n / (ms * 1e-3) / 1e12, 3),
            "paper_ai": round(paper_ai(b, s, n, DT_BYTES[dtype]), 1)}


# Gram shapes of the roofline study: the dense 2^20 x 2048 workload at
# s = 16, 32 (b = 64), the precision-sweep shape (4096 x 256, b = 128, s = 32)
# and the paper's per-kernel roofline shape (Fig. 5: m = 8192, n = 16384,
# b = 32, s = 32 .. 128).
GRAM_SHAPES = [(1 << 20, 2048, 64, 16), (1 << 20, 2048, 64, 32), (4096, 256, 128, 32),
               (8192, 16384, 32, 32), (8192, 16384, 32, 64), (8192, 16384, 32, 128)]


def gram_shapes_bench(cg, dtypes, reps=10, shapes=None):
    """Standalone Gram launches (casgd_gram_margin without margins: one
    counter-clearing, one gather and one Gram launch per call) at the roofline
    shapes, for each storage type. Timed with HIP events per call (gather
    included); the Gram kernel alone is read from a kernel trace of this mode."""
    import torch
    stream = torch.cuda.current_stream()
    rows = []
    for (m, n, b, s) in (shapes or GRAM_SHAPES):
        g = torch.Generator(device="cuda")
        g.manual_seed(m * 7 + n)
        X32 = torch.randn(m, n, device="cuda", generator=g) * (1.0 / math.sqrt(n))
        for dt in dtypes:
            if dt == "f32":
                X = cg.dense_matrix(X32)
                keep = None
            else:
                keep = cg.casgd_quantize(X32, DT_NAME[dt])
                X = cg.dense_matrix(keep[0], keep[1], n=n)
            sb = s * b
            G = torch.empty(sb, sb, device="cuda")
            base = cg.casgd_workspace_size(X, b, s)
            split = cg.casgd_gram_workspace_size(X, b, s)
            ws = cg.workspace(split)
            kinds = [(64, base), (128, base)] + ([(128, split)] if split > base else [])
            for tile, nb in kinds:
                o = cg.opts(gram_tile=tile)
                ksplit = nb > base
                wsv = ws[:nb]
                for h in range(2):
                    cg.casgd_gram_margin(X, None, b, s, SEED, h, G=G, ws=wsv, stream=stream, opts=o)
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for h in range(reps):
                    cg.casgd_gram_margin(X, None, b, s, SEED, h, G=G, ws=wsv, stream=stream, opts=o)
                e1.record(stream)
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) * 1e3 / reps
                fl = gram_flops(b, s, n)
                rows.append({"m": m, "n": n, "b": b, "s": s, "storage": dt, "gram_tile": tile,
                             "k_split": ksplit, "us_per_call_with_gather": round(us, 3),
                             "gram_flops": fl, "paper_flops": 2.0 * sb * sb * n})
                log(f"[gram] m={m} n={n} b={b} s={s} {dt} tile {tile}"
                    f"{' split along K' if ksplit else ''}: {us:.2f} us per call "
                    f"({fl / (us * 1e-6) / 1e12:.1f} TFLOP/s incl. gather)")
            del G, ws, wsv, X, keep
        del X32
        torch.cuda.empty_cache()
    return {"metric": "standalone Gram launches at the roofline shapes", "rows": rows}


def e2e_study(cg, H: int = 320_000, snaps: int = 64):
    """Error study of the precision recipes on the 4096 x 256 workload
    (logistic, b = 32, s = 16, eta = 0.1, lambda = 0, the paper's long-horizon
    setting): FP32 everywhere; BF16 and FP16 storage with FP32 elsewhere (the
    mixed recipes); and the end-to-end BF16 and FP16 baselines (every slot
    rounded to the format). Relative test-loss gap to the FP32 run at every
    snapshot."""
    import torch
    from workloads import dense_c1
    p = dense_c1(SEED)
    b, s, eta, lam = 32, 16, 0.1, 0.0
    Xt = cg.dense_matrix(torch.from_numpy(p.X_test.astype(np.float32)).cuda())
    yt = torch.from_numpy(p.y_test.astype(np.float32)).cuda()
    y = torch.from_numpy(p.y.astype(np.float32)).cuda()
    X32 = torch.from_numpy(p.X.astype(np.float32)).cuda()
    every = H // snaps
    out = {}
    for name, dt, e2e in (("fp32", cg.F32, 0), ("bf16 storage", cg.BF16, 0),
                          ("fp16 storage", cg.F16, 0), ("e2e fp16", cg.F16, 2),
                          ("e2e bf16", cg.BF16, 1)):
        v, sc = cg.casgd_quantize(X32, dt)
        X = cg.dense_matrix(v, sc, n=256)
        hist = torch.zeros(snaps, 256, device="cuda")
        x = torch.zeros(256, device="cuda")
        o = cg.opts(snapshot_every=every, x_history=hist, e2e=e2e)
        t0 = time.perf_counter()
        ws = cg.casgd_fit(X, y, x, eta, lam, b, s, SEED, 0, snaps * every, opts=o)
        torch.cuda.synchronize()
        cg.casgd_check(ws)
        out[name] = cg.casgd_logloss(Xt, yt, hist).cpu().numpy()
        log(f"[e2e-study] {name}: {time.perf_counter() - t0:.1f}s, final test loss "
            f"{out[name][-1]:.8f}")
    ref = out["fp32"]
    rows = {k: {"final_rel_gap": float(abs(v[-1] - ref[-1]) / ref[-1]),
                "max_rel_gap": float(np.max(np.abs(v - ref) / ref)),
                "final_test_loss": float(v[-1])} for k, v in out.items()}
    return {"metric": "relative test-loss gap to FP32 (precision recipes)",
            "workload": "dense 4096x256 logistic (N(0,1/256)), b=32, s=16, eta=0.1, lambda=0",
            "outer_iterations": snaps * every, "snapshots": snaps, "recipes": rows}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl: Workload, b, s, eta, lam, budget_s=12.0, budget1_s=8.0):
    """The FP64 oracle (as it stands) on the host cores: outer iterations of the
    same workload until about `budget_s` seconds have been spent with every
    thread the oracle uses, then about `budget1_s` seconds on one thread."""
    from oracle import reference as R

    def run(budget):
        x = np.zeros(wl.n)
        t = time.perf_counter()
        x = R.casgd(wl.p.X, wl.p.y, x, eta, lam, b, s, SEED, 0, 1)
        t1 = time.perf_counter() - t
        k = max(1, min(10_000, int(budget / max(t1, 1e-6))))
        t = time.perf_counter()
        R.casgd(wl.p.X, wl.p.y, x, eta, lam, b, s, SEED, 1, k)
        return k, time.perf_counter() - t

    cores = R.threads()
    k, dt = run(budget_s)
    R.set_threads(1)
    k1, dt1 = run(budget1_s)
    R.set_threads(cores)
    return {"value": round(s * k / dt, 2), "unit": "SGD updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread_value": round(s * k1 / dt1, 2),
            "sample": f"{k} outer iterations (b={b}, s={s}) of the 2^20x2048 workload, "
                      f"FP64 C oracle, {dt:.1f}s on {cores} threads; {k1} outer iterations, "
                      f"{dt1:.1f}s on one thread"}


def eta_sweep(cg, wl: Workload, etas):
    """One epoch of plain FP32 SGD (s = 1) per step size; test loss of each."""
    import torch
    X, y, _ = upload(cg, wl, "f32")
    Xt = cg.dense_matrix(torch.from_numpy(wl.p.X_test).cuda())
    yt = torch.from_numpy(wl.p.y_test).cuda()
    steps = wl.m // B_C2
    out = {}
    for eta in etas:
        x = torch.zeros(wl.n, device="cuda")
        ws = cg.casgd_fit(X, y, x, eta, LAMBDA_C2, B_C2, 1, SEED, 0, steps)
        try:
            cg.casgd_check(ws)
            out[eta] = float(cg.casgd_logloss(Xt, yt, x))
        except cg.CasgdError:
            out[eta] = float("inf")
        log(f"[eta-sweep] eta={eta:g} test loss {out[eta]:.6f}")
    return out


TARGET_GAP = 1e-3   # time-to-target: first snapshot with test loss <= L* (1 + gap)


def golden_target():
    """L*: the FP64 oracle's plain SGD test loss after the full 20-epoch budget
    (tests/golden/c2_target.json, written by tests/golden/make_c2_target.py)."""
    with open(os.path.join(ROOT, "tests", "golden", "c2_target.json")) as f:
        return json.load(f)


def time_to_target(cg, wl: Workload, Xt, yt, dtype: str, s: int, epochs: float, snaps_per_epoch: int,
                   L_star: float):
    """Fit from zero for `epochs` epochs in one fused launch with snapshots of x
    (and the device clock) every 1/snaps_per_epoch epoch; the test losses of
    the snapshots are computed afterwards, outside the timed launch."""
    import torch
    X, y, keep = upload(cg, wl, dtype)
    b = B_C2
    steps_per_epoch = wl.m // b
    every = max(1, steps_per_epoch // (snaps_per_epoch * s))      # outer iterations
    H = int(epochs * steps_per_epoch / s) // every * every
    k = H // every
    hist = torch.zeros(k, wl.n, device="cuda")
    th = torch.zeros(k + 1, dtype=torch.int64, device="cuda")
    x = torch.zeros(wl.n, device="cuda")
    o = cg.opts(exec_mode=1, snapshot_every=every, x_history=hist, t_history=th)
    ws = cg.casgd_fit(X, y, x, ETA_C2, LAMBDA_C2, b, s, SEED, 0, H, opts=o)
    torch.cuda.synchronize()
    cg.casgd_check(ws)
    losses = cg.casgd_logloss(Xt, yt, hist).cpu().numpy()
    t = (th.cpu().numpy() - int(th[0])) * 1e-8           # device clock: 100 MHz
    target = L_star * (1.0 + TARGET_GAP)
    first = trailing_hit(losses, target, max(2, snaps_per_epoch // 2))
    del X, keep
    return {"storage": dtype, "s": s, "b": b, "updates_per_snapshot": every * s,
            "updates_to_target": None if first is None else (first + 1) * every * s,
            "seconds_to_target": None if first is None else round(float(t[first + 1]), 6),
            "seconds_total": round(float(t[-1]), 6), "updates_total": H * s,
            "trailing_mean_at_target": None if first is None else round(float(
                np.mean(losses[first + 1 - max(2, snaps_per_epoch // 2):first + 1])), 7),
            "final_loss": round(float(losses[-1]), 7),
            "updates_per_s": round(H * s / float(t[-1]), 1)}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3):
    """A plain device copy of known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    a = torch.empty(nbytes // 4, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}))


def sources_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_18463_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))
                    + glob.glob(os.path.join(csrc, "*.cpp"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(name: str, outer_per_launch: int):
    """HBM bytes per launch from a committed PMC summary (profiles/<name>.json),
    or None when it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_hash") != sources_hash():
        return None
    return round(d["hbm_bytes_per_outer"] * outer_per_launch)


def c4_bench(cg, steps: int, warmup: int):
    """Sparse CSR regularisation path: 10^6 x 2^17, ~50 nnz/row (Zipf 1.1), 32
    lambdas in one persistent launch sharing every sampled block and its Gram,
    b = 128, s = 16, FP32."""
    import torch
    from workloads import lambda_path_c4, sparse_c4
    t = time.perf_counter()
    p = sparse_c4(SEED)
    log(f"[c4] generated CSR {p.m}x{p.n}, {p.values.size} nnz in {time.perf_counter() - t:.1f}s")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    X = cg.csr_matrix(dev(p.row_ptr), dev(p.col_idx), dev(p.values), p.n)
    Xt = cg.csr_matrix(dev(p.test_row_ptr), dev(p.test_col_idx), dev(p.test_values), p.n)
    y, yt = dev(p.y), dev(p.y_test)
    lams = [float(v) for v in lambda_path_c4()]
    L, b, s = len(lams), 128, 16
    ws = cg.casgd_sparse_prepare(X, b, s, L)
    # step size: best lane's test loss after a quarter epoch, eta in 2^k
    quarter = max(1, p.m // (4 * b * s))
    best = None
    for k in range(0, 10):
        eta = 2.0 ** k
        xl = torch.zeros(p.n, L, device="cuda")
        cg.casgd_fit_path(X, y, xl, lams, eta, b, s, SEED, 0, quarter, ws=ws)
        try:
            cg.casgd_check(ws)
        except cg.CasgdError as err:   # diverged: larger steps will too
            log(f"[c4] eta={eta:g}: {err}")
            cg.casgd_reset(ws)
            break
        loss = float(cg.casgd_logloss(Xt, yt, xl.t().contiguous()).min())
        log(f"[c4] eta={eta:g}: best-lane test loss {loss:.6f}")
        if math.isfinite(loss) and (best is None or loss < best[0]):
            best = (loss, eta)
    eta = best[1]
    xl = torch.zeros(p.n, L, device="cuda")
    stream = torch.cuda.current_stream()
    cg.casgd_fit_path(X, y, xl, lams, eta, b, s, SEED, 0, warmup, ws=ws, stream=stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    cg.casgd_fit_path(X, y, xl, lams, eta, b, s, SEED, warmup, steps, ws=ws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    cg.casgd_check(ws)
    ms = e0.elapsed_time(e1)
    losses = cg.casgd_logloss(Xt, yt, xl.t().contiguous()).cpu().numpy()
    # algorithmic bytes of one outer iteration, from one sampled block: its
    # nonzeros (value + column) and row offsets once, and the lane rows of x
    # for the distinct columns it touches, read and written
    idx = cg.casgd_sample_indices(SEED, warmup * s * b, s * b, p.m).cpu().numpy()
    nnz = int((p.row_ptr[idx + 1] - p.row_ptr[idx]).sum())
    cols = np.unique(np.concatenate([p.col_idx[p.row_ptr[i]:p.row_ptr[i + 1]] for i in idx]))
    by = nnz * 8 + 16 * s * b + cols.size * L * 8
    ups = s * steps / (ms * 1e-3)
    ach = by * steps / (ms * 1e-3) / 1e9
    return {"metric": "SGD updates/s per lambda lane (sparse CSR lambda path)",
            "value": round(ups, 1), "unit": "SGD updates/s", "lanes": L,
            "lane_updates_per_s": round(ups * L, 1), "steps": steps, "warmup": warmup,
            "ms_per_step": round(ms / steps, 6), "eta": eta, "dtype": "f32",
            "config": {"workload": f"sparse CSR {p.m}x{p.n}, ~50 nnz/row Zipf(1.1), "
                                   f"{L} lambdas 1e-7..1e-2, b={b}, s={s}"},
            "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": PEAK["hbm_GBps"],
                         "unit": "GB/s", "frac": round(ach / PEAK["hbm_GBps"], 5),
                         "algorithmic_bytes_per_outer": by, "sampled_nnz": nnz,
                         "distinct_columns": int(cols.size)},
            "test_loss_by_lane": [round(float(v), 6) for v in losses]}


def autotune_bench(cg, wl):
    """The tuner on the 2^20 x 2048 FP32 workload at b = 64: every candidate
    (s, execution form) it measures and the choice it stores."""
    from paper_2606_18463_amd import autotune as at
    X, y, _keep = upload(cg, wl, "f32")
    res = []
    c = at.tune(X, y, B_C2, ETA_C2, LAMBDA_C2, SEED, s_grid=(1, 4, 16, 32),
                budget_s=0.05, results=res)
    name = {(0, 1): "fused v1", (0, 2): "fused v2", (0, 3): "fused v3", (2, 0): "stream"}
    for r in res:
        log(f"[autotune] s={r.s:2d} {name[(r.exec_mode, r.variant)]:9s} {r.updates_per_s:10.0f} updates/s")
    return {"metric": "autotuner candidates (SGD updates/s)",
            "workload": f"dense {wl.m}x{wl.n} FP32, lambda={LAMBDA_C2}, eta={ETA_C2}", "b": B_C2,
            "choice": {"s": c.s, "form": name[(c.exec_mode, c.variant)],
                       "updates_per_s": round(c.updates_per_s, 1)},
            "candidates": [{"s": r.s, "form": name[(r.exec_mode, r.variant)],
                            "updates_per_s": round(r.updates_per_s, 1)} for r in res]}


def c5_batch_bench(cg, H: int, count: int = 64):
    """The uneven workload at full size: `count` problems, m log-uniform in
    [1e4, 2e5], n in [128, 4096], BF16 storage, b = 64, s = 16, H outer
    iterations each. One batched launch (automatic groups) against the same
    problems launched one after another; both timed with HIP events."""
    import torch
    from workloads import uneven_problem, uneven_problem_specs
    b, s, lam = 64, 16, 1e-5
    t = time.perf_counter()
    probs = []
    for i, sp in enumerate(uneven_problem_specs(count, 2024)):
        p = uneven_problem(sp)
        stored, scale = cg.casgd_quantize(torch.from_numpy(p.X).cuda(), cg.BF16)
        rows = p.X[:: max(1, p.m // 2048)].astype(np.float64)
        eta = 0.5 / float((rows ** 2).sum(axis=1).mean())
        probs.append(dict(X=cg.dense_matrix(stored, scale, n=p.n), y=torch.from_numpy(p.y).cuda(),
                          n=p.n, m=p.m, eta=eta, seed=300 + i))
        del p
    log(f"[c5-batch] {count} problems generated and stored in BF16 in {time.perf_counter() - t:.1f}s")
    stream = torch.cuda.current_stream()
    wss = [cg.workspace(cg.casgd_workspace_size(q["X"], b, s)) for q in probs]

    def batch_run(h0, nh):
        xs = [torch.zeros(q["n"], device="cuda") for q in probs]
        batch = [dict(X=q["X"], y=q["y"], x=xs[i], eta=q["eta"], lam=lam, b=b, s=s,
                      seed=q["seed"], outer_begin=h0, n_outer=nh, ws=wss[i])
                 for i, q in enumerate(probs)]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cg.casgd_fit_batch(batch, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        for ws in wss:
            cg.casgd_check(ws)
        return e0.elapsed_time(e1)

    def solo_run(h0, nh):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        xs = [torch.zeros(q["n"], device="cuda") for q in probs]
        e0.record(stream)
        for i, q in enumerate(probs):
            cg.casgd_fit(q["X"], q["y"], xs[i], q["eta"], lam, b, s, q["seed"], h0, nh, ws=wss[i],
                         stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        for ws in wss:
            cg.casgd_check(ws)
        return e0.elapsed_time(e1)

    batch_run(0, 2)
    solo_run(0, 2)
    ms_b = batch_run(0, H)
    ms_s = solo_run(0, H)
    updates = count * s * H
    log(f"[c5-batch] batched {ms_b:.2f} ms, one launch per problem {ms_s:.2f} ms for "
        f"{updates} SGD updates")
    return {"metric": "SGD updates/s over 64 uneven problems (one batched launch)",
            "value": round(updates / (ms_b * 1e-3), 1), "unit": "SGD updates/s",
            "solo_launches_value": round(updates / (ms_s * 1e-3), 1),
            "speedup_vs_solo_launches": round(ms_s / ms_b, 3), "outer_per_problem": H,
            "dtype": "bf16", "data": "synthetic",
            "config": {"workload": f"{count} uneven dense problems, m 1e4..2e5, n 128..4096, "
                                   f"column-scale spread <= 1e3, BF16 X, b={b}, s={s}"},
            "problems": [dict(m=q["m"], n=q["n"]) for q in probs]}


def trailing_hit(losses, target, window):
    """First snapshot k (0-based) at which the mean loss of snapshots
    k-window+1 .. k is <= target (k >= window-1), or None."""
    c = np.cumsum(np.concatenate([[0.0], np.asarray(losses, np.float64)]))
    for k in range(window - 1, len(losses)):
        if (c[k + 1] - c[k + 1 - window]) / window <= target:
            return k
    return None


def c5_bench(cg, n_train: int, n_eval: int, epochs: float = 4.0):
    """The combined target on the uneven workload: plain FP32 SGD (s = 1) against
    CA-SGD with BF16 storage (s = 16), without and with the learned diagonal
    preconditioner, each method one batched launch over the 64 unseen
    problems for the same budget (epochs), with per-problem snapshots and
    device clocks. Target per problem: L* (1 + 1e-3), L* from the FP64 oracle
    (tests/golden/c5_targets.json, written by make_c5_targets.py, which also
    fixes the plain step size); hit = first snapshot whose trailing half-epoch
    mean test loss is at or below the target."""
    import torch
    from paper_2606_18463_amd import learned as Lm
    from workloads import uneven_problem, uneven_problem_specs
    b, s, lam = 64, 16, 1e-5
    rng = dict(m_range=(1e4, 2e5), n_range=(128, 4096), spread_range=(1.0, 1e3))
    with open(os.path.join(ROOT, "tests", "golden", "c5_targets.json")) as f:
        gold = json.load(f)["problems"]
    t0 = time.perf_counter()
    stats, tds, tetas = [], [], []
    for sp in uneven_problem_specs(n_train, 101, **rng):
        dp = Lm.upload(uneven_problem(sp), dtype=cg.BF16)
        t_d, log_eta, _ = Lm.targets(dp, lam, b, s, SEED, epochs=1.0)
        stats.append(cg.casgd_colstats(Lm.stored(dp)))
        tds.append(t_d)
        tetas.append(log_eta)
        del dp
    t_targets = time.perf_counter() - t0
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    model, hist = Lm.train(stats, tds, tetas, steps=1500, lr=1e-2, log_every=500)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    log(f"[c5] targets for {n_train} problems in {t_targets:.1f}s, MLP trained in {t_train:.1f}s: "
        f"{hist}")

    specs = uneven_problem_specs(n_eval, 202, **rng)
    evals = []
    for i, sp in enumerate(specs):
        g = gold[i]
        assert g["spec"] == sp, "golden targets were written for other problems"
        p = uneven_problem(sp)
        dp = Lm.upload(p, dtype=cg.BF16)
        vf, _ = cg.casgd_quantize(dp.X32, cg.F32)         # FP32 storage, rows padded
        Xf = cg.dense_matrix(vf, None, n=dp.n)
        Xb = Lm.stored(dp)                                 # BF16 storage
        Xl, Xtl, q, eta_l = Lm.apply(model, dp)
        per_epoch = dp.m // b
        every = max(1, per_epoch // (16 * s))             # outer iterations per snapshot
        nsnap = max(4, int(epochs * per_epoch) // (every * s))
        evals.append(dict(dp=dp, Xf=Xf, Xb=Xb, Xl=Xl, Xtl=Xtl,
                          eta_p=g["eta"], eta_l=eta_l, L_star=g["L_star"], every=every,
                          nsnap=nsnap, window=max(2, round(per_epoch / (every * s) / 2))))
        del p
    torch.cuda.synchronize()

    def run(kind):
        """One batched launch over every problem; returns (losses per problem,
        device seconds per snapshot per problem, launch ms)."""
        batch, hists, ths = [], [], []
        for i, e in enumerate(evals):
            dp = e["dp"]
            ss = 1 if kind == "plain" else s
            ev = e["every"] * (s if kind == "plain" else 1)
            H = e["nsnap"] * ev
            hist_x = torch.zeros(e["nsnap"], dp.n, device="cuda")
            th = torch.zeros(e["nsnap"] + 1, dtype=torch.int64, device="cuda")
            hists.append(hist_x)
            ths.append(th)
            X = {"plain": e["Xf"], "mixed": e["Xb"], "learned": e["Xl"]}[kind]
            batch.append(dict(X=X, y=dp.y, x=torch.zeros(dp.n, device="cuda"),
                              eta=e["eta_l"] if kind == "learned" else e["eta_p"], lam=lam,
                              b=b, s=ss, seed=SEED, n_outer=H, snapshot_every=ev,
                              x_history=hist_x, t_history=th))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        wss = cg.casgd_fit_batch(batch)
        e1.record()
        torch.cuda.synchronize()
        for w in wss:
            cg.casgd_check(w)
        used = [(q["variant_used"], q["groups_used"]) for q in batch]
        log(f"[c5] {kind}: workgroups {sum(g for _, g in used)}, variants "
            f"{dict((v, sum(1 for u in used if u[0] == v)) for v in set(u[0] for u in used))}")
        losses, secs = [], []
        for i, e in enumerate(evals):
            Xt = e["Xtl"] if kind == "learned" else e["dp"].Xt
            losses.append(cg.casgd_logloss(Xt, e["dp"].yt, hists[i]).cpu().numpy())
            t = ths[i].cpu().numpy()
            secs.append((t[1:] - t[0]) * 1e-8)
        return losses, secs, e0.elapsed_time(e1)

    res = {}
    for kind in ("plain", "mixed", "learned"):
        run(kind)                                          # warm-up launch
        res[kind] = run(kind)
        log(f"[c5] {kind}: batched launch {res[kind][2]:.1f} ms")
    rows = []
    for i, e in enumerate(evals):
        target = e["L_star"] * (1 + TARGET_GAP)
        row = {"m": e["dp"].m, "n": e["dp"].n, "L_star": round(e["L_star"], 7),
               "eta_plain": e["eta_p"], "eta_learned": round(e["eta_l"], 6)}
        for kind in ("plain", "mixed", "learned"):
            losses, secs, _ = res[kind]
            k = trailing_hit(losses[i], target, e["window"])
            row[f"{kind}_seconds_to_target"] = None if k is None else round(float(secs[i][k]), 6)
            row[f"{kind}_final_loss"] = round(float(losses[i][-1]), 7)
        for kind in ("mixed", "learned"):
            tp, tk = row["plain_seconds_to_target"], row[f"{kind}_seconds_to_target"]
            row[f"{kind}_speedup_vs_plain"] = None if not (tp and tk) else round(tp / tk, 3)
        rows.append(row)

    def agg(kind):
        sp = [r[f"{kind}_speedup_vs_plain"] for r in rows if r[f"{kind}_speedup_vs_plain"]]
        reached = sum(1 for r in rows if r[f"{kind}_seconds_to_target"] is not None)
        faster = sum(1 for r in rows if r[f"{kind}_seconds_to_target"] is not None and
                     (r["plain_seconds_to_target"] is None or
                      r[f"{kind}_seconds_to_target"] < r["plain_seconds_to_target"]))
        return {"reached_target": reached, "faster_than_plain": faster,
                "median_speedup": None if not sp else float(np.median(sp)),
                "geomean_speedup": None if not sp else float(np.exp(np.mean(np.log(sp)))),
                "launch_ms": round(res[kind][2], 3)}
    plain_reached = sum(1 for r in rows if r["plain_seconds_to_target"] is not None)
    return {"metric": "time to the FP64 oracle's test loss within 1e-3: mixed + batched + learned "
                      "CA-SGD vs plain FP32 SGD (uneven problems, batched)",
            "train_problems": n_train, "eval_problems": n_eval, "b": b, "s": s,
            "budget_epochs": epochs, "mlp_loss": hist,
            "target_rule": "L* (1 + 1e-3), L* = FP64 oracle plain-SGD test loss averaged over "
                           "epochs 3-4 (tests/golden/c5_targets.json); hit on the trailing "
                           "half-epoch mean of snapshot losses",
            "methods": {"plain": "plain SGD (s = 1), FP32 X, oracle step size, batched",
                        "mixed": "CA-SGD s = 16, BF16 X, oracle step size, batched",
                        "learned": "CA-SGD s = 16, BF16 X~ = X diag(q), MLP q and step size, "
                                   "batched"},
            "plain_reached_target": plain_reached, "mixed": agg("mixed"),
            "learned": agg("learned"), "problems": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed outer iterations")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--s", type=int, default=16)
    ap.add_argument("--dtype", default="f32", choices=list(DT_NAME))
    ap.add_argument("--exec-mode", type=int, default=0, help="0 automatic, 1 fused, 2 stream")
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0, help="workgroups of the fused launch (0 = auto)")
    ap.add_argument("--grid-sweep", action="store_true",
                    help="time the fused launch at --s over grid sizes 8 .. 256")
    ap.add_argument("--m", type=int, default=1 << 20)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--eta-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gram", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-target runs")
    ap.add_argument("--ttt-epochs", type=float, default=6.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--source-hash", action="store_true")
    ap.add_argument("--c4", action="store_true", help="sparse lambda-path workload only")
    ap.add_argument("--c5", action="store_true", help="learned preconditioner workload only")
    ap.add_argument("--autotune", action="store_true",
                    help="run the autotuner on the dense workload and list its candidates")
    ap.add_argument("--c5-batch", action="store_true",
                    help="uneven problems at full size: batched vs one launch per problem")
    ap.add_argument("--gram-shapes", action="store_true",
                    help="standalone Gram launches at the roofline shapes (all storage types)")
    ap.add_argument("--gram-dtype", default=None, choices=list(DT_NAME),
                    help="with --gram-shapes: only this storage type")
    ap.add_argument("--gram-shape", type=int, default=None,
                    help="with --gram-shapes: only this index of the shape list")
    ap.add_argument("--e2e-study", action="store_true",
                    help="long-horizon test-loss gap of the precision recipes to FP32")
    ap.add_argument("--c5-train", type=int, default=256)
    ap.add_argument("--c5-eval", type=int, default=64)
    args = ap.parse_args()
    if args.source_hash:
        print(sources_hash())
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2606_18463_amd as cg
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cg._lib.load()
    if args.copy_calib:
        copy_calibration()
        return
    if args.c5:
        print(json.dumps(c5_bench(cg, args.c5_train, args.c5_eval)), flush=True)
        return
    if args.e2e_study:
        H = args.steps if args.steps is not None else 320_000
        print(json.dumps(e2e_study(cg, H)), flush=True)
        return
    if args.gram_shapes:
        dts = [args.gram_dtype] if args.gram_dtype else ["f32", "bf16", "fp8"]
        shapes = [GRAM_SHAPES[args.gram_shape]] if args.gram_shape is not None else GRAM_SHAPES
        print(json.dumps(gram_shapes_bench(cg, dts, shapes=shapes)), flush=True)
        return
    if args.c5_batch:
        H = args.steps if args.steps is not None else 32
        print(json.dumps(c5_batch_bench(cg, H)), flush=True)
        return
    if args.c4:
        K = args.steps if args.steps is not None else 64
        print(json.dumps(c4_bench(cg, K, args.warmup if args.warmup is not None else 8)), flush=True)
        return

    s, b, n, dtype = args.s, B_C2, args.n, args.dtype
    if args.autotune:
        print(json.dumps(autotune_bench(cg, Workload(args.m, n))), flush=True)
        return
    wl = Workload(args.m, n, with_test=args.eta_sweep or not args.no_ttt)
    if args.eta_sweep:
        res = eta_sweep(cg, wl, [2.0 ** k for k in range(-2, 7)])
        print(json.dumps({"eta_sweep": res}))
        return

    X, y, _keep = upload(cg, wl, dtype)
    # default K: 2^16 SGD updates (a few hundred ms); the warm-up launch has
    # the same length, so every launch of the kernel in a profile of this
    # command has the timed launch's duration
    K = args.steps if args.steps is not None else max(8, (1 << 16) // s)
    W = args.warmup if args.warmup is not None else K
    okw = dict(exec_mode=args.exec_mode, fused_variant=args.variant)
    if args.grid > 0:
        okw["grid_blocks"] = args.grid
    ms, x, ws = timed_fit(cg, X, y, n, b, s, ETA_C2, LAMBDA_C2, K, W, okw)
    ups = s * K / (ms * 1e-3)
    log(f"[bench] s={s} {dtype}: {K} outer in {ms:.2f} ms -> {ups:,.0f} updates/s")

    fl = outer_flops(b, s, n) * K
    by = outer_bytes(b, s, n, DT_BYTES[dtype]) * K
    peak_f = PEAK[f"{dtype}_TFLOPs"]
    ach_f = fl / (ms * 1e-3) / 1e12
    ach_b = by / (ms * 1e-3) / 1e9
    tname = f"traffic_k_fit_dense_{args.m}x{n}_{dtype}_s{s}"
    traffic = measured_traffic(tname, K)
    if s > 1:
        roof = {"kernel": "k_fit (fused launch, all steps)", "bound": "mfma",
                "achieved": round(ach_f, 3), "peak": peak_f, "unit": "TFLOP/s",
                "frac": round(ach_f / peak_f, 4), "traffic": traffic,
                "flops_per_launch": fl, "algorithmic_bytes_per_launch": by}
    else:
        roof = {"kernel": "k_fit (fused launch, all steps)", "bound": "hbm",
                "achieved": round(ach_b, 2), "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                "frac": round(ach_b / PEAK["hbm_GBps"], 5), "traffic": traffic,
                "algorithmic_bytes_per_launch": by}

    out = {
        "metric": "SGD updates/s & time-to-1e-3 loss gap: CA-SGD mixed vs plain, % roofline",
        "value": round(ups, 1), "unit": "SGD updates/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms / K, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"dense logistic regression X {args.m}x{n} FP32 "
                               f"(N(0,1/n), 10% columns x10, 5% label flips), b={b}, s={s}, "
                               f"lambda={LAMBDA_C2}, eta={ETA_C2}",
                   "b": b, "s": s, "storage": dtype, "exec_mode": args.exec_mode,
                   "variant": args.variant},
        "roofline": roof,
    }
    if not args.no_gram and s > 1:
        out["roofline_gram"] = gram_roofline(cg, X, n, b, s, dtype)
    if args.grid_sweep:
        rows = []
        for g in (8, 16, 32, 64, 128, 256):
            Kg = max(8, (1 << 15) // s)
            msg, _, _ = timed_fit(cg, X, y, n, b, s, ETA_C2, LAMBDA_C2, Kg, max(2, Kg // 20),
                                  dict(okw, grid_blocks=g))
            rows.append({"s": s, "grid": g, "us_per_outer": round(msg * 1e3 / Kg, 2),
                         "updates_per_s": round(s * Kg / (msg * 1e-3), 1)})
            log(f"[grid] s={s} grid={g}: {rows[-1]}")
        out["grid_sweep"] = rows
    if args.sweep:
        rows = []
        for ss in (1, 4, 16, 32):
            for em, var in ((1, 0), (1, 2), (2, 0)):
                if ss == 1 and var == 2:
                    continue
                Ks = max(8, (1 << 15) // ss)
                mss, _, _ = timed_fit(cg, X, y, n, b, ss, ETA_C2, LAMBDA_C2, Ks, max(2, Ks // 20),
                                      dict(exec_mode=em, fused_variant=var))
                rows.append({"s": ss, "exec_mode": em, "variant": var,
                             "updates_per_s": round(ss * Ks / (mss * 1e-3), 1),
                             "us_per_outer": round(mss * 1e3 / Ks, 3)})
                log(f"[sweep] {rows[-1]}")
        out["sweep"] = rows
    if not args.no_ttt:
        del X, y, _keep, x, ws
        torch.cuda.empty_cache()
        g = golden_target()
        Xt, _ = cg.casgd_quantize(torch.from_numpy(wl.p.X_test).cuda(), cg.F32)
        Xt = cg.dense_matrix(Xt, None, n=n)
        yt = torch.from_numpy(wl.p.y_test).cuda()
        runs = []
        for name, dt, ss in (("plain SGD, FP32", "f32", 1), ("CA-SGD, FP32", "f32", 16),
                             ("CA-SGD mixed, BF16 X", "bf16", 16),
                             ("CA-SGD mixed, FP8-e4m3 X", "fp8", 16)):
            r = time_to_target(cg, wl, Xt, yt, dt, ss, args.ttt_epochs, 16, g["L_star"])
            r["name"] = name
            runs.append(r)
            log(f"[ttt] {name}: {r}")
        plain = runs[0]["seconds_to_target"]
        ttt = {"L_star": g["L_star"], "gap": TARGET_GAP,
               "target": g["L_star"] * (1 + TARGET_GAP),
               "L_star_source": "FP64 oracle plain SGD, mean test loss over epochs 11-20 of 20 "
                                "(tests/golden/c2_target.json)",
               "hit_rule": "first snapshot whose trailing half-epoch mean test loss <= target",
               "runs": runs}
        for r in runs[1:]:
            if plain and r["seconds_to_target"]:
                r["speedup_vs_plain"] = round(plain / r["seconds_to_target"], 2)
        out["time_to_target"] = ttt
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, b, s, ETA_C2, LAMBDA_C2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
