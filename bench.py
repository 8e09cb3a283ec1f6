"""Benchmark: plain single-field quantize + dequantize on one MI355X.

Workload (one "step"): a 512^3 float32 Gaussian-random-field grid (power
spectrum k^-3, unit variance, seed 1, 0.01 % special values) quantized and
dequantized under ABS and NOA at eb = 1e-3, and its lognormal-magnitude
variant (log10|x| ~ U(-30, 30), random signs, 1 % zeros, seed 11) under REL at
eb = 1e-3.  Inputs are resident in HBM before timing starts; every stream and
decode is produced by the library's HIP kernels through the C ABI.

value = input bytes of the three fields / step time (each field quantized
once and dequantized once per step), GB/s.

Also reported: per-operation GB/s, the dominant kernel's roofline (HIP events
around each main-kernel launch inside the timed steps), the oracle's
throughput on this host, and a byte-exact comparison of the GPU streams with
the oracle's.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
METRIC = "quantize+dequantize GB/s and % HBM peak (plain vs batched); serving p50/p99 ms"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_inputs(N, eb, seed=1, rel_seed=11, frac=1e-4):
    import numpy as np
    import synth
    t0 = time.time()
    g = synth.grf_3d(N, seed, dtype=np.float64)
    x = g.astype(np.float32)
    nsp = synth.n_specials(x.size, frac)
    x, _, _ = synth.inject_specials(x, nsp, seed + 1000, eb)
    xr = synth.rel_variant(g, rel_seed, dtype=np.float32)
    del g
    xr, _, _ = synth.inject_specials(xr, nsp, rel_seed + 1000, eb)
    log(f"inputs {N}^3 generated in {time.time() - t0:.1f}s")
    return x, xr


def alg_bytes_quant(n, s, k):
    # read n values, write n int32 codes, one u64 per 1024-value chunk, k outliers
    return n * s + 4 * n + 8 * ((n + 1023) // 1024) + k * s


def alg_bytes_dequant(n, s, k):
    return 4 * n + 8 * ((n + 1023) // 1024) + k * s + n * s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape autotuner (use variant 0)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; the quantizer path has no "
                          "multi-GPU form here (see DESIGN.md for how it would shard)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2407_15037_amd as lcq

    dev = torch.device("cuda:0")
    eb = args.eb
    tuned = None
    if not args.no_tune:
        from paper_2407_15037_amd import autotune
        tuned = autotune.tune(log=log)
    x, xr = make_inputs(args.grid, eb)
    n = x.size
    s = 4
    fields = [("abs", x), ("noa", x), ("rel", xr)]
    dx = {"abs": torch.from_numpy(x).to(dev)}
    dx["noa"] = dx["abs"]
    dx["rel"] = torch.from_numpy(xr).to(dev)
    cap = lcq.max_stream_bytes(torch.float32, n)
    bufs = {q: torch.empty(cap, dtype=torch.uint8, device=dev) for q, _ in fields}
    nbs = {q: torch.zeros(1, dtype=torch.int64, device=dev) for q, _ in fields}
    ws = {q: torch.empty(lcq.workspace_bytes(q, torch.float32, n), dtype=torch.uint8, device=dev)
          for q, _ in fields}
    outs = {q: torch.empty(n, dtype=torch.float32, device=dev) for q, _ in fields}
    torch.cuda.synchronize()

    order_q = ["abs", "noa", "rel"]
    ev = {}

    def step(record):
        for q in order_q:
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(); e1.record()  # create the events before handing them over
                lcq.profile_events(e0, e1)
                ev.setdefault(("q", q), []).append((e0, e1))
            lcq.quantize(dx[q], q, eb, out=bufs[q], nbytes=nbs[q], ws=ws[q])
        for q in order_q:
            if record:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(); e1.record()
                lcq.profile_events(e0, e1)
                ev.setdefault(("d", q), []).append((e0, e1))
            lcq.dequantize(bufs[q], torch.float32, n, out=outs[q], ws=ws[q])
        lcq.profile_events(None, None)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record()
    for _ in range(args.steps):
        step(True)
    t_end.record()
    torch.cuda.synchronize()
    total_ms = t_start.elapsed_time(t_end)
    ms_per_step = total_ms / args.steps

    sizes = {q: int(nbs[q].item()) for q, _ in fields}
    ks = {}
    for q, _ in fields:
        hdr = bufs[q][:64].cpu().numpy()
        ks[q] = int(hdr[16:24].view(np.uint64)[0])

    kern = {}
    for (kind, q), pairs in ev.items():
        ms = [a.elapsed_time(b) for a, b in pairs]
        avg = sum(ms) / len(ms)
        nbytes = (alg_bytes_quant if kind == "q" else alg_bytes_dequant)(n, s, ks[q])
        kern[f"{'quantize' if kind == 'q' else 'dequantize'}_{q}"] = {
            "avg_us": avg * 1e3, "alg_bytes": nbytes, "gbs_hbm": nbytes / (avg * 1e-3) / 1e9,
            "gbs_input": n * s / (avg * 1e-3) / 1e9}
    dom_name = max(kern, key=lambda k: kern[k]["avg_us"])
    dom = kern[dom_name]
    total_input = n * s * len(fields)
    value = total_input / (ms_per_step * 1e-3) / 1e9

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"grf{args.grid}^3 float32, 0.01% specials; ABS+NOA eb={eb}, "
                               f"REL eb={eb} on lognormal variant; quantize+dequantize each",
                   "n": n, "eb": eb, "quantizers": order_q},
        "ops": {k: {"us": round(v["avg_us"], 2), "input_GBs": round(v["gbs_input"], 1),
                    "alg_GBs": round(v["gbs_hbm"], 1)} for k, v in sorted(kern.items())},
        "outlier_fraction": {q: ks[q] / n for q in order_q},
        "stream_bytes": sizes,
        "autotune": tuned,
        "roofline": {"kernel": dom_name, "bound": "hbm", "achieved": round(dom["gbs_hbm"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom["gbs_hbm"] / HBM_PEAK_GBS, 4), "traffic": None,
                     "alg_bytes_per_launch": dom["alg_bytes"], "avg_launch_us": round(dom["avg_us"], 2)},
    }

    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        cpu = {}
        parity = {}
        for q, arr in fields:
            t0 = time.perf_counter()
            st = oracle.quantize(q, arr, eb)
            t1 = time.perf_counter()
            dec = oracle.dequantize(st, np.float32, n)
            t2 = time.perf_counter()
            cpu[q] = (t1 - t0, t2 - t1)
            if not args.no_verify:
                g = bufs[q][: sizes[q]].cpu().numpy()
                gd = outs[q].cpu().numpy()
                parity[q] = bool(g.size == st.size and np.array_equal(g, st)
                                 and np.array_equal(gd.view(np.uint32), dec.view(np.uint32)))
            del st, dec
        if not args.no_cpu_baseline:
            tsum = sum(a + b for a, b in cpu.values())
            result["cpu_baseline"] = {
                "value": round(total_input / tsum / 1e9, 4), "unit": "GB/s", "cores": 1,
                "kind": "oracle",
                "sample": f"the full step's three fields ({n} float32 values each), one "
                          "single-threaded oracle quantize + dequantize per field"}
        if not args.no_verify:
            result["parity_vs_oracle"] = parity
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
