"""Benchmark of the guaranteed-error-bound quantizers on one MI355X.

Headline (the `value` field): plain single-field quantize + dequantize.  One
step = a 512^3 float32 Gaussian-random-field grid (power spectrum k^-3, unit
variance, seed 1, 0.01 % special values) quantized and dequantized under ABS
and NOA at eb = 1e-3, and its lognormal-magnitude variant (log10|x| ~
U(-30, 30), random signs, 1 % zeros, seed 11) quantized and dequantized under
REL at eb = 1e-3.  value = input bytes of the three fields / step time, GB/s.
Inputs are resident in HBM before timing starts; every stream and decode is
produced by the library's HIP kernels through the C ABI.

Also reported on the same JSON line:
  ops          per-kernel time and GB/s (HIP events around each main kernel)
  roofline     the dominant kernel against the 8 TB/s HBM peak
  packing      the lossless packing stage after each quantizer: compression
               ratio, pack / unpack time, byte-exact round trip
  ablation     section 6: ABS with vs without the double-check, REL with the
               section 3.2 approximations vs the device math library
  inline_layout the same fields in the in-line outlier layout (section 3.1):
               per-kernel time, decodes equal to the list layout's
  batched      2,000 fields, log-uniform 4 KiB - 64 MiB, 70 % float32, random
               quantizer and eb in [1e-5, 1e-1]: one graph launch vs a
               per-field launch loop, byte-equal outputs checked
  serving      Poisson requests (50/50 quantize / dequantize, 64 KiB - 256 MiB,
               mixed dtype / quantizer / eb), 64 GB admission budget: GB/s,
               p50 / p99 latency, every output checked against the same
               request run alone
  cpu_baseline the CPU oracle on this host (single thread), which also checks
               the GPU streams of the plain step and of sampled batch fields
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


def kernel_source_digest():
    """sha256 over the HIP sources (names and bytes), to tell whether stored
    hardware counter figures still describe the kernels being timed."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2407_15037_amd", "csrc", "*"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_grf512_f32.md")


def measured_traffic(op, grid, eb, variants):
    """HBM bytes per launch of `op` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary of this workload, or None if the workload differs,
    the launch variants timed (quantize, dequantize) are not the ones the
    counters were taken with, or the kernels changed since."""
    if grid != 512 or eb != 1e-3 or not os.path.exists(TRAFFIC_PROFILE):
        return None
    digest, table, counted = None, {}, None
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            if line.startswith("kernel-source-sha256:"):
                digest = line.split(":", 1)[1].strip()
            if counted is None and "--variants " in line:
                v = line.split("--variants ", 1)[1].split()[0]
                counted = tuple(int(x) for x in v.split(","))
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 4 and cells[0] and not cells[0].startswith(("op", "-", "`")):
                try:
                    table[cells[0]] = float(cells[3])
                except ValueError:
                    pass
    if digest != kernel_source_digest() or counted != tuple(variants):
        return None
    return table.get(op)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def alg_bytes_quant(n, s, k):
    # read n values, write n int32 codes, one u64 per 1024-value chunk, k outliers
    return n * s + 4 * n + 8 * ((n + 1023) // 1024) + k * s


def alg_bytes_dequant(n, s, k):
    return 4 * n + 8 * ((n + 1023) // 1024) + k * s + n * s


def header_k(buf):
    import numpy as np
    return int(buf[:64].cpu().numpy()[16:24].view(np.uint64)[0])


# ------------------------------------------------------------------- plain --
def make_plain_inputs(N, eb, seed=1, rel_seed=11, frac=1e-4):
    import synth
    t0 = time.time()
    x, xr = synth.plain_step_inputs(N, eb, seed, rel_seed, frac)
    log(f"plain inputs {N}^3 generated in {time.time() - t0:.1f}s")
    return x, xr


def run_plain(args, x, xr):
    import torch
    import paper_2407_15037_amd as lcq
    dev = torch.device("cuda:0")
    eb = args.eb
    n, s = x.size, 4
    order_q = ["abs", "noa", "rel"]
    dx = {"abs": torch.from_numpy(x).to(dev)}
    dx["noa"] = dx["abs"]
    dx["rel"] = torch.from_numpy(xr).to(dev)
    cap = lcq.max_stream_bytes(torch.float32, n)
    bufs = {q: torch.empty(cap, dtype=torch.uint8, device=dev) for q in order_q}
    nbs = {q: torch.zeros(1, dtype=torch.int64, device=dev) for q in order_q}
    ws = {q: torch.empty(lcq.workspace_bytes(q, torch.float32, n), dtype=torch.uint8, device=dev)
          for q in order_q}
    outs = {q: torch.empty(n, dtype=torch.float32, device=dev) for q in order_q}
    torch.cuda.synchronize()
    ev = {}

    def step(record):
        for kind in ("q", "d"):
            for q in order_q:
                if record:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(); e1.record()  # create the events before handing them over
                    lcq.profile_events(e0, e1)
                    ev.setdefault((kind, q), []).append((e0, e1))
                if kind == "q":
                    lcq.quantize(dx[q], q, eb, out=bufs[q], nbytes=nbs[q], ws=ws[q])
                else:
                    lcq.dequantize(bufs[q], torch.float32, n, out=outs[q], ws=ws[q])
        lcq.profile_events(None, None)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record()
    for _ in range(args.steps):
        step(True)
    t_end.record()
    torch.cuda.synchronize()
    ms_per_step = t_start.elapsed_time(t_end) / args.steps
    # NOA as a whole operation: range pass, parameters and both quantize
    # passes, events on the launch stream around the call
    whole = []
    for _ in range(max(3, args.steps // 4)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        lcq.quantize(dx["noa"], "noa", eb, out=bufs["noa"], nbytes=nbs["noa"], ws=ws["noa"])
        e1.record()
        torch.cuda.synchronize()
        whole.append(e0.elapsed_time(e1) * 1e3)
    ks = {q: header_k(bufs[q]) for q in order_q}
    kern = {}
    for (kind, q), pairs in ev.items():
        ms = [a.elapsed_time(b) for a, b in pairs]
        avg = sum(ms) / len(ms)
        nbytes = (alg_bytes_quant if kind == "q" else alg_bytes_dequant)(n, s, ks[q])
        kern[f"{'quantize' if kind == 'q' else 'dequantize'}_{q}"] = {
            "avg_us": avg * 1e3, "alg_bytes": nbytes, "gbs_hbm": nbytes / (avg * 1e-3) / 1e9,
            "gbs_input": n * s / (avg * 1e-3) / 1e9}
    value = n * s * len(order_q) / (ms_per_step * 1e-3) / 1e9
    sizes = {q: int(nbs[q].item()) for q in order_q}
    gpu_streams = {q: bufs[q][: sizes[q]].cpu().numpy() for q in order_q}
    gpu_decodes = {q: outs[q].cpu().numpy() for q in order_q}
    del dx, bufs, ws, outs
    torch.cuda.empty_cache()
    return dict(ms_per_step=ms_per_step, value=value, kern=kern, ks=ks, sizes=sizes, n=n,
                noa_whole_us=sum(whole) / len(whole),
                gpu_streams=gpu_streams, gpu_decodes=gpu_decodes)


# ----------------------------------------------------------------- float64 --
def run_f64(args):
    """The float64 single-field workload (384^3 GRF with its bin-border slice;
    ABS / NOA at 1e-6, REL at 1e-4): per-operation times of the per-value
    kernels, events on the launch stream as in the float32 step."""
    import numpy as np
    import torch
    import synth
    import paper_2407_15037_amd as lcq
    t0 = time.time()
    x, xr = synth.f64_grid_inputs()
    log(f"float64 inputs 384^3 generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ebs = {"abs": 1e-6, "noa": 1e-6, "rel": 1e-4}
    order_q = ["abs", "noa", "rel"]
    n, s = x.size, 8
    dx = {"abs": torch.from_numpy(x).to(dev)}
    dx["noa"] = dx["abs"]
    dx["rel"] = torch.from_numpy(xr).to(dev)
    cap = lcq.max_stream_bytes(torch.float64, n)
    bufs = {q: torch.empty(cap, dtype=torch.uint8, device=dev) for q in order_q}
    nbs = {q: torch.zeros(1, dtype=torch.int64, device=dev) for q in order_q}
    ws = {q: torch.empty(lcq.workspace_bytes(q, torch.float64, n), dtype=torch.uint8, device=dev)
          for q in order_q}
    outs = {q: torch.empty(n, dtype=torch.float64, device=dev) for q in order_q}
    ev = {}
    for rep in range(args.warmup + args.steps):
        for kind in ("q", "d"):
            for q in order_q:
                if rep >= args.warmup:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(); e1.record()
                    lcq.profile_events(e0, e1)
                    ev.setdefault((kind, q), []).append((e0, e1))
                if kind == "q":
                    lcq.quantize(dx[q], q, ebs[q], out=bufs[q], nbytes=nbs[q], ws=ws[q])
                else:
                    lcq.dequantize(bufs[q], torch.float64, n, out=outs[q], ws=ws[q])
            lcq.profile_events(None, None)
    torch.cuda.synchronize()
    ks = {q: header_k(bufs[q]) for q in order_q}
    ops = {}
    for (kind, q), pairs in sorted(ev.items()):
        us = 1e3 * sum(a.elapsed_time(b) for a, b in pairs) / len(pairs)
        nbytes = (alg_bytes_quant if kind == "q" else alg_bytes_dequant)(n, s, ks[q])
        ops[f"{'quantize' if kind == 'q' else 'dequantize'}_{q}"] = {
            "us": round(us, 2), "input_GBs": round(n * s / (us * 1e-6) / 1e9, 1),
            "alg_GBs": round(nbytes / (us * 1e-6) / 1e9, 1),
            "frac_of_peak": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    # every decoded value within its bound (specials bit-exact) on the GPU
    ok = {}
    for q in order_q:
        a, b = dx[q], outs[q]
        fin = torch.isfinite(a) & ~((a != 0) & (a.abs() < 2.2250738585072014e-308))
        if q == "rel":
            good = (b - a).abs() <= ebs[q] * a.abs()
        else:
            bound = float(bufs[q][40:48].cpu().numpy().view(np.float64)[0])
            good = (b - a).abs() <= bound
        same_bits = a.view(torch.int64) == b.view(torch.int64)
        ok[q] = bool(torch.where(fin, good | same_bits, same_bits).all().item())
    res = {"workload": "grf384^3 float64, 0.01% specials, 2^20-value bin-border slice at n/2; "
                       "ABS/NOA eb=1e-6, REL eb=1e-4 on the lognormal variant",
           "n": n, "ops": ops,
           "outlier_fraction": {q: ks[q] / n for q in order_q},
           "stream_bytes": {q: int(nbs[q].item()) for q in order_q},
           "decodes_within_bound": ok}
    del dx, bufs, ws, outs
    torch.cuda.empty_cache()
    return res


# ----------------------------------------------------------------- in-line --
def run_inline(args, x, xr, plain):
    """The same three fields in the in-line layout (one word per value plus a
    raw-value bitmap): per-kernel time, and decodes equal to the list
    layout's decodes of the timed plain step."""
    import torch
    import paper_2407_15037_amd as lcq
    dev = torch.device("cuda:0")
    eb = args.eb
    n, s = x.size, 4
    order_q = ["abs", "noa", "rel"]
    dx = {"abs": torch.from_numpy(x).to(dev)}
    dx["noa"] = dx["abs"]
    dx["rel"] = torch.from_numpy(xr).to(dev)
    nb = lcq.inline_stream_bytes(torch.float32, n)
    bufs = {q: torch.empty(nb, dtype=torch.uint8, device=dev) for q in order_q}
    ws = torch.empty(lcq.inline_workspace_bytes("noa"), dtype=torch.uint8, device=dev)
    outs = {q: torch.empty(n, dtype=torch.float32, device=dev) for q in order_q}
    ev = {}
    reps = max(3, args.steps // 2)
    for r in range(reps + 1):
        for kind in ("q", "d"):
            for q in order_q:
                if r:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(); e1.record()
                    lcq.profile_events(e0, e1)
                    ev.setdefault((kind, q), []).append((e0, e1))
                if kind == "q":
                    lcq.quantize_inline(dx[q], q, eb, out=bufs[q], ws=ws)
                else:
                    lcq.dequantize_inline(bufs[q], torch.float32, n, out=outs[q], ws=ws)
                lcq.profile_events(None, None)
    torch.cuda.synchronize()
    ops, same = {}, {}
    for (kind, q), pairs in ev.items():
        avg = sum(a.elapsed_time(b) for a, b in pairs) / len(pairs)
        alg = n * s + n * s + (n + 7) // 8
        name = f"{'quantize' if kind == 'q' else 'dequantize'}_inline_{q}"
        ops[name] = {"us": round(avg * 1e3, 2), "alg_GBs": round(alg / (avg * 1e-3) / 1e9, 1),
                     "input_GBs": round(n * s / (avg * 1e-3) / 1e9, 1)}
    for q in order_q:
        ref = torch.from_numpy(plain["gpu_decodes"][q]).to(dev)
        same[q] = bool(torch.equal(outs[q].view(torch.int32), ref.view(torch.int32)))
    del dx, bufs, outs, ws
    torch.cuda.empty_cache()
    return {"stream_bytes": nb, "ops": dict(sorted(ops.items())),
            "decode_equals_list_layout": same}


# ----------------------------------------------------------------- packing --
def run_packing(args, x, xr):
    """Lossless packing stage after each quantizer on the plain step's
    fields: packed size (compression ratio against the float32 input and
    against the LCQ1 stream), pack / unpack time (events around each call,
    all of its kernels), and the unpacked stream equal to the original."""
    import torch
    import paper_2407_15037_amd as lcq
    dev = torch.device("cuda:0")
    eb = args.eb
    n = x.size
    reps = max(3, args.steps // 4)
    res = {}
    for q, arr in (("abs", x), ("noa", x), ("rel", xr)):
        xt = torch.from_numpy(arr).to(dev)
        st, nb = lcq.quantize(xt, q, eb)
        size = int(nb.item())
        pk = torch.empty(lcq.pack_max_bytes(torch.float32, n), dtype=torch.uint8, device=dev)
        pnb = torch.zeros(1, dtype=torch.int64, device=dev)
        ws = torch.empty(lcq.pack_workspace_bytes(torch.float32, n), dtype=torch.uint8, device=dev)
        back = torch.empty(lcq.max_stream_bytes(torch.float32, n), dtype=torch.uint8, device=dev)
        bnb = torch.zeros(1, dtype=torch.int64, device=dev)
        tp, tu = [], []
        for r in range(reps + 1):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            lcq.pack(st, torch.float32, n, stream_bytes=size, out=pk, nbytes=pnb, ws=ws)
            e1.record()
            lcq.unpack(pk, torch.float32, n, out=back, nbytes=bnb, ws=ws)
            e2.record()
            torch.cuda.synchronize()
            if r:
                tp.append(e0.elapsed_time(e1) * 1e3)
                tu.append(e1.elapsed_time(e2) * 1e3)
        psize = int(pnb.item())
        same = int(bnb.item()) == size and torch.equal(back[:size], st[:size])
        res[q] = {"lcq1_bytes": size, "packed_bytes": psize,
                  "ratio_vs_input": round(n * 4 / psize, 3), "ratio_vs_lcq1": round(size / psize, 3),
                  "pack_us": round(sum(tp) / len(tp), 2), "unpack_us": round(sum(tu) / len(tu), 2),
                  "unpacked_equals_stream": bool(same)}
        del xt, st, pk, ws, back
        torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------- ablation --
ABL_SAMPLE = 1 << 20  # REL-libm codes kept for the CPU/GPU comparison


def run_ablation(args, x, xr, plain):
    """The paper's two ablations (section 6) on the plain step's fields, same
    kernels and launch shape: ABS with vs without the double-check, and REL
    with the section 3.2 approximations vs the device math library's
    log2 / exp2, each pair timed interleaved (events around the per-value
    kernels, as for the plain ops); the unchecked ABS decode is counted
    against the bound on the device."""
    import numpy as np
    import torch
    import paper_2407_15037_amd as lcq
    dev = torch.device("cuda:0")
    eb = args.eb
    n = x.size
    xa = torch.from_numpy(x).to(dev)
    xl = torch.from_numpy(xr).to(dev)
    cap = lcq.max_stream_bytes(torch.float32, n)
    buf = torch.empty(cap, dtype=torch.uint8, device=dev)
    nb = torch.zeros(1, dtype=torch.int64, device=dev)
    ws = torch.empty(lcq.workspace_bytes("rel", torch.float32, n), dtype=torch.uint8, device=dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    reps = max(5, args.steps // 2)

    def timed_once(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(); e1.record()
        lcq.profile_events(e0, e1)
        fn()
        lcq.profile_events(None, None)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1e3

    res = {}
    for kind, base_q, xt in (("abs_unchecked", "abs", xa), ("rel_libm", "rel", xl)):
        # the guaranteed quantizer and its ablation, interleaved rep by rep
        # so that both see the same clocks and memory state
        tq = {base_q: [], kind: []}
        td = {base_q: [], kind: []}
        for r in range(reps + 1):
            for which in (base_q, kind):
                if which == base_q:
                    tq_ = timed_once(lambda: lcq.quantize(xt, base_q, eb, out=buf, nbytes=nb, ws=ws))
                else:
                    tq_ = timed_once(lambda: lcq.quantize_ablation(xt, kind, eb, out=buf, nbytes=nb,
                                                                    ws=ws))
                size = int(nb.item())
                if which == base_q:
                    td_ = timed_once(lambda: lcq.dequantize(buf, torch.float32, n, stream_bytes=size,
                                                            out=out, ws=ws))
                else:
                    td_ = timed_once(lambda: lcq.dequantize_ablation(buf, kind, torch.float32, n,
                                                                     stream_bytes=size, out=out,
                                                                     ws=ws))
                if r:
                    tq[which].append(tq_)
                    td[which].append(td_)
        avg = lambda v: sum(v) / len(v)
        k = header_k(buf)  # the ablation's stream is the last one written
        fin = torch.isfinite(xt)
        if kind == "abs_unchecked":
            e = np.float32(eb)  # the float32 bound: largest float32 not above eb
            if float(e) > eb:
                e = np.nextafter(e, np.float32(0))
            e = float(e)
            err = (xt.double() - out.double()).abs()
            viol = int(((err > e) & fin).sum().item())
            res["abs"] = {
                "protected_quantize_us": round(avg(tq["abs"]), 2),
                "unchecked_quantize_us": round(avg(tq[kind]), 2),
                "check_cost_pct": round(100.0 * (avg(tq["abs"]) - avg(tq[kind])) / avg(tq[kind]), 2),
                "protected_dequantize_us": round(avg(td["abs"]), 2),
                "unchecked_dequantize_us": round(avg(td[kind]), 2),
                "unchecked_outliers": k, "protected_outliers": plain["ks"]["abs"],
                "unchecked_values_outside_bound": viol}
        else:
            res["rel"] = {
                "mitchell_quantize_us": round(avg(tq["rel"]), 2),
                "libm_quantize_us": round(avg(tq[kind]), 2),
                "mitchell_dequantize_us": round(avg(td["rel"]), 2),
                "libm_dequantize_us": round(avg(td[kind]), 2),
                "mitchell_outliers": plain["ks"]["rel"], "libm_outliers": k}
            codes = buf[64: 64 + 4 * ABL_SAMPLE].view(torch.int32).cpu().numpy().copy()
    del xa, xl, buf, ws, out
    torch.cuda.empty_cache()
    return res, codes


# ----------------------------------------------------------------- batched --
def make_batch_specs(nf, seed=3):
    import synth
    return synth.field_specs(nf, seed, 4 << 10, 64 << 20)


def make_masters(seed, N=256):
    import numpy as np
    import synth
    master = synth.grf_3d(N, seed, dtype=np.float64)
    return master, synth.rel_variant(master, seed + 10, dtype=np.float64)


def run_batched(args):
    import numpy as np
    import torch
    import paper_2407_15037_amd as lcq
    import synth
    from paper_2407_15037_amd.batch import BatchPlan, variants
    t0 = time.time()
    specs = make_batch_specs(args.fields)
    master, relm = make_masters(3)
    fields, total_bytes = [], 0
    for i, sp in enumerate(specs):
        x = synth.field_data(sp, master, relm, 30000 + i)
        xt = torch.from_numpy(x).cuda()
        fields.append(dict(x=xt, q=sp["q"], eb=sp["eb"]))
        total_bytes += x.nbytes
    torch.cuda.synchronize()
    log(f"batched: {len(fields)} fields, {total_bytes / 1e9:.2f} GB generated in "
        f"{time.time() - t0:.1f}s")

    def timed(fn, reps):
        ts = []
        for r in range(reps + 1):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
        ts.sort()
        return ts[len(ts) // 2]

    # tuner: each batch tile shape, quantize graph time
    best_v, tune_ms = 0, []
    for v in range(variants()):
        p = BatchPlan(fields, variant=v)
        tune_ms.append(round(timed(p.quantize, 2), 3))
        p.close()
        del p
        torch.cuda.empty_cache()
    best_v = min(range(len(tune_ms)), key=lambda i: tune_ms[i])
    log(f"batched tuner (quantize ms per variant): {tune_ms} -> {best_v}")
    plan = BatchPlan(fields, variant=best_v)
    bq = timed(plan.quantize, args.batch_reps)
    bd = timed(plan.dequantize, args.batch_reps)
    bad = plan.first_bad_field()

    # per-field launch loop on the same fields (plain entry points)
    loop_bufs = []
    for f, d in zip(fields, plan.fields):
        n = d["x"].numel()
        loop_bufs.append(dict(
            buf=torch.empty(lcq.max_stream_bytes(d["x"].dtype, n), dtype=torch.uint8, device="cuda"),
            nb=torch.zeros(1, dtype=torch.int64, device="cuda"),
            ws=torch.empty(lcq.workspace_bytes(f["q"], d["x"].dtype, n), dtype=torch.uint8, device="cuda"),
            out=torch.empty(n, dtype=d["x"].dtype, device="cuda")))

    def loop_q():
        for f, lb in zip(fields, loop_bufs):
            lcq.quantize(f["x"], f["q"], f["eb"], out=lb["buf"], nbytes=lb["nb"], ws=lb["ws"])

    def loop_d():
        for f, lb in zip(fields, loop_bufs):
            lcq.dequantize(lb["buf"], f["x"].dtype, f["x"].numel(), out=lb["out"], ws=lb["ws"])

    lq = timed(loop_q, args.batch_reps)
    ld = timed(loop_d, args.batch_reps)
    # batch output == per-field output, every field, compared on the device
    same_streams = same_decodes = 0
    for d, lb in zip(plan.fields, loop_bufs):
        s1, s2 = int(d["nbytes"].item()), int(lb["nb"].item())
        same_streams += int(s1 == s2 and torch.equal(d["stream"][:s1], lb["buf"][:s2]))
        same_decodes += int(torch.equal(d["out"].view(torch.uint8), lb["out"].view(torch.uint8)))
    res = {
        "workload": f"{len(fields)} fields, log-uniform 4 KiB-64 MiB, 70% float32, "
                    "random ABS/REL/NOA, eb log-uniform [1e-5, 1e-1], 0.01% specials",
        "total_input_GB": round(total_bytes / 1e9, 3),
        "variant": best_v, "tuner_quantize_ms": tune_ms,
        "batch_quantize_ms": round(bq, 3), "batch_dequantize_ms": round(bd, 3),
        "loop_quantize_ms": round(lq, 3), "loop_dequantize_ms": round(ld, 3),
        "batch_GBs": round(total_bytes / ((bq + bd) * 1e-3) / 1e9, 1),
        "loop_GBs": round(total_bytes / ((lq + ld) * 1e-3) / 1e9, 1),
        "speedup_vs_loop": round((lq + ld) / (bq + bd), 3),
        "fields_equal_to_plain": f"{same_streams}/{len(fields)} streams, "
                                 f"{same_decodes}/{len(fields)} decodes",
        "stream_check_first_bad": bad,
    }
    sample = [i for i in range(len(fields)) if fields[i]["x"].numel() <= (1 << 20)][:12]
    sample_data = [(specs[i], fields[i]["x"].cpu().numpy(),
                    plan.fields[i]["stream"][: int(plan.fields[i]["nbytes"].item())].cpu().numpy())
                   for i in sample]
    plan.close()
    del plan, fields, loop_bufs
    torch.cuda.empty_cache()
    return res, sample_data


# ----------------------------------------------------------------- serving --
def run_serving(args):
    import numpy as np
    import torch
    import paper_2407_15037_amd as lcq
    import synth
    from paper_2407_15037_amd import serve
    t0 = time.time()
    specs = synth.field_specs(args.pool, 4, 64 << 10, 256 << 20)
    master, relm = make_masters(4, N=256)
    pool = []
    for i, sp in enumerate(specs):
        x = synth.field_data(sp, master, relm, 40000 + i)
        xt = torch.from_numpy(x).cuda()
        tdt = xt.dtype
        # the payload processed alone once: expected bytes for the mix
        buf, nb = lcq.quantize(xt, sp["q"], sp["eb"])
        torch.cuda.synchronize()
        size = int(nb.item())
        st = buf[:size].clone()
        del buf
        dec = lcq.dequantize(st, tdt, x.size, stream_bytes=size)
        pool.append(dict(spec=sp, tdt=tdt, x=xt, stream=st, size=size,
                         dec=dec.view(torch.uint8)))
    torch.cuda.synchronize()
    log(f"serving pool of {len(pool)} payloads ready in {time.time() - t0:.1f}s")
    arr = synth.poisson_arrivals(args.rate, args.serve_seconds, 5)
    rng = np.random.default_rng(6)
    reqs, in_bytes = [], 0
    for t in arr:
        p = pool[int(rng.integers(0, len(pool)))]
        sp = p["spec"]
        es = 8 if p["tdt"] == torch.float64 else 4
        if rng.random() < 0.5:
            reqs.append(dict(op="quantize", x=p["x"], n=sp["n"], dtype=p["tdt"], q=sp["q"],
                             eb=sp["eb"], expect=p["stream"], expect_bytes=p["size"],
                             arrival_ns=int(t)))
            in_bytes += sp["n"] * es
        else:
            reqs.append(dict(op="dequantize", x=p["stream"], n=sp["n"], dtype=p["tdt"],
                             in_bytes=p["size"], expect=p["dec"], arrival_ns=int(t)))
            in_bytes += p["size"]
    arena = torch.empty(int(args.budget_gb * (1 << 30)), dtype=torch.uint8, device="cuda")
    log(f"serving {len(reqs)} requests over {args.serve_seconds}s")
    r = serve.run(reqs, n_streams=args.streams, arena=arena)
    lat = (r["done_ns"] - r["arrival_ns"]) / 1e6
    qwait = (r["admit_ns"] - r["arrival_ns"]) / 1e6
    makespan = (r["done_ns"].max() - r["arrival_ns"].min()) / 1e9
    ok = int(np.sum((r["status"] == 0) & (r["mismatched"] == 0)))
    res = {
        "workload": f"Poisson {args.rate}/s for {args.serve_seconds}s, 50/50 quantize/"
                    "dequantize, 64 KiB-256 MiB log-uniform, 70% float32, random "
                    f"ABS/REL/NOA, eb [1e-5,1e-1]; pool of {len(pool)} resident payloads; "
                    f"{args.budget_gb} GB admission budget, {args.streams} streams",
        "requests": len(reqs), "GBs": round(in_bytes / makespan / 1e9, 2),
        "offered_GBs": round(in_bytes / args.serve_seconds / 1e9, 2),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "max_ms": round(float(lat.max()), 4),
        "queue_p99_ms": round(float(np.percentile(qwait, 99)), 4),
        "outputs_equal_alone": f"{ok}/{len(reqs)}",
    }
    # saturation: the first requests of the same mix all arriving at once
    # (closed queue), so the loop admits them as fast as the budget and the
    # streams allow; every output still compared with the request alone
    m = min(len(reqs), args.saturation_requests)
    sat = [dict(r, arrival_ns=0) for r in reqs[:m]]
    sat_bytes = sum(r["n"] * (8 if r["dtype"] == torch.float64 else 4) if r["op"] == "quantize"
                    else r["in_bytes"] for r in sat)
    log(f"serving saturation: {m} requests at once")
    rs = serve.run(sat, n_streams=args.streams, arena=arena)
    span = (rs["done_ns"].max() - rs["admit_ns"].min()) / 1e9
    res["saturated"] = {
        "requests": m, "GBs": round(sat_bytes / span / 1e9, 1),
        "outputs_equal_alone": f"{int(np.sum((rs['status'] == 0) & (rs['mismatched'] == 0)))}/{m}"}
    # the smallest payloads' expected streams go to the CPU leg, which checks
    # them against the oracle
    small = sorted(range(len(pool)), key=lambda i: pool[i]["spec"]["n"])[:16]
    sample = [(pool[i]["spec"], pool[i]["x"].cpu().numpy(), pool[i]["stream"].cpu().numpy())
              for i in small]
    del arena, pool, reqs
    torch.cuda.empty_cache()
    return res, sample


# ------------------------------------------------------------ CPU baseline --
def cpu_baseline_leg(x, xr, eb, plain, batch_sample, abl_codes=None, serve_sample=()):
    """The CPU oracle, single thread, timed on the plain step's three fields
    (quantize + dequantize each); its streams also check the GPU's."""
    import numpy as np
    import oracle
    n = x.size
    tsum, parity = 0.0, {}
    for q, arr in (("abs", x), ("noa", x), ("rel", xr)):
        t0 = time.perf_counter()
        st = oracle.quantize(q, arr, eb)
        t1 = time.perf_counter()
        dec = oracle.dequantize(st, np.float32, n)
        t2 = time.perf_counter()
        tsum += t2 - t0
        g = plain["gpu_streams"][q]
        parity[q] = bool(g.size == st.size and np.array_equal(g, st) and
                         np.array_equal(plain["gpu_decodes"][q].view(np.uint32), dec.view(np.uint32)))
        del st, dec
    bparity = 0
    for sp, xv, gs in batch_sample:
        bparity += int(np.array_equal(oracle.quantize(sp["q"], xv, sp["eb"]), gs))
    if serve_sample:
        ok = sum(int(np.array_equal(oracle.quantize(sp["q"], xv, sp["eb"]), gs))
                 for sp, xv, gs in serve_sample)
        parity["serving_pool_sample"] = f"{ok}/{len(serve_sample)}"
    if abl_codes is not None:
        # REL-libm ablation: the host library's codes for the first values of
        # the field vs the GPU's (REL codes depend on the value alone)
        st = oracle.quantize("rel_libm", xr[: abl_codes.size], eb)
        oc = st[64: 64 + 4 * abl_codes.size].view(np.int32)
        parity["rel_libm_codes_differing_cpu_vs_gpu"] = (
            f"{int(np.count_nonzero(oc != abl_codes))} of {abl_codes.size}")
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    base = {"value": round(3 * n * 4 / tsum / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "host": f"{model}, {os.cpu_count()} logical CPUs visible",
            "sample": f"the plain step's three fields ({n} float32 values each): one "
                      "single-threaded oracle quantize + dequantize per field"}
    return base, parity, f"{bparity}/{len(batch_sample)}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--grid", type=int, default=512)
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape autotuner (use the built-in defaults)")
    ap.add_argument("--variants", default=None,
                    help="Q,D: fixed float32 quantize / dequantize launch variants "
                         "instead of the autotuner (for profiler runs that must time "
                         "the same kernels)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-inline", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-packing", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--fields", type=int, default=2000)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--saturation-requests", type=int, default=20000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run three 512 MiB device-to-device copies (a plain copy "
                         "kernel of known size, to scale hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the quantizer path has no multi-GPU form "
                          "(sharding is described, not implemented)", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2407_15037_amd as lcq
    if args.calib_copy:
        src = torch.ones(128 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copies: 3 x 512 MiB read + 512 MiB written")
    tuned = None
    if args.variants:
        qv, dv = (int(v) for v in args.variants.split(","))
        lcq.tune_set("quantize", torch.float32, qv)
        lcq.tune_set("dequantize", torch.float32, dv)
        tuned = {"float32": {"quantize": {"best": qv}, "dequantize": {"best": dv}}}
    elif not args.no_tune:
        from paper_2407_15037_amd import autotune
        tuned = autotune.tune(log=log)
    x, xr = make_plain_inputs(args.grid, args.eb)
    plain = run_plain(args, x, xr)
    kern = plain["kern"]
    dom_name = max(kern, key=lambda k: kern[k]["avg_us"])
    dom = kern[dom_name]
    result = {
        "metric": METRIC, "value": round(plain["value"], 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(plain["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"grf{args.grid}^3 float32, 0.01% specials; ABS+NOA eb={args.eb}, "
                               f"REL eb={args.eb} on lognormal variant; quantize+dequantize each",
                   "n": plain["n"], "eb": args.eb, "quantizers": ["abs", "noa", "rel"]},
        "ops": {k: {"us": round(v["avg_us"], 2), "input_GBs": round(v["gbs_input"], 1),
                    "alg_GBs": round(v["gbs_hbm"], 1)} for k, v in sorted(kern.items())},
        "input_GBs": {
            # input bytes of the three fields over the summed per-op times
            # (NOA quantize as a whole operation, range pass included)
            "quantize": round(3 * plain["n"] * 4 / (1e-6 * (kern["quantize_abs"]["avg_us"] +
                                                          plain["noa_whole_us"] +
                                                          kern["quantize_rel"]["avg_us"])) / 1e9, 1),
            "dequantize": round(3 * plain["n"] * 4 / (1e-6 * sum(
                kern[f"dequantize_{q}"]["avg_us"] for q in ("abs", "noa", "rel"))) / 1e9, 1),
            "combined_step": round(plain["value"], 1)},
        "quantize_noa_whole_op_us": round(plain["noa_whole_us"], 2),
        "outlier_fraction": {q: plain["ks"][q] / plain["n"] for q in plain["ks"]},
        "stream_bytes": plain["sizes"],
        "autotune": tuned,
        "roofline": {"kernel": dom_name, "bound": "hbm", "achieved": round(dom["gbs_hbm"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(dom["gbs_hbm"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom_name, args.grid, args.eb,
                                                 (lcq.tune_get("quantize", torch.float32),
                                                  lcq.tune_get("dequantize", torch.float32))),
                     "alg_bytes_per_launch": dom["alg_bytes"],
                     "avg_launch_us": round(dom["avg_us"], 2)},
    }
    # each quantizer's quantize + dequantize pair on one field: algorithmic
    # bytes of both over their summed times (NOA: whole quantize operation,
    # its range pass's read of the field included)
    pair = {}
    for q in ("abs", "noa", "rel"):
        kq, kd = kern[f"quantize_{q}"], kern[f"dequantize_{q}"]
        tq = plain["noa_whole_us"] if q == "noa" else kq["avg_us"]
        nb = kq["alg_bytes"] + kd["alg_bytes"] + (plain["n"] * 4 if q == "noa" else 0)
        pair[q] = round(nb / ((tq + kd["avg_us"]) * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
    result["quantize_dequantize_pair_frac_of_peak"] = pair
    if not args.no_f64:
        result["float64_grid"] = run_f64(args)
    if not args.no_inline:
        result["inline_layout"] = run_inline(args, x, xr, plain)
    if not args.no_packing:
        result["packing"] = run_packing(args, x, xr)
    abl_codes = None
    if not args.no_ablation:
        result["ablation"], abl_codes = run_ablation(args, x, xr, plain)
    sample = []
    if not args.no_batched:
        result["batched"], sample = run_batched(args)
    serve_sample = []
    if not args.no_serving:
        result["serving"], serve_sample = run_serving(args)
    if not args.no_cpu_baseline:
        base, parity, bpar = cpu_baseline_leg(x, xr, args.eb, plain, sample, abl_codes, serve_sample)
        result["cpu_baseline"] = base
        result["parity_vs_oracle"] = {"plain": parity, "batched_sample": bpar}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
