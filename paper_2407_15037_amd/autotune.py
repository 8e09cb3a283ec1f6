"""Launch-shape autotuner for the per-value kernels.

Every operation comes in a few kernel variants (see lcq_tune_variants in
include/lcq.h); all of them produce the same bytes.  The tuner times each
variant of quantize and dequantize per dtype on two synthetic fields resident
in HBM (an ABS field with few outliers, a REL field with 1 % of them), keeps
the fastest total (medians of repeats, HIP events around the operation's
kernels) and installs it process-wide.  The result can be cached as JSON
keyed by the device name.
"""
import json
import os

import paper_2407_15037_amd as lcq

OPS = ("quantize", "dequantize")


def _field(n, dtype, device):
    import torch
    g = torch.Generator(device="cpu").manual_seed(1234)
    x = torch.randn(n, generator=g, dtype=torch.float64).cumsum(0) * 1e-3
    return x.to(dtype).to(device)


def _rel_field(n, dtype, device):
    """Magnitudes log-uniform over 2^(+-40), random signs, 1 % zeros: a REL
    field with about 1 % of its values stored losslessly."""
    import torch
    g = torch.Generator(device=device).manual_seed(4321)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    s = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    x = torch.exp2(u * 80.0 - 40.0) * torch.where(s < 0.5, -1.0, 1.0)
    x = torch.where(s > 0.99, torch.zeros_like(x), x)
    return x.to(dtype)


def tune(n=1 << 26, reps=7, eb=1e-3, device="cuda", dtypes=None, install=True, log=None):
    """Time every launch variant of quantize and dequantize on an ABS field
    (smooth, few outliers) and a REL field (1 % outliers) per dtype; the
    fastest total wins.  Returns {dtype_name: {op: {"best": v, "us":
    [per-variant summed median us]}}}."""
    import torch
    dtypes = dtypes or (torch.float32, torch.float64)
    result = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(); e1.record()

    def timed(fn):
        ts = []
        for r in range(reps + 2):
            lcq.profile_events(e0, e1)
            fn()
            lcq.profile_events(None, None)
            torch.cuda.synchronize()
            if r >= 2:
                ts.append(e0.elapsed_time(e1) * 1e3)
        ts.sort()
        return ts[len(ts) // 2]

    for dt in dtypes:
        m = n if dt == torch.float32 else n // 2
        cases = [("abs", _field(m, dt, device)), ("rel", _rel_field(m, dt, device))]
        cap = lcq.max_stream_bytes(dt, m)
        bufs = [torch.empty(cap, dtype=torch.uint8, device=device) for _ in cases]
        nbs = [torch.empty(1, dtype=torch.int64, device=device) for _ in cases]
        ws = torch.empty(lcq.workspace_bytes("noa", dt, m), dtype=torch.uint8, device=device)
        out = torch.empty(m, dtype=dt, device=device)
        name = str(dt).replace("torch.", "")
        result[name] = {}
        saved = {op: lcq.tune_get(op, dt) for op in OPS}
        for (q, x), buf, nb in zip(cases, bufs, nbs):
            lcq.quantize(x, q, eb, out=buf, nbytes=nb, ws=ws)
        torch.cuda.synchronize()
        sizes = [int(nb.item()) for nb in nbs]
        for op in OPS:
            tot = []
            for v in range(lcq.tune_variants()):
                lcq.tune_set(op, dt, v)
                t = 0.0
                for (q, x), buf, nb, size in zip(cases, bufs, nbs, sizes):
                    if op == "quantize":
                        t += timed(lambda: lcq.quantize(x, q, eb, out=buf, nbytes=nb, ws=ws))
                    else:
                        t += timed(lambda: lcq.dequantize(buf, dt, m, stream_bytes=size, out=out,
                                                          ws=ws))
                tot.append(t)
            best = min(range(len(tot)), key=lambda i: tot[i])
            result[name][op] = {"best": best, "us": [round(t, 1) for t in tot]}
            lcq.tune_set(op, dt, best if install else saved[op])
            if log:
                log(f"autotune {name} {op}: {result[name][op]}")
        del cases, bufs, out, ws
    return result


def install(table):
    """Apply a table produced by tune() (or loaded from JSON)."""
    import torch
    for name, ops in table.items():
        dt = getattr(torch, name)
        for op, r in ops.items():
            lcq.tune_set(op, dt, r["best"])


def cache_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def load_or_tune(path=None, **kw):
    import torch
    path = path or cache_path()
    dev = torch.cuda.get_device_name(0)
    if os.path.exists(path):
        try:
            data = json.load(open(path))
            if dev in data:
                install(data[dev])
                return data[dev]
        except (OSError, ValueError):
            pass
    table = tune(**kw)
    try:
        data = json.load(open(path)) if os.path.exists(path) else {}
    except (OSError, ValueError):
        data = {}
    data[dev] = table
    try:
        json.dump(data, open(path, "w"), indent=1)
    except OSError:
        pass
    return table


def tune_batch(fields, reps=3, cpws=(1, 2, 4, 8), log=None):
    """Pick the batch plan's tuning string for a set of fields (dicts with
    x, q, eb as for batch.BatchPlan), timing the quantize graph on the
    fields themselves (512 MiB written and 512 MiB read to evict the caches
    before every run, median of `reps` after one untimed run): first each
    kernel variant; if the chunk form wins, then its chunks per wavefront
    for float32 fields (float64 at 1), then for float64 fields (float32 at
    its best).  Returns {"tune": string for lcq_batch_plan_create, "ms":
    {tuning string: median ms}}."""
    import torch
    from paper_2407_15037_amd.batch import BatchPlan, variants
    scratch = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    clean = torch.ones(64 << 20, dtype=torch.int64, device="cuda")
    ms = {}

    def timed(tune):
        if tune in ms:
            return ms[tune]
        plan = BatchPlan(fields, tune=tune)
        ts = []
        for r in range(reps + 1):
            scratch.fill_(0x5A)  # evict the caches
            clean.sum()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.quantize()
            e1.record()
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
        plan.close()
        del plan
        torch.cuda.empty_cache()
        ts.sort()
        ms[tune] = round(ts[len(ts) // 2], 3)
        return ms[tune]

    best = min((f"batch={v}" for v in range(variants())), key=timed)
    if best == "batch=0":
        c32 = min(cpws, key=lambda c: timed(f"batch=0 f32={c} f64=1"))
        c64 = min(cpws, key=lambda c: timed(f"batch=0 f32={c32} f64={c}"))
        best = f"batch=0 f32={c32} f64={c64}"
    out = {"tune": best, "ms": ms}
    if log:
        log(f"batch autotune (quantize ms): {ms} -> {best}")
    return out
