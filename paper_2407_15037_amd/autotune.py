"""Launch-shape autotuner for the per-value kernels.

Every kernel comes in a few variants (loads in flight per thread x rounds per
tile, see lcq_tune_variants in include/lcq.h); all of them produce the same
bytes.  The tuner times each variant of quantize and dequantize per dtype on a
synthetic field resident in HBM, keeps the fastest (median of repeats, HIP
events around the per-value kernel only) and installs it process-wide.  The
result can be cached as JSON keyed by the device name.
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


def tune(n=1 << 26, reps=7, quantizer="abs", eb=1e-3, device="cuda", dtypes=None, install=True,
         log=None):
    """Returns {dtype_name: {op: {"best": v, "us": [per-variant median us]}}}."""
    import torch
    dtypes = dtypes or (torch.float32, torch.float64)
    result = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(); e1.record()
    for dt in dtypes:
        m = n if dt == torch.float32 else n // 2
        x = _field(m, dt, device)
        cap = lcq.max_stream_bytes(dt, m)
        buf = torch.empty(cap, dtype=torch.uint8, device=device)
        nb = torch.empty(1, dtype=torch.int64, device=device)
        ws = torch.empty(lcq.workspace_bytes(quantizer, dt, m), dtype=torch.uint8, device=device)
        out = torch.empty(m, dtype=dt, device=device)
        name = str(dt).replace("torch.", "")
        result[name] = {}
        saved = {op: lcq.tune_get(op, dt) for op in OPS}
        for op in OPS:
            med = []
            for v in range(lcq.tune_variants()):
                lcq.tune_set(op, dt, v)
                ts = []
                for r in range(reps + 2):
                    lcq.profile_events(e0, e1)
                    if op == "quantize":
                        lcq.quantize(x, quantizer, eb, out=buf, nbytes=nb, ws=ws)
                    else:
                        lcq.dequantize(buf, dt, m, out=out, ws=ws)
                    lcq.profile_events(None, None)
                    torch.cuda.synchronize()
                    if r >= 2:
                        ts.append(e0.elapsed_time(e1) * 1e3)
                ts.sort()
                med.append(ts[len(ts) // 2])
                if op == "quantize":
                    lcq.tune_set(op, dt, saved[op])
            best = min(range(len(med)), key=lambda i: med[i])
            result[name][op] = {"best": best, "us": [round(t, 1) for t in med]}
            lcq.tune_set(op, dt, best if install else saved[op])
            if log:
                log(f"autotune {name} {op}: {result[name][op]}")
        del x, buf, out, ws
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
