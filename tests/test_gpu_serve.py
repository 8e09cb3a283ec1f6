"""Serving (continuous batching): requests admitted as slots and memory free
up, overlapping on the device; every output equals the oracle's bytes, both
when the requests run one at a time and when they run in the mix."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import announce

pytestmark = pytest.mark.gpu


def _pool(seed, m, lo=4 << 10, hi=8 << 20, grid=64):
    import torch
    master = synth.grf_3d(grid, seed, dtype=np.float64)
    relm = synth.rel_variant(master, seed + 1, dtype=np.float64)
    specs = synth.field_specs(m, seed + 2, lo, hi)
    pool = []
    for i, sp in enumerate(specs):
        x = synth.field_data(sp, master, relm, seed + 10 + i)
        st = O.quantize_mt(sp["q"], x, sp["eb"])
        dec = O.dequantize_mt(st, x.dtype, x.size)
        tdt = torch.float32 if x.dtype == np.float32 else torch.float64
        pool.append(dict(spec=sp, tdt=tdt, x=torch.from_numpy(x).cuda(),
                         stream=torch.from_numpy(st).cuda(), stream_bytes=st.size,
                         dec=torch.from_numpy(dec.view(np.uint8).copy()).cuda()))
    return pool


def _requests(pool, arrivals, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for t in arrivals:
        p = pool[int(rng.integers(0, len(pool)))]
        sp = p["spec"]
        if rng.random() < 0.5:
            reqs.append(dict(op="quantize", x=p["x"], n=sp["n"], dtype=p["tdt"], q=sp["q"],
                             eb=sp["eb"], expect=p["stream"], expect_bytes=p["stream_bytes"],
                             arrival_ns=int(t)))
        else:
            reqs.append(dict(op="dequantize", x=p["stream"], n=sp["n"], dtype=p["tdt"],
                             in_bytes=p["stream_bytes"], expect=p["dec"], arrival_ns=int(t)))
    return reqs


def test_serve_mix_and_alone_match_oracle():
    from paper_2407_15037_amd import serve
    pool = _pool(5, 24)
    arr = synth.poisson_arrivals(20000, 0.02, 6)  # ~400 requests in 20 ms
    reqs = _requests(pool, arr, 7)
    announce("serve mix", len(reqs))
    mix = serve.run(reqs, n_streams=8, arena_bytes=2 << 30)
    assert np.all(mix["status"] == 0), mix["status"]
    assert np.all(mix["mismatched"] == 0), np.flatnonzero(mix["mismatched"])
    assert np.all(mix["done_ns"] >= mix["admit_ns"])
    assert np.all(mix["admit_ns"] >= mix["arrival_ns"])
    assert len(set(mix["stream"].tolist())) > 1  # work really was spread over slots
    # the same requests one at a time (one slot, spaced arrivals)
    alone_reqs = [dict(r, arrival_ns=i * 200000) for i, r in enumerate(reqs)]
    announce("serve alone", len(alone_reqs))
    alone = serve.run(alone_reqs, n_streams=1, arena_bytes=2 << 30)
    assert np.all(alone["status"] == 0)
    assert np.all(alone["mismatched"] == 0)


def test_serve_full_size_range_matches_oracle():
    """Payloads drawn from the served size range (64 KiB - 256 MiB,
    log-uniform, mixed dtype / quantizer / bound), a Poisson mix of about
    400 requests: every output equals the oracle's bytes."""
    from paper_2407_15037_amd import serve
    pool = _pool(25, 12, 64 << 10, 256 << 20, grid=256)
    arr = synth.poisson_arrivals(2000, 0.2, 26)
    reqs = _requests(pool, arr, 27)
    announce("serve full range", len(reqs), max(p["spec"]["n"] for p in pool))
    res = serve.run(reqs, n_streams=8, arena_bytes=16 << 30)
    assert np.all(res["status"] == 0), res["status"]
    assert np.all(res["mismatched"] == 0), np.flatnonzero(res["mismatched"])


def test_serve_admission_under_tight_budget():
    """A budget that holds only a couple of requests at a time: requests wait
    for memory (first come, first served) and still all come out right."""
    from paper_2407_15037_amd import serve
    pool = _pool(15, 10)
    arr = np.zeros(120, dtype=np.int64)  # all at once
    reqs = _requests(pool, arr, 17)
    biggest = max(p["spec"]["n"] * (8 if p["tdt"].itemsize == 8 else 4) for p in pool)
    announce("serve tight", len(reqs), biggest)
    res = serve.run(reqs, n_streams=8, arena_bytes=3 * 2 * biggest + (1 << 20))
    assert np.all(res["status"] == 0)
    assert np.all(res["mismatched"] == 0)
    # admissions in arrival order
    order = np.argsort(res["admit_ns"], kind="stable")
    assert np.all(np.diff(order) > 0)
