"""Autotuning and HIP graphs on the GPU.

The tuned launch must give the same result as the oracle (the choice of
tile, workgroup size and beta never changes a result), the disk cache must
return the stored choice, and every replay of a captured graph must equal
the same launches run eagerly, with eager work between the replays.
"""
import os

import numpy as np
import pytest

import simplex_inputs as si
from oracle import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def smap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_11617_amd import binding
    binding.lib()
    yield binding
    binding.autotune_reset()


def expected(m, n, op, inp):
    out = si.sentinel_box(m, n, oracle.dtype_of(op))
    oracle.apply(m, n, op, inp, out)
    return out


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32 if a.dtype == np.uint32 else np.uint8)).cuda()


@pytest.mark.parametrize("m,n,op", [(2, 300, "accum"), (3, 45, "hash"), (4, 33, "hash"),
                                    (2, 700, "ca2"), (3, 70, "ca3")])
def test_autotune_result_and_cache(smap, tmp_path, m, n, op):
    dist = {"accum": "u31", "ca2": "bern", "ca3": "bern"}.get(op)
    inp = si.box(m, n, dist, 7000 + n, p=0.3) if dist else None
    want = expected(m, n, op, inp)
    d_in = dev(inp) if inp is not None else None
    d_out = dev(si.sentinel_box(m, n, want.dtype))
    cache = str(tmp_path / "tune.txt")
    say(f"autotune m={m} n={n} {op}")
    best = smap.autotune(m, n, op, d_in, d_out, reps=5, cache_path=cache)
    torch.cuda.synchronize()
    assert best["us"] > 0 and best["rho"] > 0
    assert best["beta"] in ((3, 4) if m == 4 else (2,))
    assert np.array_equal(d_out.cpu().numpy().view(want.dtype), want)
    # a fresh launch with the tuned choice (beta 0 = the tuned beta)
    d_out2 = dev(si.sentinel_box(m, n, want.dtype))
    smap.map_launch(m, n, op, d_in, d_out2)
    torch.cuda.synchronize()
    assert np.array_equal(d_out2.cpu().numpy().view(want.dtype), want)
    assert os.path.exists(cache) and "smap-tune-v2" in open(cache).read()
    # the cache returns the stored choice without timing
    smap.autotune_reset()
    again = smap.autotune(m, n, op, d_in, d_out, reps=5, cache_path=cache)
    keys = ("rho", "wg_threads", "tiles_per_wg", "beta")
    assert tuple(again[k] for k in keys) == tuple(best[k] for k in keys)
    assert abs(again["us"] - best["us"]) < 1e-2


def test_graph_accum_in_place_replays(smap):
    m, n, steps = 2, 500, 3
    inp = si.box(m, n, "u31", 7100, poison=True)
    buf = dev(inp)
    other = dev(si.box(m, n, "u31", 7101))
    other_want = dev(expected(m, n, "accum", si.box(m, n, "u31", 7101)))
    g = smap.Graph(m, n, "accum", buf, buf, steps=steps)
    inside = torch.from_numpy(si.inside_mask(m, n)).cuda()
    base = buf.clone()
    try:
        for k in range(1, 5):
            say(f"graph replay {k}")
            g.launch()
            torch.cuda.synchronize()
            want = torch.where(inside, base + steps * k, base)   # int32 wraps like uint32
            assert torch.equal(buf, want), k
            # eager work between the replays
            tmp = torch.full_like(other, 0)
            smap.map_launch(m, n, "accum", other, tmp)
            torch.cuda.synchronize()
            assert torch.equal(torch.where(inside, tmp, other_want), other_want)
    finally:
        g.close()


@pytest.mark.parametrize("use_bb", [False, True])
def test_graph_ca2_ping_pong_replays(smap, use_bb):
    m, n, steps = 2, 777, 4
    inp = si.box(m, n, "bern", 7200, p=0.3)
    a, b = dev(inp), dev(si.sentinel_box(m, n, np.uint8))
    ea, eb = a.clone(), b.clone()
    g = smap.Graph(m, n, "ca2", a, b, steps=steps, use_bb=use_bb)
    try:
        for k in range(3):
            say(f"ca2 graph replay {k}")
            g.launch()
            for i in range(steps):          # the same steps, eagerly, on copies
                src, dst = (ea, eb) if i % 2 == 0 else (eb, ea)
                smap.map_launch(m, n, "ca2", src, dst)
            torch.cuda.synchronize()
            assert torch.equal(a, ea) and torch.equal(b, eb), k
    finally:
        g.close()


def test_queue_graph_replays(smap):
    """A persistent work-queue launch over a fixed mix of CA2 and CA3 jobs,
    captured once and replayed several times with eager work (output resets)
    and synchronisations in between: every replay equals the single launches."""
    OP = {2: "ca2", 3: "ca3"}
    MIX = [(2, n) for n in (0, 5, 14, 15, 37, 256, 300, 2049)] + [(3, n) for n in (0, 3, 14, 16, 64, 65, 130)]
    ins = [si.box_torch(m, n, "bern", 5700 + k, p=0.25 if m == 2 else 0.2, device="cuda")
           for k, (m, n) in enumerate(MIX)]
    refs = []
    for k, (m, n) in enumerate(MIX):
        ref = si.sentinel_box_torch(m, n, True, device="cuda")
        smap.map_launch(m, n, OP[m], ins[k], ref)
        refs.append(ref)
    outs = [si.sentinel_box_torch(m, n, True, device="cuda") for m, n in MIX]
    torch.cuda.synchronize()
    for cap in (0, 7):
        g = smap.QueueGraph([(m, OP[m], n, ins[k], outs[k]) for k, (m, n) in enumerate(MIX)], max_workgroups=cap)
        try:
            for rep in range(4):
                for o in outs:
                    o.fill_(si.SENTINEL_U8)
                torch.cuda.synchronize()
                say(f"queue graph cap={cap} replay {rep}")
                g.launch(torch.cuda.current_stream())
                torch.cuda.synchronize()
                for k, (m, n) in enumerate(MIX):
                    assert torch.equal(outs[k], refs[k]), (cap, rep, m, n)
        finally:
            g.close()


def test_autotune_edm_skips_grouped_shapes(smap):
    """EDM runs one tile per workgroup only: the tuner passes over the
    grouped pointwise shapes and returns an ungrouped one, bit-for-bit the
    same distances as the default launch."""
    n = 500
    pts = torch.from_numpy(si.points(n, 7300)).cuda()
    ref = dev(si.sentinel_box(2, n, np.uint32))
    smap.map_launch(2, n, "edm", pts, ref)
    out = dev(si.sentinel_box(2, n, np.uint32))
    try:
        best = smap.autotune(2, n, "edm", pts, out, reps=3)
        torch.cuda.synchronize()
        assert best["tiles_per_wg"] == 1 and best["us"] > 0
        again = dev(si.sentinel_box(2, n, np.uint32))
        smap.map_launch(2, n, "edm", pts, again)
        torch.cuda.synchronize()
        assert torch.equal(again, ref)
    finally:
        smap.autotune_reset()
