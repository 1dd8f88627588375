"""Batched launches and the serving loop on the GPU.

Every job's result must be identical alone and in the mix: the batched
launch and both serving modes are compared, bit for bit, with the job's own
single launch (simplex_map_launch) and, at small sizes, with the oracle.
The sentinel outside each job's simplex must survive.
"""
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
    return binding


OP = {2: "ca2", 3: "ca3"}


def job_input(m, n, seed):
    return si.box_torch(m, n, "bern", seed, p=0.25 if m == 2 else 0.2, device="cuda")


def alone(smap, m, n, inp):
    out = si.sentinel_box_torch(m, n, True, device="cuda")
    smap.map_launch(m, n, OP[m], inp, out)
    return out


MIX = [(2, n) for n in (0, 1, 5, 14, 15, 16, 37, 255, 256, 257, 300, 1000, 2049)] + \
      [(3, n) for n in (0, 2, 3, 14, 15, 16, 40, 63, 64, 65, 130)]


def test_batch_matches_single_launch_and_oracle(smap):
    ins, refs, outs = [], [], []
    for k, (m, n) in enumerate(MIX):
        inp = job_input(m, n, 5100 + k)
        ins.append(inp)
        refs.append(alone(smap, m, n, inp))
        outs.append(si.sentinel_box_torch(m, n, True, device="cuda"))
    torch.cuda.synchronize()
    order = list(range(len(MIX)))
    np.random.default_rng(7).shuffle(order)          # interleave the classes
    say("batch of", len(order), "jobs")
    smap.batch_launch([(MIX[i][0], OP[MIX[i][0]], MIX[i][1], ins[i], outs[i]) for i in order])
    torch.cuda.synchronize()
    for k, (m, n) in enumerate(MIX):
        say(f"compare m={m} n={n}")
        assert torch.equal(outs[k], refs[k]), (m, n)
        if (m == 2 and n <= 300) or (m == 3 and n <= 40):
            want = si.sentinel_box(m, n, np.uint8)
            oracle.apply(m, n, OP[m], ins[k].cpu().numpy(), want)
            assert np.array_equal(outs[k].cpu().numpy(), want), (m, n)


def test_batch_many_jobs_split_over_launches(smap):
    """More jobs than one launch takes (4096): split launches, same results."""
    n = 20
    inp = job_input(2, n, 5300)
    ref = alone(smap, 2, n, inp)
    outs = [si.sentinel_box_torch(2, n, True, device="cuda") for _ in range(4100)]
    torch.cuda.synchronize()
    say("batch of 4100 jobs")
    smap.batch_launch([(2, "ca2", n, inp, o) for o in outs])
    torch.cuda.synchronize()
    stacked = torch.stack(outs)
    assert torch.equal(stacked, ref.unsqueeze(0).expand_as(stacked))


@pytest.mark.parametrize("cap", [0, 1, 7])
def test_queue_matches_single_launch_and_oracle(smap, cap):
    """One persistent launch over the mixed classes: cap 0 runs the device's
    resident workgroup count, 1 runs every unit on one workgroup, 7 makes
    workgroups claim units of several jobs and classes in turn."""
    ins, refs, outs = [], [], []
    for k, (m, n) in enumerate(MIX):
        inp = job_input(m, n, 5400 + k)
        ins.append(inp)
        refs.append(alone(smap, m, n, inp))
        outs.append(si.sentinel_box_torch(m, n, True, device="cuda"))
    torch.cuda.synchronize()
    order = list(range(len(MIX)))
    np.random.default_rng(8).shuffle(order)
    say(f"queue launch of {len(order)} jobs, cap {cap}")
    smap.queue_launch([(MIX[i][0], OP[MIX[i][0]], MIX[i][1], ins[i], outs[i]) for i in order],
                      max_workgroups=cap)
    torch.cuda.synchronize()
    for k, (m, n) in enumerate(MIX):
        say(f"compare m={m} n={n}")
        assert torch.equal(outs[k], refs[k]), (m, n)
        if (m == 2 and n <= 300) or (m == 3 and n <= 40):
            want = si.sentinel_box(m, n, np.uint8)
            oracle.apply(m, n, OP[m], ins[k].cpu().numpy(), want)
            assert np.array_equal(outs[k].cpu().numpy(), want), (m, n)


def test_queue_large_jobs_and_split(smap):
    """A large job of each class beside small ones, repeated launches
    reusing the ring, and more jobs than one launch takes (4096)."""
    big = [(2, 5000), (3, 300), (2, 20), (3, 17)]
    ins = [job_input(m, n, 5500 + k) for k, (m, n) in enumerate(big)]
    refs = [alone(smap, m, n, ins[k]) for k, (m, n) in enumerate(big)]
    torch.cuda.synchronize()
    for rep in range(3):
        outs = [si.sentinel_box_torch(m, n, True, device="cuda") for m, n in big]
        say(f"queue launch of large jobs, repeat {rep}")
        smap.queue_launch([(m, OP[m], n, ins[k], outs[k]) for k, (m, n) in enumerate(big)])
        torch.cuda.synchronize()
        for k, (m, n) in enumerate(big):
            assert torch.equal(outs[k], refs[k]), (rep, m, n)
    n = 20
    outs = [si.sentinel_box_torch(3, n, True, device="cuda") for _ in range(4100)]
    torch.cuda.synchronize()
    say("queue launch of 4100 jobs")
    inp = job_input(3, n, 5601)
    ref = alone(smap, 3, n, inp)
    torch.cuda.synchronize()
    smap.queue_launch([(3, "ca3", n, inp, o) for o in outs])
    torch.cuda.synchronize()
    stacked = torch.stack(outs)
    assert torch.equal(stacked, ref.unsqueeze(0).expand_as(stacked))


def serve_jobs(count, seed, spread_s):
    rng = np.random.default_rng(seed)
    jobs = []
    t = 0.0
    for k in range(count):
        if rng.random() < 0.6:
            m, n = 2, int(np.exp(rng.uniform(np.log(16), np.log(700))))
        else:
            m, n = 3, int(np.exp(rng.uniform(np.log(8), np.log(90))))
        t += rng.exponential(spread_s / count)
        jobs.append((m, n, t))
    return jobs


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_serve_results_same_alone_and_in_the_mix(smap, mode):
    spec = serve_jobs(40, 11, 0.02)
    ins = [job_input(m, n, 6000 + k) for k, (m, n, _) in enumerate(spec)]
    refs = [alone(smap, m, n, ins[k]) for k, (m, n, _) in enumerate(spec)]
    sizes = [((n + 1) ** m + 255) // 256 * 256 for m, n, _ in spec]
    arena = torch.full((sum(sizes) + 4096,), 0xA5, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    say(f"serve mode={mode} jobs={len(spec)}")
    recs = smap.serve_run([(m, OP[m], n, ins[k], t) for k, (m, n, t) in enumerate(spec)],
                          arena, mode, max_inflight=2, keep_outputs=True)
    torch.cuda.synchronize()
    for k, ((m, n, t), r) in enumerate(zip(spec, recs)):
        assert r["status"] == smap.OK
        assert t <= r["admit_s"] + 1e-9 and r["admit_s"] <= r["launch_s"] <= r["release_s"], r
        assert r["done_s"] <= r["release_s"] + 1e-3 and r["done_s"] >= r["launch_s"] - 1e-3, r
        box = (n + 1) ** m
        got = arena[r["out_offset"]:r["out_offset"] + box].view((n + 1,) * m)
        assert torch.equal(got, refs[k]), (k, m, n)
    if mode in (1, 2):
        assert max(r["batch"] for r in recs) < len(spec)      # some jobs shared a launch
    else:
        assert sorted(r["batch"] for r in recs) == list(range(len(spec)))


def test_serve_small_budget_queues_and_completes(smap):
    """An arena that holds two outputs: jobs wait for memory, all complete,
    and the memory in use never exceeds the arena."""
    n, count = 400, 12
    box = (n + 1) ** 2
    size = (box + 255) // 256 * 256
    ins = [job_input(2, n, 6500 + k) for k in range(count)]
    ref_last = alone(smap, 2, n, ins[-1])
    arena = torch.full((2 * size,), 0xA5, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    for mode in (0, 1, 2):
        say(f"small budget mode={mode}")
        recs = smap.serve_run([(2, "ca2", n, ins[k], 0.0) for k in range(count)], arena, mode)
        assert all(r["status"] == smap.OK for r in recs)
        assert recs[-1]["admit_s"] > recs[0]["admit_s"]           # the last job had to wait
        # host-clock interval during which each job held its output memory
        events = sorted([(r["admit_s"], 1) for r in recs] + [(r["release_s"], -1) for r in recs])
        live = 0
        for _, d in events:
            live += d
            assert live <= 2
        last = recs[-1]
        got = arena[last["out_offset"]:last["out_offset"] + box].view(n + 1, n + 1)
        assert torch.equal(got, ref_last)
