"""The no-allocation persistent launch (simplex_queue_launch_static) gives
the same bytes as simplex_queue_launch, on two calls in a row on one
stream, the second with fewer and smaller jobs, and rejects oversize job
sets before any work."""
import numpy as np
import pytest

import simplex_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def smap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_11617_amd import binding
    binding.lib()
    return binding


def _jobs(sizes, seed):
    ins, outs_a, outs_b, jobs_a, jobs_b = [], [], [], [], []
    for k, (m, n) in enumerate(sizes):
        d_in = si.box_torch(m, n, "bern", seed + k, p=0.3 if m == 2 else 0.2, device="cuda")
        a = si.sentinel_box_torch(m, n, True)
        b = si.sentinel_box_torch(m, n, True)
        op = "ca2" if m == 2 else "ca3"
        ins.append(d_in)
        outs_a.append(a)
        outs_b.append(b)
        jobs_a.append((m, op, n, d_in, a))
        jobs_b.append((m, op, n, d_in, b))
    return ins, outs_a, outs_b, jobs_a, jobs_b


def test_static_queue_matches_queue_launch(smap):
    s = torch.cuda.current_stream()
    calls = [
        [(2, 3000), (3, 300), (2, 14), (3, 14), (2, 700), (3, 129), (2, 0), (3, 1)] + [(2, 64 + k) for k in range(40)],
        [(3, 40), (2, 100), (2, 5)],     # second call: fewer and smaller jobs
    ]
    for c, sizes in enumerate(calls):
        print(f"call {c}: {len(sizes)} jobs", flush=True)
        ins, outs_a, outs_b, jobs_a, jobs_b = _jobs(sizes, 4100 + 100 * c)
        smap.queue_launch(jobs_a, stream=s)
        smap.queue_launch_static(jobs_b, stream=s)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(outs_a, outs_b)):
            assert torch.equal(a, b), (c, k, sizes[k])
        # one job checked against its own single launch too
        ref = si.sentinel_box_torch(*sizes[0], True)
        m0, n0 = sizes[0]
        smap.map_launch(m0, n0, "ca2" if m0 == 2 else "ca3", ins[0], ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, outs_b[0])


def test_static_queue_limits(smap):
    d = torch.zeros(16, dtype=torch.uint8, device="cuda")
    e = torch.zeros(16, dtype=torch.uint8, device="cuda")
    jobs = [(2, "ca2", 2, d, e)] * 257
    assert smap.queue_launch_static_raw(jobs) == smap.ERANGE
    assert smap.queue_launch_static_raw([], -1) == smap.EINVAL
    assert smap.queue_launch_static_raw([], 0) == smap.OK
