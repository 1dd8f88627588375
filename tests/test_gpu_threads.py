"""Launches from several host threads at once.

The library's calls are thread-safe (the plan cache, tile overrides and the
job-table ring are mutex-guarded).  Four threads, each on a stream of its
own, launch single steps (H and BB), batched launches and persistent
work-queue launches over their own buffers at the same time; every result
must equal the single-threaded launch of the same job.
"""
import threading

import pytest

import simplex_inputs as si

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


def test_four_threads_launching_at_once(smap):
    torch.cuda.set_device(0)
    jobs = [(2, 300), (3, 60), (2, 1000), (3, 100), (2, 37), (3, 17)]
    ins = [si.box_torch(m, n, "bern", 7000 + k, p=0.3, device="cuda") for k, (m, n) in enumerate(jobs)]
    refs = []
    for k, (m, n) in enumerate(jobs):
        out = si.sentinel_box_torch(m, n, True, device="cuda")
        smap.map_launch(m, n, OP[m], ins[k], out)
        refs.append(out)
    torch.cuda.synchronize()
    errors = []

    def worker(tid):
        try:
            torch.cuda.set_device(0)
            s = torch.cuda.Stream()
            for rep in range(5):
                outs = [si.sentinel_box_torch(m, n, True, device="cuda") for m, n in jobs]
                outs_b = [si.sentinel_box_torch(m, n, True, device="cuda") for m, n in jobs]
                outs_q = [si.sentinel_box_torch(m, n, True, device="cuda") for m, n in jobs]
                bb_out = si.sentinel_box_torch(*jobs[tid % len(jobs)], True, device="cuda")
                torch.cuda.synchronize()
                with torch.cuda.stream(s):
                    m, n = jobs[tid % len(jobs)]
                    smap.bb_launch(m, n, OP[m], ins[tid % len(jobs)], bb_out, stream=s)
                    for k, (m, n) in enumerate(jobs):
                        smap.map_launch(m, n, OP[m], ins[k], outs[k], stream=s)
                    smap.batch_launch([(m, OP[m], n, ins[k], outs_b[k]) for k, (m, n) in enumerate(jobs)], stream=s)
                    smap.queue_launch([(m, OP[m], n, ins[k], outs_q[k]) for k, (m, n) in enumerate(jobs)],
                                      max_workgroups=(0 if rep % 2 else 5), stream=s)
                s.synchronize()
                assert torch.equal(bb_out, refs[tid % len(jobs)]), (tid, rep, "bb")
                for k in range(len(jobs)):
                    assert torch.equal(outs[k], refs[k]), (tid, rep, k, "single")
                    assert torch.equal(outs_b[k], refs[k]), (tid, rep, k, "batch")
                    assert torch.equal(outs_q[k], refs[k]), (tid, rep, k, "queue")
        except Exception as e:   # collected and re-raised in the main thread
            errors.append(e)

    say("4 threads x 5 rounds of single, batched and queue launches")
    threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads), "a launching thread did not finish"
    assert not errors, repr(errors[0])
