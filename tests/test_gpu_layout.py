"""The 3-D automaton under each native layout set explicitly: batched and
work-queue launches (which default to the packed layout) and one-job
launches of one step or several generations (which default to the
level-ordered one), each bit-exact against the oracle."""
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


def oracle_ca3(n, inp, steps=1):
    cur = inp.copy()
    for _ in range(steps):
        nxt = si.sentinel_box(3, n, np.uint8)
        oracle.apply(3, n, "ca3", cur, nxt)
        cur = nxt
    return cur


SIZES = [0, 1, 14, 15, 16, 40, 65, 130, 200]


@pytest.mark.parametrize("layout", ["packed", "levels"])
def test_every_ca3_launch_kind_under_layout(smap, layout):
    smap.set_layout(3, smap.LAYOUT_LEVELS if layout == "levels" else smap.LAYOUT_PACKED)
    try:
        ins = {n: si.box(3, n, "bern", 9100 + n, p=0.3) for n in SIZES}
        want1 = {n: oracle_ca3(n, ins[n]) for n in SIZES}
        d_in = {n: torch.from_numpy(ins[n].copy()).cuda() for n in SIZES}

        def fresh(n):
            return torch.from_numpy(si.sentinel_box(3, n, np.uint8)).cuda()

        for n in SIZES:
            say(f"{layout} single n={n}")
            d = fresh(n)
            smap.map_launch(3, n, "ca3", d_in[n], d)
            torch.cuda.synchronize()
            assert np.array_equal(d.cpu().numpy(), want1[n]), ("single", layout, n)

        say(f"{layout} batch of {len(SIZES)}")
        outs = {n: fresh(n) for n in SIZES}
        smap.batch_launch([(3, "ca3", n, d_in[n], outs[n]) for n in SIZES])
        torch.cuda.synchronize()
        for n in SIZES:
            assert np.array_equal(outs[n].cpu().numpy(), want1[n]), ("batch", layout, n)

        for mw in (0, 7):
            say(f"{layout} queue of {len(SIZES)} max_workgroups={mw}")
            outs = {n: fresh(n) for n in SIZES}
            smap.queue_launch([(3, "ca3", n, d_in[n], outs[n]) for n in SIZES], max_workgroups=mw)
            torch.cuda.synchronize()
            for n in SIZES:
                assert np.array_equal(outs[n].cpu().numpy(), want1[n]), ("queue", layout, mw, n)

        for n in (15, 65, 130):
            for steps in (1, 5, 17):
                say(f"{layout} steps n={n} steps={steps}")
                want = oracle_ca3(n, ins[n], steps)
                a = torch.from_numpy(ins[n].copy()).cuda()
                d = fresh(n)
                smap.map_launch_steps(3, n, "ca3", steps, a, d)
                torch.cuda.synchronize()
                assert np.array_equal(d.cpu().numpy(), want), ("steps", layout, n, steps)
    finally:
        smap.set_layout(3, smap.LAYOUT_AUTO)
