"""Several automaton generations per pass (temporal blocking) against the
oracle applied generation by generation; bit-exact, H and BB, with the
sentinel outside the simplex intact and the input untouched when one pass
suffices."""
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


def oracle_steps(n, inp, steps, m=2):
    cur = inp.copy()
    for _ in range(steps):
        nxt = si.sentinel_box(m, n, np.uint8)
        oracle.apply(m, n, "ca2" if m == 2 else "ca3", cur, nxt)
        cur = nxt
    return cur


SIZES = [0, 1, 5, 14, 15, 16, 63, 100, 127, 128, 129, 159, 160, 161, 255, 300, 700]
STEPS = [1, 2, 7, 16, 17, 33, 40]


@pytest.mark.parametrize("kind", ["h", "bb"])
def test_steps_match_oracle(smap, kind):
    launch = smap.map_launch_steps if kind == "h" else smap.bb_launch_steps
    for n in SIZES:
        inp = si.box(2, n, "bern", 8000 + n, p=0.35)
        inside = si.inside_mask(2, n)
        for steps in STEPS:
            if n > 300 and steps > 17:
                continue
            say(f"{kind} n={n} steps={steps}")
            want = oracle_steps(n, inp, steps)
            d_in = torch.from_numpy(inp.copy()).cuda()
            d_out = torch.from_numpy(si.sentinel_box(2, n, np.uint8)).cuda()
            launch(2, n, "ca2", steps, d_in, d_out)
            torch.cuda.synchronize()
            got = d_out.cpu().numpy()
            assert np.array_equal(got, want), (kind, n, steps)
            after_in = d_in.cpu().numpy()
            assert np.array_equal(after_in[~inside], inp[~inside])      # outside never written
            if steps <= 32:
                assert np.array_equal(after_in, inp)                   # one pass: input untouched


def test_steps_workload_size_matches_single_steps(smap):
    """n = 16384: 16 generations in one pass equal 16 single-step launches."""
    w = si.WORKLOADS["c2"]
    n = w["n"]
    a = si.box_torch(2, n, "bern", w["seed"], p=w["p"], device="cuda")
    b = si.sentinel_box_torch(2, n, True, device="cuda")
    orig = a.clone()
    ref_a, ref_b = a.clone(), b.clone()
    say("single steps x16")
    for i in range(16):
        src, dst = (ref_a, ref_b) if i % 2 == 0 else (ref_b, ref_a)
        smap.map_launch(2, n, "ca2", src, dst)
    out = si.sentinel_box_torch(2, n, True, device="cuda")
    say("one pass of 16")
    smap.map_launch_steps(2, n, "ca2", 16, a, out)
    torch.cuda.synchronize()
    r = torch.arange(n + 1, device="cuda")
    inside = (r.view(-1, 1) + r.view(1, -1)) <= n          # x_1 + x_2 <= n (symmetric)
    # 16 single steps end in ref_a; outside the simplex ref_a keeps the input's
    # poison and `out` its sentinel, neither written
    assert torch.equal(out[inside], ref_a[inside])
    assert bool((out[~inside] == si.SENTINEL_U8).all())
    assert torch.equal(a, orig)             # one pass leaves the input untouched


SIZES3 = [0, 1, 5, 14, 15, 16, 31, 32, 33, 40, 63, 64, 65, 100, 130]
STEPS3 = [1, 2, 3, 5, 9, 16, 17, 33]


@pytest.mark.parametrize("kind", ["h", "bb"])
def test_steps_3d_match_oracle(smap, kind):
    """3-D: passes of up to 16 generations (64^3 tiles, 16-cell halo, one
    bit per cell in LDS); 17 and 33 steps take several passes."""
    launch = smap.map_launch_steps if kind == "h" else smap.bb_launch_steps
    for n in SIZES3:
        inp = si.box(3, n, "bern", 8100 + n, p=0.2)
        inside = si.inside_mask(3, n)
        for steps in STEPS3:
            if n > 65 and steps not in (1, 16, 17):
                continue
            say(f"3-D {kind} n={n} steps={steps}")
            want = oracle_steps(n, inp, steps, m=3)
            d_in = torch.from_numpy(inp.copy()).cuda()
            d_out = torch.from_numpy(si.sentinel_box(3, n, np.uint8)).cuda()
            launch(3, n, "ca3", steps, d_in, d_out)
            torch.cuda.synchronize()
            got = d_out.cpu().numpy()
            assert np.array_equal(got, want), (kind, n, steps)
            after_in = d_in.cpu().numpy()
            assert np.array_equal(after_in[~inside], inp[~inside])      # outside never written
            if steps <= 16:
                assert np.array_equal(after_in, inp)                   # one pass: input untouched


def test_steps_3d_workload_size_matches_single_steps(smap):
    """m = 3, n = 1024: 4 generations in one pass equal 4 single-step launches."""
    w = si.WORKLOADS["c3"]
    n = w["n"]
    a = si.box_torch(3, n, "bern", w["seed"], p=w["p"], device="cuda")
    orig = a.clone()
    ref_a, ref_b = a.clone(), si.sentinel_box_torch(3, n, True, device="cuda")
    say("3-D single steps x4")
    for i in range(4):
        src, dst = (ref_a, ref_b) if i % 2 == 0 else (ref_b, ref_a)
        smap.map_launch(3, n, "ca3", src, dst)
    out = si.sentinel_box_torch(3, n, True, device="cuda")
    say("3-D one pass of 4")
    smap.map_launch_steps(3, n, "ca3", 4, a, out)
    torch.cuda.synchronize()
    r = torch.arange(n + 1, device="cuda", dtype=torch.int16)
    inside = (r.view(-1, 1, 1) + r.view(1, -1, 1) + r.view(1, 1, -1)) <= n
    assert torch.equal(out[inside], ref_a[inside])
    assert bool((out[~inside] == si.SENTINEL_U8).all())
    assert torch.equal(a, orig)
