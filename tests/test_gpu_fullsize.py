"""GPU parity at the workload sizes: whole boxes, element by element.

Every cell of the output box -- the simplex cells against the oracle, the
cells outside against the untouched sentinel -- for the H and BB launches
(and beta 3 and 4 for m = 4) at the sizes the benchmark runs:
  * m = 2, n = 16384: one Life step (B3/S23);
  * m = 3, n = 1024: one B6/S567 step, with the default tile, and with the
    256^3 tile at sizes where its sub-blocks meet neighbouring tiles across
    every face (n = 511, 512, 513, 767), in both 3-D layouts;
  * m = 4, n = 128: the coordinate hash;
  * several generations per pass (m = 2 and m = 3, 4 generations) against
    the oracle stepped generation by generation.
The oracle's slabs run on several host threads (tests/fullsize.py).
"""
import numpy as np
import pytest

from tests import fullsize
import simplex_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def smap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2208_11617_amd import binding  # raises if the library is missing
    binding.lib()
    return binding


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32 if a.dtype == np.uint32 else np.uint8)).cuda()


def fresh(m, n, u8):
    return si.sentinel_box_torch(m, n, u8)


def run(smap, kind, m, n, op, d_in, d_out, beta=0):
    say(f"  launch {kind} m={m} n={n} op={op} beta={beta}")
    if kind == "h":
        smap.map_launch(m, n, op, d_in, d_out, beta=beta)
    else:
        smap.bb_launch(m, n, op, d_in, d_out)
    torch.cuda.synchronize()


def first_difference(got, want):
    g = got.reshape(-1).cpu().numpy()
    w = want.reshape(-1).cpu().numpy()
    i = int(np.flatnonzero(g != w)[0])
    return i, int(g[i]), int(w[i])


@pytest.mark.parametrize("name", ["c2", "c3", "c4"])
def test_workload_whole_box(smap, name):
    w = si.WORKLOADS[name]
    m, n, op = w["m"], w["n"], w["op"]
    u8 = op.startswith("ca")
    say(f"workload {name}: m={m} n={n} op={op}: inputs and oracle on {fullsize.THREADS} threads")
    inp = fullsize.box(m, n, w["dist"], w["seed"], w["p"]) if w["dist"] else None
    want = dev(fullsize.expected(m, n, op, inp))
    d_in = dev(inp) if inp is not None else None
    del inp
    kinds = [("h", 0), ("bb", 0)] + ([("h", 4)] if m == 4 else [])
    for kind, beta in kinds:
        d_out = fresh(m, n, u8)
        run(smap, kind, m, n, op, d_in, d_out, beta)
        if not torch.equal(d_out, want):
            pytest.fail(f"{name} {kind} beta={beta}: first difference (index, got, want) "
                        f"{first_difference(d_out, want)}")
        del d_out


@pytest.mark.parametrize("layout", ["packed", "levels"])
def test_ca3_rho256_across_tile_faces(smap, layout):
    """The 256^3 CA3 tile (256- and 128-thread sub-block shapes) with
    neighbouring tiles on every face: whole boxes at n = 511, 512, 513 (two
    tiles per side, the last one ragged) and 767."""
    smap.set_layout(3, {"packed": smap.LAYOUT_PACKED, "levels": smap.LAYOUT_LEVELS}[layout])
    try:
        for n in (511, 512, 513, 767):
            inp = fullsize.box(3, n, "bern", 3700 + n, 0.2 if n % 2 else 0.3)
            want = dev(fullsize.expected(3, n, "ca3", inp))
            d_in = dev(inp)
            for wg in (256, 128):
                smap.set_tile(3, "ca3", 256, wg)
                say(f"ca3 rho 256 threads {wg} layout={layout} n={n}")
                for kind in ("h", "bb"):
                    d_out = fresh(3, n, True)
                    run(smap, kind, 3, n, "ca3", d_in, d_out)
                    if not torch.equal(d_out, want):
                        pytest.fail(f"n={n} threads={wg} {kind}: first difference {first_difference(d_out, want)}")
    finally:
        smap.set_tile(3, "ca3", 0)
        smap.set_layout(3, smap.LAYOUT_AUTO)


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_generations_whole_box(smap, name):
    """Four generations in one pass against the oracle stepped four times."""
    w = si.WORKLOADS[name]
    m, n, op, gens = w["m"], w["n"], w["op"], 4
    say(f"{name}: {gens} generations, oracle stepped generation by generation")
    inp = fullsize.box(m, n, w["dist"], w["seed"], w["p"])
    want = inp
    for g in range(gens):
        want = fullsize.expected(m, n, op, want)
    want = dev(want)
    for kind in ("h", "bb"):
        d_in, d_out = dev(inp), fresh(m, n, True)
        say(f"  {kind} launch_steps")
        if kind == "h":
            smap.map_launch_steps(m, n, op, gens, d_in, d_out)
        else:
            smap.bb_launch_steps(m, n, op, gens, d_in, d_out)
        torch.cuda.synchronize()
        if not torch.equal(d_out, want):
            pytest.fail(f"{name} {kind}: first difference {first_difference(d_out, want)}")
        del d_in, d_out
