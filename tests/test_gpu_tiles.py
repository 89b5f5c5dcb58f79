"""GPU checks of the tile shapes: the 4^3-cell tile (2x2x2 octs) and the
8^3-cell tile (4x4x4 octs assembled from small tiles), chosen for all
levels or level by level, give bit-identical FP64 results (each face flux
is the same expression of the same primitives whichever tile computes it),
and match the oracle at the parity bar; base sides of 2 mod 4 cells (an odd
number of octs per axis: tiles cut by the domain's high side) on both
boundary rules; the batched boxes with such sides.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle

import cases

pytestmark = pytest.mark.gpu

TOL = 1e-12
SMALL = dict(tiles_per_wg=1, persistent=0, waves_per_cu=4, batch=1, waves_per_tile=1, tile_cells=4)
BIG = dict(tiles_per_wg=1, persistent=0, waves_per_cu=4, batch=1, waves_per_tile=8, tile_cells=8)
# the 8^3-cell tile on 4 wavefronts: two core cells per thread
BIG4 = dict(BIG, waves_per_tile=4)


@pytest.fixture(scope="module")
def ry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_14631_amd import ry as mod
    mod.lib()
    return mod


def compare_levels(g, o, tol=TOL):
    worst = 0.0
    for lv in g.levels:
        ng, leaf_g = g.level_info(lv)
        no, leaf_o = o.level_info(lv)
        assert (ng, leaf_g) == (no, leaf_o), lv
        if ng == 0:
            continue
        kg, rg = g.mesh(lv)
        ko, ro = o.mesh(lv)
        np.testing.assert_array_equal(kg, ko)
        np.testing.assert_array_equal(rg, ro)
        worst = max(worst, cases.rel_err(g.download(lv), o.download(lv)))
    assert worst <= tol, worst
    return worst


def states(h):
    return [h.download(lv) for lv in h.levels]


def run(ry, prob, n, prec="fp64", tuning=None, per_level=None):
    h = ry.Hydro(prob, prec)
    if tuning:
        h.set_tuning(**tuning)
    for lv, t in (per_level or {}).items():
        h.set_level_tuning(lv, **t)
    h.advance(n)
    return h


def outflow(prob):
    return dataclasses.replace(prob, bc=(W.BC_OUTFLOW,) * 6)


PROBLEMS = {
    "blob_periodic": lambda: cases.amr_blob(),
    "blob_outflow": lambda: cases.amr_blob(bc=(W.BC_OUTFLOW,) * 6, centre=(0.1, 0.5, 0.5)),
    "uniform32": lambda: W.random_smooth(32, seed=21, mach=1.5),
    "twolevel64": lambda: W.twolevel(64, 0.5),
}


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_big_tile_matches_oracle_and_small_tile_bit_exact(ry, name):
    prob = PROBLEMS[name]()
    small = run(ry, prob, 4, tuning=SMALL)
    o = Oracle(prob)
    o.advance(4)
    for t in (BIG, BIG4):
        big = run(ry, prob, 4, tuning=t)
        assert big.tuning()["tile_cells"] == 8
        for a, b in zip(states(small), states(big)):
            np.testing.assert_array_equal(a, b)
        compare_levels(big, o)
        assert big.floors() == small.floors()


def test_big_tile_mixed_form_bit_exact(ry):
    prob = cases.amr_blob()
    a = run(ry, prob, 3, "mixed", tuning=SMALL)
    for t in (BIG, BIG4):
        b = run(ry, prob, 3, "mixed", tuning=t)
        for x, y in zip(states(a), states(b)):
            np.testing.assert_array_equal(x, y)


def test_per_level_tile_shapes_bit_exact(ry):
    """Every mixture of tile shapes over the levels gives the same state
    (graph path and host-driven path), and a regrid rebuilds the 8^3-cell
    tile tables of the new mesh."""
    prob = cases.amr_blob(level_min=3, level_max=5)
    ref = run(ry, prob, 3)
    for per in ({3: BIG}, {4: BIG}, {5: BIG}, {3: BIG, 5: BIG}, {4: BIG, 5: BIG}, {3: BIG4, 4: BIG4, 5: BIG}):
        h = run(ry, prob, 3, per_level=per)
        for lv, t in per.items():
            assert h.level_tuning(lv)["tile_cells"] == 8
        for a, b in zip(states(ref), states(h)):
            np.testing.assert_array_equal(a, b)
    g = ry.Hydro(prob)
    g.set_tuning(**BIG)
    for _ in range(3):
        g.coarse_step(g.cfl_dt())
    for a, b in zip(states(ref), states(g)):
        np.testing.assert_array_equal(a, b)
    # regrid, then more steps on both tile shapes
    ref.regrid()
    g2 = run(ry, prob, 3, tuning=BIG)
    g2.regrid()
    ref.advance(2)
    g2.advance(2)
    for a, b in zip(states(ref), states(g2)):
        np.testing.assert_array_equal(a, b)


def test_autotune_per_level_keeps_results(ry):
    prob = cases.amr_blob()
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    best, times = a.autotune()
    assert len(times) >= 5 and all(t > 0 for t in times)
    chosen = [a.level_tuning(lv) for lv in a.levels]
    assert chosen[0] == best
    a.advance(3)
    b.advance(3)
    for x, y in zip(states(a), states(b)):
        np.testing.assert_array_equal(x, y)


def test_autotune_cache(ry, tmp_path):
    """A tuning stored in the cache file for a workload, precision and GPU
    architecture is applied without timing; other keys time and add theirs."""
    import json
    path = str(tmp_path / "tune.json")
    prob = cases.amr_blob()
    a = ry.Hydro(prob)
    best, times = a.autotune(cache=path)
    assert times
    chosen = [a.level_tuning(lv) for lv in a.levels]
    b = ry.Hydro(prob)
    best_b, times_b = b.autotune(cache=path)
    assert times_b == [] and best_b == best
    assert [b.level_tuning(lv) for lv in b.levels] == chosen
    m = ry.Hydro(prob, "mixed")
    assert m.autotune(cache=path)[1]
    boxes = [W.batch_box(60, 16, 1.0, 1.5), W.batch_box(61, 24, 0.7, 0.8)]
    b1 = ry.BatchHydro(boxes)
    assert b1.autotune(cache=path)[1]
    b2 = ry.BatchHydro(boxes)
    assert b2.autotune(cache=path)[1] == [] and b2.tuning() == b1.tuning()
    assert len(json.load(open(path))) == 3
    for h in (b1, b2):
        h.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_big_tile_bit_exact(ry, prec):
    """Batched boxes on 8^3-cell tiles (sides of 8 mod 16 and 2 mod 4 give
    super-tiles cut by the box's high side): the same boxes and times as on
    4^3-cell tiles, FP64 also against the oracle; the autotuner may pick
    either shape."""
    boxes = [W.batch_box(40, 24, 1.0, 1.5), W.batch_box(41, 18, 0.7, 0.8), W.batch_box(42, 32, 1.2, 2.0),
             W.batch_box(43, 10, 0.5, 1.0), W.batch_box(44, 16, 1.0, 1.0)]
    out = []
    for t in (SMALL, BIG, BIG4, None):
        bh = ry.BatchHydro(boxes, prec)
        if t is None:
            bh.autotune()
        else:
            bh.set_tuning(**t)
        bh.run(4)
        out.append(([bh.download(b) for b in range(len(boxes))], [bh.box_info(b)[1] for b in range(len(boxes))]))
        bh.close()
    for states, times in out[1:]:
        assert times == out[0][1]
        for a, b in zip(states, out[0][0]):
            np.testing.assert_array_equal(a, b)
    if prec == "fp64":
        for b, p in enumerate(boxes):
            o = Oracle(p)
            o.advance(4)
            assert cases.rel_err(out[1][0][b], o.download(p.level_min)) <= TOL, b


def test_big_tile_rejected_where_unsupported(ry):
    g = ry.Hydro(cases.with_scalars(cases.amr_blob(), 1))
    with pytest.raises(ry.RyError) as e:
        g.set_tuning(**BIG)
    assert e.value.code == ry.RY_EINVAL
    h = ry.Hydro(cases.amr_blob())
    with pytest.raises(ry.RyError) as e:
        h.set_tuning(**dict(BIG, waves_per_tile=2))
    assert e.value.code == ry.RY_EINVAL


# ------------------------------------------------ base sides of 2 mod 4 cells
@pytest.mark.parametrize("n", [18, 30])
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_base_side_2_mod_4_uniform(ry, n, bc):
    prob = W.random_smooth(n, seed=n, mach=1.2)
    if bc == "outflow":
        prob = outflow(prob)
    o = Oracle(prob)
    o.advance(4)
    for t in (SMALL, BIG):
        g = run(ry, prob, 4, tuning=t)
        compare_levels(g, o)


@pytest.mark.parametrize("n_fine", [36, 60])
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_base_side_2_mod_4_amr(ry, n_fine, bc):
    prob = W.twolevel(n_fine, 0.5)
    if bc == "outflow":
        prob = outflow(prob)
    o = Oracle(prob)
    assert o.level_info(prob.level_max)[0] > 0
    o.advance(3)
    for t in (SMALL, BIG):
        g = run(ry, prob, 3, tuning=t)
        compare_levels(g, o)


@pytest.mark.parametrize("level_max", [3, 5])
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_non_cubic_box(ry, level_max, bc):
    """A box of 8 x 16 x 12 base cells (4 x 8 x 6 octs: 8^3-cell tiles cut
    along z), uniform and with two refined levels, on every tile shape,
    against the oracle."""
    prob = cases.noncubic_blob(bc=(W.BC_OUTFLOW if bc == "outflow" else W.BC_PERIODIC,) * 6, level_max=level_max)
    o = Oracle(prob)
    o.advance(3)
    for t in (SMALL, BIG, BIG4):
        g = run(ry, prob, 3, tuning=t)
        compare_levels(g, o)


def test_batch_accepts_sides_2_mod_4(ry):
    boxes = [W.batch_box(30, 18, 1.0, 1.5), W.batch_box(31, 30, 0.7, 0.8), W.batch_box(32, 16, 1.2, 2.0),
             W.batch_box(33, 6, 0.5, 1.0)]
    bh = ry.BatchHydro(boxes)
    bh.run(5)
    for b, p in enumerate(boxes):
        o = Oracle(p)
        o.advance(5)
        assert cases.rel_err(bh.download(b), o.download(p.level_min)) <= TOL, b
        assert abs(bh.box_info(b)[1] - o.t) <= 1e-14 * o.t

