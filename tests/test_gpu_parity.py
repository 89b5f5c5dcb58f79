"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU
oracle, element by element on identical seeded inputs.

Bar: FP64 form within 1e-12 relative per cell per variable, with the
relative error of a value b taken against max(|b|, 1e-3 max|b_v|) so that
components crossing zero are measured on their variable's scale; mesh keys
and refinement maps bit-exact; invariants (uniform state, stationary
contact) bit-exact; conservation to 1e-13.  The mixed form is compared with
the FP64 form (relative L1 density error <= 1e-5 after 10 steps).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle

import cases

pytestmark = pytest.mark.gpu

TOL = 1e-12


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
        ng, _ = g.level_info(lv)
        no, _ = o.level_info(lv)
        assert ng == no, (lv, ng, no)
        if ng == 0:
            continue
        kg, rg = g.mesh(lv)
        ko, ro = o.mesh(lv)
        np.testing.assert_array_equal(kg, ko)
        np.testing.assert_array_equal(rg, ro)
        worst = max(worst, cases.rel_err(g.download(lv), o.download(lv)))
    assert worst <= tol, worst
    return worst


def step_both(g, o, n):
    for _ in range(n):
        dt = o.cfl_dt()
        dg = g.cfl_dt()
        assert abs(dg - dt) <= 1e-14 * dt, (dg, dt)
        o.coarse_step(dt)
        g.coarse_step(dt)


# ------------------------------------------------------------ single level
def test_uniform_small_host_driven(ry):
    prob = W.random_smooth(16, seed=3, mach=1.5)
    g, o = ry.Hydro(prob), Oracle(prob)
    compare_levels(g, o, 0.0)
    step_both(g, o, 3)
    compare_levels(g, o)
    assert g.floors() == 0


def test_uniform_small_graph_advance(ry):
    prob = W.random_smooth(16, seed=4, mach=2.0)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(5)
    o.advance(5)
    compare_levels(g, o)


def test_sod_full_run(ry):
    prob = W.sod(32)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(1000, prob.t_end)
    n = o.advance(1000, prob.t_end)
    assert g.t == o.t == 0.1 and n > 10
    compare_levels(g, o)


def test_minimum_box_single_tile(ry):
    prob = W.random_smooth(4, seed=9)
    prob.nbase = (4, 4, 4)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(3)
    o.advance(3)
    compare_levels(g, o)


# -------------------------------------------------------------------- AMR
@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_amr_blob_host_driven(ry, bc):
    kw = {} if bc == "periodic" else dict(bc=(W.BC_OUTFLOW,) * 6, centre=(0.1, 0.5, 0.5))
    prob = cases.amr_blob(**kw)
    g, o = ry.Hydro(prob), Oracle(prob)
    assert g.level_info(5)[0] > 0
    compare_levels(g, o, 0.0)
    step_both(g, o, 3)
    compare_levels(g, o)


def test_amr_graph_equals_host_driven_bit_exact(ry):
    prob = cases.amr_blob()
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    for _ in range(3):
        a.coarse_step(a.cfl_dt())
    b.advance(3)
    for lv in a.levels:
        np.testing.assert_array_equal(a.download(lv), b.download(lv))


@pytest.mark.parametrize("n", [11, 16, 23])
def test_multi_step_graphs_equal_eager_bit_exact(ry, n):
    """Runs that use the multi-step graphs (11 = 8 + 2 + 1 steps, 16 = one
    16-step graph, 23 = 16 + 4 + 2 + 1) give the eager result bit for bit,
    and so does a run whose t_end falls inside a multi-step graph."""
    prob = cases.amr_blob(level_min=3, level_max=4)
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    a.set_timing(True)
    a.advance(n)
    b.advance(n)
    assert a.t == b.t
    for lv in a.levels:
        np.testing.assert_array_equal(a.download(lv), b.download(lv))
    t_end = 0.6 * a.t
    c, d = ry.Hydro(prob), ry.Hydro(prob)
    c.set_timing(True)
    c.advance(n, t_end)
    d.advance(n, t_end)
    assert c.t == d.t == t_end
    for lv in c.levels:
        np.testing.assert_array_equal(c.download(lv), d.download(lv))


@pytest.mark.parametrize("n_coarse", [19, 1001])
def test_sod_t_end_with_odd_skipped_steps(ry, n_coarse):
    """t_end is reached after 18 steps: the remaining n_coarse - 18 steps
    (odd here) are skipped on the device, and the state returned is the one
    at t_end, on the graph path and on the eager path."""
    prob = W.sod(32)
    o = Oracle(prob)
    n = o.advance(n_coarse, prob.t_end)
    assert (n_coarse - n) % 2 == 1
    for eager in (False, True):
        g = ry.Hydro(prob)
        g.set_timing(eager)
        g.advance(n_coarse, prob.t_end)
        assert g.t == o.t == prob.t_end
        compare_levels(g, o)


@pytest.mark.parametrize("n_coarse", [11, 16])
def test_amr_t_end_inside_graph_matches_oracle(ry, n_coarse):
    """AMR run whose t_end falls inside a multi-step graph with an odd number
    of steps left over; then further steps continue from the right buffers."""
    prob = cases.amr_blob(level_min=3, level_max=4)
    probe = Oracle(prob)
    probe.advance(n_coarse)
    t_full = probe.t
    # pick a t_end that leaves an odd number of the n_coarse steps unused
    for frac in (0.45, 0.5, 0.55, 0.6, 0.65, 0.7, 0.75):
        o = Oracle(prob)
        k = o.advance(n_coarse, frac * t_full)
        if (n_coarse - k) % 2 == 1:
            break
    assert (n_coarse - k) % 2 == 1
    t_end = frac * t_full
    for eager in (False, True):
        g = ry.Hydro(prob)
        g.set_timing(eager)
        g.advance(n_coarse, t_end)
        assert g.t == t_end
        compare_levels(g, o)
    o.advance(3)
    g.advance(3)
    compare_levels(g, o)


def test_amr_eager_timing_equals_graph_bit_exact(ry):
    prob = cases.amr_blob(level_min=3, level_max=4)
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    a.set_timing(True)
    a.advance(3)
    b.advance(3)
    n, ms = a.kernel_time("hydro")
    assert n == 3 * 3 and ms > 0
    for lv in a.levels:
        np.testing.assert_array_equal(a.download(lv), b.download(lv))


def test_twolevel_small_advance(ry):
    prob = W.twolevel(32, 0.5)
    g, o = ry.Hydro(prob), Oracle(prob)
    assert g.level_info(5)[0] > 0
    g.advance(3)
    o.advance(3)
    compare_levels(g, o)


# ------------------------------------------------------------- invariants
def test_uniform_state_bit_exact(ry):
    for prob in (W.uniform_state(8), cases.analytic_problem(
            "amr_uniform", 3, 5,
            lambda pos: (np.full(len(pos), 1.3), np.full(len(pos), 0.3), np.full(len(pos), -0.2),
                         np.full(len(pos), 0.1), np.full(len(pos), 0.7)), rho_thr=1.0)):
        for prec in ("fp64", "mixed"):
            g = ry.Hydro(prob, prec)
            before = [g.download(lv) for lv in g.levels]
            g.advance(3)
            for lv, U0 in zip(g.levels, before):
                np.testing.assert_array_equal(g.download(lv), U0)


def test_stationary_contact_bit_exact(ry):
    def state(pos):
        d = pos - 0.5
        rho = 1.0 + 30.0 * np.exp(-(d * d).sum(1) / 0.01) + 0.5 * np.sin(6.28 * pos[:, 1])
        z = np.zeros(len(pos))
        return rho, z, z, z, np.full(len(pos), 2.0)
    prob = cases.analytic_problem("contact_amr", 3, 5, state, rho_thr=2.0)
    g = ry.Hydro(prob)
    before = [g.download(lv) for lv in g.levels]
    g.advance(3)
    for lv, U0 in zip(g.levels, before):
        np.testing.assert_array_equal(g.download(lv), U0)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_conservation(ry, prec):
    for prob in (W.random_smooth(16, seed=5, mach=1.2), cases.amr_blob()):
        g = ry.Hydro(prob, prec)
        t0 = g.totals()
        o = Oracle(prob)
        np.testing.assert_allclose(t0, o.totals(), rtol=1e-13, atol=1e-13 * np.abs(t0).max())
        msum = sum(np.abs(g.download(lv)[1:4]).sum() * (1.0 / (prob.nbase[0] << (lv - prob.level_min))) ** 3
                   for lv in g.levels)
        g.advance(4)
        t1 = g.totals()
        assert abs(t1[0] - t0[0]) <= 1e-13 * abs(t0[0])
        assert abs(t1[4] - t0[4]) <= 1e-13 * abs(t0[4])
        for v in (1, 2, 3):
            assert abs(t1[v] - t0[v]) <= 1e-13 * msum


# ---------------------------------------------------- scheduling invariance
def test_tuning_invariance_bit_exact(ry):
    prob = cases.amr_blob()
    ref = None
    for t in ([1, 0, 4, 1, 4], [1, 0, 4, 1, 1], [2, 0, 4, 1, 1], [2, 0, 4, 1, 2], [1, 0, 4, 1, 2],
              [4, 0, 4, 1, 1], [1, 1, 16, 1, 4], [2, 1, 8, 4, 1], [4, 1, 8, 2, 1], [1, 1, 2, 2, 2]):
        g = ry.Hydro(prob)
        g.set_tuning(*t)
        g.advance(2)
        out = [g.download(lv) for lv in g.levels]
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)


def test_repeat_runs_bit_identical(ry):
    prob = W.random_smooth(16, seed=8)
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    a.advance(4)
    b.advance(4)
    np.testing.assert_array_equal(a.download(4), b.download(4))


def test_autotune_keeps_state_and_results(ry):
    prob = cases.amr_blob()
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    best, times = a.autotune()
    assert len(times) >= 4 and all(t > 0 for t in times)
    a.advance(2)
    b.advance(2)
    for lv in a.levels:
        np.testing.assert_array_equal(a.download(lv), b.download(lv))


# ------------------------------------------------------------ mixed form
def test_mixed_form_error_budget(ry):
    prob = W.uniform(32, n_steps=10)
    f, m = ry.Hydro(prob, "fp64"), ry.Hydro(prob, "mixed")
    f.advance(10)
    m.advance(10)
    rf, rm = f.download(5)[0], m.download(5)[0]
    l1 = np.abs(rm - rf).sum() / np.abs(rf).sum()
    assert l1 <= 1e-5, l1
    assert m.floors() == 0


# ------------------------------------------------------------------ batch
def test_batch_equals_single_box_runs(ry):
    boxes = [W.batch_box(0, 16, 1.0, 2.0), W.batch_box(1, 24, 0.7, 0.6), W.batch_box(2, 8, 1.4, 2.5),
             W.batch_box(3, 40, 0.5, 1.0)]
    bh = ry.BatchHydro(boxes)
    bh.run(5)
    for b, p in enumerate(boxes):
        s = ry.Hydro(p)
        s.advance(5)
        np.testing.assert_array_equal(bh.download(b), s.download(p.level_min))
        o = Oracle(p)
        o.advance(5)
        assert cases.rel_err(bh.download(b), o.download(p.level_min)) <= TOL
        assert abs(bh.box_info(b)[1] - o.t) <= 1e-14 * o.t


# ----------------------------------------------------------- error paths
def test_order_rule_enforced(ry):
    prob = cases.amr_blob()
    g = ry.Hydro(prob)
    dt = g.cfl_dt()
    with pytest.raises(ry.RyError) as e:
        g.hydro_step(3, dt)                      # finer levels have not stepped
    assert e.value.code == ry.RY_ESTATE
    g.hydro_step(5, dt / 4)
    with pytest.raises(ry.RyError) as e:
        g.hydro_step(5, dt / 8)                  # second substep with another dt
    assert e.value.code == ry.RY_EINVAL
    g.hydro_step(5, dt / 4)
    with pytest.raises(ry.RyError) as e:
        g.hydro_step(5, dt / 4)                  # a third substep
    assert e.value.code == ry.RY_ESTATE
    with pytest.raises(ry.RyError) as e:
        g.advance(1)                             # inside a coarse step
    assert e.value.code == ry.RY_ESTATE


def test_numeric_fault_latched(ry):
    prob = W.random_smooth(8, seed=2)
    g = ry.Hydro(prob)
    U = g.download(3)
    U[0, 17] = np.nan
    g.upload(3, U)
    with pytest.raises(ry.RyError) as e:
        g.cfl_dt()
    assert e.value.code == ry.RY_ENUMERIC


# ------------------------------------------------------- full-size cases
def test_uniform128_full_size_config_steps(ry):
    """The 128^3 box over its configuration's 10 steps (each side with its
    own dt), checked after the first step and accumulated after the tenth."""
    prob = W.uniform(128)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(1)
    o.advance(1)
    compare_levels(g, o)
    g.advance(prob.n_steps - 1)
    o.advance(prob.n_steps - 1)
    assert abs(g.t - o.t) <= 1e-13 * o.t
    compare_levels(g, o)


def test_twolevel128_full_size_config_steps(ry):
    """The two-level mesh (theta 0.70) over its 10 coarse steps."""
    prob = W.twolevel(128, 0.70)
    g, o = ry.Hydro(prob), Oracle(prob)
    assert g.level_info(7)[0] == 65018
    g.advance(1)
    o.advance(1)
    compare_levels(g, o)
    g.advance(prob.n_steps - 1)
    o.advance(prob.n_steps - 1)
    assert abs(g.t - o.t) <= 1e-13 * o.t
    compare_levels(g, o)


def test_batch_tunings_bit_exact(ry):
    """The batched launch is independent of its tuning: the plain launch and
    the persistent queue-fed kernel (several grid sizes, queue batches and
    waves per tile) give bit-identical boxes, and the autotuner leaves the
    state untouched."""
    boxes = [W.batch_box(4, 16, 1.2, 1.5), W.batch_box(5, 32, 0.8, 2.0), W.batch_box(6, 24, 1.0, 0.5)]
    ref = None
    for t in ([1, 0, 4, 1, 1], [1, 1, 14, 4, 2], [1, 1, 8, 1, 1], [2, 1, 20, 4, 1], [1, 0, 4, 1, 4], None):
        bh = ry.BatchHydro(boxes)
        if t is None:
            best, times = bh.autotune()
            assert len(times) >= 4 and all(x > 0 for x in times)
            assert bh.tuning() == best
        else:
            bh.set_tuning(*t)
        bh.run(3)
        out = [bh.download(b) for b in range(len(boxes))]
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)
        bh.close()


def test_batch512_full_size_sampled_boxes(ry):
    """All 512 uneven boxes advanced together 20 steps; 16 boxes spread over
    the list are recomputed one by one by the oracle."""
    boxes = W.batch(512)
    for prec in ("fp64",):
        bh = ry.BatchHydro(boxes, prec)
        bh.run(20)
        for b in range(0, 512, 32):
            o = Oracle(boxes[b])
            o.advance(20)
            assert cases.rel_err(bh.download(b), o.download(1)) <= TOL, b
            assert abs(bh.box_info(b)[1] - o.t) <= 1e-13 * o.t


# ------------------------------------------------ failure paths, checkpoints
class _FailingMemory:
    """dev_alloc hook that succeeds `budget` times, then returns NULL."""

    def __init__(self, ry, budget):
        import torch
        self.live = {}
        self.calls = 0

        def alloc(nbytes, user):
            self.calls += 1
            if self.calls > budget:
                return None
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def free(p, user):
            self.live.pop(p, None)

        self.alloc_cb = ry.ALLOC_FN(alloc)
        self.free_cb = ry.FREE_FN(free)


def test_allocation_failure_reports_enomem_and_frees(ry):
    prob = cases.amr_blob()
    for budget in (0, 3, 12):
        mem = _FailingMemory(ry, budget)
        with pytest.raises(ry.RyError) as e:
            ry.Hydro(prob, memory=mem)
        assert e.value.code == ry.RY_ENOMEM
        assert not mem.live          # every successful allocation was released
    ok = ry.Hydro(prob)              # the library still works afterwards
    ok.advance(1)


def test_checkpoint_resume_bit_exact(ry):
    prob = cases.amr_blob()
    full = ry.Hydro(prob)
    full.advance(4)
    a = ry.Hydro(prob)
    a.advance(2)
    saved = [a.download(lv) for lv in a.levels]
    t_saved = a.t
    b = ry.Hydro(prob)
    for lv, U in zip(b.levels, saved):
        b.upload(lv, U)
    b.t = t_saved
    b.advance(2)
    for lv in full.levels:
        np.testing.assert_array_equal(b.download(lv), full.download(lv))


def test_amr_with_empty_refinement_equals_single_level(ry):
    base = W.random_smooth(16, seed=12)
    amr = W.Problem("unref", 4, 6, (16, 16, 16), base.gamma, base.U_base, refine=W.REFINE_MASS,
                    refine_param=1e30, fill=lambda l, ijk: np.zeros((5, len(ijk))))
    g, s = ry.Hydro(amr), ry.Hydro(base)
    assert g.level_info(5)[0] == 0 and g.level_info(6)[0] == 0
    g.advance(3)
    s.advance(3)
    np.testing.assert_array_equal(g.download(4), s.download(4))


@pytest.mark.parametrize("n_fine,theta", [(64, 0.5), (128, 0.70)])
def test_floor_census_equals_oracle(ry, n_fine, theta):
    """Floor activations counted once per event of a step (a leaf cell's own
    conversion, each used face's states, each ghost cell per parent step):
    the GPU's count equals the oracle's on the two-level meshes, whose
    interpolated ghost cells can have less total energy than kinetic energy,
    with either tile shape, on the graph path and host-driven."""
    prob = W.twolevel(n_fine, theta)
    o = Oracle(prob)
    o.advance(2)
    assert o.floors() > 0
    for t in ([1, 0, 4, 1, 1, 4], [1, 0, 4, 1, 2, 4], [1, 0, 4, 1, 8, 8]):
        g = ry.Hydro(prob)
        g.set_tuning(*t)
        g.advance(2)
        assert g.floors() == o.floors(), (t, g.floors(), o.floors())
    h, o1 = ry.Hydro(prob), Oracle(prob)
    step_both(h, o1, 1)
    assert h.floors() == o1.floors() > 0


def test_floor_census_equals_oracle_deep_hierarchy(ry):
    """The census on a four-level zoom mesh (32^3 base, levels 5-8), where a
    ghost oct's covering leaf can sit two or more levels up: after 12 coarse
    steps the GPU counts what the oracle counts, on both tile shapes, and
    the states agree at the parity bar."""
    prob = W.zoom(level_min=5, level_max=8)
    o = Oracle(prob)
    o.advance(12)
    assert o.floors() > 0
    for t in ([1, 0, 4, 1, 1, 4], [1, 0, 4, 1, 8, 8]):
        g = ry.Hydro(prob)
        g.set_tuning(*t)
        g.advance(12)
        assert g.floors() == o.floors(), (t, g.floors(), o.floors())
        for lv in g.levels:
            assert cases.rel_err(g.download(lv), o.download(lv)) <= 1e-12, (t, lv)
