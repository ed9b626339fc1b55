"""Batched solves through the C ABI: every instance of a batch must compute
exactly what it computes alone (DET schedule: same classes, same order,
same kernels), whatever the launch configuration the tuner picks."""
import sys

import numpy as np
import pytest

from paper_1311_2661_amd import instances as I

pytestmark = pytest.mark.gpu
T = None


def setup_module(module):
    global T
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_2661_amd import thetis as TT
    T = TT
    torch.cuda.set_device(0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mixed_instances():
    return [I.vc_er(300, 1200, seed=1), I.vc_ba(5000, seed=2), I.mis_regular(800, 7, seed=3),
            I.vc_er(40, 90, seed=4), I.mis_regular(2000, 16, seed=5), I.vc_ba(20000, seed=6)]


def pair(insts, **kw):
    a = [T.Solver(T.Instance(x), seed=10 + k, **kw) for k, x in enumerate(insts)]
    b = [T.Solver(T.Instance(x), seed=10 + k, **kw) for k, x in enumerate(insts)]
    return a, b


def assert_same(sa, sb):
    ya, yb = sa.y, sb.y
    assert np.array_equal(ya, yb), np.abs(ya - yb).max()
    ma, mb = sa.metrics(), sb.metrics()
    for k in ("F", "lp_value", "dual_bound", "linf", "max_viol"):
        assert ma[k] == mb[k], k


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16"])
def test_batch_equals_alone_fixed_epochs(prec):
    say(f"case batch vs alone {prec}")
    p = dict(fp32=None, fp64=None, bf16=None)
    precision = {"fp32": T.PREC_FP32, "fp64": T.PREC_FP64, "bf16": T.PREC_BF16X}[prec]
    alone, batched = pair(mixed_instances(), precision=precision)
    for s in alone:
        s.run(23)
    b = T.Batch(batched)
    done = b.run(23)
    assert list(done) == [23] * len(batched)
    for sa, sb in zip(alone, batched):
        assert sb.epoch == 23
        assert_same(sa, sb)


@pytest.mark.parametrize("kind", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_alone_on_mixed_lps(kind, prec):
    """General LPs of mixed shape (instances.mixed_lp: all three senses,
    zero / finite / infinite bounds, a column of more than 64 entries), one
    batch per way of storing the values (all 1, +-1, general)."""
    say(f"case batch vs alone, mixed LPs kind {kind} {prec}")
    precision = {"fp32": T.PREC_FP32, "fp64": T.PREC_FP64}[prec]
    alone, batched = pair([I.mixed_lp(kind + 3 * t) for t in range(4)], beta=4.0, precision=precision)
    for s in alone:
        s.run(17)
    done = T.Batch(batched).run(17)
    assert list(done) == [17] * len(batched)
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)


def test_batch_gap_stop_per_instance():
    say("case batch gap stop")
    insts = [I.vc_er(200, 800, seed=7), I.mis_regular(600, 4, seed=8), I.vc_ba(3000, seed=9)]
    alone, batched = pair(insts)
    ref = [s.run(2000, gap_tol=1e-4) for s in alone]
    done = T.Batch(batched).run(2000, gap_tol=1e-4)
    say(f"  epochs alone {ref} batched {list(done)}")
    assert list(done) == ref
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)
        assert sb.metrics()["gap"] <= 1e-4 + 1e-12


def test_batch_multiway_cut_blocks():
    say("case batch multiway cut")
    insts = [I.mc_grid(side=12, k=4, seed=1), I.mc_grid(side=20, k=8, seed=2), I.mc_grid(side=7, k=3, seed=3)]
    alone, batched = pair(insts)
    for s in alone:
        s.run(17)
    T.Batch(batched).run(17)
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)


@pytest.mark.parametrize("widen,grid,strided,cols", [(1, 1, 1, 1), (2, 4, 0, 1), (4, 8, 1, 1), (1, 8, 0, 1),
                                                     (1, 2, 1, 2), (1, 1, 0, 4), (2, 2, 1, 4), (4, 1, 1, 4),
                                                     (1, 0, 1, 4), (1, 0, 0, 1)])
def test_batch_launch_configuration_does_not_change_results(widen, grid, strided, cols):
    insts = mixed_instances()[:4]
    alone, batched = pair(insts)
    for s in alone:
        s.run(12)
    b = T.Batch(batched)
    b.configure(widen, grid, strided, cols)
    b.run(12)
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)


def test_batch_autotune_and_continue():
    say("case batch autotune")
    insts = mixed_instances()
    alone, batched = pair(insts)
    b = T.Batch(batched)
    w, g, st, c = b.autotune(epochs_per_candidate=2)
    assert w in (1, 2) and g in (0, 1, 2, 4) and st in (0, 1) and c in (1, 2, 4)
    ran = batched[0].epoch            # the tuner's epochs are real epochs
    b.run(10)
    for sa in alone:
        sa.run(ran + 10)
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)


@pytest.mark.parametrize("window", [1, 2, 5])
def test_batch_window_equals_alone(window):
    """With a window, waiting instances start on the device as others
    retire; each still computes exactly its solo trajectory, and the batch
    runs until every instance has retired."""
    say(f"case batch window {window}")
    insts = [I.vc_er(200, 800, seed=7), I.mis_regular(600, 4, seed=8), I.vc_ba(3000, seed=9),
             I.vc_er(40, 90, seed=4), I.mis_regular(900, 9, seed=5), I.vc_er(300, 1200, seed=1)]
    alone, batched = pair(insts)
    ref = [s.run(300, gap_tol=1e-4) for s in alone]
    b = T.Batch(batched)
    b.set_window(window)
    done = b.run(300, gap_tol=1e-4)
    say(f"  epochs alone {ref} batched {list(done)}")
    assert list(done) == ref
    assert all(int(v) in (1, 2) for v in b.last_status)
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)


def test_batch_window_fixed_epochs():
    """Without a gap every instance runs exactly max_epochs, in turns."""
    insts = mixed_instances()[:5]
    alone, batched = pair(insts)
    for s in alone:
        s.run(11)
    b = T.Batch(batched)
    b.set_window(2)
    done = b.run(11)
    assert list(done) == [11] * 5
    for sa, sb in zip(alone, batched):
        assert_same(sa, sb)


def test_batch_many_uneven_instances():
    """256 independent-set instances of uneven size and degree, as in the
    batched workload, against solo runs of a sample."""
    say("case batch 256 uneven")
    rng = np.random.default_rng(0)
    insts = [I.mis_regular(int(rng.integers(200, 3000)), int(rng.integers(3, 17)), seed=100 + k)
             for k in range(256)]
    batched = [T.Solver(T.Instance(x), seed=k) for k, x in enumerate(insts)]
    done = T.Batch(batched).run(40, gap_tol=1e-4)
    for k in rng.choice(256, 6, replace=False):
        s = T.Solver(T.Instance(insts[k]), seed=int(k))
        e = s.run(40, gap_tol=1e-4)
        assert e == done[k]
        assert_same(s, batched[k])
        s.round(T.ROUND_MIS_THRESH)
        assert s.check(T.ROUND_MIS_THRESH) == (True, 0)


def test_solver_in_a_batch_cannot_be_destroyed():
    sa = T.Solver(T.Instance(I.vc_er(300, 1200, seed=1)))
    sb = T.Solver(T.Instance(I.vc_er(200, 700, seed=2)))
    b = T.Batch([sa, sb])
    with pytest.raises(T.ThetisError) as e:
        sa.close()
    assert e.value.code == T.EBUSY
    b.set(0, None)
    sa.close()                                # the slot is empty now
    assert list(b.run(3)) == [0, 3]
    b.set(0, sb)                              # one solver in two slots
    b.set(1, None)
    with pytest.raises(T.ThetisError):
        sb.close()
    b.close()
    sb.close()


def test_batch_rejects_mixed_kinds():
    a = T.Solver(T.Instance(I.vc_er(50, 100, seed=1)), precision=T.PREC_FP32)
    b = T.Solver(T.Instance(I.vc_er(50, 100, seed=2)), precision=T.PREC_FP64)
    with pytest.raises(T.ThetisError):
        T.Batch([a, b])
    c = T.Solver(T.Instance(I.vc_er(50, 100, seed=3)), schedule=T.SCHED_ASYNC)
    with pytest.raises(T.ThetisError):
        T.Batch([a, c])
    d = T.Solver(T.Instance(I.mc_grid(side=5, k=3, seed=1)))
    with pytest.raises(T.ThetisError):
        T.Batch([a, d])


def test_batch_run_lengths_around_the_graph_period():
    """One captured graph runs several epochs (the refresh period): runs of
    0 epochs, fewer than, exactly and more than a period, one after another
    on the same batch, leave every instance where the same runs alone do."""
    say("case batch run lengths 0, 3, 5, 7, 13")
    insts = mixed_instances()[:4]
    alone, batched = pair(insts, precision=T.PREC_FP64, refresh_every=5)
    b = T.Batch(batched)
    total = 0
    for n in (0, 3, 5, 7, 13):
        done = b.run(n)
        assert list(done) == [n] * len(batched)
        for s in alone:
            s.run(n)
        total += n
        for sa, sb in zip(alone, batched):
            assert sb.epoch == total
            assert np.array_equal(sa.y, sb.y)


def test_batch_with_a_hub_past_the_lds_tile():
    """A 5000-entry hub column (its scatter re-reads the entries past the
    2048-entry LDS tile) batched with ordinary instances: every instance
    equals its solve alone, bit for bit (FP32 and FP64)."""
    say("case batch with a hub past the LDS tile")
    rng = np.random.default_rng(31)
    n = 5001
    star = np.stack([np.zeros(n - 1, np.int64), np.arange(1, n, dtype=np.int64)], axis=1)
    extra = rng.integers(1, n, (8000, 2))
    extra = extra[extra[:, 0] != extra[:, 1]]
    edges = np.unique(np.sort(np.concatenate([star, extra]), axis=1), axis=0)
    hub = I.vc_lp(n, edges, rng.uniform(1, 10, n))
    for prec in (T.PREC_FP32, T.PREC_FP64):
        insts = [hub, I.vc_ba(5000, seed=2), I.mis_regular(800, 7, seed=3)]
        alone, batched = pair(insts, precision=prec)
        for s in alone:
            s.run(17)
        done = T.Batch(batched).run(17)
        assert list(done) == [17] * len(insts)
        for sa, sb in zip(alone, batched):
            assert_same(sa, sb)
