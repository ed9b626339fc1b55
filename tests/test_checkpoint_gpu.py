"""Checkpoint and resume (thetis_solver_save / thetis_solver_load): in the
DET schedule, 25 epochs, save, load into a fresh solver and 25 more epochs
give bit for bit the same state as 50 epochs in one solver, also across
multiplier steps (ubar, shifted costs, beta, prox centre) and with simplex
blocks; mismatched checkpoints are refused."""
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


@pytest.mark.parametrize("maker,precision", [(lambda: I.vc_er(5000, 20000, seed=3), "fp32"),
                                             (lambda: I.vc_er(2000, 8000, seed=4), "bf16"),
                                             (lambda: I.mc_grid(side=32, k=4, seed=2), "fp32"),
                                             (lambda: I.mis_regular(3000, 5, seed=5), "fp64")])
def test_save_load_resumes_bit_for_bit(maker, precision):
    inst = maker()
    prec = {"fp32": T.PREC_FP32, "fp64": T.PREC_FP64, "bf16": T.PREC_BF16X}[precision]
    h = T.Instance(inst)
    a = T.Solver(h, precision=prec, seed=7)
    a.run(25)
    blob = a.save()
    a.run(25)
    b = T.Solver(h, precision=prec, seed=7)
    b.load(blob)
    assert b.epoch == 25
    b.run(25)
    assert np.array_equal(a.y, b.y)
    ma, mb = a.metrics(), b.metrics()
    assert ma["F"] == mb["F"] and ma["dual_bound"] == mb["dual_bound"]


@pytest.mark.parametrize("prox", [False, True])
def test_resume_across_multiplier_steps(prox):
    inst = I.vc_er(3000, 12000, seed=6)
    yb = np.zeros(inst.n + inst.m) if prox else None
    h = T.Instance(inst)

    def solver():
        return T.Solver(h, beta=5.0, prox=prox, ybar=yb, ubar=np.zeros(inst.m), seed=6)

    a = solver()
    a.run(10)
    a.multiplier_step(move_centre=prox, beta=20.0)
    a.run(5)
    blob = a.save()
    a.run(10)
    sa = a.multiplier_step(move_centre=prox)
    b = solver()
    b.load(blob)
    b.run(10)
    sb = b.multiplier_step(move_centre=prox)
    assert np.array_equal(a.y, b.y)
    assert np.array_equal(a.ubar, b.ubar)
    assert sa["lp_value"] == sb["lp_value"] and sa["lp_dual"] == sb["lp_dual"]
    if prox:
        assert np.array_equal(a.ybar, b.ybar)
    # a reset after the load returns to the creation values
    b.reset()
    assert np.all(b.ubar == 0.0)


def test_mismatched_checkpoints_are_refused():
    h1 = T.Instance(I.vc_er(500, 1500, seed=1))
    h2 = T.Instance(I.vc_er(600, 1500, seed=1))
    h3 = T.Instance(I.vc_er(500, 1500, seed=2))       # same sizes, other edges and costs
    a = T.Solver(h1)
    a.run(3)
    blob = a.save()
    for other in (T.Solver(h2), T.Solver(h3), T.Solver(h1, precision=T.PREC_FP64),
                  T.Solver(h1, ubar=np.zeros(1500))):
        with pytest.raises(T.ThetisError) as e:
            other.load(blob)
        assert e.value.code == T.EINVAL
    with pytest.raises(T.ThetisError):
        T.Solver(h1).load(blob[:-4])
    with pytest.raises(T.ThetisError):
        T.Solver(h1).load(b"x" * len(blob))
    # a checkpoint stores y and r in the internal row and column order, and
    # records a digest of it (bytes 64..71 of the header): another layout is
    # refused
    other_layout = bytearray(blob)
    other_layout[64] ^= 0xFF
    with pytest.raises(T.ThetisError) as e:
        T.Solver(h1).load(bytes(other_layout))
    assert e.value.code == T.EINVAL and "layout" in str(e.value)
