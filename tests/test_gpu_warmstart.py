"""Training pipeline of the learned warm start: labels are the plain
RTG-GMRES solutions (spot-checked against the float64 oracle), and a few
training steps on them reduce the loss."""
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.operator import Operator, make_observation
from oracle.sketch import Sketch
from oracle.gmres import rtg_gmres
import _util as U

pytestmark = pytest.mark.gpu


def test_labels_are_plain_solver_solutions_and_training_learns():
    import torch
    from paper_2603_00839_amd import rtg, warmstart
    print("[case] warm-start pipeline, 16 pairs", file=sys.stderr, flush=True)
    C_all, Y_all, iters = warmstart.make_pairs(None, 16, seed=3, chunk=8, log=lambda s: None)
    assert all(i == 50 for i in iters)
    for p in (0, 11):
        pr = synth.cfg5_problem(3, p)
        op, sk = Operator(pr.a1_band, pr.a2_band, pr.b_band), Sketch(pr.om1, pr.om2, pr.om3)
        C = synth.from_device_layout(C_all[p].cpu().numpy()).astype(np.float64)
        # the same C (formed on the GPU) and delta = nu ||Phi(X)|| from the oracle
        _, delta, _ = make_observation(op, pr.x_true, pr.noise_dir, pr.nu)
        ref = rtg_gmres(op, sk, C, 50, delta=delta, eta=1.01)
        X = synth.from_device_layout(Y_all[p].cpu().numpy())
        assert U.rel(X, ref.X) < 2e-4
    net = rtg.WarmStartNet(warmstart.initial_params(0))
    losses = [float(net.train_step(C_all[:8].contiguous(), Y_all[:8].contiguous(), 2e-3).item()) for _ in range(40)]
    assert losses[-1] < losses[0]
